"""Pins of the oracle's lattice Boltzmann part (Sec. II A, Guo forcing, App. C walls) against
conservation laws and closed-form flows."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_14889_amd import workload as wl
from tests.helpers import oracle_sim

FLUID_ONLY = dict(ericksen=0, polymer_force=0, evolve_sigma=0, evolve_P=0)


def _momentum(h):
    return np.array([np.tensordot(oracle.CX, h, axes=(0, 0)).sum(),
                     np.tensordot(oracle.CY, h, axes=(0, 0)).sum()])


def test_mass_conserved_in_coupled_run():
    w = wl.small_case(21, 40, 36, n_bodies=2, radius=4.0)
    s = oracle_sim(w.sims[0])
    m0 = s.h.sum()
    s.run(60)
    assert abs(s.h.sum() / m0 - 1.0) < 1e-13


def test_momentum_grows_by_total_external_force():
    # Guo forcing adds exactly F per site per step; divergence forces telescope on the periodic
    # lattice, internal body forces cancel and the kernel sums to one, so the total momentum
    # grows by exactly the total pull every step
    w = wl.small_case(22, 40, 36, n_bodies=2, radius=4.0, pull=3e-4)
    s = oracle_sim(w.sims[0])
    s.run(5)
    pull = np.sum([b.pull for b in s.bodies], axis=0)
    for _ in range(4):
        obs = s.observe()
        F = np.array([obs["Fx"].sum(), obs["Fy"].sum()])
        assert np.max(np.abs(F - pull)) < 1e-15
        m0 = _momentum(s.h)
        s.run(1)
        assert np.max(np.abs(_momentum(s.h) - m0 - pull)) < 1e-14


def test_shear_wave_decay_gives_viscosity():
    # nu = cs^2 (tau - 1/2) (Sec. II A): a transverse wave u_x = U sin(k y) decays as exp(-nu k^2 t)
    n, tau, U = 64, 0.8, 1e-4
    y = np.arange(n)
    ux = np.broadcast_to((U * np.sin(2 * np.pi * y / n))[:, None], (n, 4)).copy()
    rho = np.ones((n, 4))
    h = oracle.equilibrium(rho, ux, np.zeros_like(ux))
    s = oracle.Sim(dict(nx=4, ny=n, tau=tau, **FLUID_ONLY), h=h)
    s.run(100)
    a1 = (s.observe()["vx"][:, 0] * np.sin(2 * np.pi * y / n)).sum()
    s.run(400)
    a2 = (s.observe()["vx"][:, 0] * np.sin(2 * np.pi * y / n)).sum()
    k = 2 * np.pi / n
    nu = -math.log(a2 / a1) / (400 * k * k)
    assert abs(nu / ((tau - 0.5) / 3.0) - 1.0) < 2e-3


def test_poiseuille_between_bounce_back_walls():
    # body-force-driven channel between halfway bounce-back walls at y = -1/2 and y = H - 1/2
    # (App. C: Dirichlet zero-velocity walls by bounce-back).  At tau = 1/2 + sqrt(3)/4 the
    # halfway wall sits exactly mid-link for BGK and the parabola is reproduced to round-off.
    H, g = 16, 1e-6
    tau = 0.5 + math.sqrt(3.0) / 4.0
    s = oracle.Sim(dict(nx=2, ny=H, tau=tau, walls=1, gx=g, **FLUID_ONLY))
    s.run(12000)
    vx = s.observe()["vx"][:, 0]
    nu = (tau - 0.5) / 3.0
    y = np.arange(H)
    ref = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    assert np.max(np.abs(vx - ref)) / ref.max() < 1e-9


def test_poiseuille_second_order_at_other_tau():
    tau, g = 0.8, 1e-6
    errs = []
    for H in (8, 16, 32):
        s = oracle.Sim(dict(nx=2, ny=H, tau=tau, walls=1, gx=g, **FLUID_ONLY))
        s.run(int(12 * H * H / ((tau - 0.5) / 3.0) / 10))
        vx = s.observe()["vx"][:, 0]
        nu = (tau - 0.5) / 3.0
        y = np.arange(H)
        ref = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
        errs.append(np.max(np.abs(vx - ref)) / ref.max())
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(order) > 1.8, (errs, order)


def test_rest_state_is_stationary():
    s = oracle.Sim(dict(nx=8, ny=8, **FLUID_ONLY))
    h0 = s.h.copy()
    s.run(10)
    assert np.max(np.abs(s.h - h0)) < 1e-15


# --- the closed box (walls on all four sides) -----------------------------------------------

# D2Q9 directions under the reflection x <-> y: c_n = (cx, cy) -> (cy, cx)
TRANSPOSE_DIR = [0, 2, 1, 4, 3, 5, 8, 7, 6]


def _box_state(seed, n):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal((n, n))
    ux, uy = 0.01 * rng.standard_normal((2, n, n))
    h = oracle.equilibrium(rho, ux, uy)
    sigma = 1e-4 * rng.standard_normal((3, n, n))
    th = rng.uniform(0, math.pi, (n, n))
    P = 0.9 * np.stack([np.cos(th), np.sin(th)])
    R = oracle.polygon(n / 2 + 0.3, n / 2 - 0.7, 4.0, 25) + 0.1 * rng.standard_normal((25, 2))
    return h, sigma, P, R


def _transpose_state(h, sigma, P, R):
    hT = np.empty_like(h)
    for q in range(9):
        hT[TRANSPOSE_DIR[q]] = h[q].T
    sT = np.stack([sigma[1].T, sigma[0].T, sigma[2].T])
    PT = np.stack([P[1].T, P[0].T])
    return hT, sT, PT, R[:, ::-1].copy()


@pytest.mark.parametrize("walls", [2, 0])
def test_reflection_across_the_diagonal(walls):
    """x <-> y reflection covariance of the whole coupled step (the aligned stiffness is even in
    y, so the law is covariant): the reflected initial state gives the reflected fields.  With
    walls = 2 this pins the x-walls against the y-walls."""
    n = 24
    h, sigma, P, R = _box_state(5, n)
    hT, sT, PT, RT = _transpose_state(h, sigma, P, R)
    par = dict(nx=n, ny=n, walls=walls, D_p=0.02, eta_p=2.0, gx=3e-6, gy=-1e-6)
    parT = dict(par, gx=-1e-6, gy=3e-6)
    bA = oracle.Body(R=R, k_spring=0.05, eps_angle=0.01, l_eq=1.0, pull=(2e-4, 1e-4))
    bB = oracle.Body(R=RT, k_spring=0.05, eps_angle=0.01, l_eq=1.0, pull=(1e-4, 2e-4))
    a = oracle.Sim(par, bodies=[bA], h=h, sigma=sigma, P=P).run(30)
    b = oracle.Sim(parT, bodies=[bB], h=hT, sigma=sT, P=PT).run(30)
    oa, ob = a.observe(), b.observe()
    assert np.max(np.abs(ob["vx"] - oa["vy"].T)) < 1e-15 + 1e-12 * np.abs(oa["vy"]).max()
    assert np.max(np.abs(ob["vy"] - oa["vx"].T)) < 1e-15 + 1e-12 * np.abs(oa["vx"]).max()
    assert np.max(np.abs(b.sigma[0] - a.sigma[1].T)) < 1e-12 * np.abs(a.sigma).max()
    assert np.max(np.abs(b.sigma[2] - a.sigma[2].T)) < 1e-12 * np.abs(a.sigma).max()
    assert np.max(np.abs(b.P[0] - a.P[1].T)) < 1e-12
    assert np.max(np.abs(bB.R - bA.R[:, ::-1])) < 1e-12


def test_box_conserves_mass():
    n = 20
    h, sigma, P, R = _box_state(6, n)
    s = oracle.Sim(dict(nx=n, ny=n, walls=2, gx=1e-5), bodies=[oracle.Body(R=R, pull=(1e-4, 0.0))],
                   h=h, sigma=sigma, P=P)
    m0 = s.h.sum()
    s.run(50)
    assert abs(s.h.sum() - m0) < 1e-12 * m0
