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
