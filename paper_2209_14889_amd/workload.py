"""Seeded synthetic workloads shaped like the paper's simulations (arXiv 2209.14889).

This module produces INPUTS only: lattice sizes, coefficients, initial polarization fields and
immersed-body node sets.  It holds none of the method's arithmetic and serves both the GPU
library and the CPU oracle.  Every random draw comes from numpy's PCG64 ``default_rng(seed)``.

Coefficients follow the paper's Tables III-IV as lattice units: xi = 1.1, alpha = -0.9,
beta = 1, kappa = 0.001, Gamma = 1, K^x = (0.01, 0.005, 0.005, 0.005).  The polymer viscosity is
eta_p = relax_time * 0.009375, where 0.009375 = (3*0.01 + 2*0.005 + 4*0.005 + 3*0.005)/8 is the
isotropic stiffness C~11 of that K^x (Sec. II C 3), so relax_time is the Maxwell time of the
isotropic medium.  Initial polarization vectors are rounded to float32 so that the FP32 GPU state
and the FP64 oracle state start from identical values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KX_TABLE_IV = (0.01, 0.005, 0.005, 0.005)   # K1111, K1122, K2222, K1212
C11_ISO_TABLE_IV = 0.009375                 # isotropic C~11 of KX_TABLE_IV
BE_TABLE_III = dict(xi=1.1, alpha=-0.9, beta=1.0, kappa=0.001, Gamma=1.0)


@dataclass
class BodySpec:
    R: np.ndarray                     # (n, 2) FP64 node positions (regular polygon at t = 0)
    k_spring: float
    eps_angle: float
    l_eq: float
    pull: tuple                       # total external force (Fx, Fy)
    t_on: float = 0.0                 # logistic switch-on centre (steps); width 0 = constant pull
    t_off: float = 0.0                # logistic switch-off centre (steps)
    width: float = 0.0                # logistic scale (steps)
    trap: dict | None = None          # harmonic trap: k, x0, y0, dx, dy, t1, t2, w (include/lb.h)


@dataclass
class SimSpec:
    nx: int
    ny: int
    params: dict                      # tau, Kx, eta_p, D_p, xi, alpha, beta, kappa, Gamma, P_clamp, ericksen
    P0: np.ndarray                    # (2, ny, nx) FP64, float32-representable
    bodies: list = field(default_factory=list)
    sigma0: np.ndarray | None = None  # (3, ny, nx) or None (zero stress)
    meta: dict = field(default_factory=dict)


@dataclass
class Workload:
    name: str
    sims: list
    steps: int
    precision: str = "fp32"           # "fp32" or "fp16" population storage
    meta: dict = field(default_factory=dict)

    @property
    def sites(self) -> int:
        return sum(s.nx * s.ny for s in self.sims)


def polygon_nodes(cx: float, cy: float, radius: float, n: int) -> np.ndarray:
    a = 2.0 * math.pi * np.arange(n) / n
    return np.stack([cx + radius * np.cos(a), cy + radius * np.sin(a)], axis=1)


def make_body(cx, cy, radius, n, pull, k_spring=0.05, **sched) -> BodySpec:
    """Regular polygon at rest: l_eq is its chord so springs start unstretched; the bending
    stiffness keeps the paper's ratio eps_angle / (k_spring l_eq^2) = 1e-20 / (1e-5 * (2e-8)^2)
    = 2.5 (Table II)."""
    l_eq = 2.0 * radius * math.sin(math.pi / n)
    return BodySpec(R=polygon_nodes(cx, cy, radius, n), k_spring=k_spring,
                    eps_angle=2.5 * k_spring * l_eq * l_eq, l_eq=l_eq, pull=tuple(pull), **sched)


def base_params(relax_time: float, D_p: float, tau: float = 0.8, **over) -> dict:
    p = dict(tau=tau, Kx=KX_TABLE_IV, eta_p=relax_time * C11_ISO_TABLE_IV, D_p=D_p,
             P_clamp=0.99, ericksen=1, **BE_TABLE_III)
    p.update(over)
    return p


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def director_field(angles: np.ndarray, magnitude: float) -> np.ndarray:
    return _f32(np.stack([magnitude * np.cos(angles), magnitude * np.sin(angles)]))


def c1(seed: int = 1001, nx: int = 64, ny: int = 64, steps: int = 500) -> Workload:
    """64x64 periodic; directors uniform in [0, pi) per site; one body R=6, N=40, pull 1e-4 x."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi, size=(ny, nx))
    Peq = math.sqrt(0.9)
    sim = SimSpec(nx, ny, base_params(50.0, 0.05), director_field(th, Peq),
                  [make_body(nx / 2, ny / 2, 6.0, 40, (1e-4, 0.0))])
    return Workload("c1", [sim], steps, "fp32", dict(seed=seed))


def c2(seed: int = 1002, n: int = 512, steps: int = 5000) -> Workload:
    """512x512 periodic; directors at 30 deg plus N(0, 0.1 rad); one body R=16, N=100, pull 5e-5 x."""
    rng = np.random.default_rng(seed)
    th = math.radians(30.0) + rng.normal(0.0, 0.1, size=(n, n))
    sim = SimSpec(n, n, base_params(200.0, 0.02), director_field(th, math.sqrt(0.9)),
                  [make_body(n / 2, n / 2, 16.0, 100, (5e-5, 0.0))])
    return Workload("c2", [sim], steps, "fp32", dict(seed=seed))


def c3(seed: int = 1003, n: int = 2048, steps: int = 20000, n_bodies: int = 8) -> Workload:
    """2048x2048 with FP16 population storage; 8 bodies R ~ U[12, 24] at seeded positions
    (periodic centre distance >= R_i + R_j + 16), pull directions uniform in angle, |F| = 5e-5."""
    rng = np.random.default_rng(seed)
    th = math.radians(30.0) + rng.normal(0.0, 0.1, size=(n, n))
    bodies, placed = [], []
    while len(placed) < n_bodies:
        R = rng.uniform(12.0, 24.0)
        cx, cy = rng.uniform(0.0, n), rng.uniform(0.0, n)
        ok = True
        for (px, py, pr) in placed:
            dx = abs(cx - px); dx = min(dx, n - dx)
            dy = abs(cy - py); dy = min(dy, n - dy)
            if math.hypot(dx, dy) < R + pr + 16.0:
                ok = False
                break
        if not ok:
            continue
        placed.append((cx, cy, R))
        ang = rng.uniform(0.0, 2.0 * math.pi)
        bodies.append(make_body(cx, cy, R, int(round(2 * math.pi * R)),
                                (5e-5 * math.cos(ang), 5e-5 * math.sin(ang))))
    sim = SimSpec(n, n, base_params(200.0, 0.02), director_field(th, math.sqrt(0.9)), bodies)
    return Workload("c3", [sim], steps, "fp16", dict(seed=seed))


def ensemble_member(i: int, sizes=(64, 128, 256, 512), seed_base: int = 2000, squares: bool = False) -> SimSpec:
    """One member of the batched parameter sweep: nx, ny drawn independently from `sizes`,
    D_p log-uniform in [0.001, 0.2], relax time 200, uniform director at theta0 ~ U[0, 90] deg
    to the +x pull, one centred body R ~ U[4, 32] redrawn until 2R + 8 <= min(nx, ny)/2."""
    rng = np.random.default_rng(seed_base + i)
    nx = int(rng.choice(sizes))
    ny = nx if squares else int(rng.choice(sizes))
    D_p = float(math.exp(rng.uniform(math.log(0.001), math.log(0.2))))
    th0 = float(rng.uniform(0.0, math.pi / 2))
    while True:
        R = float(rng.uniform(4.0, 32.0))
        if 2 * R + 8 <= min(nx, ny) / 2:
            break
    P0 = director_field(np.full((ny, nx), th0), math.sqrt(0.9))
    body = make_body(nx / 2, ny / 2, R, int(round(2 * math.pi * R)), (5e-5, 0.0))
    return SimSpec(nx, ny, base_params(200.0, D_p), P0, [body],
                   meta=dict(D_p=D_p, theta0=th0, radius=R, seed=seed_base + i))


def c4(n_sims: int = 256, steps: int = 5000, squares: bool = False) -> Workload:
    sims = [ensemble_member(i, squares=squares) for i in range(n_sims)]
    return Workload("c4", sims, steps, "fp32", dict(n_sims=n_sims))


# Surrogate sweep: 128^2 runs of 4096 steps; the pull is switched on by a logistic of scale 30
# steps centred at step 120 (a 30-step rest plus three scales) and off at step 2048; the
# restoring force along the pull is sampled every 64 steps (64 samples).
C5_N = 128
C5_STEPS = 4096
C5_SAMPLE_EVERY = 64
C5_T_ON, C5_T_OFF, C5_WIDTH = 120.0, 2048.0, 30.0


def surrogate_inputs(seed: int) -> dict:
    rng = np.random.default_rng(seed)
    return dict(
        D_p=float(math.exp(rng.uniform(math.log(0.001), math.log(0.2)))),
        relax=float(math.exp(rng.uniform(math.log(20.0), math.log(400.0)))),
        radius=float(rng.uniform(4.0, 16.0)),
        theta0=float(rng.uniform(0.0, math.pi / 2)),
        P_eq=float(rng.uniform(0.0, 0.95)),
    )


def surrogate_member(seed: int, n: int = C5_N) -> SimSpec:
    x = surrogate_inputs(seed)
    P_eq = x["P_eq"]
    params = base_params(x["relax"], x["D_p"], alpha=-(P_eq * P_eq), beta=1.0)
    P0 = director_field(np.full((n, n), x["theta0"]), P_eq)
    R = x["radius"]
    body = make_body(n / 2, n / 2, R, int(round(2 * math.pi * R)), (5e-5, 0.0),
                     t_on=C5_T_ON, t_off=C5_T_OFF, width=C5_WIDTH)
    return SimSpec(n, n, params, P0, [body], meta=dict(x, seed=seed))


def c5(seeds, n: int = C5_N) -> Workload:
    return Workload("c5", [surrogate_member(s, n) for s in seeds], C5_STEPS, "fp32",
                    dict(sample_every=C5_SAMPLE_EVERY))


def small_case(seed: int, nx: int, ny: int, n_bodies: int = 1, radius: float = 5.0,
               random_dirs: bool = True, D_p: float = 0.05, relax: float = 50.0,
               pull: float = 1e-4, tau: float = 0.8, **over) -> Workload:
    """Parity-sized case with ragged (non power of two) extents and optional several bodies."""
    rng = np.random.default_rng(seed)
    if random_dirs:
        th = rng.uniform(0.0, math.pi, size=(ny, nx))
    else:
        th = math.radians(30.0) + rng.normal(0.0, 0.1, size=(ny, nx))
    bodies = []
    for b in range(n_bodies):
        cx = (b + 0.5) * nx / n_bodies + rng.uniform(-0.5, 0.5)
        cy = ny / 2 + rng.uniform(-0.5, 0.5)
        ang = rng.uniform(0, 2 * math.pi)
        nn = max(8, int(round(2 * math.pi * radius)))
        bodies.append(make_body(cx, cy, radius, nn, (pull * math.cos(ang), pull * math.sin(ang))))
    sim = SimSpec(nx, ny, base_params(relax, D_p, tau=tau, **over), director_field(th, math.sqrt(0.9)), bodies)
    return Workload(f"small{nx}x{ny}", [sim], 0, "fp32", dict(seed=seed))


def trap_body(cx: float, cy: float, radius: float, d_pull: float, T_pull: float, k_trap: float,
              t_rest: float = 30.0, width: float = 30.0, k_spring: float = 0.05) -> BodySpec:
    """A body pulled along +x by the harmonic trap protocol (App. A, App. C): a t_rest rest, the
    stiffness switched on by a logistic of scale `width` centred three scales later, the trap moved
    d_pull at constant speed over T_pull with logistic starts and stops, then let go."""
    b = make_body(cx, cy, radius, int(round(2 * math.pi * radius)), (0.0, 0.0), k_spring=k_spring)
    c = b.R.mean(axis=0)
    t1 = t_rest + 3.0 * width
    b.trap = dict(k=k_trap, x0=float(c[0]), y0=float(c[1]), dx=float(d_pull), dy=0.0, t1=t1, t2=t1 + T_pull,
                  w=width)
    return b


def trap_case(seed: int, nx: int, ny: int, radius: float = 6.0, d_pull: float = 4.0, T_pull: float = 800.0,
              k_trap: float = 0.01, relax: float = 200.0, D_p: float = 0.01, walls: int = 1, P_eq: float = 0.0,
              theta0: float = 0.0, **over) -> Workload:
    """The paper's driven-droplet experiment at small size: one body pulled by the trap through the
    polymer solution between walls, a uniform director at theta0 to the pull with magnitude P_eq
    (alpha = -P_eq^2, beta = 1)."""
    params = base_params(relax, D_p, walls=walls, alpha=-(P_eq * P_eq), beta=1.0, **over)
    P0 = director_field(np.full((ny, nx), theta0), P_eq)
    body = trap_body(nx / 2 - d_pull / 2, ny / 2, radius, d_pull, T_pull, k_trap)
    return Workload(f"trap{nx}x{ny}", [SimSpec(nx, ny, params, P0, [body], meta=dict(seed=seed))], 0, "fp32",
                    dict(d_pull=d_pull, T_pull=T_pull))


# The paper's own parameters (Tables I-IV) in lattice units of its unit map: dx = 4e-8 m,
# dt = 8e-6 s, rho_s = 2e7 kg/m^3, so stress 500 Pa, viscosity 4e-3 Pa s, diffusivity
# 2e-10 m^2/s, stiffness (N/m) 2e-5, energy 3.2e-20 J, length 4e-8 m, time 8e-6 s.
PAPER_STEPS = 187_500
PAPER_UNITS = dict(stress=500.0, viscosity=4e-3, diffusivity=2e-10, stiffness=2e-5, energy=3.2e-20, length=4e-8,
                   time=8e-6)


def paper_case(D_p: float = 1e-13, radius_m: float = 5e-7, T_pull_s: float = 0.2, d_pull_m: float = 4e-6,
               theta0: float = 0.0, alpha: float = -0.9, n: int = 250, scalar: bool = False,
               fe_units: str = "Pa") -> Workload:
    """The paper's experiment at its own size (Tables I-IV, App. C): a 250 x 250 closed box, tau 1.25,
    a droplet of radius 0.5 um (12.5 sites, nodes 0.5 sites apart) dragged 4 um (100 sites) over
    0.2 s (25 000 steps) by the trap and let go, 187 500 steps in all; stress-related values
    divided by the 500 Pa stress unit.  Physical inputs in SI units, converted here.

    scalar=True gives the scalar model of Sec. II B (eqMaxDiff, C = 0.01 Pa of Table IV): no
    polarization, and an isotropic K^x = (C, 0, C, C/2), for which the stiffness operator is C times
    the identity on (Xxx, Xyy, Xxy) whatever P is, so the tensorial step reduces exactly to
    C Psi - (C / eta_p) sigma + D_p lap sigma.

    fe_units: the unit of the free-energy coefficients alpha, beta, kappa (Table III prints no unit).
    "Pa" (default) converts them with the 500 Pa stress unit like every other stress in Tables I-IV
    (alpha = -0.9 -> -1.8e-3, beta 2e-3, kappa 2e-6), which keeps |P|_eq = sqrt(-alpha / beta) and
    the quasi-static flow-alignment viscosity xi^2 |P|^2 / Gamma and puts the magnitude relaxation at
    1 / (2 Gamma beta |P|^2) = 280 steps.  "lattice" takes the printed numbers as lattice units, where
    that relaxation takes 0.55 steps and the coupled flow-magnitude response carries waves faster than
    one site per step: the explicit step then grows a grid-scale mode at the walls and the protocol
    stops after 5 000 - 45 000 steps for every alpha != 0."""
    U = PAPER_UNITS
    if scalar:
        C = 0.01 / U["stress"]
        Kx = (C, 0.0, C, 0.5 * C)
    else:
        Kx = tuple(v / U["stress"] for v in (0.01, 0.005, 0.005, 0.005))
    if fe_units not in ("Pa", "lattice"):
        raise ValueError("fe_units must be 'Pa' or 'lattice'")
    fe = U["stress"] if fe_units == "Pa" else 1.0
    params = dict(tau=1.25, Kx=Kx, eta_p=0.1 / U["viscosity"], D_p=D_p / U["diffusivity"], P_clamp=0.99,
                  ericksen=0 if scalar else 1, xi=1.1, alpha=alpha / fe, beta=1.0 / fe, kappa=0.001 / fe,
                  Gamma=1.0, walls=2)
    P_eq = 0.0 if scalar else math.sqrt(max(0.0, -alpha))
    P0 = director_field(np.full((n, n), theta0), P_eq)
    R = radius_m / U["length"]
    l_eq = 2e-8 / U["length"]
    nn = int(round(2 * math.pi * R / l_eq))
    d_pull = d_pull_m / U["length"]
    T_pull = T_pull_s / U["time"]
    x0 = n / 2 - d_pull / 2
    body = make_body(x0, n / 2, R, nn, (0.0, 0.0), k_spring=1e-5 / U["stiffness"])
    body.eps_angle = 1e-20 / U["energy"]
    c = body.R.mean(axis=0)
    t1 = 30.0 + 3 * 30.0
    body.trap = dict(k=1e-6 / U["stiffness"], x0=float(c[0]), y0=float(c[1]), dx=float(d_pull), dy=0.0, t1=t1,
                     t2=t1 + T_pull, w=30.0)
    return Workload("paper_scalar" if scalar else "paper", [SimSpec(n, n, params, P0, [body], meta=dict(d_pull=d_pull))],
                    PAPER_STEPS, "fp32",
                    dict(d_pull=d_pull, T_pull=T_pull))


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4}
