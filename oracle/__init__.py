"""Plain FP64 CPU oracle for the viscoelastic IB-LB coupled step (arXiv 2209.14889).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously-correct reference that the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  It shares no code with the GPU library, and the GPU library
never imports it.

The arithmetic lives in ``velb_oracle.c`` (plain C99, FP64, optional OpenMP over sites only).
This module is argument marshalling plus the textbook equilibrium used to build initial
populations.  Every function cites the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")

# D2Q9 lattice, same ordering as velb_oracle.c
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)
WQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("walls", ctypes.c_int),
        ("tau", ctypes.c_double), ("Kx", ctypes.c_double * 4),
        ("eta_p", ctypes.c_double), ("D_p", ctypes.c_double),
        ("xi", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("kappa", ctypes.c_double), ("Gamma", ctypes.c_double), ("P_clamp", ctypes.c_double),
        ("ericksen", ctypes.c_int), ("polymer_force", ctypes.c_int),
        ("evolve_sigma", ctypes.c_int), ("evolve_P", ctypes.c_int), ("kinematic", ctypes.c_int),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
    ]


class _Body(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("k_spring", ctypes.c_double), ("eps_angle", ctypes.c_double),
        ("l_eq", ctypes.c_double), ("pull_fx", ctypes.c_double), ("pull_fy", ctypes.c_double),
        ("t_on", ctypes.c_double), ("t_off", ctypes.c_double), ("width", ctypes.c_double),
        ("trap_k", ctypes.c_double), ("trap_x0", ctypes.c_double), ("trap_y0", ctypes.c_double),
        ("trap_dx", ctypes.c_double), ("trap_dy", ctypes.c_double), ("trap_t1", ctypes.c_double),
        ("trap_t2", ctypes.c_double), ("trap_w", ctypes.c_double),
        ("R", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liborc.so (built by oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_bessel_i.restype = ctypes.c_double
        L.orc_bessel_i.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_k_of_p.restype = ctypes.c_double
        L.orc_k_of_p.argtypes = [ctypes.c_double]
        L.orc_stiffness.argtypes = [ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.orc_phi.restype = ctypes.c_double
        L.orc_phi.argtypes = [ctypes.c_double]
        L.orc_node_forces.argtypes = [ctypes.POINTER(_Body), ctypes.c_double, _dp]
        L.orc_pull_factor.restype = ctypes.c_double
        L.orc_pull_factor.argtypes = [ctypes.POINTER(_Body), ctypes.c_double]
        L.orc_body_energy.restype = ctypes.c_double
        L.orc_trap_k.restype = ctypes.c_double
        L.orc_trap_k.argtypes = [ctypes.POINTER(_Body), ctypes.c_double]
        L.orc_trap_energy.restype = ctypes.c_double
        L.orc_trap_energy.argtypes = [ctypes.POINTER(_Body), ctypes.c_double]
        L.orc_trap_pos.argtypes = [ctypes.POINTER(_Body), ctypes.c_double, _dp]
        L.orc_body_energy.argtypes = [ctypes.POINTER(_Body)]
        L.orc_spread.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_interp.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(_Body),
                              _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int]
        L.orc_observe.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(_Body),
                                  _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.orc_body_force.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Body), _dp, _dp]
        L.orc_body_force_area.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Body), _dp, _dp]
        L.orc_cell_area.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double]
        L.orc_cell_area.restype = ctypes.c_double
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def bessel_i(n: int, k: float) -> float:
    return lib().orc_bessel_i(int(n), float(k))


def k_of_p(p: float) -> float:
    return lib().orc_k_of_p(float(p))


def stiffness(Px: float, Py: float, Kx, P_clamp: float = 0.99) -> np.ndarray:
    """3x3 plain-component stiffness operator C~(P) (App. B)."""
    K = np.ascontiguousarray(np.asarray(Kx, dtype=np.float64))
    C = np.zeros(9)
    lib().orc_stiffness(float(Px), float(Py), _ptr(K), float(P_clamp), _ptr(C))
    return C.reshape(3, 3)


def phi(r: float) -> float:
    return lib().orc_phi(float(r))


def equilibrium(rho: np.ndarray, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    """Standard second-order D2Q9 equilibrium (the form the paper cites for h^eq)."""
    uu = ux * ux + uy * uy
    out = np.empty((9,) + rho.shape)
    for n in range(9):
        cu = CX[n] * ux + CY[n] * uy
        out[n] = WQ[n] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
    return out


DEFAULT_PARAMS = dict(
    nx=64, ny=64, walls=0, tau=0.8, Kx=(0.01, 0.005, 0.005, 0.005), eta_p=0.46875, D_p=0.05,
    xi=1.1, alpha=-0.9, beta=1.0, kappa=0.001, Gamma=1.0, P_clamp=0.99,
    ericksen=1, polymer_force=1, evolve_sigma=1, evolve_P=1, kinematic=0, gx=0.0, gy=0.0,
)


def make_params(**kw) -> _Params:
    d = dict(DEFAULT_PARAMS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown oracle parameters {sorted(unknown)}")
    d.update(kw)
    p = _Params()
    for k, v in d.items():
        if k == "Kx":
            p.Kx = (ctypes.c_double * 4)(*[float(x) for x in v])
        elif isinstance(getattr(p, k), int):
            setattr(p, k, int(v))
        else:
            setattr(p, k, float(v))
    return p


@dataclass
class Body:
    R: np.ndarray                 # (n, 2) unwrapped node positions, FP64
    k_spring: float = 0.05
    eps_angle: float = 0.0
    l_eq: float = 1.0
    pull: tuple = (0.0, 0.0)      # total external force on the body
    t_on: float = 0.0             # logistic pull schedule (width 0: constant pull)
    t_off: float = 0.0
    width: float = 0.0
    trap: dict | None = None      # k, x0, y0, dx, dy, t1, t2, w (harmonic trap, see orc_body)
    _c: _Body = field(default=None, repr=False)

    def cstruct(self) -> _Body:
        self.R = np.ascontiguousarray(self.R, dtype=np.float64).reshape(-1, 2)
        b = _Body()
        b.n = self.R.shape[0]
        b.k_spring, b.eps_angle, b.l_eq = self.k_spring, self.eps_angle, self.l_eq
        b.pull_fx, b.pull_fy = float(self.pull[0]), float(self.pull[1])
        b.t_on, b.t_off, b.width = float(self.t_on), float(self.t_off), float(self.width)
        if self.trap:
            tr = self.trap
            b.trap_k, b.trap_x0, b.trap_y0 = float(tr["k"]), float(tr["x0"]), float(tr["y0"])
            b.trap_dx, b.trap_dy = float(tr["dx"]), float(tr["dy"])
            b.trap_t1, b.trap_t2, b.trap_w = float(tr["t1"]), float(tr["t2"]), float(tr["w"])
        b.R = self.R.ctypes.data_as(_dp)
        self._c = b
        return b

    def forces(self, t: float = 0.0) -> np.ndarray:
        f = np.zeros(2 * self.R.shape[0])
        lib().orc_node_forces(ctypes.byref(self.cstruct()), float(t), _ptr(f))
        return f.reshape(-1, 2)

    def pull_factor(self, t: float) -> float:
        return lib().orc_pull_factor(ctypes.byref(self.cstruct()), float(t))

    def energy(self) -> float:
        return lib().orc_body_energy(ctypes.byref(self.cstruct()))

    def trap_k(self, t: float) -> float:
        return lib().orc_trap_k(ctypes.byref(self.cstruct()), float(t))

    def trap_pos(self, t: float) -> np.ndarray:
        out = np.zeros(2)
        lib().orc_trap_pos(ctypes.byref(self.cstruct()), float(t), _ptr(out))
        return out

    def trap_energy(self, t: float) -> float:
        return lib().orc_trap_energy(ctypes.byref(self.cstruct()), float(t))


class Sim:
    """State of one oracle simulation: populations h (9, ny, nx), sigma (3, ny, nx),
    P (2, ny, nx) and the bodies' nodes, all FP64."""

    def __init__(self, params: dict | None = None, bodies=(), h=None, sigma=None, P=None, u_kin=None):
        self.pdict = dict(DEFAULT_PARAMS)
        self.pdict.update(params or {})
        self.p = make_params(**self.pdict)
        nx, ny = self.p.nx, self.p.ny
        self.bodies = list(bodies)
        # private copies: the C code updates the state in place
        self.h = np.array(h, dtype=np.float64, order="C", copy=True) if h is not None else \
            np.ascontiguousarray(np.broadcast_to(WQ[:, None, None], (9, ny, nx)), dtype=np.float64)
        self.sigma = np.array(sigma, dtype=np.float64, order="C", copy=True) if sigma is not None else np.zeros((3, ny, nx))
        self.P = np.array(P, dtype=np.float64, order="C", copy=True) if P is not None else np.zeros((2, ny, nx))
        self.u_kin = np.array(u_kin, dtype=np.float64, order="C", copy=True) if u_kin is not None else np.zeros((2, ny, nx))
        assert self.h.shape == (9, ny, nx) and self.sigma.shape == (3, ny, nx) and self.P.shape == (2, ny, nx)
        self.t = 0

    def _bodies_c(self):
        arr = (_Body * max(1, len(self.bodies)))()
        for i, b in enumerate(self.bodies):
            arr[i] = b.cstruct()
        return arr

    def run(self, n_steps: int) -> "Sim":
        arr = self._bodies_c()
        lib().orc_run(ctypes.byref(self.p), len(self.bodies), arr, _ptr(self.h), _ptr(self.sigma),
                      _ptr(self.P), _ptr(self.u_kin), int(self.t), int(n_steps))
        self.t += n_steps
        return self

    def observe(self) -> dict:
        nx, ny = self.p.nx, self.p.ny
        out = np.zeros((7, ny, nx))
        arr = self._bodies_c()
        lib().orc_observe(ctypes.byref(self.p), len(self.bodies), arr, _ptr(self.h), _ptr(self.sigma),
                          _ptr(self.P), _ptr(self.u_kin), int(self.t), _ptr(out))
        names = ["rho", "vx", "vy", "fpx", "fpy", "Fx", "Fy"]
        d = {k: out[i].copy() for i, k in enumerate(names)}
        d.update(sxx=self.sigma[0].copy(), syy=self.sigma[1].copy(), sxy=self.sigma[2].copy(),
                 Px=self.P[0].copy(), Py=self.P[1].copy())
        return d

    def body_force(self, b: int) -> np.ndarray:
        out = np.zeros(4)
        bc = self.bodies[b].cstruct()
        lib().orc_body_force(ctypes.byref(self.p), ctypes.byref(bc), _ptr(self.sigma), _ptr(out))
        return out

    def body_force_area(self, b: int) -> np.ndarray:
        """Area-weighted restoring force of body b (see orc_body_force_area)."""
        out = np.zeros(2)
        bc = self.bodies[b].cstruct()
        lib().orc_body_force_area(ctypes.byref(self.p), ctypes.byref(bc), _ptr(self.sigma), _ptr(out))
        return out

    def spread(self, R: np.ndarray, f: np.ndarray):
        nx, ny = self.p.nx, self.p.ny
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        fx = np.zeros((ny, nx)); fy = np.zeros((ny, nx))
        lib().orc_spread(ctypes.byref(self.p), R.size // 2, _ptr(R), _ptr(f), _ptr(fx), _ptr(fy))
        return fx, fy

    def interp(self, R: np.ndarray, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        ux = np.ascontiguousarray(ux, dtype=np.float64)
        uy = np.ascontiguousarray(uy, dtype=np.float64)
        out = np.zeros(R.size)
        lib().orc_interp(ctypes.byref(self.p), R.size // 2, _ptr(R), _ptr(ux), _ptr(uy), _ptr(out))
        return out.reshape(-1, 2)


def cell_area(R: np.ndarray, x0: float, x1: float, y0: float, y1: float) -> float:
    """Area of the polygon with nodes R (n, 2) inside the box [x0, x1] x [y0, y1]."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    return float(lib().orc_cell_area(R.shape[0], _ptr(R), x0, x1, y0, y1))


def polygon(cx: float, cy: float, radius: float, n: int) -> np.ndarray:
    """Regular polygon, node 0 at angle 0 (a test helper for building bodies)."""
    a = 2.0 * math.pi * np.arange(n) / n
    return np.stack([cx + radius * np.cos(a), cy + radius * np.sin(a)], axis=1)
