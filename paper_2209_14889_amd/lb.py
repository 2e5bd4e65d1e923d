"""ctypes binding of liblb (include/lb.h): argument marshalling only.

PyTorch provides the device arena (one uint8 tensor) and the HIP stream; every step of the
method runs in the library's HIP kernels.  Importing this module never falls back to a CPU
path: if liblb.so is missing or no GPU is present, creating a simulation raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .workload import SimSpec, Workload

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblb.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ERANGE = 0, -1, -2, -3, -4, -5
FIELDS = ["rho", "vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy"]
F_NODES = 1 << 10
F_ALL = 0x7FF

_dp = ctypes.POINTER(ctypes.c_double)


class BodyDesc(ctypes.Structure):
    _fields_ = [
        ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("radius", ctypes.c_double),
        ("n_nodes", ctypes.c_int32),
        ("k_spring", ctypes.c_double), ("eps_angle", ctypes.c_double), ("l_eq", ctypes.c_double),
        ("pull_fx", ctypes.c_double), ("pull_fy", ctypes.c_double),
        ("pull_t_on", ctypes.c_double), ("pull_t_off", ctypes.c_double), ("pull_width", ctypes.c_double),
        ("trap_k", ctypes.c_double), ("trap_x0", ctypes.c_double), ("trap_y0", ctypes.c_double),
        ("trap_dx", ctypes.c_double), ("trap_dy", ctypes.c_double), ("trap_t1", ctypes.c_double),
        ("trap_t2", ctypes.c_double), ("trap_w", ctypes.c_double),
        ("nodes", _dp),
    ]


class SimParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
        ("Kx", ctypes.c_double * 4), ("eta_p", ctypes.c_double), ("D_p", ctypes.c_double),
        ("xi", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("kappa", ctypes.c_double), ("Gamma", ctypes.c_double), ("P_clamp", ctypes.c_double),
        ("ericksen", ctypes.c_int32), ("walls", ctypes.c_int32), ("gx", ctypes.c_double),
        ("gy", ctypes.c_double), ("n_bodies", ctypes.c_int32),
        ("bodies", ctypes.POINTER(BodyDesc)),
        ("init_P", _dp), ("init_sigma", _dp), ("init_h", _dp),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("fp16_shift", ctypes.c_int32),
        ("watchdog_every", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
        ("kernel", ctypes.c_int32), ("timing", ctypes.c_int32), ("seg_rows", ctypes.c_int32),
        ("fused_threads", ctypes.c_int32), ("autotune", ctypes.c_int32), ("grid", ctypes.c_int32),
        ("autotune_cache", ctypes.c_char_p),
    ]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblb error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.lb_query_arena_bytes.argtypes = [ctypes.POINTER(SimParams), ctypes.c_int32, ctypes.POINTER(Options),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.lb_create.argtypes = [ctypes.POINTER(SimParams), ctypes.c_int32, ctypes.POINTER(Options), vp,
                                ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.lb_step.argtypes = [vp, ctypes.c_int32]
        L.lb_read_fields.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32, _dp, ctypes.c_size_t]
        L.lb_body_force.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _dp]
        L.lb_conservation.argtypes = [vp, ctypes.c_int32, _dp]
        L.lb_body_forces.argtypes = [vp, _dp, ctypes.c_size_t]
        L.lb_sync.argtypes = [vp]
        L.lb_time.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.lb_timing.argtypes = [vp, _dp, ctypes.POINTER(ctypes.c_int64), _dp, ctypes.POINTER(ctypes.c_int64),
                                ctypes.c_int32]
        L.lb_destroy.argtypes = [vp]
        L.lb_launch_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _dp]
        L.lb_body_forces_device.argtypes = [vp, vp, ctypes.c_size_t]
        L.lb_state_bytes.argtypes = [vp, _dp]
        L.lb_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.lb_last_error.restype = ctypes.c_char_p
        for name in ("lb_query_arena_bytes", "lb_create", "lb_step", "lb_read_fields", "lb_body_force",
                     "lb_conservation", "lb_sync", "lb_time", "lb_timing", "lb_destroy", "lb_launch_shape",
                     "lb_body_forces", "lb_body_forces_device", "lb_state_bytes", "lb_stream_copy"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != LB_OK:
        raise LBError(rc, lib().lb_last_error().decode())


def stream_copy(src, dst, stream=None) -> None:
    """dst[:] = src with the library's streaming copy kernel (cuda tensors of equal byte size, a
    multiple of 16); asynchronous on `stream` (default: torch's current stream)."""
    import torch
    n = src.numel() * src.element_size()
    assert n == dst.numel() * dst.element_size() and src.is_contiguous() and dst.is_contiguous()
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    check(lib().lb_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(n),
                               ctypes.c_void_p(st.cuda_stream)))


def make_options(precision: int = 0, fp16_shift: int = 0, watchdog_every: int = 0, graph_chunk: int = 0,
                 kernel: int = 0, timing: int = 0, seg_rows: int = 0, fused_threads: int = 0,
                 autotune: int = 0, grid: int = 0, autotune_cache: str | None = None) -> Options:
    o = Options()
    o.precision, o.fp16_shift, o.watchdog_every, o.graph_chunk = precision, fp16_shift, watchdog_every, graph_chunk
    o.kernel, o.timing, o.seg_rows, o.fused_threads = kernel, timing, seg_rows, fused_threads
    o.autotune, o.grid = autotune, grid
    o.autotune_cache = None if autotune_cache is None else os.fsencode(autotune_cache)
    return o


class _Marshal:
    """Owns the ctypes structs and numpy buffers that describe a list of SimSpecs."""

    def __init__(self, sims: list):
        self.keep = []
        self.params = (SimParams * len(sims))()
        for i, s in enumerate(sims):
            self.params[i] = self._sim(s)

    def _arr(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.keep.append(a)
        return a.ctypes.data_as(_dp)

    def _sim(self, s: SimSpec) -> SimParams:
        p = SimParams()
        p.nx, p.ny = s.nx, s.ny
        q = s.params
        p.tau = q["tau"]
        p.Kx = (ctypes.c_double * 4)(*q["Kx"])
        p.eta_p, p.D_p = q["eta_p"], q["D_p"]
        p.xi, p.alpha, p.beta, p.kappa, p.Gamma = q["xi"], q["alpha"], q["beta"], q["kappa"], q["Gamma"]
        p.P_clamp = q["P_clamp"]
        p.ericksen = int(q.get("ericksen", 1))
        p.walls = int(q.get("walls", 0))
        p.gx, p.gy = float(q.get("gx", 0.0)), float(q.get("gy", 0.0))
        bodies = (BodyDesc * max(1, len(s.bodies)))()
        for j, b in enumerate(s.bodies):
            d = BodyDesc()
            d.n_nodes = b.R.shape[0]
            d.k_spring, d.eps_angle, d.l_eq = b.k_spring, b.eps_angle, b.l_eq
            d.pull_fx, d.pull_fy = b.pull
            d.pull_t_on, d.pull_t_off, d.pull_width = b.t_on, b.t_off, b.width
            if getattr(b, "trap", None):
                tr = b.trap
                d.trap_k, d.trap_x0, d.trap_y0 = tr["k"], tr["x0"], tr["y0"]
                d.trap_dx, d.trap_dy, d.trap_t1, d.trap_t2, d.trap_w = tr["dx"], tr["dy"], tr["t1"], tr["t2"], tr["w"]
            d.nodes = self._arr(b.R.reshape(-1))
            d.cx, d.cy = float(b.R[:, 0].mean()), float(b.R[:, 1].mean())
            d.radius = float(np.max(np.hypot(b.R[:, 0] - d.cx, b.R[:, 1] - d.cy)))
            bodies[j] = d
        self.keep.append(bodies)
        p.n_bodies = len(s.bodies)
        p.bodies = ctypes.cast(bodies, ctypes.POINTER(BodyDesc))
        p.init_P = self._arr(s.P0.reshape(-1)) if s.P0 is not None else None
        p.init_sigma = self._arr(s.sigma0.reshape(-1)) if s.sigma0 is not None else None
        p.init_h = self._arr(s.h0.reshape(-1)) if getattr(s, "h0", None) is not None else None
        return p


def arena_bytes(sims: list, options: Options | None = None) -> int:
    m = _Marshal(sims)
    n = ctypes.c_size_t(0)
    check(lib().lb_query_arena_bytes(m.params, len(sims), ctypes.byref(options) if options else None,
                                     ctypes.byref(n)))
    return int(n.value)


class Sim:
    """One handle: a single simulation or a batched ensemble of independent ones."""

    def __init__(self, sims, options: Options | None = None, device: str = "cuda:0", library_stream: bool = False):
        import torch
        if isinstance(sims, Workload):
            sims = sims.sims
        if isinstance(sims, SimSpec):
            sims = [sims]
        self.specs = list(sims)
        self.options = options or make_options()
        if not torch.cuda.is_available():
            raise RuntimeError("liblb needs a ROCm GPU (torch.cuda.is_available() is False)")
        self._torch = torch
        self.device = torch.device(device)
        m = _Marshal(self.specs)
        n = ctypes.c_size_t(0)
        check(lib().lb_query_arena_bytes(m.params, len(self.specs), ctypes.byref(self.options), ctypes.byref(n)))
        self.arena = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        # a stream of our own (default priority): graph capture is not allowed on the legacy
        # default stream.  library_stream: pass NULL, so the library creates (and destroys) one.
        self.stream = None if library_stream else torch.cuda.Stream(device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        h = ctypes.c_void_p()
        check(lib().lb_create(m.params, len(self.specs), ctypes.byref(self.options),
                              ctypes.c_void_p(self.arena.data_ptr()), ctypes.c_size_t(self.arena.numel()),
                              ctypes.c_void_p(None if library_stream else self.stream.cuda_stream),
                              ctypes.byref(h)))
        self.h = h

    # -- stepping ------------------------------------------------------------------------------
    def step(self, n: int = 1) -> "Sim":
        check(lib().lb_step(self.h, int(n)))
        return self

    def sync(self) -> None:
        check(lib().lb_sync(self.h))

    @property
    def t(self) -> int:
        v = ctypes.c_int64(0)
        check(lib().lb_time(self.h, ctypes.byref(v)))
        return int(v.value)

    # -- observables ---------------------------------------------------------------------------
    def fields(self, sim: int = 0, names=None) -> dict:
        names = FIELDS if names is None else list(names)
        mask = 0
        for nm in names:
            mask |= 1 << FIELDS.index(nm)
        s = self.specs[sim]
        N = s.nx * s.ny
        out = np.empty(len(names) * N)
        check(lib().lb_read_fields(self.h, sim, mask, out.ctypes.data_as(_dp), out.size))
        order = [f for f in FIELDS if f in names]
        return {nm: out[i * N:(i + 1) * N].reshape(s.ny, s.nx).copy() for i, nm in enumerate(order)}

    def nodes(self, sim: int = 0) -> list:
        s = self.specs[sim]
        counts = [b.R.shape[0] for b in s.bodies]
        out = np.empty(2 * sum(counts))
        check(lib().lb_read_fields(self.h, sim, F_NODES, out.ctypes.data_as(_dp), out.size))
        res, o = [], 0
        for c in counts:
            res.append(out[o:o + 2 * c].reshape(c, 2).copy())
            o += 2 * c
        return res

    def body_force(self, sim: int = 0, body: int = 0) -> dict:
        out = np.empty(8)
        check(lib().lb_body_force(self.h, sim, body, out.ctypes.data_as(_dp)))
        return dict(restoring=out[0:2].copy(), pull=out[2:4].copy(), com=out[4:6].copy(), node_force=out[6:8].copy())

    def body_forces(self) -> np.ndarray:
        """(total bodies, 10): restoring force as the inside-site sum (2), pull (2), centre of
        mass (2), node force (2), area-weighted restoring force (2)."""
        nb = sum(len(s.bodies) for s in self.specs)
        out = np.empty(10 * max(1, nb))
        check(lib().lb_body_forces(self.h, out.ctypes.data_as(_dp), out.size))
        return out[:10 * nb].reshape(nb, 10).copy()

    def body_forces_device(self, out) -> None:
        """Queue the body observables into `out`, a float64 cuda tensor of 8 values per body (site-sum
        restoring force, centre of mass, node force, area-weighted restoring force), without
        synchronising: the values are there once the handle's stream has reached this point."""
        assert out.dtype == self._torch.float64 and out.is_cuda and out.is_contiguous()
        check(lib().lb_body_forces_device(self.h, ctypes.c_void_p(out.data_ptr()), out.numel()))

    def state_bytes(self) -> float:
        """Stored state bytes read and written per site update in this handle's storage form."""
        v = ctypes.c_double(0)
        check(lib().lb_state_bytes(self.h, ctypes.byref(v)))
        return float(v.value)

    def conservation(self, sim: int = 0) -> np.ndarray:
        out = np.empty(3)
        check(lib().lb_conservation(self.h, sim, out.ctypes.data_as(_dp)))
        return out

    def timing(self, reset: bool = False) -> dict:
        fm, im = ctypes.c_double(0), ctypes.c_double(0)
        fn, inn = ctypes.c_int64(0), ctypes.c_int64(0)
        check(lib().lb_timing(self.h, ctypes.byref(fm), ctypes.byref(fn), ctypes.byref(im), ctypes.byref(inn),
                              int(reset)))
        return dict(field_ms=fm.value, field_launches=fn.value, ib_ms=im.value, ib_launches=inn.value)

    def launch_shape(self) -> dict:
        t, sg, ni, gr = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        ms = ctypes.c_double(0)
        check(lib().lb_launch_shape(self.h, ctypes.byref(t), ctypes.byref(sg), ctypes.byref(ni), ctypes.byref(gr),
                                    ctypes.byref(ms)))
        return dict(threads=t.value, seg_rows=sg.value, n_items=ni.value, grid=gr.value, tuned_ms=ms.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            lib().lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
