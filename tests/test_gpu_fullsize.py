"""The 2048 x 2048 workload at its full size, in the configuration the benchmark times (FP16
population storage, 256-thread work items of 19 rows, the shape its autotuner settles on; steps
replayed from HIP graphs), checked against the oracle on sampled windows.

A site's value after k steps depends only on the sites within 4k of it: one coupled step reads the
polarization 4 sites away (the molecular field's Laplacian inside the Ericksen stress, inside the
force, inside the velocity gradient of the Heun corrector), and everything else less far.  So the
oracle can compute sampled outputs of the full lattice on small windows cut from the full initial
state. Each window is run periodically for k steps with a margin of 4k + 8 sites, holds either
one whole body or no body, and has no node of any other body in it.  Inside the margin the window's
values must equal the full lattice's, to the FP16 bar (1e-3, L-infinity normalised over the
compared region), and the body's nodes must agree within 1e-4 sites."""
import math
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import lb, workload as wl
from tests.helpers import linf_rel, oracle_sim

pytestmark = pytest.mark.gpu

K = 50                 # steps (windows of about 470 sites around four of the eight bodies)
H = 4 * K + 8          # margin of a window
FIELDS = ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def window(spec: wl.SimSpec, x0: int, y0: int, side: int, bodies) -> wl.SimSpec:
    """The periodic side x side window at (x0, y0) of the initial state, with the given bodies
    moved into window coordinates."""
    n = spec.nx
    ys = np.arange(y0, y0 + side) % spec.ny
    xs = np.arange(x0, x0 + side) % n
    P = spec.P0[:, ys][:, :, xs]
    moved = []
    for b in bodies:
        R = np.mod(b.R - np.array([x0, y0], dtype=np.float64), n)
        moved.append(wl.BodySpec(R=R, k_spring=b.k_spring, eps_angle=b.eps_angle, l_eq=b.l_eq, pull=b.pull))
    return wl.SimSpec(side, side, dict(spec.params), P, moved)


def nodes_in(spec: wl.SimSpec, x0: int, y0: int, side: int, skip: int = -1) -> bool:
    for i, b in enumerate(spec.bodies):
        if i == skip:
            continue
        d = np.mod(b.R - np.array([x0, y0], dtype=np.float64), spec.nx)
        if np.any((d[:, 0] < side) & (d[:, 1] < side)):
            return True
    return False


def test_full_size_bench_configuration_on_sampled_windows():
    w = wl.c3()
    s = w.sims[0]
    say(f"case c3 2048x2048 seed=1003 FP16, 256 threads x 19 rows, graph chunks of 100, {K} steps; "
        f"oracle windows with a {H}-site margin")
    g = lb.Sim(w, lb.make_options(precision=1, fused_threads=256, seg_rows=19, graph_chunk=100))
    assert g.launch_shape()["threads"] == 256 and g.launch_shape()["seg_rows"] == 19
    g.step(K)
    f = g.fields(names=["rho", *FIELDS])
    nodes = g.nodes()
    g.close()

    samples = []
    for i, b in enumerate(s.bodies):   # a window around each body that no other body reaches
        c = b.R.mean(axis=0)
        ext = int(math.ceil(float(np.max(np.hypot(*(b.R - c).T))))) + 4
        side = 2 * (ext + H)
        x0, y0 = int(math.floor(c[0])) - ext - H, int(math.floor(c[1])) - ext - H
        if not nodes_in(s, x0, y0, side, skip=i):
            samples.append((f"body {i}", x0, y0, side, [b], i))
    rng = np.random.default_rng(77)
    while sum(1 for t in samples if t[4] == []) < 3:   # windows of fluid only
        side = 64 + 2 * H
        x0, y0 = (int(v) for v in rng.integers(0, s.nx, size=2))
        if not nodes_in(s, x0, y0, side):
            samples.append((f"fluid at ({x0}, {y0})", x0, y0, side, [], -1))
    assert sum(1 for t in samples if t[4]) >= 4, "too few bodies without a neighbour in their window"

    for name, x0, y0, side, bodies, ib in samples:
        ws = window(s, x0, y0, side, bodies)
        r = oracle_sim(ws)
        r.run(K)
        o = r.observe()
        ys = np.arange(y0 + H, y0 + side - H) % s.ny
        xs = np.arange(x0 + H, x0 + side - H) % s.nx
        inner = (slice(H, side - H), slice(H, side - H))
        errs = {}
        for k in FIELDS:
            errs[k] = linf_rel(f[k][ys][:, xs], o[k][inner])
        errs["rho"] = linf_rel(f["rho"][ys][:, xs] - 1.0, o["rho"][inner] - 1.0)
        say(f"  {name}, window {side}x{side}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        for k, v in errs.items():
            assert v <= 1e-3, (name, k, v)
        if ib >= 0:   # the body's nodes, back in lattice coordinates
            d = nodes[ib] - (r.bodies[0].R + np.array([x0, y0], dtype=np.float64))
            d = (d + s.nx / 2) % s.nx - s.nx / 2
            say(f"    node error {float(np.max(np.abs(d))):.1e}")
            assert float(np.max(np.abs(d))) <= 1e-4, name
