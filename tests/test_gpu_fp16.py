"""Precision form: populations stored as FP16 offsets from the rest weights (scaled by 2^S) with FP32
arithmetic, against the FP64 oracle.  Bar: L-infinity-normalised relative error <= 1e-3 on velocity
and stress after 1000 steps, on a 256 x 256 periodic window shaped like the 2048 x 2048 workload
(near-uniform directors, two bodies of radius 12 and 16)."""
import math
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import lb, workload as wl
from tests.helpers import linf_rel, oracle_sim

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def crop_case():
    rng = np.random.default_rng(1003)
    n = 256
    th = math.radians(30.0) + rng.normal(0.0, 0.1, size=(n, n))
    bodies = [wl.make_body(80.0, 96.0, 12.0, 75, (5e-5 * math.cos(0.7), 5e-5 * math.sin(0.7))),
              wl.make_body(176.0, 160.0, 16.0, 101, (5e-5 * math.cos(2.9), 5e-5 * math.sin(2.9)))]
    sim = wl.SimSpec(n, n, wl.base_params(200.0, 0.02), wl.director_field(th, math.sqrt(0.9)), bodies)
    return wl.Workload("c3-crop", [sim], 1000, "fp16")


def test_fp16_storage_within_1e3_of_oracle():
    w = crop_case()
    say("case fp16 precision form 256x256 two bodies, 1000 steps")
    g = lb.Sim(w, lb.make_options(precision=1, graph_chunk=100))
    r = oracle_sim(w.sims[0])
    g.step(1000)
    r.run(1000)
    a, o = g.fields(), r.observe()
    worst = 0.0
    for k in ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py"):
        e = linf_rel(a[k], o[k])
        worst = max(worst, e)
        say(f"  {k} {e:.2e}")
    for k in ("vx", "vy", "sxx", "syy", "sxy"):
        assert linf_rel(a[k], o[k]) <= 1e-3, k
    nodes = g.nodes()
    for b in range(2):
        d = float(np.max(np.abs(nodes[b] - r.bodies[b].R)))
        say(f"  body {b} node error {d:.2e}")
        assert d <= 1e-4


def test_fp16_shift_changes_nothing_structural():
    # a different exponent shift keeps the result within the same bar (the shift only moves the
    # FP16 window of representable offsets)
    w = crop_case()
    say("case fp16 shift 12 vs 10, 200 steps")
    a = lb.Sim(w, lb.make_options(precision=1, fp16_shift=10))
    b = lb.Sim(w, lb.make_options(precision=1, fp16_shift=12))
    a.step(200)
    b.step(200)
    fa, fb = a.fields(), b.fields()
    for k in ("vx", "vy", "sxx"):
        assert linf_rel(fa[k], fb[k]) <= 1e-3, k
