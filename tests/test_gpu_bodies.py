"""GPU parity of the immersed-boundary path at its limits, against the FP64 oracle:

* the most bodies a simulation may hold (64), packed so that more body patches reach every work
  item of the fused kernel than it lists (8): those sites scan every body of the simulation
  instead of the item's list.  Both body-update forms are run: one launch (at most 512 patch
  tiles) and two launches (more tiles);
* the most nodes a body may have (1024), whose update walks its nodes in four 256-thread rounds.

Bar as for every FP32 parity case: L-infinity-normalised relative error <= 1e-4 on the fields,
node positions within 1e-5 sites."""
import math
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import lb, workload as wl
from tests.helpers import linf_rel, oracle_sim

pytestmark = pytest.mark.gpu

FIELDS = ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def crowded(seed: int, n: int, spacing: float, radius: float) -> wl.Workload:
    """64 bodies on an 8 x 8 grid `spacing` sites apart, random small pulls, random directors."""
    rng = np.random.default_rng(seed)
    bodies = []
    nodes = max(8, int(round(2 * math.pi * radius)))
    for i in range(8):
        for j in range(8):
            ang = rng.uniform(0.0, 2 * math.pi)
            bodies.append(wl.make_body((i + 0.5) * spacing + rng.uniform(-0.3, 0.3),
                                       (j + 0.5) * spacing + rng.uniform(-0.3, 0.3), radius, nodes,
                                       (1e-4 * math.cos(ang), 1e-4 * math.sin(ang))))
    th = rng.uniform(0.0, math.pi, size=(n, n))
    sim = wl.SimSpec(n, n, wl.base_params(50.0, 0.05), wl.director_field(th, math.sqrt(0.9)), bodies)
    return wl.Workload("crowded", [sim], 0, "fp32", dict(seed=seed))


def check(g: lb.Sim, r, steps: int):
    g.step(steps)
    r.run(steps)
    f = g.fields()
    o = r.observe()
    for k in FIELDS:
        e = linf_rel(f[k], o[k])
        say(f"  {k}: {e:.2e}")
        assert e <= 1e-4, (k, e)
    nodes = g.nodes()
    worst = max(float(np.max(np.abs(nodes[b] - body.R))) for b, body in enumerate(r.bodies))
    say(f"  worst node error {worst:.2e}")
    assert worst <= 1e-5


def patches_per_item(sim: wl.SimSpec, threads: int, seg: int) -> list:
    """How many body patches reach each fused work item at t = 0.  Items are strips of threads - 8
    columns and segments of about `seg` rows (nearly equal parts); an item touches its columns
    with 4 of halo on each side and its rows with 2; a patch is 2 * ceil(extent) + 24 sites wide,
    starting 3 sites below the lowest node."""
    n_x, n_y = sim.nx, sim.ny
    ns, ng = -(-n_x // (threads - 8)), max(1, -(-n_y // seg))

    def meets(a0, alen, b0, blen, n):
        return any((a0 + k - b0) % n < blen for k in range(alen))

    pats = []
    for b in sim.bodies:
        c = b.R.mean(axis=0)
        ps = min(2 * math.ceil(float(np.max(np.hypot(*(b.R - c).T)))) + 24, n_x, n_y)
        pats.append((math.floor(b.R[:, 0].min()) - 3, math.floor(b.R[:, 1].min()) - 3, ps))
    out = []
    for g in range(ng):
        y0, y1 = g * n_y // ng, (g + 1) * n_y // ng
        for k in range(ns):
            x0, x1 = k * n_x // ns, (k + 1) * n_x // ns
            out.append(sum(1 for ox, oy, ps in pats if meets(x0 - 4, x1 - x0 + 8, ox, ps, n_x)
                           and meets(y0 - 2, y1 - y0 + 4, oy, ps, n_y)))
    return out


@pytest.mark.parametrize("radius,tiles", [(2.5, 256), (6.0, 576)], ids=["one-launch", "two-launch"])
def test_most_bodies_crowding_one_work_item(radius, tiles):
    spacing = 16.0
    n = int(8 * spacing)
    w = crowded(61, n, spacing, radius)
    # every 64-thread item reaches more patches than it can list, so all its sites scan
    counts = patches_per_item(w.sims[0], 64, 25)
    assert min(counts) > 8, counts
    ps = [min(2 * math.ceil(radius) + 24, n)] * 64
    assert sum(((p + 15) // 16) ** 2 for p in ps) == tiles   # 512 or fewer: one launch, else two
    say(f"case 64 bodies R={radius} on {n}x{n} seed=61 ({tiles} patch tiles), 200 steps, 64-thread items "
        f"reaching {min(counts)}-{max(counts)} patches each")
    g = lb.Sim(w, lb.make_options(fused_threads=64, seg_rows=25))
    check(g, oracle_sim(w.sims[0]), 200)
    g.close()


def test_body_with_the_most_nodes():
    rng = np.random.default_rng(62)
    n, R, nodes = 192, 72.0, 1024
    th = rng.uniform(0.0, math.pi, size=(n, n))
    body = wl.make_body(n / 2 + 0.3, n / 2 - 0.2, R, nodes, (2e-4, 1e-4))
    sim = wl.SimSpec(n, n, wl.base_params(50.0, 0.05), wl.director_field(th, math.sqrt(0.9)), [body])
    w = wl.Workload("bignodes", [sim], 0, "fp32", dict(seed=62))
    say(f"case one body of {nodes} nodes R={R} on {n}x{n} seed=62, 200 steps")
    g = lb.Sim(w, lb.make_options())
    check(g, oracle_sim(w.sims[0]), 200)
    g.close()
