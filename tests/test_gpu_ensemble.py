"""Batched ensemble on the GPU: several independent simulations of different sizes advanced by one
fused launch per step.  Each member must equal the same simulation run alone, bit for bit (the
per-site arithmetic does not depend on how sites are grouped into work items), and one member is
checked against the FP64 oracle."""
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import lb, workload as wl
from tests.helpers import linf_rel, oracle_sim

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def members(n=6):
    return [wl.ensemble_member(i, sizes=(64, 96, 128)) for i in range(n)]


@pytest.mark.parametrize("grid", [0, 64], ids=["item-grid", "persistent-64"])
def test_ensemble_members_equal_single_runs(grid):
    sims = members()
    say(f"case ensemble of {len(sims)} sims sizes", [(s.nx, s.ny) for s in sims], f"grid={grid} steps=80")
    ens = lb.Sim(sims, lb.make_options(seg_rows=10, grid=grid, graph_chunk=8))
    ens.step(80)
    for i, s in enumerate(sims):
        one = lb.Sim([s], lb.make_options(seg_rows=7))
        one.step(80)
        a, b = ens.fields(i), one.fields(0)
        for k in lb.FIELDS:
            assert np.array_equal(a[k], b[k]), (i, k)
        assert np.array_equal(ens.nodes(i)[0], one.nodes(0)[0]), i
        one.close()


def test_ensemble_member_matches_oracle():
    sims = members(4)
    say("case ensemble member 2 vs oracle, 200 steps")
    ens = lb.Sim(sims, lb.make_options(autotune=1))
    say("  launch shape", ens.launch_shape())
    ens.step(200)
    r = oracle_sim(sims[2])
    r.run(200)
    g, o = ens.fields(2), r.observe()
    for k in ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py"):
        e = linf_rel(g[k], o[k])
        say(f"  {k} {e:.2e}")
        assert e <= 1e-4, k


def test_body_update_paths_agree():
    """Many patch tiles (here about a thousand) take the two-launch body update (nodes once, then
    the spreading tiles); a single simulation takes the one-launch form in which every tile block
    repeats its body's node update.  Both must give the same bits."""
    sims = [wl.ensemble_member(i, sizes=(128,)) for i in range(48)]
    say("case 48 sims 128x128, two-launch body update vs one-launch single runs, 40 steps")
    ens = lb.Sim(sims, lb.make_options(seg_rows=16))
    ens.step(40)
    for i in (0, 23, 47):
        one = lb.Sim([sims[i]], lb.make_options(seg_rows=16))
        one.step(40)
        a, b = ens.fields(i), one.fields(0)
        for k in lb.FIELDS:
            assert np.array_equal(a[k], b[k]), (i, k)
        assert np.array_equal(ens.nodes(i)[0], one.nodes(0)[0]), i
        one.close()
