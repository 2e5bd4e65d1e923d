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
    for k in ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy"):
        e = linf_rel(g[k], o[k])
        say(f"  {k} {e:.2e}")
        assert e <= 1e-4, k


@pytest.mark.timeout(900)
def test_full_ensemble_in_the_bench_configuration():
    """The 256-member ensemble (sides 64 to 512 drawn independently, 14.7 M sites per step) at full
    size, in the configuration the benchmark times: FP32, 128-thread items of 17 rows (the shape its
    autotuner settles on), graph chunks of 100.  After 100 steps eight sampled members equal their single runs bit for bit and
    the three smallest of them match the oracle; after 1000 steps the smallest member of the
    ensemble and one of median size match the oracle at the FP32 bar."""
    w = wl.c4()
    sims = w.sims
    say(f"case full ensemble c4: {len(sims)} sims, {sum(s.nx * s.ny for s in sims)} sites, 128 x 17 items, "
        "graph chunks of 100, 100 then 1000 steps")
    ens = lb.Sim(sims, lb.make_options(fused_threads=128, seg_rows=17, graph_chunk=100))
    shape = ens.launch_shape()
    say("  launch shape", shape)
    assert shape["threads"] == 128 and shape["seg_rows"] == 17
    ens.step(100)
    pick = sorted(int(i) for i in np.random.default_rng(78).choice(len(sims), 8, replace=False))
    for i in pick:
        s = sims[i]
        say(f"  member {i}: {s.nx}x{s.ny}")
        one = lb.Sim([s], lb.make_options())
        one.step(100)
        a, b = ens.fields(i), one.fields(0)
        for k in lb.FIELDS:
            assert np.array_equal(a[k], b[k]), (i, k)
        assert np.array_equal(ens.nodes(i)[0], one.nodes(0)[0]), i
        one.close()
    for i in sorted(pick, key=lambda j: sims[j].nx * sims[j].ny)[:3]:
        r = oracle_sim(sims[i])
        r.run(100)
        g, o = ens.fields(i), r.observe()
        errs = {k: linf_rel(g[k], o[k]) for k in ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy")}
        say(f"  member {i} vs oracle: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        for k, v in errs.items():
            assert v <= 1e-4, (i, k, v)
    ens.step(900)
    by_size = sorted(range(len(sims)), key=lambda j: (sims[j].nx * sims[j].ny, j))
    for i in (by_size[0], by_size[len(sims) // 2]):
        s = sims[i]
        say(f"  member {i} ({s.nx}x{s.ny}, D_p {s.meta['D_p']:.3g}, R {s.meta['radius']:.1f}) vs oracle at 1000 steps")
        r = oracle_sim(s)
        r.run(1000)
        g, o = ens.fields(i), r.observe()
        errs = {k: linf_rel(g[k], o[k]) for k in ("vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy")}
        say("    " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        for k, v in errs.items():
            assert v <= 1e-4, (i, k, v)
        d = float(np.max(np.abs(ens.nodes(i)[0] - r.bodies[0].R)))
        say(f"    node error {d:.1e}")
        assert d <= 1e-5
    ens.close()


def test_autotune_cache(tmp_path):
    """lb_options.autotune_cache: the first tuned create appends its shape under the workload's key;
    a second create of the same workload takes the shape from the file without timing (the same
    shape and stored milliseconds, no new line); another workload adds its own line; a garbled
    file only means tuning again."""
    cache = str(tmp_path / "tune.txt")
    opt = lb.make_options(autotune=1, autotune_cache=cache)
    w = wl.small_case(65, 96, 80, n_bodies=1)
    say("case autotune cache 96x80 and 64x48 seed=65")

    def shape(work):
        g = lb.Sim(work, opt)
        s = g.launch_shape()
        g.step(4)
        g.sync()
        g.close()
        return s

    def lines():
        with open(cache) as f:
            return f.read().splitlines()

    a = shape(w)
    assert len(lines()) == 1 and lines()[0].startswith("lbtune1 ") and a["tuned_ms"] > 0
    b = shape(w)
    assert b == a, (a, b)
    assert len(lines()) == 1
    shape(wl.small_case(65, 64, 48, n_bodies=1))
    assert len(lines()) == 2
    with open(cache, "w") as f:
        f.write("garbage\nlbtune1 zz 1 2\n")
    c = shape(w)
    assert (c["threads"] in (64, 128, 256)) and c["tuned_ms"] > 0
    assert len(lines()) == 3


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


def test_scalar_variant_matches_tensorial_path():
    """With P = 0 in every simulation the field kernel runs its variant without the polarization
    work (the scalar model, Sec. II B).  At P = 0 the tensorial arithmetic reduces to the same
    operations plus exact zeros (Ericksen stress, anisotropic stiffness), so a P = 0 simulation
    alone (scalar variant) and batched with a polarized one (tensorial variant) agree to FP32
    rounding (the compiler may fuse multiply-adds differently in the two instantiations)."""
    scalar = wl.trap_case(52, 72, 56, k_trap=0.5, walls=2, P_eq=0.0).sims[0]
    polar = wl.small_case(53, 64, 48).sims[0]
    say("case scalar variant vs tensorial path, 72x56 box trap + 64x48 polarized, 300 steps")
    one = lb.Sim([scalar], lb.make_options(seg_rows=8))
    both = lb.Sim([scalar, polar], lb.make_options(seg_rows=8))
    one.step(300)
    both.step(300)
    a, b = one.fields(0), both.fields(0)
    for k in ("vx", "vy", "sxx", "syy", "sxy"):
        e = linf_rel(a[k], b[k])
        say(f"  {k} {e:.1e}")
        assert e <= 1e-6, k
    assert np.max(np.abs(a["rho"] - b["rho"])) <= 1e-6
    assert np.all(a["Px"] == 0) and np.all(a["Py"] == 0) and np.all(b["Px"] == 0)
    assert np.max(np.abs(one.nodes(0)[0] - both.nodes(0)[0])) <= 1e-7


def test_scalar_variant_matches_oracle():
    w = wl.trap_case(54, 64, 48, k_trap=0.5, walls=2, P_eq=0.0)
    say("case scalar variant vs oracle, 64x48 box trap, 600 steps")
    g = lb.Sim(w, lb.make_options(seg_rows=12))
    r = oracle_sim(w.sims[0])
    g.step(600)
    r.run(600)
    gf, of = g.fields(), r.observe()
    for k in ("vx", "vy", "sxx", "syy", "sxy"):
        e = linf_rel(gf[k], of[k])
        say(f"  {k} {e:.2e}")
        assert e <= 1e-4, k
    assert np.max(np.abs(g.nodes()[0] - r.bodies[0].R)) <= 1e-5
