"""The largest lattice the library accepts: 16384 columns (the side limit) by 6103 rows, 99 991 552
sites under the 1e8-site limit.  There the 32-bit byte offsets into the population planes reach
3.6 GB (FP32) and every work-item table, site-block grid and read-back buffer is at its largest.

The oracle cannot step 1e8 sites inside a test, so the check is a property that holds at any size.
A state that repeats every 128 columns stays periodic: every site's update depends only on its
neighbours, and the fused kernel's results do not depend on how the lattice is cut into work
items (the launch-shape test shows it bit for bit).  So each step of the large lattice must equal,
bit for bit, the same steps of one 128-column period, tiled across it.  That period is checked
against the oracle like every other parity case."""
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import lb, workload as wl
from tests.helpers import linf_rel, oracle_sim

pytestmark = pytest.mark.gpu

NX, NY, PERIOD, STEPS = 16384, 6103, 128, 3
NAMES = ["rho", "vx", "vy", "sxx", "syy", "sxy", "Px", "Py", "fpx", "fpy"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def periodic_pair(seed: int, walls: int):
    """(one period, the largest lattice made of NX / PERIOD copies of it): random directors of
    magnitude sqrt(0.9) and a random initial stress, both FP32-representable, no bodies."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, np.pi, size=(NY, PERIOD))
    P = wl.director_field(th, np.sqrt(0.9))
    sig = rng.normal(0.0, 2e-3, size=(3, NY, PERIOD)).astype(np.float32).astype(np.float64)
    params = wl.base_params(50.0, 0.05, walls=walls)
    small = wl.Workload("period", [wl.SimSpec(PERIOD, NY, params, P, [], sigma0=sig)], STEPS, "fp32", {})
    reps = NX // PERIOD
    big = wl.Workload("largest", [wl.SimSpec(NX, NY, params, np.tile(P, (1, 1, reps)), [],
                                             sigma0=np.tile(sig, (1, 1, reps)))], STEPS, "fp32", {})
    return small, big


@pytest.mark.parametrize("precision,walls,tol", [(0, 0, 1e-4), (1, 0, 1e-3), (0, 1, 1e-4)],
                         ids=["fp32-periodic", "fp16-periodic", "fp32-channel"])
def test_largest_lattice_equals_its_tiled_period(precision, walls, tol):
    small, big = periodic_pair(52, walls)
    say(f"case largest lattice {NX}x{NY} ({NX * NY} sites) = {NX // PERIOD} x period {PERIOD}x{NY}, "
        f"seed=52 precision={precision} walls={walls}, {STEPS} steps")
    opt = lb.make_options(precision=precision)
    g = lb.Sim(small, opt)
    g.step(STEPS)
    fs = g.fields(names=NAMES)
    g.close()
    r = oracle_sim(small.sims[0])
    r.run(STEPS)
    o = r.observe()
    for nm in NAMES:
        # the density as its offset rho - 1, which is what the populations store
        e = linf_rel(fs[nm] - 1.0, o[nm] - 1.0) if nm == "rho" else linf_rel(fs[nm], o[nm])
        say(f"  period vs oracle {nm}: {e:.2e}")
        assert e <= tol, (nm, e)
    if precision == 0:
        assert float(np.max(np.abs(fs["rho"] - o["rho"]))) <= 1e-6
    if walls:
        # the walls act: the rows next to them differ from the periodic run of the same state
        g = lb.Sim(periodic_pair(52, 0)[0], opt)
        g.step(STEPS)
        fp = g.fields(names=["vy"])["vy"]
        g.close()
        assert np.max(np.abs(fs["vy"][0] - fp[0])) > 0 and np.max(np.abs(fs["vy"][-1] - fp[-1])) > 0
    say("  period done; stepping the largest lattice")
    g = lb.Sim(big, opt)
    g.step(STEPS)
    fb = g.fields(names=NAMES)
    g.close()
    for nm in NAMES:
        tiled = np.tile(fs[nm], (1, NX // PERIOD))
        same = np.array_equal(fb[nm], tiled)
        if not same:
            bad = np.argwhere(fb[nm] != tiled)
            say(f"  {nm}: {len(bad)} sites differ, first at (y, x) = {tuple(bad[0])}")
        assert same, nm
    say("  largest lattice equals the tiled period in every field")
