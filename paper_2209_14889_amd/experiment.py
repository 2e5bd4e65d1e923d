"""The paper's pull-and-release experiment (Sec. III, App. C) run through the library at its own
size: the droplet is dragged by the switched, moving harmonic trap and let go, and the distance of
its centre of mass from where it started is followed to the end of the protocol.

    Return = 1 - d_rec / d_pull   (Sec. III), d_rec the final distance from the starting point.

Sweeps: the tensorial model over the equilibrium polarization (through alpha, |P| = sqrt(-alpha))
and the initial director angle theta0 with the pull along x, as in the results on anisotropy; the
scalar model (Sec. II B) over the stress diffusion D_p.

Each run is its own simulation, so a run the library stops (its watchdog: a non-finite or drifting
mass, a body outgrowing its force patch) is reported with the step it stopped at and does not end
the sweep.  Besides the trajectory every run reports the largest speed in the two site rows along
the walls and elsewhere: a flow that grows at the walls rather than around the droplet is the wall
mode of the explicit flow-alignment coupling and makes a run's Return meaningless.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lb
from . import workload as wl


def return_value(com0, com_end, d_pull: float) -> float:
    """Return = 1 - d_rec / d_pull (Sec. III); d_rec is the Euclidean distance of the final centre
    of mass from the initial one (the droplet may leave the pull axis when the director is oblique)."""
    d = np.asarray(com_end, dtype=np.float64) - np.asarray(com0, dtype=np.float64)
    return 1.0 - float(math.hypot(d[0], d[1])) / d_pull


def wall_speeds(sim: "lb.Sim", band: int = 2) -> tuple[float, float]:
    """(largest |v| within `band` sites of a wall, largest |v| elsewhere) for a closed box."""
    f = sim.fields(names=["vx", "vy"])
    v = np.hypot(f["vx"], f["vy"])
    mask = np.zeros(v.shape, dtype=bool)
    mask[:band, :] = mask[-band:, :] = True
    mask[:, :band] = mask[:, -band:] = True
    return float(v[mask].max()), float(v[~mask].max())


def run_protocol(w: "wl.Workload", steps: int = wl.PAPER_STEPS, every: int = 2500, graph_chunk: int = 100,
                 log=None) -> dict:
    """Run one single-simulation workload through `steps` steps, sampling the centre of mass every
    `every` steps; returns the trajectory, the Return and the wall diagnostics."""
    spec = w.sims[0]
    d_pull = float(spec.meta["d_pull"])
    sim = lb.Sim(w, lb.make_options(graph_chunk=graph_chunk))
    try:
        com0 = sim.body_forces()[0, 4:6].copy()
        traj, failure, t = [], None, 0
        t0 = time.perf_counter()
        while t < steps:
            n = min(every, steps - t)
            try:
                sim.step(n)
                sim.sync()
            except lb.LBError as e:
                failure = f"stopped at step {sim.t}: {e}"
                break
            t += n
            com = sim.body_forces()[0, 4:6]
            traj.append((t, round(float(math.hypot(*(com - com0))), 5)))
        wall_s = time.perf_counter() - t0
        out = dict(steps=t, seconds=round(wall_s, 3), failure=failure, trajectory=traj)
        if failure is None:
            com = sim.body_forces()[0, 4:6]
            out["return"] = round(return_value(com0, com, d_pull), 5)
            out["final_com"] = [round(float(c), 4) for c in com]
            vw, vb = wall_speeds(sim)
            out["wall_v"], out["bulk_v"] = vw, vb
        else:
            out["return"] = None
        return out
    finally:
        sim.close()


def alpha_theta_sweep(alphas, thetas, steps: int = wl.PAPER_STEPS, fe_units: str = "Pa", log=print):
    """Return over (alpha, theta0) for the tensorial model, pull along x (results on anisotropy).
    alpha is Table III's number; fe_units says what unit it and beta, kappa are read in."""
    rows = []
    for a in alphas:
        for th in thetas:
            w = wl.paper_case(alpha=a, theta0=th, fe_units=fe_units)
            r = run_protocol(w, steps)
            r.update(alpha=a, theta0=round(th, 6), fe_units=fe_units)
            rows.append(r)
            if log:
                log(json.dumps({k: v for k, v in r.items() if k != "trajectory"}))
    return rows


def dp_sweep(dps, steps: int = wl.PAPER_STEPS, scalar: bool = True, log=print):
    """Return over the stress diffusion D_p (m^2/s) for the scalar model (results on D_p)."""
    rows = []
    for d in dps:
        w = wl.paper_case(D_p=d, scalar=scalar)
        r = run_protocol(w, steps)
        r.update(D_p=d, model="scalar" if scalar else "tensorial")
        rows.append(r)
        if log:
            log(json.dumps({k: v for k, v in r.items() if k != "trajectory"}))
    return rows


def scalar_sweep(name: str, values, steps: int = wl.PAPER_STEPS, log=print):
    """Return of the scalar model over the droplet radius (name "radius_m", metres) or the pull
    time (name "T_pull_s", seconds), the other inputs at Tables I-IV."""
    rows = []
    for v in values:
        w = wl.paper_case(scalar=True, **{name: v})
        r = run_protocol(w, steps)
        r.update(model="scalar", **{name: v})
        rows.append(r)
        if log:
            log(json.dumps({k: v for k, v in r.items() if k != "trajectory"}))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--sweep", choices=["alpha-theta", "dp", "radius", "tpull"], default="alpha-theta")
    ap.add_argument("--alphas", default="0,-0.3,-0.6,-0.9")
    ap.add_argument("--thetas", default="0,30,60,90,120,150", help="degrees")
    ap.add_argument("--dps", default="1e-15,1e-14,1e-13,1e-12", help="m^2/s")
    ap.add_argument("--radii", default="3.2e-7,5e-7,7.2e-7,9.2e-7,1.12e-6", help="m")
    ap.add_argument("--tpulls", default="0.05,0.1,0.2,0.4", help="s")
    ap.add_argument("--steps", type=int, default=wl.PAPER_STEPS)
    ap.add_argument("--fe-units", choices=["Pa", "lattice"], default="Pa",
                    help="unit of Table III's free-energy coefficients (see workload.paper_case)")
    ap.add_argument("--out", default="", help="write every run (with its trajectory) as JSON here")
    a = ap.parse_args(argv)

    def log(s):
        print(s, flush=True)

    if a.sweep == "alpha-theta":
        rows = alpha_theta_sweep([float(x) for x in a.alphas.split(",")],
                                 [math.radians(float(x)) for x in a.thetas.split(",")], a.steps, a.fe_units, log)
    elif a.sweep == "dp":
        rows = dp_sweep([float(x) for x in a.dps.split(",")], a.steps, True, log)
    elif a.sweep == "radius":
        rows = scalar_sweep("radius_m", [float(x) for x in a.radii.split(",")], a.steps, log)
    else:
        rows = scalar_sweep("T_pull_s", [float(x) for x in a.tpulls.split(",")], a.steps, log)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
