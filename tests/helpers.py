"""Shared test helpers: turn a seeded workload into an oracle simulation, and compare fields.

Only inputs are shared between the oracle and the GPU path (paper_2209_14889_amd.workload)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2209_14889_amd import workload as wl


def oracle_params(sim: "wl.SimSpec", **over) -> dict:
    p = sim.params
    d = dict(nx=sim.nx, ny=sim.ny, tau=p["tau"], Kx=p["Kx"], eta_p=p["eta_p"], D_p=p["D_p"],
             xi=p["xi"], alpha=p["alpha"], beta=p["beta"], kappa=p["kappa"], Gamma=p["Gamma"],
             P_clamp=p["P_clamp"], ericksen=p["ericksen"], walls=p.get("walls", 0), gx=p.get("gx", 0.0),
             gy=p.get("gy", 0.0))
    d.update(over)
    return d


def oracle_sim(sim: "wl.SimSpec", **over) -> oracle.Sim:
    bodies = [oracle.Body(R=b.R.copy(), k_spring=b.k_spring, eps_angle=b.eps_angle, l_eq=b.l_eq,
                          pull=b.pull, t_on=b.t_on, t_off=b.t_off, width=b.width, trap=b.trap)
              for b in sim.bodies]
    sig = sim.sigma0 if sim.sigma0 is not None else None
    return oracle.Sim(oracle_params(sim, **over), bodies=bodies, P=sim.P0.copy(), sigma=sig)


def linf_rel(a: np.ndarray, ref: np.ndarray) -> float:
    """max |a - ref| / max |ref| (the L-infinity-normalised relative error)."""
    den = float(np.max(np.abs(ref)))
    num = float(np.max(np.abs(a - ref)))
    if den == 0.0:
        return num
    return num / den
