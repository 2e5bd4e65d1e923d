"""Pins of the host-side inputs of the paper-size run and of its observable.

The unit system of the paper's experiment follows from Table I (lattice spacing, time step and
solvent density), and every converted parameter of `workload.paper_case` is checked here against
the printed SI values of Tables I-IV (tests/golden/paper_values.json) through that unit system,
not through the workload's own table of units.  The Return of Sec. III is checked on closed forms.
"""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2209_14889_amd import experiment
from paper_2209_14889_amd import workload as wl

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
T1 = GOLD["table_I_lattice"]["value"]
T2 = GOLD["table_II_droplet"]["value"]
T4 = GOLD["table_IV_si"]["value"]
T3 = GOLD["table_III_beris_edwards"]["value"]


def units_from_table_I():
    """Lattice units in SI: length dx, time dt, mass rho_s dx^3 (lattice density 1)."""
    dx, dt, rho = T1["dx_m"], T1["dt_s"], T1["rho_kg_m3"]
    mass = rho * dx ** 3
    force = mass * dx / dt ** 2
    return dict(length=dx, time=dt, stress=force / dx ** 2, viscosity=force / dx ** 2 * dt,
                diffusivity=dx ** 2 / dt, stiffness=force / dx, energy=force * dx)


def test_unit_system_follows_from_table_I():
    ref = units_from_table_I()
    assert math.isclose(ref["stress"], 500.0, rel_tol=1e-12)   # rho_s dx^2 / dt^2
    for k, v in ref.items():
        assert math.isclose(wl.PAPER_UNITS[k], v, rel_tol=1e-12), k


def test_tau_gives_the_solvent_viscosity_of_table_I():
    # eta_s = rho nu = rho cs^2 (tau - 1/2) in lattice units (Sec. II A), rho = 1
    p = wl.paper_case().sims[0].params
    assert p["tau"] == T1["tau"]
    cs2 = GOLD["viscosity_relation"]["value"]["cs2"]
    eta = cs2 * (p["tau"] - 0.5) * units_from_table_I()["viscosity"]
    assert math.isclose(eta, T1["eta_s_Pa_s"], rel_tol=1e-12)


def test_paper_case_converts_tables_I_to_IV():
    U = units_from_table_I()
    w = wl.paper_case()
    s = w.sims[0]
    p = s.params
    assert (s.nx, s.ny) == (T1["nx"], T1["ny"]) and w.steps == T1["steps"] and p["walls"] == 2
    # Table IV through the stress, viscosity and diffusivity units
    kx = [T4[k] / U["stress"] for k in ("K1111_Pa", "K1122_Pa", "K2222_Pa", "K1212_Pa")]
    assert np.allclose(p["Kx"], kx, rtol=1e-12, atol=0)
    assert math.isclose(p["eta_p"], T4["eta_p_Pa_s"] / U["viscosity"], rel_tol=1e-12)   # 25
    assert math.isclose(p["D_p"], T4["D_p_m2_s"] / U["diffusivity"], rel_tol=1e-12)      # 5e-4
    # Table III: free-energy coefficients in units of the stress (the default reading)
    assert p["xi"] == T3["xi"] and p["Gamma"] == T3["Gamma"]
    for k in ("alpha", "beta", "kappa"):
        assert math.isclose(p[k], T3[k] / U["stress"], rel_tol=1e-12), k
    # the initial polarization has the equilibrium magnitude sqrt(-alpha / beta) of the printed
    # numbers (unchanged by the common unit) along theta0 = 0
    P_eq = GOLD["equilibrium_polarization"]["value"]
    assert np.allclose(s.P0[0], P_eq, rtol=1e-6) and np.all(s.P0[1] == 0)
    # Table II: droplet and trap
    b = s.bodies[0]
    R = T2["R_m"] / U["length"]                      # 12.5 sites
    n = round(2 * math.pi * R / (T2["l_eq_m"] / U["length"]))
    assert len(b.R) == n == 157
    c = b.R.mean(axis=0)
    assert np.allclose(np.hypot(*(b.R - c).T), R, rtol=1e-12)
    assert math.isclose(b.l_eq, T2["l_eq_m"] / U["length"], rel_tol=2e-3)   # chord of the polygon
    assert math.isclose(b.k_spring, T2["k_spring_N_m"] / U["stiffness"], rel_tol=1e-12)      # 0.5
    assert math.isclose(b.eps_angle, T2["eps_angle_N_m"] / U["energy"], rel_tol=1e-12)       # 0.3125
    tr = b.trap
    assert math.isclose(tr["k"], T2["k_trap_N_m"] / U["stiffness"], rel_tol=1e-12)           # 0.05
    assert math.isclose(tr["dx"], T2["d_pull_m"] / U["length"], rel_tol=1e-12) and tr["dy"] == 0.0
    assert math.isclose(tr["t2"] - tr["t1"], T2["T_pull_s"] / U["time"], rel_tol=1e-12)      # 25 000
    assert (tr["x0"], tr["y0"]) == (float(c[0]), float(c[1]))     # the trap starts on the droplet
    # the droplet is pulled along x and ends centred in the box
    assert math.isclose(c[0] + tr["dx"] / 2, s.nx / 2, abs_tol=1e-9)


def test_paper_case_readings_and_scalar_model():
    U = units_from_table_I()
    p = wl.paper_case(fe_units="lattice").sims[0].params
    for k in ("alpha", "beta", "kappa"):
        assert p[k] == T3[k], k
    with pytest.raises(ValueError):
        wl.paper_case(fe_units="kPa")
    s = wl.paper_case(scalar=True).sims[0]
    C = T4["C_Pa"] / U["stress"]
    assert np.allclose(s.params["Kx"], (C, 0.0, C, C / 2), rtol=1e-12, atol=0)
    assert s.params["ericksen"] == 0 and not np.any(s.P0)


def test_return_closed_forms():
    # Return = 1 - d_rec / d_pull (Sec. III), d_rec the distance of the final centre from the start
    assert experiment.return_value((10.0, 20.0), (10.0, 20.0), 100.0) == 1.0     # back at the start
    assert experiment.return_value((0.0, 0.0), (100.0, 0.0), 100.0) == 0.0       # no recoil at all
    assert experiment.return_value((5.0, 5.0), (55.0, 5.0), 100.0) == 0.5
    assert math.isclose(experiment.return_value((0.0, 0.0), (30.0, 40.0), 100.0), 0.5)   # off axis
    assert experiment.return_value((0.0, 0.0), (-50.0, 0.0), 100.0) == 0.5       # overshoot back


def test_wall_speeds_split_the_box_into_wall_band_and_bulk():
    """The wall-mode diagnostic of the sweeps: the largest speed within `band` sites of any wall,
    and elsewhere.  A stand-in for the simulation supplies the two velocity planes."""
    class Fields:
        def __init__(self, vx, vy):
            self.vx, self.vy = vx, vy

        def fields(self, names=None):
            return {"vx": self.vx, "vy": self.vy}

    ny, nx = 20, 30
    vx, vy = np.zeros((ny, nx)), np.zeros((ny, nx))
    vx[1, 15] = 3.0          # inside the band at the south wall
    vy[10, 28] = 4.0         # inside the band at the east wall
    vx[10, 15], vy[10, 15] = 0.6, 0.8   # bulk, |v| = 1
    vx[2, 2] = 2.0           # just outside a two-site band: bulk
    wall, bulk = experiment.wall_speeds(Fields(vx, vy), band=2)
    assert wall == 4.0 and bulk == 2.0
    wall, bulk = experiment.wall_speeds(Fields(vx, vy), band=3)   # (2, 2) joins the band
    assert wall == 4.0 and bulk == 1.0


def test_bench_refuses_several_gpus():
    bench = os.path.join(os.path.dirname(HERE), "bench.py")
    r = subprocess.run([sys.executable, bench, "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
