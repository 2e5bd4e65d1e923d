"""Host-side logic of the surrogate (no GPU): the input normalisation, the calibration of the error
estimate and the fallback rule.  The networks' predictions and the LB runs are replaced by
stand-ins, so only the arithmetic of these three steps is under test."""
import math

import numpy as np

from paper_2209_14889_amd import surrogate as sg
from paper_2209_14889_amd import workload as wl


def test_features_map_the_sampled_ranges_onto_the_unit_box():
    lo = dict(D_p=0.001, relax=20.0, radius=4.0, theta0=0.0, P_eq=0.0)
    hi = dict(D_p=0.2, relax=400.0, radius=16.0, theta0=math.pi / 2, P_eq=0.95)
    mid = dict(D_p=math.sqrt(0.001 * 0.2), relax=math.sqrt(20.0 * 400.0), radius=10.0, theta0=math.pi / 4,
               P_eq=0.475)
    x = sg.features([lo, hi, mid])
    assert x.dtype == np.float32 and x.shape == (3, 5)
    assert np.allclose(x[0], -1.0, atol=1e-6) and np.allclose(x[1], 1.0, atol=1e-6)
    assert np.allclose(x[2], 0.0, atol=1e-6)   # log-scaled inputs at their geometric means
    xs = sg.features([wl.surrogate_inputs(s) for s in range(3000, 3200)])
    assert np.all(np.abs(xs) <= 1.0 + 1e-6)


def _surrogate_with(mean, spread):
    s = object.__new__(sg.Surrogate)   # no networks: predict() is the stand-in below
    s.predict = lambda X: (mean, spread)
    s.factor, s.threshold = 1.0, 0.02
    return s


def test_calibration_bounds_the_error_on_the_requested_share_of_rows():
    rng = np.random.default_rng(5)
    n, k = 400, 64
    Y = rng.normal(1.0, 0.1, size=(n, k))
    spread = rng.uniform(1e-3, 1e-2, size=n)
    # errors about 3x the spread, with scatter
    err_dir = rng.normal(size=(n, k))
    err_dir /= np.linalg.norm(err_dir, axis=1, keepdims=True)
    rel = 3.0 * spread * rng.lognormal(0.0, 0.3, size=n)
    mean = Y + err_dir * (rel * np.linalg.norm(Y, axis=1))[:, None]
    s = _surrogate_with(mean, spread)
    thr = s.calibrate(None, Y, target=0.02, coverage=0.95)
    err = np.linalg.norm(mean - Y, axis=1) / np.linalg.norm(Y, axis=1)
    covered = np.mean(s.factor * spread >= err - 1e-15)
    assert 0.95 <= covered <= 0.95 + 2.0 / n    # the estimate bounds the error on 95% of the rows
    assert math.isclose(thr, 0.02 / s.factor) and math.isclose(s.threshold, thr)
    assert 3.0 < s.factor < 6.0                 # close to the planted ratio of about 3


def test_fallback_replaces_exactly_the_rows_whose_spread_exceeds_the_threshold(monkeypatch):
    n, k = 10, 4
    mean = np.arange(n * k, dtype=np.float64).reshape(n, k)
    spread = np.array([0.001, 0.02, 0.003, 0.5, 0.0, 0.011, 0.01, 0.2, 0.009, 0.0101])
    s = _surrogate_with(mean, spread)
    s.threshold = 0.01
    calls = []

    def fake_simulate(seeds, batch=512, **kw):
        calls.append(list(seeds))
        return None, -np.ones((len(seeds), k)) * np.asarray(seeds, dtype=np.float64)[:, None]

    monkeypatch.setattr(sg, "simulate", fake_simulate)
    seeds = list(range(100, 100 + n))
    out, info = s.predict_with_fallback(seeds, X=np.zeros((n, 5), dtype=np.float32))
    fb = [1, 3, 5, 7, 9]                          # spread > 0.01 (0.01 itself stays)
    assert list(info["fallback"]) == fb and calls == [[seeds[i] for i in fb]]
    for i in range(n):
        expect = -np.full(k, seeds[i], dtype=np.float64) if i in fb else mean[i]
        assert np.array_equal(out[i], expect), i
