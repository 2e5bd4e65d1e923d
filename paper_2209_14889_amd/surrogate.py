"""Learned surrogate of the body's restoring-force time series, with the lattice Boltzmann run as
fallback and as the reference for its error.

Inputs (5): stress diffusion D_p, relaxation time, body radius, director angle to the pull, and
polarization magnitude P_eq (alpha = -P_eq^2).  Output: the viscoelastic restoring force on the
body along the pull (the integral of div sigma^p over the body, Sec. III and Fig. 6) sampled every
64 steps of a 4096-step pull-and-release run on a 128 x 128 lattice (64 samples).  The integral is
taken with area weights (each site's div sigma^p times the area of its unit cell inside the node
polygon): the plain sum over the sites inside jumps by whole sites as the outline moves across the
lattice, by around 10 per cent between radii 0.1 apart, which no smooth map of the five inputs can
follow to a few per cent; the area-weighted form varies continuously.

Training data comes from batched LB ensembles run by the library; the networks (an ensemble of M
members with different seeds) are trained by the library's own forward/backward/Adam kernels.  The
spread of the members estimates the error of their mean; rows whose estimate exceeds the threshold
are simulated instead.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import lb, mlp
from . import workload as wl

WIDTHS = [5, 256, 256, 256, 64]


def features(inputs) -> np.ndarray:
    """Map the five parameters to [-1, 1]."""
    x = []
    for d in inputs:
        x.append([
            math.log(d["D_p"] / 0.001) / math.log(200.0),
            math.log(d["relax"] / 20.0) / math.log(20.0),
            (d["radius"] - 4.0) / 12.0,
            d["theta0"] / (math.pi / 2),
            d["P_eq"] / 0.95,
        ])
    return (2.0 * np.asarray(x, dtype=np.float64) - 1.0).astype(np.float32)


OBSERVABLES = ("force", "force_sites", "distance")


def simulate(seeds, batch: int = 512, n: int = wl.C5_N, steps: int = wl.C5_STEPS,
             every: int = wl.C5_SAMPLE_EVERY, observable: str = "force", log=None):
    """Run the LB method for the given seeds in batched ensembles; returns (inputs, series) with
    series[i, k] the observable after (k+1)*every steps: "force" (area-weighted restoring force
    along the pull, +x), "force_sites" (the inside-site sum along +x), "distance" (centre-of-mass
    displacement along +x), or "all" (a dict of the three)."""
    seeds = list(seeds)
    inputs, series = [], {k: [] for k in OBSERVABLES}
    import torch
    for c0 in range(0, len(seeds), batch):
        chunk = seeds[c0:c0 + batch]
        specs = [wl.surrogate_member(s, n) for s in chunk]
        sim = lb.Sim(specs, lb.make_options(graph_chunk=every if every % 2 == 0 else 0))
        x0 = sim.body_forces()[:, 4]
        n_samples = steps // every
        # every sample is queued on the device and read back once at the end: no synchronisation
        # inside the run
        samples = torch.empty((n_samples, len(chunk), 8), dtype=torch.float64, device=sim.device)
        for k in range(n_samples):
            sim.step(every)
            sim.body_forces_device(samples[k])
        sim.sync()
        raw = samples.cpu().numpy()
        cur = {"force": raw[:, :, 6].T.copy(), "force_sites": raw[:, :, 0].T.copy(),
               "distance": raw[:, :, 2].T - x0[:, None]}
        sim.close()
        inputs += [s.meta for s in specs]
        for k in OBSERVABLES:
            series[k].append(cur[k])
        if log:
            log(f"surrogate: simulated {c0 + len(chunk)}/{len(seeds)} runs")
    out = {k: np.concatenate(v) for k, v in series.items()}
    return inputs, (out if observable == "all" else out[observable])


class Surrogate:
    def __init__(self, members: int = 4, widths=WIDTHS, seed: int = 0, max_batch: int = 4096,
                 device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.widths = list(widths)
        self.device = device
        self.nets = [mlp.MLP(widths, max_batch, device) for _ in range(members)]
        for i, net in enumerate(self.nets):
            net.set_params(mlp.init_params(widths, seed + 1000 * i))
        self.scale = 1.0
        self.factor = 1.0
        self.threshold = 0.02

    def _t(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)

    def fit(self, X, Y, epochs: int = 3600, batch: int = 256, lr: float = 2e-3, lr_min: float = 2e-5,
            seed: int = 0, log=None):
        """Adam with cosine learning-rate decay on the mean squared relative error of each series.
        The members train concurrently, each on its own stream and its own shuffling of the data."""
        torch = self.torch
        self.scale = float(np.sqrt(np.mean(np.asarray(Y) ** 2)))
        Xt, Yt = self._t(X), self._t(np.asarray(Y) / self.scale)
        n = Xt.shape[0]
        rngs = [np.random.default_rng(seed + 7919 * m) for m in range(len(self.nets))]
        steps_per_epoch = max(1, n // batch)
        total = epochs * steps_per_epoch
        losses = [torch.zeros(1, dtype=torch.float32, device=self.device) for _ in self.nets]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step = 0
        for ep in range(epochs):
            shuffled = []
            for r in rngs:
                perm = torch.as_tensor(r.permutation(n)[:steps_per_epoch * batch], device=self.device)
                shuffled.append((Xt[perm].contiguous(), Yt[perm].contiguous()))
            torch.cuda.synchronize()   # the shuffled copies are complete before the networks' streams read them
            for b in range(steps_per_epoch):
                lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / total))
                for net, (Xe, Ye), loss in zip(self.nets, shuffled, losses):
                    net.train_step(Xe[b * batch:(b + 1) * batch], Ye[b * batch:(b + 1) * batch], lr_t, loss)
                step += 1
            for net in self.nets:
                net.stream.synchronize()   # before the shuffled copies are released
            if log and (ep + 1) % max(1, epochs // 6) == 0:
                log(f"surrogate: epoch {ep + 1}/{epochs} batch losses " +
                    " ".join(f"{float(l.item()):.3e}" for l in losses))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def predict(self, X):
        """Ensemble mean, and the relative spread |std| / |mean| of each row (the error estimate)."""
        Xt = self._t(X)
        outs = np.stack([net.forward(Xt).cpu().numpy() for net in self.nets]) * self.scale
        mean = outs.astype(np.float64).mean(axis=0)
        spread = np.linalg.norm(outs.std(axis=0), axis=1) / np.maximum(np.linalg.norm(mean, axis=1), 1e-300)
        return mean, spread

    def calibrate(self, X, Y, target: float = 0.02, coverage: float = 0.95):
        """Error estimate = c * spread, with c the `coverage` quantile over validation rows of
        (true relative error) / spread, so the estimate bounds the error on that share of them.
        A row falls back to the LB when its estimate exceeds `target`; returns the spread
        threshold target / c."""
        mean, spread = self.predict(X)
        err = np.linalg.norm(mean - Y, axis=1) / np.linalg.norm(Y, axis=1)
        self.factor = float(np.quantile(err / np.maximum(spread, 1e-30), coverage))
        self.threshold = target / self.factor
        return self.threshold

    def predict_with_fallback(self, seeds, X=None, batch: int = 512, **sim_kw):
        """Surrogate rows where the spread is at most the threshold; LB for the rest."""
        seeds = list(seeds)
        if X is None:
            X = features([wl.surrogate_inputs(s) for s in seeds])
        t0 = time.perf_counter()
        mean, spread = self.predict(X)
        t_inf = time.perf_counter() - t0
        fb = np.nonzero(spread > self.threshold)[0]
        out = mean.astype(np.float64)
        t1 = time.perf_counter()
        if fb.size:
            _, Yfb = simulate([seeds[i] for i in fb], batch=batch, **sim_kw)
            out[fb] = Yfb
        t_lb = time.perf_counter() - t1
        return out, dict(fallback=fb, t_inference=t_inf, t_fallback=t_lb, spread=spread)


def study(train: int = 4096, test: int = 512, val: int = 512, members: int = 4, epochs: int = 3600,
          batch: int = 256, lr: float = 2e-3, sim_batch: int = 1024, target: float = 0.02, data=None, log=None):
    """Full surrogate study: `train` LB runs (seeds 3000 on; the last `val` held back to calibrate
    the threshold), `test` held-out runs (seeds 9000 on) for the error and the speedup
    T(batched LB of all held-out runs) / (T(ensemble inference) + T(batched LB of the fallback rows)).
    `data`: optional dict with X, Y of the training runs (skips simulating them)."""
    import torch

    seeds = list(range(9000, 9000 + test))
    Xt = features([wl.surrogate_inputs(x) for x in seeds])
    t0 = time.perf_counter()
    if data is not None:
        X, Y = data["X"][:train], data["Y"][:train]
    else:
        inp, Y = simulate(range(3000, 3000 + train), batch=sim_batch, log=log)
        X = features(inp)
    t_data = time.perf_counter() - t0
    ntr = train - val
    s = Surrogate(members=members, max_batch=max(batch, test, val))
    t_fit = s.fit(X[:ntr], Y[:ntr], epochs=epochs, batch=batch, lr=lr, log=log)
    th = s.calibrate(X[ntr:], Y[ntr:], target=target)
    if log:
        log(f"surrogate: error estimate = {s.factor:.3g} x spread; LB when the spread exceeds {th:.4g}")

    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, Yt = simulate(seeds, batch=test)
    t_lb = time.perf_counter() - t1
    s.predict(Xt)   # first call pays one-off costs
    out, info = s.predict_with_fallback(seeds, Xt, batch=test)
    mean, _ = s.predict(Xt)
    err = np.linalg.norm(out - Yt, axis=1) / np.linalg.norm(Yt, axis=1)
    err_nn = np.linalg.norm(mean - Yt, axis=1) / np.linalg.norm(Yt, axis=1)
    t_sur = info["t_inference"] + info["t_fallback"]

    def stats(e):
        return dict(mean=round(float(e.mean()), 6), p95=round(float(np.quantile(e, 0.95)), 6),
                    max=round(float(e.max()), 6), frac_le_target=float(np.mean(e <= target)))

    return dict(
        observable="area-weighted restoring force along the pull, 64 samples", target_rel_l2=target,
        train_runs=train, held_out_runs=test, members=members, widths=s.widths,
        t_lb_data_s=round(t_data, 3), t_fit_s=round(t_fit, 3), estimate_factor=round(s.factor, 4),
        spread_threshold=round(th, 6),
        t_lb_all_s=round(t_lb, 4), t_inference_s=round(info["t_inference"], 5),
        t_fallback_s=round(info["t_fallback"], 4), n_fallback=int(info["fallback"].size),
        speedup=round(t_lb / t_sur, 2), err_with_fallback=stats(err), err_network_only=stats(err_nn),
        # context: the speedup without any fallback, which the target allows only when every
        # held-out row of the network alone is within it (err_network_only.frac_le_target == 1)
        speedup_network_only=round(t_lb / info["t_inference"], 1))


def main(argv=None):
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=study.__doc__)
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--val", type=int, default=512)
    ap.add_argument("--members", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=3600)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--sim-batch", type=int, default=1024)
    ap.add_argument("--target", type=float, default=0.02)
    ap.add_argument("--out", default="")
    ap.add_argument("--save-data", default="", help="only simulate; write every observable of both sets to this .npz")
    ap.add_argument("--load-data", default="", help="read the training series from this .npz")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if a.save_data:
        inp, Yb = simulate(range(3000, 3000 + a.train), batch=a.sim_batch, observable="all", log=log)
        seeds = list(range(9000, 9000 + a.test))
        _, Ytb = simulate(seeds, batch=a.test, observable="all")
        np.savez(a.save_data, X=features(inp), Y=Yb["force"], Yt=Ytb["force"],
                 Xt=features([wl.surrogate_inputs(x) for x in seeds]),
                 **{f"{k}_train": Yb[k] for k in OBSERVABLES}, **{f"{k}_test": Ytb[k] for k in OBSERVABLES})
        return None
    data = dict(np.load(a.load_data)) if a.load_data else None
    res = study(a.train, a.test, a.val, a.members, a.epochs, a.batch, a.lr, a.sim_batch, a.target, data, log)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    return res


if __name__ == "__main__":
    main()
