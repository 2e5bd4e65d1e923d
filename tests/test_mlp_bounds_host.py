"""Host checks of the element-wise bounds the GPU network tests use (tests/mlp_bounds.py):

* the bounded references are the oracle network's own layers and gradients;
* a float32 emulation of the GPU's arithmetic (BF16 operands, FP32 accumulation in another order,
  FP32 epilogues), checked layer by layer on its own inputs as the GPU test does, stays inside
  the bounds on every element;
* the bounds are tight enough to mean something: a small fraction of each element's size, far
  below the change a plausible mistake (a dropped bias) makes."""
import numpy as np

import oracle.mlp as omlp
from tests import mlp_bounds as mb

WIDTHS = [5, 256, 256, 256, 64]


def _params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for l in range(len(WIDTHS) - 1):
        k = 1.0 / np.sqrt(WIDTHS[l])
        out += [rng.uniform(-k, k, WIDTHS[l + 1] * WIDTHS[l]), rng.uniform(-0.1, 0.1, WIDTHS[l + 1])]
    return np.concatenate(out).astype(np.float32).astype(np.float64)


def _data(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(B, WIDTHS[0])).astype(np.float32)
    t = np.linspace(0, 1, WIDTHS[-1])
    Y = np.sin(np.outer(1 + X[:, 0], 3 * t) + X[:, 1:2]) * (1.5 + X[:, 2:3]) + 0.3 * X[:, 3:4] * X[:, 4:5]
    return X.astype(np.float64), Y.astype(np.float32).astype(np.float64)


def _bf32(a):
    return mb.bf16(a).astype(np.float32)


def _emulate(params, X, Y):
    """The GPU's arithmetic in float32: BF16 operands, float32 products and sums (numpy's order),
    float32 bias, tanh and derivative epilogues.  Returns the output, the flat gradients and the
    pre-activation gradient of every layer (index l: layer l)."""
    layers = omlp.unpack(params, WIDTHS)
    a = X.astype(np.float32)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = _bf32(a) @ _bf32(W).T + b.astype(np.float32)
        a = np.tanh(z) if l + 1 < len(layers) else z
        acts.append(a.astype(np.float32))
    Y32 = Y.astype(np.float32)
    B = Y.shape[0]
    y2 = np.sum(Y32 * Y32, axis=1, keepdims=True, dtype=np.float32)
    dz = (np.float32(2.0) * (acts[-1] - Y32) * (np.float32(1.0) / y2) / np.float32(B)).astype(np.float32)
    grads, dzs = [], {}
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dzs[l] = dz
        gW = _bf32(dz).T @ _bf32(acts[l])
        gb = dz.sum(axis=0, dtype=np.float32)
        grads.append((gW, gb))
        if l > 0:
            dz = (_bf32(dz) @ _bf32(W)) * (np.float32(1.0) - acts[l] * acts[l])
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return acts[-1], np.concatenate(flat), dzs


def _split(flat):
    out, o = [], 0
    for l in range(len(WIDTHS) - 1):
        n = WIDTHS[l + 1] * WIDTHS[l]
        out.append((flat[o:o + n].reshape(WIDTHS[l + 1], WIDTHS[l]), flat[o + n:o + n + WIDTHS[l + 1]]))
        o += n + WIDTHS[l + 1]
    return out


def _emulated_prefixes(p, X):
    """Pre-activations of every layer of the float32 emulation (what prefix networks return)."""
    layers = omlp.unpack(p, WIDTHS)
    a = X.astype(np.float32)
    zs = []
    for l, (W, b) in enumerate(layers):
        z = (_bf32(a) @ _bf32(W).T + b.astype(np.float32)).astype(np.float32)
        zs.append(z)
        a = np.tanh(z)
    return zs


def _layer_checks(p, X, zs):
    """Per-layer reference and bound on the emulation's own inputs; returns the activations and
    bounds the gradient check takes."""
    layers = omlp.unpack(p, WIDTHS)
    A, EA = X.astype(np.float64), np.zeros(X.shape)
    acts, errs, out = [A], [EA], []
    for l, (W, b) in enumerate(layers):
        z, ez = mb.layer_bound(A, EA, W, b)
        out.append((z, ez))
        if l + 1 < len(layers):
            A, EA = mb.hidden(zs[l])
            acts.append(A)
            errs.append(EA)
    return acts, errs, out


def test_bounded_reference_is_the_oracle_network():
    p = _params(1)
    X, Y = _data(2, 97)
    # fed the oracle's own values (zero bounds), the layers and the backward steps are the oracle's
    layers = omlp.unpack(p, WIDTHS)
    ref = omlp.forward(p, WIDTHS, X, mb.bf16)
    for l, (W, b) in enumerate(layers):
        z, _ = mb.layer_bound(ref[l], np.zeros(ref[l].shape), W, b)
        assert np.allclose(np.tanh(z) if l + 1 < len(layers) else z, ref[l + 1], rtol=1e-13, atol=1e-15)
    dz, _ = mb.output_grad_bound(ref[-1], Y, X.shape[0])
    flat = []
    for l in range(len(layers) - 1, -1, -1):
        gW, _, gb, _, dz, _ = mb.backward_layer_bound(dz, ref[l], np.zeros(ref[l].shape), layers[l][0], l == 0)
        flat = [gW.ravel(), gb] + flat
    assert np.allclose(np.concatenate(flat), omlp.gradients(p, WIDTHS, X, Y, mb.bf16), rtol=1e-12, atol=1e-18)


def _check_emulation(p, X, Y, tight=False):
    zs = _emulated_prefixes(p, X)
    acts, errs, out = _layer_checks(p, X, zs)
    for (z, ez), zg in zip(out, zs):
        assert np.all(np.abs(zg - z) <= ez)
        if tight:   # the FP32 accumulation bound of K <= 256 terms: a few 1e-5 of the largest value
            rel = ez / np.max(np.abs(z))
            assert np.median(rel) < 1e-4 and np.max(rel) < 2e-3, (np.median(rel), np.max(rel))
    B = X.shape[0]
    y32, g32, dzs = _emulate(p, X, Y)
    assert np.array_equal(y32, zs[-1])
    layers = omlp.unpack(p, WIDTHS)
    dz, edz = mb.output_grad_bound(y32, Y, B)
    assert np.all(np.abs(dzs[3] - dz) <= edz)
    got = _split(g32)
    for l in range(len(layers) - 1, -1, -1):
        gW, egW, gb, egb, dzp, edzp = mb.backward_layer_bound(dzs[l], acts[l], errs[l], layers[l][0], l == 0)
        assert np.all(np.abs(got[l][0] - gW) <= egW), l
        assert np.all(np.abs(got[l][1] - gb) <= egb), l
        if tight:
            assert np.median(egW) < 1e-4 * np.max(np.abs(gW)), (l, np.median(egW) / np.max(np.abs(gW)))
        if l > 0:
            assert np.all(np.abs(dzs[l - 1] - dzp) <= edzp), l


def test_float32_emulation_stays_inside_the_bounds():
    for seed in (3, 4):
        p = _params(seed)
        X, Y = _data(seed + 10, 256)
        _check_emulation(p, X, Y)
        # one row at a time: its bias gradients are its pre-activation gradients
        _check_emulation(p, X[:3], Y[:3])
        _check_emulation(p, X[7:8], Y[7:8])


def test_bounds_are_tight():
    p = _params(5)
    X, Y = _data(15, 256)
    _check_emulation(p, X, Y, tight=True)
    # a plausible mistake (the last bias dropped) breaks the bound on most elements
    zs = _emulated_prefixes(p, X)
    _, _, out = _layer_checks(p, X, zs)
    layers = omlp.unpack(p, WIDTHS)
    z, ez = out[-1]
    assert np.mean(np.abs((z - layers[-1][1]) - z) > ez) > 0.9
