"""Plain FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY: used by tests/ to
check the GPU network's products and gradients; it shares no code with the GPU library).

Network: widths w[0] -> ... -> w[L], tanh after every layer but the last; parameters in one flat
array, layer by layer: W_l (w[l+1] x w[l], row major) then b_l.  Loss: mean over rows of the
squared relative L2 error |yhat_i - y_i|^2 / |y_i|^2.  Gradients follow the chain rule layer by
layer (no automatic differentiation).

`rnd`, if given, is applied to both operands of every matrix product (e.g. rounding to BF16), so
that a reduced-precision product can be checked against the same products taken in FP64."""
from __future__ import annotations

import numpy as np


def unpack(params: np.ndarray, widths):
    out, o = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = params[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == params.size
    return out


def _identity(a):
    return a


def forward(params, widths, X, rnd=_identity):
    """Activations of every layer; the last entry is the output."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    for l, (W, b) in enumerate(layers):
        z = rnd(acts[-1]) @ rnd(W).T + b
        acts.append(np.tanh(z) if l + 1 < len(layers) else z)
    return acts


def loss(params, widths, X, Y):
    Yh = forward(params, widths, X)[-1]
    Y = np.asarray(Y, dtype=np.float64)
    return float(np.mean(np.sum((Yh - Y) ** 2, axis=1) / np.sum(Y ** 2, axis=1)))


def gradients(params, widths, X, Y, rnd=_identity):
    params = np.asarray(params, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    acts = forward(params, widths, X, rnd)
    layers = unpack(params, widths)
    B = Y.shape[0]
    y2 = np.sum(Y ** 2, axis=1, keepdims=True)
    dz = 2.0 * (acts[-1] - Y) / y2 / B          # output layer is linear
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gW = rnd(dz).T @ rnd(acts[l])
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if l > 0:
            dz = (rnd(dz) @ rnd(W)) * (1.0 - acts[l] ** 2)   # through tanh of layer l-1
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return np.concatenate(flat)
