"""Element-wise error bounds for the surrogate network's GPU products (test helper, no GPU).

The library rounds both operands of every matrix product to BF16 (nearest even, from FP32) and
accumulates exact BF16 x BF16 products in FP32; bias, tanh and the tanh derivative are FP32
epilogues.  Each layer is checked as a function of the GPU's own inputs to it: the reference is
the oracle's layer (oracle/mlp.py: the same BF16-rounded operands, FP64 arithmetic) applied to the
GPU's inputs to that layer, which the tests read back:

* forward: from prefixes of the network (a network of the first k layers runs the same kernels on
  the same data, so it returns the full network's k-th pre-activation bit for bit);
* backward: from single-row gradient calls, whose bias gradients are the row's pre-activation
  gradients themselves; a batch of 2^m rows then scales each row's values by exactly 2^-m.

Per element the two can then differ only by:

* FP32 accumulation: at most gamma_n = n u / (1 - n u) times the sum of |terms| (u = 2^-24, any
  order of the n additions);
* an operand the GPU holds in FP32 within a bound e of the reference's value (its own tanhf, or
  an upstream result of the backward pass) and rounds to another BF16 neighbour: rounding is
  monotone, so the two BF16 values differ by at most bf16(x + e) - bf16(x - e), zero unless a
  rounding midpoint lies within e of x;
* the FP32 epilogues: tanhf within a few ulp (TANH_ULPS) of its result, products and differences
  rounded once each."""
from __future__ import annotations

import numpy as np

import oracle.mlp as omlp

U = 2.0 ** -24          # FP32 unit roundoff
TANH_ULPS = 8.0         # allowance for the GPU's tanhf against tanh, in units of u |result|


def bf16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(torch.bfloat16).to(
        torch.float64).numpy()


def gamma(n: int) -> float:
    return n * U / (1.0 - n * U)


def bf16_spread(x: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Largest possible |bf16(y) - bf16(x)| over y within e of x (monotone rounding)."""
    return bf16(x + e) - bf16(x - e)


def hidden(z_gpu: np.ndarray):
    """The input the next layer takes from an FP32 pre-activation: tanh in FP64 and the bound on
    the GPU's tanhf of the same FP32 value."""
    a = np.tanh(np.asarray(z_gpu, dtype=np.float64))
    return a, TANH_ULPS * U * np.abs(a) + 1e-38


def layer_bound(A, EA, W, b):
    """Reference pre-activation bf16(A) bf16(W)^T + b in FP64 and a per-element bound on the GPU's
    FP32 result for an input within EA of A."""
    K = W.shape[1]
    bA, dA, bW = bf16(A), bf16_spread(A, EA), bf16(W)
    z = bA @ bW.T + b
    ez = dA @ np.abs(bW).T + gamma(K + 1) * ((np.abs(bA) + dA) @ np.abs(bW).T + np.abs(b))
    return z, ez


def output_grad_bound(Yh_gpu, Y, batch: int):
    """Reference d loss / d yhat = 2 (yhat - y) / (|y|^2 batch) from the GPU's FP32 output, and the
    bound on the GPU's FP32 value: an FP32 sum of N squares for |y|^2, one reciprocal, a
    difference, products and a division."""
    Yh = np.asarray(Yh_gpu, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N = Y.shape[1]
    dz = 2.0 * (Yh - Y) / np.sum(Y * Y, axis=1, keepdims=True) / batch
    return dz, (N + 8) * U * np.abs(dz) + 1e-45


def backward_layer_bound(dz, A, EA, W, first: bool):
    """One layer of the backward pass from the GPU's own FP32 gradient dz (batch x N) of the layer's
    pre-activation and the layer's input A (batch x K, within EA of the GPU's): reference dW
    (N x K), db (N) and, unless first, the previous layer's pre-activation gradient
    (bf16(dz) bf16(W)) * (1 - A^2), each with a per-element bound on the GPU's FP32 result."""
    dz = np.asarray(dz, dtype=np.float64)
    B = dz.shape[0]
    bdz = bf16(dz)
    bA, dA = bf16(A), bf16_spread(A, EA)
    gW = bdz.T @ bA
    egW = np.abs(bdz).T @ dA + gamma(B) * (np.abs(bdz).T @ (np.abs(bA) + dA))
    gb = dz.sum(axis=0)
    egb = gamma(B) * np.abs(dz).sum(axis=0) + 1e-45
    if first:
        return gW, egW, gb, egb, None, None
    bW = bf16(W)
    s = bdz @ bW
    es = gamma(W.shape[0]) * (np.abs(bdz) @ np.abs(bW))
    g = 1.0 - A * A
    eg = 2.0 * np.abs(A) * EA + EA * EA + U * (A * A + np.abs(g))
    dzp = s * g
    edzp = np.abs(g) * es + (np.abs(s) + es) * eg + U * np.abs(dzp) + 1e-45
    return gW, egW, gb, egb, dzp, edzp


def prefix_params(params, widths, k: int) -> np.ndarray:
    """Parameters of the network made of the first k layers."""
    n = sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(k))
    return np.asarray(params)[:n]
