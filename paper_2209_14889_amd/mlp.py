"""ctypes binding of the surrogate network library (include/lb_mlp.h): argument marshalling only.
PyTorch provides the device arena, input/output tensors and the stream; the forward, backward and
Adam kernels are the library's own (BF16 matrix-core products, FP32 accumulation)."""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import lb as _lb


class MLPConfig(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("widths", ctypes.c_int32 * 9), ("max_batch", ctypes.c_int32),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_fp = ctypes.POINTER(ctypes.c_float)
_ready = False


def lib():
    global _ready
    L = _lb.lib()
    if not _ready:
        vp = ctypes.c_void_p
        cfgp = ctypes.POINTER(MLPConfig)
        L.lb_mlp_query_bytes.argtypes = [cfgp, ctypes.POINTER(ctypes.c_size_t)]
        L.lb_mlp_n_params.argtypes = [cfgp, ctypes.POINTER(ctypes.c_size_t)]
        L.lb_mlp_create.argtypes = [cfgp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.lb_mlp_set_params.argtypes = [vp, _fp]
        L.lb_mlp_get_params.argtypes = [vp, _fp]
        L.lb_mlp_forward.argtypes = [vp, vp, ctypes.c_int32, vp]
        L.lb_mlp_gradients.argtypes = [vp, vp, vp, ctypes.c_int32, _fp, _fp]
        L.lb_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp]
        L.lb_mlp_destroy.argtypes = [vp]
        L.lb_mlp_gemm_bf16.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        L.lb_mlp_forward_noalloc.argtypes = [cfgp, vp, vp, ctypes.c_int32, vp, vp]
        for n in ("lb_mlp_query_bytes", "lb_mlp_n_params", "lb_mlp_create", "lb_mlp_set_params", "lb_mlp_get_params",
                  "lb_mlp_forward", "lb_mlp_gradients", "lb_mlp_train_step", "lb_mlp_destroy", "lb_mlp_gemm_bf16",
                  "lb_mlp_forward_noalloc"):
            getattr(L, n).restype = ctypes.c_int
        _ready = True
    return L


def make_config(widths, max_batch: int) -> MLPConfig:
    c = MLPConfig()
    c.n_layers = len(widths) - 1
    c.widths = (ctypes.c_int32 * 9)(*(list(widths) + [0] * (9 - len(widths))))
    c.max_batch = int(max_batch)
    return c


def n_params(widths) -> int:
    n = ctypes.c_size_t(0)
    _lb.check(lib().lb_mlp_n_params(ctypes.byref(make_config(widths, 1)), ctypes.byref(n)))
    return int(n.value)


def init_params(widths, seed: int) -> np.ndarray:
    """Seeded Glorot-uniform weights, zero biases (an input to the network, drawn on the host)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        a = math.sqrt(6.0 / (widths[l] + widths[l + 1]))
        parts.append(rng.uniform(-a, a, size=widths[l + 1] * widths[l]))
        parts.append(np.zeros(widths[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def gemm_bf16(A, B, stream=None):
    """D = A B on the matrix cores (BF16 operands, FP32 accumulation); torch float32 cuda tensors."""
    import torch
    A = A.contiguous()
    B = B.contiguous()
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    D = torch.empty((M, N), dtype=torch.float32, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    _lb.check(lib().lb_mlp_gemm_bf16(_dev(A), _dev(B), _dev(D), M, N, K, ctypes.c_void_p(st.cuda_stream)))
    return D


def forward_noalloc(widths, params, X, Y, stream=None) -> None:
    """Y = network(X) through lb_mlp_forward_noalloc: params, X and Y are float32 cuda tensors the
    caller owns (Y preallocated, batch x widths[-1]); nothing is allocated by the call."""
    import torch
    assert params.is_contiguous() and X.is_contiguous() and Y.is_contiguous()
    st = stream if stream is not None else torch.cuda.current_stream(X.device)
    _lb.check(lib().lb_mlp_forward_noalloc(ctypes.byref(make_config(widths, 1)), _dev(params), _dev(X), X.shape[0],
                                           _dev(Y), ctypes.c_void_p(st.cuda_stream)))


class MLP:
    def __init__(self, widths, max_batch: int, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.widths = list(widths)
        self.cfg = make_config(widths, max_batch)
        self.max_batch = int(max_batch)
        n = ctypes.c_size_t(0)
        _lb.check(lib().lb_mlp_query_bytes(ctypes.byref(self.cfg), ctypes.byref(n)))
        self.arena = torch.empty(int(n.value), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        torch.cuda.current_stream(device).synchronize()
        h = ctypes.c_void_p()
        _lb.check(lib().lb_mlp_create(ctypes.byref(self.cfg), _dev(self.arena), ctypes.c_size_t(self.arena.numel()),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.n_params = n_params(widths)
        self.device = device

    def set_params(self, p: np.ndarray) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        _lb.check(lib().lb_mlp_set_params(self.h, p.ctypes.data_as(_fp)))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        _lb.check(lib().lb_mlp_get_params(self.h, p.ctypes.data_as(_fp)))
        return p

    def _after_torch(self):
        # inputs made on torch's current stream must be complete before the library's stream reads
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def forward(self, X):
        X = X.contiguous()
        self._after_torch()
        Y = self.torch.empty((X.shape[0], self.widths[-1]), dtype=self.torch.float32, device=X.device)
        _lb.check(lib().lb_mlp_forward(self.h, _dev(X), X.shape[0], _dev(Y)))
        self.stream.synchronize()
        return Y

    def gradients(self, X, Y):
        X, Y = X.contiguous(), Y.contiguous()
        self._after_torch()
        loss = np.zeros(1, dtype=np.float32)
        g = np.empty(self.n_params, dtype=np.float32)
        _lb.check(lib().lb_mlp_gradients(self.h, _dev(X), _dev(Y), X.shape[0], loss.ctypes.data_as(_fp),
                                         g.ctypes.data_as(_fp)))
        return float(loss[0]), g

    def train_step(self, X, Y, lr: float, loss_out=None) -> None:
        """Asynchronous on the network's stream; X and Y must already be complete there."""
        _lb.check(lib().lb_mlp_train_step(self.h, _dev(X), _dev(Y), X.shape[0], float(lr),
                                          _dev(loss_out) if loss_out is not None else None))

    def close(self):
        if getattr(self, "h", None):
            lib().lb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
