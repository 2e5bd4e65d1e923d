"""lb_mlp_forward_noalloc: the network's forward pass with its hidden activations in the library's
fixed scratch array, called through the C ABI with caller-owned parameters, inputs and outputs, and
no allocation in the call.  It runs the same kernels on the same data as lb_mlp_forward, so its
outputs must equal that entry point's bit for bit: two calls in a row, the second with a smaller
batch (the scratch keeps the first call's values, which the second must not read)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WIDTHS = [5, 256, 256, 256, 64]


def _data(seed, B):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(B, WIDTHS[0])).astype(np.float32)


def test_noalloc_forward_equals_handle_forward():
    import torch
    from paper_2209_14889_amd import lb, mlp
    params = mlp.init_params(WIDTHS, 21)
    rng = np.random.default_rng(22)
    o = 0
    for l in range(len(WIDTHS) - 1):   # non-zero biases
        o += WIDTHS[l + 1] * WIDTHS[l]
        params[o:o + WIDTHS[l + 1]] = rng.uniform(-0.1, 0.1, WIDTHS[l + 1])
        o += WIDTHS[l + 1]
    net = mlp.MLP(WIDTHS, 512)
    net.set_params(params)
    p_dev = torch.from_numpy(params).cuda()
    for batch, seed in ((512, 23), (77, 24)):
        print(f"case noalloc forward batch {batch} seed {seed}", flush=True)
        X = torch.from_numpy(_data(seed, batch)).cuda()
        ref = net.forward(X).cpu().numpy()
        Y = torch.full((batch, WIDTHS[-1]), float("nan"), dtype=torch.float32, device="cuda")
        mlp.forward_noalloc(WIDTHS, p_dev, X, Y)
        torch.cuda.synchronize()
        got = Y.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    net.close()


def test_noalloc_forward_rejects_batches_beyond_the_scratch():
    """batch x widest hidden layer beyond 2^19 values is refused before anything is queued."""
    import torch
    from paper_2209_14889_amd import lb, mlp
    cfg = mlp.make_config(WIDTHS, 1)
    batch = (1 << 19) // 256 + 1
    p = torch.zeros(mlp.n_params(WIDTHS), dtype=torch.float32, device="cuda")
    X = torch.zeros((1, WIDTHS[0]), dtype=torch.float32, device="cuda")
    Y = torch.zeros((1, WIDTHS[-1]), dtype=torch.float32, device="cuda")
    rc = mlp.lib().lb_mlp_forward_noalloc(ctypes.byref(cfg), ctypes.c_void_p(p.data_ptr()),
                                          ctypes.c_void_p(X.data_ptr()), batch, ctypes.c_void_p(Y.data_ptr()), None)
    assert rc == lb.LB_ERANGE
