"""bamg_mlp_loss_grad_noalloc (the entry point for callers that cannot
allocate device memory) against bamg_mlp_loss_grad, through the C ABI: the
same kernels on the same inputs, so loss and gradient agree bit for bit.
Two calls in a row, the second with fewer points (the fixed scratch keeps
the first call's contents), then a call beyond the documented maximum,
which is rejected without running anything."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

bamg = pytest.importorskip("paper_1402_4005_amd")

MAX_POINTS = 60000  # BAMG_MLP_NOALLOC_MAX_POINTS in include/bamg.h


def _data(seed, n):
    import torch
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, bamg.MLP_IN)).astype(np.float32)
    T = rng.standard_normal((n, bamg.MLP_OUT)).astype(np.float32)
    M = (rng.random((n, bamg.MLP_OUT)) < 0.6).astype(np.float32)
    return [torch.from_numpy(a).cuda() for a in (X, T, M)]


def _call(fn, net, X, T, M, n):
    import torch
    g = torch.full((bamg.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    loss = C.c_double(float("nan"))
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(net.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), C.c_void_p(M.data_ptr()),
            C.c_int64(n), C.byref(loss), C.c_void_p(g.data_ptr()), s)
    return st, loss.value, g.cpu().numpy()


def test_noalloc_loss_grad_equals_allocating_entry_point():
    lib = bamg.lib()
    fn = lib.bamg_mlp_loss_grad_noalloc
    fn.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
    ref = lib.bamg_mlp_loss_grad
    net = bamg.MLP(bamg.mlp_init_params(7))
    for seed, n in ((1, 50000), (2, 3001)):
        X, T, M = _data(seed, n)
        st_a, loss_a, g_a = _call(fn, net, X, T, M, n)
        st_b, loss_b, g_b = _call(ref, net, X, T, M, n)
        assert st_a == 0 and st_b == 0
        assert np.isfinite(loss_a) and np.all(np.isfinite(g_a))
        assert loss_a == loss_b, (n, loss_a, loss_b)
        assert np.array_equal(g_a, g_b), (n, np.abs(g_a - g_b).max())
    # beyond the fixed scratch: a clean argument error
    X, T, M = _data(3, 8)
    st, _, _ = _call(fn, net, X, T, M, MAX_POINTS + 1)
    assert st == -1
    assert b"no-allocation maximum" in lib.bamg_last_error()
    net.close()
