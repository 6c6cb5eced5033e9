"""Allocation-free isotropic loss entry point: called through the C ABI, it
matches rgx_isotropic_loss bit for bit (same kernels, fixed per-device
workspace instead of an allocated one) on two calls in a row, the second
with fewer Gaussians than the first."""
import ctypes as C

import numpy as np
import pytest

from paper_2509_07782_amd import lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _call(fn, ctx, t, r0, loss, grad, accumulate, stream):
    rc = fn(ctx.h, int(t.shape[0]), C.c_void_p(t.data_ptr()), C.c_float(r0),
            C.c_void_p(loss.data_ptr()), C.c_void_p(grad.data_ptr()), int(accumulate),
            C.c_void_p(stream))
    lib.check(rc, ctx.h, fn.__name__)


def test_noalloc_matches_allocating_entry_point(torch_cuda):
    torch = torch_cuda
    L = lib.load()
    ctx = lib.Context(0)
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(11)
    r0 = 10.0
    for n in (1_000_003, 70_001):                   # second call smaller than the first
        ls = torch.from_numpy(rng.normal(-4.0, 1.0, (n, 3)).astype(np.float32)).cuda()
        out = {}
        for name in ("rgx_isotropic_loss", "rgx_isotropic_loss_noalloc"):
            loss = torch.full((), float("nan"), device="cuda")
            grad = torch.full((n, 3), float("nan"), device="cuda")
            _call(getattr(L, name), ctx, ls, r0, loss, grad, 0, stream)
            # accumulate mode adds the same gradient again
            grad2 = grad.clone()
            _call(getattr(L, name), ctx, ls, r0, loss, grad2, 1, stream)
            torch.cuda.synchronize()
            out[name] = (float(loss), grad.cpu().numpy(), grad2.cpu().numpy())
        a, b = out["rgx_isotropic_loss"], out["rgx_isotropic_loss_noalloc"]
        assert np.isfinite(a[0]) and a[0] > 0
        assert a[0] == b[0], (n, a[0], b[0])
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[2], b[2])
        assert np.array_equal(b[2], 2 * b[1])
    # sizes past the fixed workspace are rejected before anything runs
    loss = torch.zeros((), device="cuda")
    grad = torch.zeros((4, 3), device="cuda")
    rc = L.rgx_isotropic_loss_noalloc(ctx.h, (1 << 23) + 1, C.c_void_p(grad.data_ptr()),
                                      C.c_float(r0), C.c_void_p(loss.data_ptr()),
                                      C.c_void_p(grad.data_ptr()), 0, C.c_void_p(stream))
    assert rc == -1
    ctx.close()
