"""mxp_residual_noalloc: the regenerating residual with the library's own
file-scope scratch array instead of a caller work buffer, for callers that
cannot allocate.  Checked through the C ABI against mxp_residual (same
kernels, so equal bit for bit) on two calls in a row, the second smaller,
and for its size limit."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu


def _noalloc():
    f = mxp.lib().mxp_residual_noalloc
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    f.restype = ctypes.c_int
    f.argtypes = [I64, ctypes.c_uint64, ctypes.c_int, P, P, I64, P, I64, P, I64, I64, P]
    return f


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def test_noalloc_residual_matches_residual_twice():
    f = _noalloc()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, nrhs, kind, gamma, seed in ((20001, 5, mxp.GEN_DOMINANT, 0.0, 3), (1027, 2, mxp.GEN_SQRTN, 0.6, 4)):
        print("noalloc residual", n, nrhs, kind, flush=True)
        prob = mxp.mxp_generate(n, nrhs, seed, store="f16", with_matrix=False, kind=kind, gamma=gamma)
        X = torch.from_numpy(np.random.default_rng(n).uniform(-1, 1, (nrhs, n))).cuda()
        want = mxp.mxp_residual(prob, X, prob.B)
        R = torch.full((nrhs, n), float("nan"), dtype=torch.float64, device="cuda")
        rc = f(n, seed, kind, _ptr(prob.diag), _ptr(X), n, _ptr(prob.B), n, _ptr(R), n, nrhs, stream)
        assert rc == 0, mxp.lib().mxp_last_error()
        torch.cuda.synchronize()
        assert torch.equal(R, want)
        # without B: R = A X
        want2 = mxp.mxp_residual(prob, X, None)
        rc = f(n, seed, kind, _ptr(prob.diag), _ptr(X), n, None, n, _ptr(R), n, nrhs, stream)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(R, want2)


def test_noalloc_residual_rejects_sizes_beyond_its_scratch():
    f = _noalloc()
    L = mxp.lib()
    n = 1 << 20
    assert L.mxp_residual_work_bytes(n, 8) > 32 << 20
    fake = ctypes.c_void_p(256)
    rc = f(n, 1, mxp.GEN_DOMINANT, fake, fake, n, None, n, fake, n, 8, None)
    assert rc == mxp.EINVAL
    assert b"scratch" in L.mxp_last_error()
