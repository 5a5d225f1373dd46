"""GPU tests of single kernels through the C ABI.

The trailing update C <- C - diag(ia) Aq Bq^T diag(ib) is checked against its
definition evaluated in FP64 from the same quantised operands; the bound is
FP32 accumulation (K+2 roundings of 2^-24 relative to the magnitudes
involved) plus one rounding to the storage format.
"""
import numpy as np
import pytest
import torch

import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu

TORCH_OP = {"f16": torch.float16, "bf16": torch.bfloat16, "f8": torch.float8_e4m3fn, "f32": torch.float32}
TORCH_ST = {"f16": torch.float16, "bf16": torch.bfloat16, "f32": torch.float32}
U_ST = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8, "f32": 2.0 ** -24}
# half the spacing of the storage format's subnormals: the absolute error of a
# rounding that lands below its smallest normal number
SUB_ST = {"f16": 2.0 ** -25, "bf16": 2.0 ** -134, "f32": 2.0 ** -150}


def _pad(x, m):
    return (x + m - 1) // m * m


@pytest.mark.parametrize("M,N,K,update,store", [
    (256, 256, 512, "f16", "f16"),
    (300, 520, 512, "f16", "f16"),
    (1000, 777, 256, "bf16", "bf16"),
    (513, 257, 128, "f8", "f16"),
    (640, 384, 512, "f8", "bf16"),
    (200, 333, 64, "f32", "f32"),
    (384, 129, 128, "f16", "f32"),
    (1, 1, 64, "bf16", "f32"),
])
def test_trailing_update_matches_definition(M, N, K, update, store):
    _run_update(M, N, K, update, store, aligned=False)


# ldc a multiple of 8 elements (16-byte columns) with whole 256 x 128 tiles:
# the production epilogue (C half-tile loaded at the first stage, LDS-staged
# read-modify-write, streaming stores); the last shapes mix full and edge tiles
@pytest.mark.parametrize("M,N,K,update,store", [
    (1024, 1024, 512, "f16", "f16"),
    (1024, 768, 512, "bf16", "bf16"),
    (768, 1024, 512, "f8", "f16"),
    (512, 512, 1024, "f8", "bf16"),
    (1000, 900, 512, "f16", "f16"),
    (1300, 517, 256, "f8", "f16"),
])
def test_trailing_update_full_tiles_aligned(M, N, K, update, store):
    _run_update(M, N, K, update, store, aligned=True)


# two block steps in one pass (mxp_trailing_update2): the second segment
# with other scale factors, some rows and columns with both
@pytest.mark.parametrize("M,N,K1,K2,update,store,aligned", [
    (1024, 1024, 512, 512, "f16", "f16", True),
    (1000, 900, 512, 512, "bf16", "bf16", True),
    (768, 1024, 256, 256, "f8", "f16", True),
    (1300, 517, 128, 128, "f8", "bf16", True),
    (300, 520, 512, 512, "f16", "f16", False),
    (200, 333, 64, 64, "f32", "f32", False),
    (384, 129, 128, 256, "f16", "f32", False),
])
def test_two_step_update_matches_definition(M, N, K1, K2, update, store, aligned):
    _run_update(M, N, K1, update, store, aligned=aligned, K2=K2)


def _operands(g, Mp, Np, K, update):
    A = torch.rand((Mp, K), generator=g, dtype=torch.float64) * 2 - 1
    B = torch.rand((Np, K), generator=g, dtype=torch.float64) * 2 - 1
    scale_op = 200.0 if update == "f8" else 1.0
    Aq = (A.float() * scale_op).to(TORCH_OP[update])
    Bq = (B.float() * scale_op).to(TORCH_OP[update])
    ia = torch.pow(2.0, torch.randint(-20, -5, (Mp // 32,), generator=g).double()).float()
    ib = torch.pow(2.0, torch.randint(-8, 3, (Np // 32,), generator=g).double()).float()
    return Aq, Bq, ia, ib


def _run_update(M, N, K, update, store, aligned, K2=0):
    print("gemm", M, N, K, K2, update, store, "aligned" if aligned else "", flush=True)
    g = torch.Generator().manual_seed(M * 7 + N + K2)
    Mp, Np = _pad(M, 256), _pad(N, 256)
    segs = [_operands(g, Mp, Np, K, update)] + ([_operands(g, Mp, Np, K2, update)] if K2 else [])
    if aligned:
        ldc = _pad(M, 8) + 64
    else:
        ldc = M + 3 if store != "f32" else M + 4
    C = (torch.rand((N, ldc), generator=g, dtype=torch.float64) * 8 - 4).to(TORCH_ST[store])
    Cd = C.cuda()
    if K2:
        (A1, B1, a1, b1), (A2, B2, a2, b2) = segs
        mxp.mxp_trailing_update2(Cd, ldc, M, N, K, K2, update, store, A1.cuda(), B1.cuda(), a1.cuda(), b1.cuda(),
                                 A2.cuda(), B2.cuda(), a2.cuda(), b2.cuda())
    else:
        Aq, Bq, ia, ib = segs[0]
        mxp.mxp_trailing_update(Cd, ldc, M, N, K, update, store, Aq.cuda(), Bq.cuda(), ia.cuda(), ib.cuda())
    got = Cd.cpu().double()
    C0 = C.double().numpy()[:, :M].T           # M x N
    prod = np.zeros((M, N))
    mag = np.abs(C0)
    for Aq, Bq, ia, ib in segs:
        a = Aq.double()[:M].numpy()
        b = Bq.double()[:N].numpy()
        da = np.repeat(ia.double().numpy(), 32)[:M]
        db = np.repeat(ib.double().numpy(), 32)[:N]
        prod += (a @ b.T) * da[:, None] * db[None, :]
        mag = mag + (np.abs(a) @ np.abs(b).T) * da[:, None] * db[None, :]
    ref = C0 - prod
    bound = U_ST[store] * np.abs(ref) + SUB_ST[store] + (K + K2 + 2) * 2.0 ** -24 * mag
    err = np.abs(got.numpy()[:, :M].T - ref)
    assert np.all(err <= bound), float((err / bound).max())
    # padding rows of C (ld > M) untouched
    assert torch.equal(got[:, M:], C.double()[:, M:])
