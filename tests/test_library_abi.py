"""CPU checks of the C-ABI library: it loads and exports every function that
include/mxp.h declares, and the size queries and argument checks behave
(no device work is launched by these calls)."""
import ctypes
import os
import re

import pytest

import paper_2509_19618_amd as mxp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mxp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mxp_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("mxp_generate", "mxp_factor", "mxp_solve_ir"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(mxp.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(mxp.exported_symbols()) == set(_declared())


def test_size_queries():
    L = mxp.lib()
    n, nb = 32768, 512
    aux = L.mxp_factor_aux_bytes(n, nb)
    # FP32 diagonal blocks + two sets of 64x64 inverses dominate
    assert aux >= n * nb * 4 + 2 * n * 64 * 4
    w16 = L.mxp_factor_work_bytes(n, nb, mxp.F16)
    w8 = L.mxp_factor_work_bytes(n, nb, mxp.F8E4M3)
    assert w16 > w8 > 0
    assert L.mxp_solve_work_bytes(n, 1, 30) >= n * 31 * 8
    assert L.mxp_solve_work_bytes(n, 1, 0) == 0
    assert L.mxp_factor_work_bytes(n, nb, 99) == 0


def test_argument_errors_return_einval_without_device_work():
    L = mxp.lib()
    # NULL diag / a_inf, bad n: rejected before anything is enqueued
    assert L.mxp_generate(0, 0, 1, mxp.GEN_DOMINANT, 0.0, mxp.F16, None, 0, None, 0, None, None, None,
                          None) == mxp.EINVAL
    assert L.mxp_generate(16, 0, 1, mxp.GEN_DOMINANT, 0.0, mxp.F16, None, 16, None, 16, None, None, None,
                          None) == mxp.EINVAL
    assert b"mxp_generate" in L.mxp_last_error()
    fake = ctypes.c_void_p(256)
    # an unknown matrix kind, a sqrt(n) diagonal without a positive coefficient
    assert L.mxp_generate(16, 0, 1, 7, 0.0, mxp.F16, None, 16, None, 16, fake, None, fake, None) == mxp.EINVAL
    assert L.mxp_generate(16, 0, 1, mxp.GEN_SQRTN, 0.0, mxp.F16, None, 16, None, 16, fake, None, fake,
                          None) == mxp.EINVAL
    assert L.mxp_generate(16, 0, 1, mxp.GEN_SQRTN, -1.0, mxp.F16, None, 16, None, 16, fake, None, fake,
                          None) == mxp.EINVAL
    # bad (update, store) pair, bad nb
    fake = ctypes.c_void_p(256)
    assert L.mxp_factor(64, 64, mxp.F16, mxp.BF16, 0, None, fake, 64, fake, fake, 1 << 30, None, None) == mxp.EINVAL
    assert L.mxp_factor(64, 96, mxp.F16, mxp.F16, 0, None, fake, 64, fake, fake, 1 << 30, None, None) == mxp.EINVAL
    assert L.mxp_factor(64, 64, mxp.F8E4M3, mxp.F16, 0, None, fake, 64, fake, fake, 1 << 30, None, None) == mxp.EINVAL
    # workspace too small
    assert L.mxp_factor(64, 64, mxp.F16, mxp.F16, 0, None, fake, 64, fake, fake, 16, None, None) == mxp.EWORKSPACE
    # row equilibration without the diagonal
    assert L.mxp_factor(64, 64, mxp.F16, mxp.F16, 1, None, fake, 64, fake, fake, 1 << 30, None, None) == mxp.EINVAL
    # the two-step update: a second segment of zero or ragged length, a bad format pair
    f = fake
    assert L.mxp_trailing_update2(64, 64, 64, 0, mxp.F16, mxp.F16, f, 64, f, f, f, f, f, f, f, f, None) == mxp.EINVAL
    assert L.mxp_trailing_update2(64, 64, 64, 48, mxp.F16, mxp.F16, f, 64, f, f, f, f, f, f, f, f, None) == mxp.EINVAL
    assert L.mxp_trailing_update2(64, 64, 64, 64, mxp.F16, mxp.BF16, f, 64, f, f, f, f, f, f, f, f, None) == mxp.EINVAL
    assert L.mxp_trailing_update2(64, 64, 64, 64, mxp.F16, mxp.F16, f, 64, f, f, f, f, None, f, f, f, None) == mxp.EINVAL
    # nothing to update: no device work, no error
    assert L.mxp_trailing_update2(0, 64, 64, 64, mxp.F16, mxp.F16, None, 1, None, None, None, None, None, None, None,
                                  None, None) == mxp.OK


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(mxp, "_lib", None)
    monkeypatch.setattr(mxp, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        mxp.lib()


def test_server_request_bytes_and_argument_checks():
    L = mxp.lib()
    b = [mxp.server_request_bytes(n, 1, 256) for n in (512, 1024, 4096, 16384)]
    assert all(x > 0 for x in b) and b == sorted(b)
    # at least A (16-bit, padded leading dimension) plus B, X and the factor's aux space
    for n, x in zip((512, 1024, 4096, 16384), b):
        assert x >= n * n * 2 + 2 * n * 8 + L.mxp_factor_aux_bytes(n, 256)
    assert mxp.server_request_bytes(4096, 8, 256) > mxp.server_request_bytes(4096, 1, 256)
    assert mxp.server_request_bytes(0, 1, 256) == 0
    assert mxp.server_request_bytes(512, 0, 256) == 0
    # invalid configurations are rejected before any device call
    cfg = mxp._ServerCfg(0, mxp.BF16, mxp.BF16, 0, 0, 30, 50, 16.0, 2.0 ** -50)
    h = ctypes.c_void_p()
    assert L.mxp_server_create(0, ctypes.c_void_p(256), 1 << 20, ctypes.byref(cfg), ctypes.byref(h)) == mxp.EINVAL
    cfg = mxp._ServerCfg(2, mxp.BF16, mxp.BF16, 96, 0, 30, 50, 16.0, 2.0 ** -50)
    assert L.mxp_server_create(0, ctypes.c_void_p(256), 1 << 20, ctypes.byref(cfg), ctypes.byref(h)) == mxp.EINVAL
    assert L.mxp_server_submit(None, 512, 1, 1, None, ctypes.byref(ctypes.c_uint64())) == mxp.EINVAL


def test_profile_classes_mask_and_read_without_device_work():
    """mxp_profile_enable takes a bitmask of kernel classes; reading a class
    with nothing timed returns zeros, an unknown class is rejected (no HIP
    call is made by any of these)."""
    L = ctypes.CDLL(mxp.LIB_PATH)
    L.mxp_profile_read.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4
    assert L.mxp_profile_reset() == 0
    assert L.mxp_profile_enable(1 << mxp.PROF_GEMM) == 0
    ms, fl, by = ctypes.c_double(-1), ctypes.c_double(-1), ctypes.c_double(-1)
    cnt = ctypes.c_int64(-1)
    args = [ctypes.addressof(ms), ctypes.addressof(fl), ctypes.addressof(by), ctypes.addressof(cnt)]
    assert L.mxp_profile_read(mxp.PROF_TRSM, *args) == 0
    assert (ms.value, fl.value, by.value, cnt.value) == (0.0, 0.0, 0.0, 0)
    assert L.mxp_profile_read(99, *args) != 0
    assert L.mxp_profile_read(-1, *args) != 0
    assert L.mxp_profile_enable(0) == 0
    mxp.profile_enable(True, classes=[mxp.PROF_GEMM, mxp.PROF_DIAG])
    mxp.profile_enable(False)


def test_factor_layout_query():
    """The aux/work layout query: parts in order, inside the sizes the
    *_bytes queries give, 256-byte aligned, and rejected for bad sizes."""
    L = mxp.lib()
    for n, nb, up in ((32768, 512, mxp.F16), (1000, 128, mxp.F8E4M3), (65, 64, mxp.F32)):
        lay = mxp.factor_layout(n, nb, up)
        aux = [lay.T, lay.Trm, lay.linv, lay.uinv, lay.lsc, lay.rowscale, lay.linv_full, lay.uinv_full, lay.aux_bytes]
        work = [lay.Lq, lay.Uq, lay.inv_sa, lay.inv_sb, lay.info, lay.work_bytes]
        assert aux == sorted(aux) and work == sorted(work)
        assert all(x % 256 == 0 for x in aux + work)
        assert lay.aux_bytes == L.mxp_factor_aux_bytes(n, nb)
        assert lay.work_bytes == L.mxp_factor_work_bytes(n, nb, up)
        nblk = -(-n // nb)
        assert lay.strips == -(-n // 32) and lay.op_rows >= n
        assert lay.Trm - lay.T >= nblk * nb * nb * 4 and lay.rowscale - lay.lsc >= nblk * lay.strips * 4
        esz = {mxp.F16: 2, mxp.F8E4M3: 1, mxp.F32: 4}[up]
        assert lay.Uq - lay.Lq >= 2 * lay.op_rows * nb * esz
    with pytest.raises(mxp.MxpError):
        mxp.factor_layout(0, 64, mxp.F16)
    with pytest.raises(mxp.MxpError):
        mxp.factor_layout(100, 96, mxp.F16)
