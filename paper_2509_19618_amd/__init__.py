"""paper_2509_19618_amd -- MI355X (gfx950) mixed-precision LU + GMRES-IR solver.

A thin ctypes binding over ``libmxp.so`` (C ABI declared in
``include/mxp.h``).  Every step of the solve runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch provides device
memory and the current HIP stream.  There is no CPU fallback: if the
library has not been built, every call raises.

Matrices are column-major.  A matrix with leading dimension ``lda`` and
``ncols`` columns is held in a torch tensor of shape ``(ncols, lda)`` whose
row ``j`` is column ``j``; :func:`as_matrix` returns the ``(rows, cols)``
view.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmxp.so")

F64, F32, F16, BF16, F8E4M3 = 0, 1, 2, 3, 4
OK, EINVAL, EWORKSPACE, EHIP, ESINGULAR, ENOCONV, ECRITERION, PENDING = 0, -1, -2, -3, 1, 2, 3, 4
SCALE_NONE, SCALE_ROW_EQUIL = 0, 1
GEN_DOMINANT, GEN_SQRTN, GEN_UNIFORM = 0, 1, 2

_DTYPE = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "f8": F8E4M3, "e4m3": F8E4M3, "fp8": F8E4M3}
_TORCH = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16, F64: torch.float64}


class MxpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libmxp error %d: %s" % (code, msg))
        self.code = code


class _RhsReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("cycles", ctypes.c_int64), ("eta", ctypes.c_double),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class FactorLayout(ctypes.Structure):
    """Byte offsets of the parts of mxp_factor's aux and work buffers (mxp_factor_layout)."""
    _fields_ = [(k, ctypes.c_size_t) for k in ("T", "Trm", "linv", "uinv", "lsc", "rowscale", "linv_full",
                                               "uinv_full", "aux_bytes", "Lq", "Uq", "inv_sa", "inv_sb", "info",
                                               "work_bytes")] + [("op_rows", ctypes.c_int64), ("strips", ctypes.c_int64)]


class _FactorItem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nb", ctypes.c_int64), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("aux", ctypes.c_void_p), ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


TILE_256x128, TILE_128x128 = 0, 1


class _ServerCfg(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("update", ctypes.c_int), ("store", ctypes.c_int), ("nb", ctypes.c_int),
                ("autotune", ctypes.c_int), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("tol", ctypes.c_double), ("tau", ctypes.c_double)]


class _RequestResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("n", ctypes.c_int64), ("nrhs", ctypes.c_int64), ("nb", ctypes.c_int64),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("eta", ctypes.c_double), ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("peak_in_flight", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes_in_use", ctypes.c_size_t), ("groups", ctypes.c_int64),
                ("grouped_requests", ctypes.c_int64), ("peak_group", ctypes.c_int64), ("streams", ctypes.c_int64)]


_lib = None

# (name, restype, argtypes)
_P, _I64, _U64, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = [
    ("mxp_last_error", ctypes.c_char_p, []),
    ("mxp_version", ctypes.c_char_p, []),
    ("mxp_generate", _I, [_I64, _I64, _U64, _I, _D, _I, _P, _I64, _P, _I64, _P, _P, _P, _P]),
    ("mxp_factor_aux_bytes", _SZ, [_I64, _I64]),
    ("mxp_factor_work_bytes", _SZ, [_I64, _I64, _I]),
    ("mxp_factor", _I, [_I64, _I64, _I, _I, _I, _P, _P, _I64, _P, _P, _SZ, _P, _P]),
    ("mxp_factor_get_layout", _I, [_I64, _I64, _I, _P]),
    ("mxp_factor_group", _I, [_I, _P, _I, _I, _I, _P, _P]),
    ("mxp_solve_work_bytes", _SZ, [_I64, _I64, _I]),
    ("mxp_solve_ir", _I, [_I64, _I64, _I, _I, _U64, _I, _P, _I64, _P, _P, _P, _P, _I64, _P, _I64, _I64, _I, _I, _D,
                          _D, _P, _P, _SZ, _P]),
    ("mxp_residual_work_bytes", _SZ, [_I64, _I64]),
    ("mxp_residual", _I, [_I64, _U64, _I, _P, _P, _I64, _P, _I64, _P, _I64, _I64, _P, _SZ, _P]),
    ("mxp_residual_noalloc", _I, [_I64, _U64, _I, _P, _P, _I64, _P, _I64, _P, _I64, _I64, _P]),
    ("mxp_apply_prec_work_bytes", _SZ, [_I64, _I64]),
    ("mxp_apply_prec", _I, [_I64, _I64, _I, _I, _P, _I64, _P, _P, _I64, _P, _I64, _I64, _P, _SZ, _P]),
    ("mxp_hpl_eta_work_bytes", _SZ, [_I64]),
    ("mxp_hpl_eta", _I, [_I64, _U64, _I, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    ("mxp_trailing_update", _I, [_I64, _I64, _I64, _I, _I, _P, _I64, _P, _P, _P, _P, _P]),
    ("mxp_trailing_update2", _I, [_I64, _I64, _I64, _I64, _I, _I, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("mxp_lu64_work_bytes", _SZ, [_I64]),
    ("mxp_trailing_update64", _I, [_I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P]),
    ("mxp_lu64_factor", _I, [_I64, _P, _I64, _P, _I, _P, _SZ, _P, _P]),
    ("mxp_lu64_solve", _I, [_I64, _P, _I64, _P, _P, _I64, _I64, _P]),
    ("mxp_profile_enable", _I, [_I]),
    ("mxp_profile_reset", _I, []),
    ("mxp_profile_read", _I, [_I, _P, _P, _P, _P]),
    ("mxp_server_request_bytes", _SZ, [_I64, _I64, _I64, _I, _I, _I]),
    ("mxp_server_create", _I, [_I, _P, _SZ, _P, _P]),
    ("mxp_server_submit", _I, [_P, _I64, _I64, _U64, _P, _P]),
    ("mxp_server_poll", _I, [_P, _U64, _P]),
    ("mxp_server_wait", _I, [_P, _U64, _P]),
    ("mxp_server_drain", _I, [_P]),
    ("mxp_server_get_stats", _I, [_P, _P]),
    ("mxp_server_block_size", _I64, [_P, _I64]),
    ("mxp_server_tile", _I, [_P, _I64]),
    ("mxp_server_destroy", _I, [_P]),
]

PROF_GEMM, PROF_TRSM, PROF_DIAG, PROF_PREC, PROF_REGEN, PROF_GEMM64 = 0, 1, 2, 3, 4, 6


def lib():
    """Load libmxp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmxp.so is not built (run __graft_entry__.build() or "
                              "python paper_2509_19618_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def dtype_code(d) -> int:
    if isinstance(d, int):
        return d
    return _DTYPE[d]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(code: int, allow_positive: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_positive):
        raise MxpError(code, lib().mxp_last_error().decode())
    return code


def _bytes(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def as_matrix(t: torch.Tensor, rows: int) -> torch.Tensor:
    """(cols, ld) storage -> (rows, cols) view of a column-major matrix."""
    return t[:, :rows].t()


def round_up(a: int, b: int) -> int:
    return (a + b - 1) // b * b


# ------------------------------------------------------------------ problem
@dataclass
class Problem:
    n: int
    nrhs: int
    seed: int
    store: int
    A: torch.Tensor | None      # (n, lda) storage, column-major matrix
    lda: int
    B: torch.Tensor | None      # (nrhs, n) FP64, column-major n x nrhs
    diag: torch.Tensor          # (n,) FP64
    a_inf: torch.Tensor         # (1,) FP64
    kind: int = GEN_DOMINANT
    gamma: float = 0.0
    row_l1: torch.Tensor | None = None   # (n,) FP64


def mxp_generate(n: int, nrhs: int, seed: int, store="f16", with_matrix: bool = True, lda: int | None = None,
                 device="cuda", stream=None, kind: int = GEN_DOMINANT, gamma: float = 0.0) -> Problem:
    st = dtype_code(store)
    lda = lda or round_up(n, 128)
    A = torch.empty((n, lda), dtype=_TORCH[st], device=device) if with_matrix else None
    B = torch.empty((max(nrhs, 1), n), dtype=torch.float64, device=device)
    diag = torch.empty(n, dtype=torch.float64, device=device)
    row_l1 = torch.empty(n, dtype=torch.float64, device=device)
    a_inf = torch.empty(1, dtype=torch.float64, device=device)
    _check(lib().mxp_generate(n, nrhs, seed, kind, gamma, st, _ptr(A), lda, _ptr(B) if nrhs else None, n, _ptr(diag),
                              _ptr(row_l1), _ptr(a_inf), _stream(stream)))
    return Problem(n, nrhs, seed, st, A, lda, B if nrhs else None, diag, a_inf, kind, gamma, row_l1)


# ------------------------------------------------------------------ factor
@dataclass
class Factor:
    n: int
    nb: int
    update: int
    store: int
    LU: torch.Tensor
    lda: int
    aux: torch.Tensor
    info: int
    status: int
    work: torch.Tensor | None = None


def mxp_factor(prob: Problem, nb: int, update="f16", scaling: int = SCALE_NONE, work: torch.Tensor | None = None,
               aux: torch.Tensor | None = None, sync_info: bool = True, stream=None) -> Factor:
    """Factor prob.A in place (A becomes L\\U).  Returns the Factor handle."""
    up = dtype_code(update)
    n, dev = prob.n, prob.A.device
    L = lib()
    if aux is None:
        aux = _bytes(L.mxp_factor_aux_bytes(n, nb), dev)
    wb = L.mxp_factor_work_bytes(n, nb, up)
    if work is None:
        work = _bytes(wb, dev)
    info = ctypes.c_int64(0)
    st = L.mxp_factor(n, nb, up, prob.store, scaling, _ptr(prob.diag), _ptr(prob.A), prob.lda, _ptr(aux),
                      _ptr(work), work.numel(), ctypes.byref(info) if sync_info else None, _stream(stream))
    _check(st, allow_positive=True)
    return Factor(n, nb, up, prob.store, prob.A, prob.lda, aux, int(info.value), st, work)


def mxp_factor_group(probs, nbs, update="bf16", tile: int = TILE_256x128, stream=None):
    """Factor several problems (same storage format) with one launch per kernel
    and block step (mxp_factor_group); returns a Factor per problem."""
    up = dtype_code(update)
    L = lib()
    items = (_FactorItem * len(probs))()
    facs = []
    for i, (prob, nb) in enumerate(zip(probs, nbs)):
        aux = _bytes(L.mxp_factor_aux_bytes(prob.n, nb), prob.A.device)
        work = _bytes(L.mxp_factor_work_bytes(prob.n, nb, up), prob.A.device)
        items[i] = _FactorItem(prob.n, nb, prob.A.data_ptr(), prob.lda, aux.data_ptr(), work.data_ptr(), work.numel())
        facs.append(Factor(prob.n, nb, up, prob.store, prob.A, prob.lda, aux, 0, 0, work))
    info = (ctypes.c_int64 * len(probs))()
    st = L.mxp_factor_group(len(probs), items, up, probs[0].store, tile, info, _stream(stream))
    _check(st, allow_positive=True)
    for f, v in zip(facs, info):
        f.info, f.status = int(v), st
    return facs


def factor_layout(n: int, nb: int, update="f16") -> FactorLayout:
    """Offsets of the parts of mxp_factor's aux and work buffers."""
    out = FactorLayout()
    _check(lib().mxp_factor_get_layout(n, nb, dtype_code(update), ctypes.byref(out)))
    return out


# ------------------------------------------------------------------ solve
@dataclass
class SolveResult:
    X: torch.Tensor          # (nrhs, n) FP64
    iters: list
    cycles: list
    eta: list
    status: list
    code: int


def mxp_solve_ir(prob: Problem, fac: Factor, B: torch.Tensor | None = None, restart: int = 30, max_iters: int = 50,
                 tol: float = 16.0, tau: float = 2.0 ** -50, work: torch.Tensor | None = None,
                 X: torch.Tensor | None = None, stream=None) -> SolveResult:
    B = prob.B if B is None else B
    nrhs, n = B.shape[0], prob.n
    L = lib()
    if work is None:
        work = _bytes(L.mxp_solve_work_bytes(n, nrhs, restart), B.device)
    if X is None:
        X = torch.empty((nrhs, n), dtype=torch.float64, device=B.device)
    reps = (_RhsReport * nrhs)()
    code = L.mxp_solve_ir(n, fac.nb, fac.update, fac.store, prob.seed, prob.kind, _ptr(fac.LU), fac.lda, _ptr(fac.aux),
                          _ptr(prob.diag), _ptr(prob.a_inf), _ptr(B), n, _ptr(X), n, nrhs, restart, max_iters, tol,
                          tau, reps, _ptr(work), work.numel(), _stream(stream))
    _check(code, allow_positive=True)
    return SolveResult(X, [r.iters for r in reps], [r.cycles for r in reps], [r.eta for r in reps],
                       [r.status for r in reps], code)


def mxp_residual(prob: Problem, X: torch.Tensor, B: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """R = B - A X (or A X when B is None) with A regenerated; X is (nrhs, n)."""
    nrhs, n = X.shape[0], prob.n
    L = lib()
    work = _bytes(L.mxp_residual_work_bytes(n, nrhs), X.device)
    R = torch.empty((nrhs, n), dtype=torch.float64, device=X.device)
    _check(L.mxp_residual(n, prob.seed, prob.kind, _ptr(prob.diag), _ptr(X), n, _ptr(B), n, _ptr(R), n, nrhs,
                          _ptr(work), work.numel(), _stream(stream)))
    return R


def mxp_apply_prec(fac: Factor, V: torch.Tensor, stream=None) -> torch.Tensor:
    """Z = M^-1 V for V of shape (nrhs, n)."""
    nrhs, n = V.shape[0], fac.n
    L = lib()
    work = _bytes(L.mxp_apply_prec_work_bytes(n, nrhs), V.device)
    Z = torch.empty_like(V)
    _check(L.mxp_apply_prec(n, fac.nb, fac.update, fac.store, _ptr(fac.LU), fac.lda, _ptr(fac.aux), _ptr(V), n,
                            _ptr(Z), n, nrhs, _ptr(work), work.numel(), _stream(stream)))
    return Z


def mxp_hpl_eta(prob: Problem, x: torch.Tensor, b: torch.Tensor, stream=None) -> float:
    n = prob.n
    L = lib()
    work = _bytes(L.mxp_hpl_eta_work_bytes(n), x.device)
    eta = ctypes.c_double(0.0)
    _check(L.mxp_hpl_eta(n, prob.seed, prob.kind, _ptr(prob.diag), _ptr(prob.a_inf), _ptr(x), _ptr(b),
                         ctypes.byref(eta), _ptr(work), work.numel(), _stream(stream)))
    return float(eta.value)


def mxp_trailing_update(C: torch.Tensor, ldc: int, M: int, N: int, K: int, update, store, Aq: torch.Tensor,
                        Bq: torch.Tensor, inv_sa: torch.Tensor, inv_sb: torch.Tensor, stream=None) -> None:
    """C <- C - diag(inv_sa) Aq Bq^T diag(inv_sb) (see include/mxp.h)."""
    _check(lib().mxp_trailing_update(M, N, K, dtype_code(update), dtype_code(store), _ptr(C), ldc, _ptr(Aq),
                                     _ptr(Bq), _ptr(inv_sa), _ptr(inv_sb), _stream(stream)))


def mxp_trailing_update2(C: torch.Tensor, ldc: int, M: int, N: int, K1: int, K2: int, update, store,
                         Aq1: torch.Tensor, Bq1: torch.Tensor, inv_sa1: torch.Tensor, inv_sb1: torch.Tensor,
                         Aq2: torch.Tensor, Bq2: torch.Tensor, inv_sa2: torch.Tensor, inv_sb2: torch.Tensor,
                         stream=None) -> None:
    """The updates of two block steps in one pass (see include/mxp.h)."""
    _check(lib().mxp_trailing_update2(M, N, K1, K2, dtype_code(update), dtype_code(store), _ptr(C), ldc, _ptr(Aq1),
                                      _ptr(Bq1), _ptr(inv_sa1), _ptr(inv_sb1), _ptr(Aq2), _ptr(Bq2),
                                      _ptr(inv_sa2), _ptr(inv_sb2), _stream(stream)))


# ------------------------------------------------------------------ FP64 LU
@dataclass
class Factor64:
    n: int
    LU: torch.Tensor           # (n, lda) FP64 storage, column-major L\U
    lda: int
    ipiv: torch.Tensor | None  # (n,) int64, 0-based swap rows; None without pivoting
    info: int
    status: int


GEMM64_OWN, GEMM64_ROCBLAS = 0, 1


def mxp_lu64_factor(A: torch.Tensor, n: int, lda: int, pivot: bool, sync_info: bool = True,
                    work: torch.Tensor | None = None, stream=None, gemm: int = GEMM64_OWN) -> Factor64:
    """FP64 LU in place of A ((n, lda) FP64 storage), with or without partial
    pivoting; gemm: the trailing update (GEMM64_OWN or GEMM64_ROCBLAS)."""
    L = lib()
    if work is None:
        work = _bytes(L.mxp_lu64_work_bytes(n), A.device)
    ipiv = torch.empty(n, dtype=torch.int64, device=A.device) if pivot else None
    info = ctypes.c_int64(0)
    st = L.mxp_lu64_factor(n, _ptr(A), lda, _ptr(ipiv), gemm, _ptr(work), work.numel(),
                           ctypes.byref(info) if sync_info else None, _stream(stream))
    _check(st, allow_positive=True)
    return Factor64(n, A, lda, ipiv, int(info.value), st)


def mxp_trailing_update64(C: torch.Tensor, ldc: int, M: int, N: int, K: int, A: torch.Tensor, lda: int,
                          B: torch.Tensor, ldb: int, stream=None) -> None:
    """C <- C - A B in FP64 (column-major, see include/mxp.h)."""
    _check(lib().mxp_trailing_update64(M, N, K, _ptr(C), ldc, _ptr(A), lda, _ptr(B), ldb, _stream(stream)))


def mxp_lu64_solve(fac: Factor64, B: torch.Tensor, stream=None) -> torch.Tensor:
    """X = U^-1 L^-1 P B for B of shape (nrhs, n) FP64 (a new tensor)."""
    X = B.clone()
    _check(lib().mxp_lu64_solve(fac.n, _ptr(fac.LU), fac.lda, _ptr(fac.ipiv), _ptr(X), fac.n, X.shape[0],
                                _stream(stream)))
    return X


def exported_symbols():
    return [name for name, _, _ in SIGNATURES]


def profile_enable(on: bool = True, classes=None) -> None:
    """Time the given kernel classes (PROF_*; all when None) with HIP events, or stop timing."""
    mask = 0
    if on:
        mask = (1 << 7) - 1 if classes is None else sum(1 << int(c) for c in set(classes))
    _check(lib().mxp_profile_enable(mask))


def profile_reset() -> None:
    _check(lib().mxp_profile_reset())


def profile_read(cls: int) -> dict:
    """Summed event time (ms), algorithmic flops and bytes, launches of a kernel class."""
    ms, fl, by, cnt = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().mxp_profile_read(cls, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by), ctypes.byref(cnt)))
    return {"ms": ms.value, "flops": fl.value, "bytes": by.value, "launches": cnt.value}


def server_request_bytes(n: int, nrhs: int, nb: int, update="bf16", store="bf16", restart: int = 30) -> int:
    """Device bytes one served request needs (see include/mxp.h)."""
    return int(lib().mxp_server_request_bytes(n, nrhs, nb, dtype_code(update), dtype_code(store), restart))


@dataclass
class RequestResult:
    id: int
    n: int
    nrhs: int
    nb: int
    status: int
    iters: int
    eta: float
    t_submit_ns: int
    t_start_ns: int
    t_done_ns: int

    @property
    def latency_ms(self) -> float:
        return (self.t_done_ns - self.t_submit_ns) / 1e6


class Server:
    """Continuous-batching solve server on one device (mxp_server_* in
    include/mxp.h).  The arena is a torch uint8 device tensor held by this
    object; solutions land in host numpy arrays given at submission."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, update="bf16", store="bf16", nb: int = 0,
                 autotune: bool = False, restart: int = 30, max_iters: int = 50, tol: float = 16.0,
                 tau: float = 2.0 ** -50, device: int = 0):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda:%d" % device)
        cfg = _ServerCfg(max_slots, dtype_code(update), dtype_code(store), nb, 1 if autotune else 0, restart,
                         max_iters, tol, tau)
        torch.cuda.synchronize(device)
        h = ctypes.c_void_p()
        _check(lib().mxp_server_create(device, _ptr(self.arena), self.arena.numel(), ctypes.byref(cfg),
                                       ctypes.byref(h)))
        self._h = h
        self._x = {}

    def submit(self, n: int, nrhs: int, seed: int, want_x: bool = True) -> int:
        import numpy as np
        x = np.empty((nrhs, n), dtype=np.float64) if want_x else None
        rid = ctypes.c_uint64()
        _check(lib().mxp_server_submit(self._h, n, nrhs, seed, x.ctypes.data if x is not None else None,
                                       ctypes.byref(rid)))
        self._x[rid.value] = x
        return rid.value

    @staticmethod
    def _result(r: _RequestResult) -> RequestResult:
        return RequestResult(r.id, r.n, r.nrhs, r.nb, r.status, r.iters, r.eta, r.t_submit_ns, r.t_start_ns,
                             r.t_done_ns)

    def poll(self, rid: int):
        r = _RequestResult()
        code = lib().mxp_server_poll(self._h, rid, ctypes.byref(r))
        if code == PENDING:
            return None
        _check(code)
        return self._result(r)

    def wait(self, rid: int) -> RequestResult:
        r = _RequestResult()
        _check(lib().mxp_server_wait(self._h, rid, ctypes.byref(r)))
        return self._result(r)

    def solution(self, rid: int):
        """The solution of a finished request, shape (nrhs, n) (row r = x_r)."""
        return self._x[rid]

    def drain(self) -> None:
        _check(lib().mxp_server_drain(self._h))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().mxp_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def block_size(self, n: int) -> int:
        return int(lib().mxp_server_block_size(self._h, n))

    def tile(self, n: int) -> int:
        """trailing-update tile (TILE_256x128 / TILE_128x128) of a request of size n"""
        return int(lib().mxp_server_tile(self._h, n))

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().mxp_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
