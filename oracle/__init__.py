"""CPU FP64 oracle for the HPL-MxP solve path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (``paper_2509_19618_amd``) never
imports it and shares no code with it.

The arithmetic lives in ``mxp_oracle.c`` (plain C, FP64); this module only
builds/loads it and marshals numpy arrays.  Each wrapper names the passage of
the paper it follows:

* generation -- "Matrix Generation" (scalable, counter-based generation; a
  diagonal large enough that LU needs no pivoting);
* ``lu_nopiv`` / ``lu_solve`` -- "Algorithmic Framework" (LU without
  pivoting, the factors used to get x0 and as the preconditioner);
* ``gmres_ir`` -- "Algorithmic Framework" (GMRES as the non-stationary
  refinement with the LU factors as a left preconditioner, at most 50
  iterations);
* ``hpl_eta`` -- "Algorithmic Framework" (the HPL backward-error formula,
  eps = 2^-53, valid below 16).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mxp_oracle.c")
_LIB = os.path.join(_HERE, "libmxp_oracle.so")

FMT_F32, FMT_F16, FMT_BF16, FMT_E4M3 = 0, 1, 2, 3
EPS = 2.0 ** -53
# matrix kinds ("Matrix Generation"; "Experimental Results"): row-dominant
# diagonal, diagonal u_ii + gamma sqrt(n), uniform in [-1, 1) without scaling
GEN_DOMINANT, GEN_SQRTN, GEN_UNIFORM = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, u64, u32, dbl, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
        P = ctypes.c_void_p
        sig = {
            "orc_philox4x32_10": (None, [P, P, P]),
            "orc_draw": (u32, [u64, u32, i64, i64]),
            "orc_entry_draw": (dbl, [u64, i64, i64]),
            "orc_rhs": (dbl, [u64, i64, i64]),
            "orc_diag": (dbl, [i64, u64, ci, dbl, i64]),
            "orc_entry": (dbl, [i64, u64, ci, dbl, i64, i64]),
            "orc_generate": (None, [i64, u64, ci, dbl, P, i64, P, P]),
            "orc_generate_rhs": (None, [i64, i64, u64, P, i64]),
            "orc_anorm_inf_regen": (dbl, [i64, u64, ci, dbl]),
            "orc_norm_inf_mat": (dbl, [i64, P, i64]),
            "orc_matvec": (None, [i64, P, i64, P, P]),
            "orc_lu_nopiv": (i64, [i64, P, i64]),
            "orc_lu_solve": (None, [i64, P, i64, P]),
            "orc_lu_pp": (i64, [i64, P, i64, P]),
            "orc_apply_pivots": (None, [i64, P, P]),
            "orc_hpl_eta": (dbl, [i64, P, i64, P, P]),
            "orc_residual_regen": (None, [i64, u64, ci, dbl, P, P, P]),
            "orc_residual_rows": (None, [i64, u64, ci, dbl, P, P, P, i64, P]),
            "orc_hpl_eta_regen": (dbl, [i64, u64, ci, dbl, P, P, dbl]),
            "orc_jacobi_regen": (i64, [i64, u64, ci, dbl, P, P, i64, dbl]),
            "orc_diag_all": (None, [i64, u64, ci, dbl, P]),
            "orc_jacobi_sweep_regen": (dbl, [i64, u64, ci, dbl, P, P, P]),
            "orc_gmres_cycle": (i64, [i64, P, i64, P, i64, P, P, i64, dbl, P, i64, P, P, P, P]),
            "orc_gmres_ir": (ctypes.c_int, [i64, P, i64, P, i64, P, P, i64, i64, dbl, dbl, P, P, P]),
            "orc_round_fmt": (dbl, [ctypes.c_int, dbl, ctypes.c_int]),
            "orc_encode_fmt": (u32, [ctypes.c_int, dbl]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- generator
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, stream: int, i: int, j: int) -> int:
    return int(lib().orc_draw(seed, stream, i, j))


def entry(n: int, seed: int, i: int, j: int, kind: int = GEN_DOMINANT, gamma: float = 0.0) -> float:
    return float(lib().orc_entry(n, seed, kind, gamma, i, j))


def generate(n: int, seed: int, kind: int = GEN_DOMINANT, gamma: float = 0.0, row_l1: bool = False):
    """Dense FP64 A (column-major, returned as a Fortran-ordered array) and
    diag (and the row 1-norms when row_l1)."""
    A = np.zeros((n, n), dtype=np.float64, order="F")
    d = np.zeros(n, dtype=np.float64)
    l1 = np.zeros(n, dtype=np.float64)
    lib().orc_generate(n, seed, kind, gamma, _p(A), n, _p(d), _p(l1))
    return (A, d, l1) if row_l1 else (A, d)


def generate_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    B = np.zeros((n, nrhs), dtype=np.float64, order="F")
    lib().orc_generate_rhs(n, nrhs, seed, _p(B), n)
    return B


def anorm_inf_regen(n: int, seed: int, kind: int = GEN_DOMINANT, gamma: float = 0.0) -> float:
    return float(lib().orc_anorm_inf_regen(n, seed, kind, gamma))


# ---------------------------------------------------------------- dense LA
def lu_nopiv(A: np.ndarray):
    """Unpivoted LU of a copy of A; returns (LU packed, info)."""
    LU = np.array(A, dtype=np.float64, order="F", copy=True)
    n = LU.shape[0]
    info = lib().orc_lu_nopiv(n, _p(LU), n)
    return LU, int(info)


def lu_pp(A: np.ndarray):
    """LU with partial pivoting of a copy of A ("Experimental Results");
    returns (LU packed, ipiv with 0-based swap rows, info)."""
    LU = np.array(A, dtype=np.float64, order="F", copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(n, dtype=np.int64)
    info = lib().orc_lu_pp(n, _p(LU), n, ipiv.ctypes.data_as(ctypes.c_void_p))
    return LU, ipiv, int(info)


def lu_pp_solve(LU: np.ndarray, ipiv, b) -> np.ndarray:
    """x = U^-1 L^-1 P b for the factors of lu_pp"""
    x = _f64(b).copy()
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int64)
    lib().orc_apply_pivots(LU.shape[0], ipiv.ctypes.data_as(ctypes.c_void_p), _p(x))
    return lu_solve(LU, x)


def lu_solve(LU: np.ndarray, b) -> np.ndarray:
    assert LU.flags.f_contiguous
    x = _f64(b).copy()
    lib().orc_lu_solve(LU.shape[0], _p(LU), LU.shape[0], _p(x))
    return x


def matvec(A: np.ndarray, x) -> np.ndarray:
    assert A.flags.f_contiguous
    x = _f64(x)
    y = np.zeros(A.shape[0])
    lib().orc_matvec(A.shape[0], _p(A), A.shape[0], _p(x), _p(y))
    return y


def hpl_eta(A: np.ndarray, x, b) -> float:
    assert A.flags.f_contiguous
    return float(lib().orc_hpl_eta(A.shape[0], _p(A), A.shape[0], _p(_f64(x)), _p(_f64(b))))


def residual_regen(n: int, seed: int, x, b, kind: int = GEN_DOMINANT, gamma: float = 0.0) -> np.ndarray:
    r = np.zeros(n)
    lib().orc_residual_regen(n, seed, kind, gamma, _p(_f64(x)), _p(_f64(b)), _p(r))
    return r


def residual_rows(n: int, seed: int, x, b, rows, kind: int = GEN_DOMINANT, gamma: float = 0.0) -> np.ndarray:
    """r[rows] of r = b - A x, A regenerated (sampled rows of residual_regen)."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(len(rows))
    lib().orc_residual_rows(n, seed, kind, gamma, _p(_f64(x)), _p(_f64(b)), rows.ctypes.data_as(ctypes.c_void_p),
                            len(rows), _p(out))
    return out


def hpl_eta_regen(n: int, seed: int, x, b, kind: int = GEN_DOMINANT, gamma: float = 0.0,
                  a_inf: float | None = None) -> float:
    """HPL scaled residual with A regenerated; a_inf (from anorm_inf_regen) may be passed to skip its pass."""
    return float(lib().orc_hpl_eta_regen(n, seed, kind, gamma, _p(_f64(x)), _p(_f64(b)),
                                         -1.0 if a_inf is None else float(a_inf)))


def jacobi_regen(n: int, seed: int, b, max_sweeps: int = 200, tol: float = 2.0 ** -50, kind: int = GEN_DOMINANT,
                 gamma: float = 0.0, progress=None):
    """Jacobi from x = 0 with A regenerated (orc_jacobi_regen).  With progress
    (a callable taking the sweep count and the sweep's largest change) the
    sweeps are run one call at a time -- the same arithmetic in the same
    order -- and reported as they finish."""
    x = np.zeros(n)
    if progress is None:
        sweeps = lib().orc_jacobi_regen(n, seed, kind, gamma, _p(_f64(b)), _p(x), max_sweeps, tol)
        return x, int(sweeps)
    bb = _f64(b)
    d = np.empty(n)
    lib().orc_diag_all(n, seed, kind, gamma, _p(d))
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        dmax = lib().orc_jacobi_sweep_regen(n, seed, kind, gamma, _p(d), _p(bb), _p(x))
        progress(sweeps, dmax)
        if dmax <= tol * np.abs(x).max():
            break
    return x, sweeps


# ---------------------------------------------------------------- GMRES-IR
def gmres_cycle(A, P, b, x, m: int, tau: float, it: int = 0, max_iters: int = 50):
    """One restart cycle; returns (x_new, k, it, V, H_rotated, H_raw, g)."""
    n = A.shape[0]
    x = _f64(x).copy()
    V = np.zeros((n, m + 1), order="F")
    H = np.zeros((m + 1, m), order="F")
    Hraw = np.zeros((m + 1, m), order="F")
    g = np.zeros(m + 1)
    itc = ctypes.c_int64(it)
    Pp, ldp = (_p(P), P.shape[0]) if P is not None else (None, 1)
    k = lib().orc_gmres_cycle(n, _p(A), n, Pp, ldp, _p(_f64(b)), _p(x), m, tau, ctypes.byref(itc),
                              max_iters, _p(V), _p(H), _p(Hraw), _p(g))
    return x, int(k), int(itc.value), V, H, Hraw, g


def gmres_ir(A, P, b, restart: int = 30, max_iters: int = 50, tol: float = 16.0, tau: float = 2.0 ** -50):
    """GMRES-IR; returns dict(x, status, iters, cycles, eta)."""
    n = A.shape[0]
    x = np.zeros(n)
    it, cyc, eta = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_double(0)
    Pp, ldp = (_p(P), P.shape[0]) if P is not None else (None, 1)
    st = lib().orc_gmres_ir(n, _p(A), n, Pp, ldp, _p(_f64(b)), _p(x), restart, max_iters, tol, tau,
                            ctypes.byref(it), ctypes.byref(cyc), ctypes.byref(eta))
    return {"x": x, "status": int(st), "iters": int(it.value), "cycles": int(cyc.value), "eta": float(eta.value)}


def solve(n: int, seed: int, nrhs: int = 1, restart: int = 30, max_iters: int = 50, tol: float = 16.0,
          tau: float = 2.0 ** -50, kind: int = GEN_DOMINANT, gamma: float = 0.0):
    """Full oracle solve at small n: generate, FP64 LU, GMRES-IR per RHS."""
    A, d = generate(n, seed, kind, gamma)
    B = generate_rhs(n, nrhs, seed)
    LU, info = lu_nopiv(A)
    if info:
        raise ArithmeticError("zero pivot at column %d" % info)
    X = np.zeros((n, nrhs), order="F")
    reps = []
    for r in range(nrhs):
        rep = gmres_ir(A, LU, B[:, r], restart, max_iters, tol, tau)
        X[:, r] = rep["x"]
        reps.append(rep)
    return A, B, X, reps


# ---------------------------------------------------------------- formats
def round_fmt(fmt: int, x: float, sat: bool = True) -> float:
    return float(lib().orc_round_fmt(fmt, float(x), 1 if sat else 0))


def encode_fmt(fmt: int, y: float) -> int:
    return int(lib().orc_encode_fmt(fmt, float(y)))


def round_array(fmt: int, a, sat: bool = True) -> np.ndarray:
    f = lib().orc_round_fmt
    s = 1 if sat else 0
    flat = np.asarray(a, dtype=np.float64).ravel()
    return np.array([f(fmt, float(v), s) for v in flat]).reshape(np.shape(a))
