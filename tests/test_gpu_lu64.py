"""GPU tests of the FP64 LU (mxp_lu64_*): the FP64 baseline of the solve
("Background") and the LU of the pivoting study ("Experimental Results",
Figures 2-4).

* The FP64 trailing update against numpy's product (FP64; the bound is the
  accumulation error of K products).
* Without pivoting: the factor against the oracle's unpivoted FP64 LU and
  the solution against the oracle's FP64 solve, at 1e-12 relative.
* With partial pivoting, on matrices uniform in [-1, 1): the pivot rows,
  where no near-tie makes several choices correct, equal the oracle's
  (the largest magnitude, first among equals); every chosen pivot is a
  largest-magnitude entry of its column within rounding; P A = L U; the
  solution matches the oracle's pivoted solve.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


@pytest.mark.parametrize("M,N,K", [(128, 128, 64), (300, 517, 128), (1000, 77, 64), (1, 1, 4), (513, 640, 128)])
def test_gemm64_matches_product(M, N, K):
    print("gemm64", M, N, K, flush=True)
    rng = np.random.default_rng(M + N + K)
    ld = M + 5
    C = rng.uniform(-1, 1, (N, ld))
    A = rng.uniform(-1, 1, (K, M + 3))
    B = rng.uniform(-1, 1, (N, K + 1))
    Cd, Ad, Bd = (torch.from_numpy(x).cuda() for x in (C, A, B))
    mxp.mxp_trailing_update64(Cd, ld, M, N, K, Ad, M + 3, Bd, K + 1)
    got = Cd.cpu().numpy()
    a = A[:, :M].T                      # M x K (column-major storage: row k of A holds column k)
    b = B[:, :K].T                      # K x N
    want = C[:, :M].T - a @ b
    bound = (K + 2) * EPS * (np.abs(C[:, :M].T) + np.abs(a) @ np.abs(b))
    assert np.all(np.abs(got[:, :M].T - want) <= bound)
    assert np.array_equal(got[:, M:], C[:, M:])


def _problem(n, seed, kind, gamma=0.0):
    prob = mxp.mxp_generate(n, 2, seed, store="f64", kind=kind, gamma=gamma)
    torch.cuda.synchronize()
    return prob


@pytest.mark.parametrize("gemm", [mxp.GEMM64_OWN, mxp.GEMM64_ROCBLAS])
@pytest.mark.parametrize("n,seed", [(1, 1), (127, 2), (1000, 3), (1100, 4), (2500, 5)])
def test_lu64_nopiv_matches_oracle(n, seed, gemm):
    print("lu64 nopiv", n, "gemm", gemm, flush=True)
    prob = _problem(n, seed, mxp.GEN_DOMINANT)
    fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=False, gemm=gemm)
    assert fac.info == 0
    X = mxp.mxp_lu64_solve(fac, prob.B)
    A, _ = oracle.generate(n, seed)
    LU0, info = oracle.lu_nopiv(A)
    assert info == 0
    got = mxp.as_matrix(fac.LU, n).cpu().numpy()
    L0, U0 = np.tril(LU0, -1) + np.eye(n), np.triu(LU0)
    # both FP64 with different summation orders: within n eps |L||U|
    bound = 4 * n * EPS * (np.abs(L0) @ np.abs(U0))
    assert np.all(np.abs(np.triu(got) - U0) <= np.triu(bound) + 1e-300)
    assert np.all(np.abs(np.tril(got, -1) - np.tril(LU0, -1)) * np.abs(np.diag(U0))[None, :]
                  <= np.tril(bound, -1) + 1e-300)
    B = oracle.generate_rhs(n, 2, seed)
    for r in range(2):
        want = oracle.lu_solve(LU0, B[:, r])
        x = X[r].cpu().numpy()
        assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()


def _perm(ipiv):
    n = len(ipiv)
    P = np.arange(n)
    for k in range(n):
        P[[k, ipiv[k]]] = P[[ipiv[k], k]]
    return P


@pytest.mark.parametrize("n,seed,gemm", [(1, 1, 0), (64, 2, 0), (200, 3, 0), (1000, 4, 0), (1301, 5, 0), (3000, 6, 0),
                                         (1301, 5, 1), (3000, 6, 1)])
def test_lu64_partial_pivoting_matches_oracle(n, seed, gemm):
    print("lu64 pivoted", n, "gemm", gemm, flush=True)
    prob = _problem(n, seed, mxp.GEN_UNIFORM)
    fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=True, gemm=gemm)
    assert fac.info == 0
    X = mxp.mxp_lu64_solve(fac, prob.B)
    ipiv = fac.ipiv.cpu().numpy()
    got = mxp.as_matrix(fac.LU, n).cpu().numpy()
    A, _ = oracle.generate(n, seed, oracle.GEN_UNIFORM)
    LU0, ipiv0, info = oracle.lu_pp(A)
    assert info == 0
    # every swap row is valid, the permutation reproduces A: P A = L U
    assert np.all((ipiv >= np.arange(n)) & (ipiv < n))
    P = _perm(ipiv)
    L, U = np.tril(got, -1) + np.eye(n), np.triu(got)
    assert np.abs(np.tril(got, -1)).max() <= 1.0 + 1e-15
    assert np.abs(A[P] - L @ U).max() <= 8 * n * EPS * (np.abs(L) @ np.abs(U)).max()
    # pivots are unique unless two candidates tie within rounding: compare where the oracle's choice was clear
    first = np.nonzero(ipiv != ipiv0)[0]
    k_same = first[0] if len(first) else n
    print("  pivots equal to the oracle's for %d of %d columns" % (k_same, n), flush=True)
    if k_same < n:
        # the first differing choice must be a near-tie: the GPU's pivot (final
        # position k) is within rounding of the largest candidate of column k
        k = k_same
        S = (A[P] - L[:, :k] @ U[:k, :])[k:, k]     # column k of the Schur complement, final row order
        assert abs(abs(S[0]) - abs(S).max()) <= 64 * n * EPS * np.abs(A).max() * np.sqrt(n)
    else:
        assert np.abs(got - LU0).max() <= 64 * n * EPS * np.abs(LU0).max()
    B = oracle.generate_rhs(n, 2, seed)
    for r in range(2):
        want = oracle.lu_pp_solve(LU0, ipiv0, B[:, r])
        x = X[r].cpu().numpy()
        cond = np.linalg.cond(A, np.inf) if n <= 1301 else 1e6
        assert np.abs(x - want).max() <= min(1e-6, 64 * n * EPS * cond) * np.abs(want).max()


def test_lu64_zero_pivot_reported():
    n = 100
    prob = _problem(n, 1, mxp.GEN_DOMINANT)
    M = torch.eye(n, dtype=torch.float64, device="cuda") * 3
    M[5, 5] = 0.0
    prob.A[:, :n] = M.t()
    fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=False)
    assert fac.status == mxp.ESINGULAR and fac.info == 6
    # with pivoting a zero column is the only way to a zero pivot
    prob = _problem(n, 1, mxp.GEN_UNIFORM)
    prob.A[7, :n] = 0.0
    fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=True)
    assert fac.status == mxp.ESINGULAR and fac.info >= 1
