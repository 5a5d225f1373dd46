"""Pins for the oracle's unpivoted LU and triangular solves.

Paper, "Algorithmic Framework": the low-precision phase must numerically be
an LU factorisation, and no partial pivoting is needed for the generated
matrices.  Pinned against (1) exact rational Gaussian elimination on tiny
matrices, (2) a library LU with partial pivoting, which on these matrices
chooses no row swap, (3) the textbook invariants of diagonally dominant
elimination (dominance kept by Schur complements, growth factor <= 2).
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle

EPS = 2.0 ** -53


def _exact_lu_solve(A, b):
    """Doolittle elimination in exact rationals; returns (L, U, x)."""
    n = len(A)
    U = [[Fraction(v) for v in row] for row in A]
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for k in range(n):
        for i in range(k + 1, n):
            L[i][k] = U[i][k] / U[k][k]
            for j in range(k, n):
                U[i][j] -= L[i][k] * U[k][j]
    y = [Fraction(v) for v in b]
    for i in range(n):
        for j in range(i):
            y[i] -= L[i][j] * y[j]
    x = [Fraction(0)] * n
    for i in reversed(range(n)):
        s = y[i]
        for j in range(i + 1, n):
            s -= U[i][j] * x[j]
        x[i] = s / U[i][i]
    return L, U, x


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 4), (3, 2), (5, 9), (8, 1), (8, 123)])
def test_lu_and_solve_match_exact_rationals(n, seed):
    A, _ = oracle.generate(n, seed)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    Lx, Ux, xx = _exact_lu_solve(A.tolist(), b.tolist())  # generator values are exact dyadics
    LU, info = oracle.lu_nopiv(A)
    assert info == 0
    for i in range(n):
        for j in range(n):
            want = Ux[i][j] if j >= i else Lx[i][j]
            got = Fraction(LU[i, j])
            scale = max(abs(Ux[i][j]), Fraction(1)) if j >= i else Fraction(1)
            assert abs(got - want) <= 8 * n * EPS * scale
    x = oracle.lu_solve(LU, b)
    xn = max(abs(v) for v in xx)
    assert max(abs(Fraction(x[i]) - xx[i]) for i in range(n)) <= 8 * n * EPS * xn


def test_exact_pin_catches_dropped_term():
    # plant a mistake in a copy of the oracle's output: a dropped
    # elimination term must fail the exact comparison used above
    n, seed = 6, 3
    A, _ = oracle.generate(n, seed)
    Lx, Ux, _ = _exact_lu_solve(A.tolist(), [0.0] * n)
    LU, _ = oracle.lu_nopiv(A)
    bad = LU.copy()
    bad[4, 5] += LU[4, 2] * LU[2, 5]  # undo one update
    assert abs(Fraction(bad[4, 5]) - Ux[4][5]) > 8 * n * EPS * max(abs(Ux[4][5]), 1)


@pytest.mark.parametrize("n,seed", [(64, 1), (257, 2), (512, 3)])
def test_matches_library_lu_which_pivots_nothing(n, seed):
    A, _ = oracle.generate(n, seed)
    lu, piv = scipy.linalg.lu_factor(A)
    assert np.array_equal(piv, np.arange(n)), "partial pivoting chose a swap"
    LU, info = oracle.lu_nopiv(A)
    assert info == 0
    scale = np.abs(A).max()
    assert np.abs(np.triu(LU) - np.triu(lu)).max() <= 64 * EPS * scale * np.sqrt(n)
    assert np.abs(np.tril(LU, -1) - np.tril(lu, -1)).max() <= 64 * EPS * np.sqrt(n)


def test_solve_matches_numpy():
    n, seed = 300, 17
    A, _ = oracle.generate(n, seed)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    LU, _ = oracle.lu_nopiv(A)
    x = oracle.lu_solve(LU, b)
    xr = np.linalg.solve(A, b)
    assert np.abs(x - xr).max() <= 1e-13 * np.abs(xr).max()


def test_schur_complements_stay_dominant_and_growth_bounded():
    n, seed = 200, 8
    A, _ = oracle.generate(n, seed)
    LU, _ = oracle.lu_nopiv(A)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    for k in (1, 7, 50, 120, 199):
        S = L[k:, k:] @ U[k:, k:]          # Schur complement after k eliminations
        off = np.abs(S).sum(axis=1) - np.abs(np.diag(S))
        assert np.all(np.diag(S) > off)
    growth = np.abs(U).max() / np.abs(A).max()
    assert growth <= 2.0                   # Wilkinson: <= 2 for diagonally dominant
    # multipliers are small: |l_ij| < 1 (dominance), in practice about 2/n
    assert np.abs(np.tril(LU, -1)).max() < 1.0


def test_zero_pivot_reported_with_column():
    A = np.array([[1.0, 2.0, 0.0], [0.5, 1.0, 1.0], [0.0, 1.0, 1.0]], order="F")
    LU, info = oracle.lu_nopiv(A)
    assert info == 2                       # second pivot is 1 - 0.5*2 = 0
    A2 = np.array([[np.nan, 0.0], [0.0, 1.0]], order="F")
    assert oracle.lu_nopiv(A2)[1] == 1


# ---------------------------------------------------------------- partial pivoting
@pytest.mark.parametrize("n,seed", [(50, 1), (257, 2), (600, 3)])
def test_partial_pivoting_matches_library_lu(n, seed):
    # "Experimental Results": LU with partial pivoting on entries uniform in
    # [-1, 1) without diagonal scaling; LAPACK's getrf (scipy) takes the same
    # pivot rule (largest magnitude, first among equals)
    A, _ = oracle.generate(n, seed, oracle.GEN_UNIFORM)
    LU, ipiv, info = oracle.lu_pp(A)
    assert info == 0
    lu, piv = scipy.linalg.lu_factor(A)
    assert np.array_equal(ipiv, piv)
    assert np.abs(LU - lu).max() <= 64 * n * EPS * np.abs(lu).max()
    # P A = L U
    P = np.arange(n)
    for k in range(n):
        P[[k, ipiv[k]]] = P[[ipiv[k], k]]
    L, U = np.tril(LU, -1) + np.eye(n), np.triu(LU)
    assert np.abs(A[P] - L @ U).max() <= 8 * n * EPS * (np.abs(L) @ np.abs(U)).max()
    assert np.abs(np.tril(LU, -1)).max() <= 1.0            # |multipliers| <= 1 by construction
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    x = oracle.lu_pp_solve(LU, ipiv, b)
    xr = scipy.linalg.lu_solve((lu, piv), b)
    assert np.abs(x - xr).max() <= 1e-10 * np.abs(xr).max()


def test_partial_pivoting_plant_mistake_is_caught():
    # a dropped row swap in the L part (a plausible slip) breaks P A = L U
    n = 40
    A, _ = oracle.generate(n, 9, oracle.GEN_UNIFORM)
    LU, ipiv, _ = oracle.lu_pp(A)
    k = int(np.nonzero(ipiv != np.arange(n))[0][3])
    bad = LU.copy()
    bad[[k, ipiv[k]], :k] = bad[[ipiv[k], k], :k]
    P = np.arange(n)
    for j in range(n):
        P[[j, ipiv[j]]] = P[[ipiv[j], j]]
    L, U = np.tril(bad, -1) + np.eye(n), np.triu(bad)
    assert np.abs(A[P] - L @ U).max() > 1e-3


def test_largest_pivot_grows_like_sqrt_n():
    # Figure 2's experiment: the largest pivot |u_kk| of partial pivoting on
    # these matrices grows like sqrt(n) (the paper's curves: sqrt(n),
    # 5/8 sqrt(n), n^0.45) and is found late in the elimination; without
    # pivoting the same matrices give far larger pivots
    for n in (256, 1024):
        A, _ = oracle.generate(n, 4, oracle.GEN_UNIFORM)
        LU, ipiv, _ = oracle.lu_pp(A)
        d = np.abs(np.diag(LU))
        assert 0.5 * np.sqrt(n) < d.max() < 2.0 * np.sqrt(n)
        assert np.argmax(d) >= n // 2
        LU0, _ = oracle.lu_nopiv(A)
        assert np.abs(np.diag(LU0)).max() > 2.0 * d.max()
