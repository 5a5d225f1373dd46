"""Pins for the oracle's matrix kinds beyond the diagonally dominant one.

Paper, "Matrix Generation": the row-dominant matrices are for debugging and
tuning only; production inputs depart from diagonal dominance so that GMRES
without a preconditioner does not converge spuriously fast (fewer than 50
iterations; over 700 were seen for larger matrices).  "Experimental
Results": random-matrix theory suggests a diagonal scaled by sqrt(n); the
pivoting experiments use entries uniform in [-1, 1) without scaling.

Pinned by the circular law (the eigenvalues of an n x n matrix with i.i.d.
entries of variance s^2 fill a disk of radius s sqrt(n): s^2 = 1/12 for
[-1/2, 1/2), 1/3 for [-1, 1)), by the exact diagonal identities, and by
the GMRES behaviour the paper states.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.mark.parametrize("n,gamma", [(7, 0.3), (300, 0.5), (1025, 1.25)])
def test_sqrtn_kind_diagonal_and_offdiagonal(n, gamma):
    seed = 19
    A, d, l1 = oracle.generate(n, seed, oracle.GEN_SQRTN, gamma, row_l1=True)
    Ad, _ = oracle.generate(n, seed)                 # same draws, dominant diagonal
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(A[off], Ad[off])
    shift = gamma * math.sqrt(n)                     # both operations rounded once (IEEE)
    own = np.array([oracle.draw(seed, 0, i, i) for i in range(n)], dtype=np.float64) * 2.0 ** -32 - 0.5
    assert np.array_equal(d, own + shift)
    assert np.array_equal(np.diag(A), d)
    assert np.allclose(l1, np.abs(A).sum(axis=1), rtol=2 ** -50, atol=0)


def test_uniform_kind_entries_and_distribution():
    n, seed = 600, 23
    A, d = oracle.generate(n, seed, oracle.GEN_UNIFORM)
    Ad, _ = oracle.generate(n, seed)
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(A[off], 2.0 * Ad[off])
    own = np.array([oracle.draw(seed, 0, i, i) for i in range(n)], dtype=np.float64) * 2.0 ** -31 - 1.0
    assert np.array_equal(d, own)
    assert A.min() >= -1.0 and A.max() < 1.0
    assert stats.kstest(A.ravel()[::7], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("kind,gamma,radius", [(oracle.GEN_SQRTN, 0.4, 1 / math.sqrt(12)),
                                               (oracle.GEN_UNIFORM, 0.0, 1 / math.sqrt(3))])
def test_circular_law_spectrum(kind, gamma, radius):
    # eigenvalues of R + c I lie in a disk of radius s sqrt(n) about c
    n = 1024
    A, _ = oracle.generate(n, 5, kind, gamma)
    c = gamma * math.sqrt(n) if kind == oracle.GEN_SQRTN else 0.0
    r = np.abs(np.linalg.eigvals(A) - c).max() / math.sqrt(n)
    assert 0.9 * radius < r < 1.1 * radius, (r, radius)


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_sqrtn_kind_defeats_unpreconditioned_gmres(n):
    # gamma = 0.3, just outside the spectral disk (radius 0.289 sqrt(n)):
    # GMRES(30) without a preconditioner needs far more than 50 iterations,
    # with the FP64 LU factors as the preconditioner x0 already passes
    seed = 3
    A, _ = oracle.generate(n, seed, oracle.GEN_SQRTN, 0.3)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    rep = oracle.gmres_ir(A, None, b, restart=30, max_iters=50)
    assert rep["status"] == 2 and rep["eta"] > 16
    long = oracle.gmres_ir(A, None, b, restart=30, max_iters=5000)
    assert long["status"] == 0 and long["iters"] > 200
    LU, info = oracle.lu_nopiv(A)
    assert info == 0
    pre = oracle.gmres_ir(A, LU, b)
    assert pre["status"] == 0 and pre["iters"] <= 2


def test_dominant_kind_lets_unpreconditioned_gmres_converge():
    # the debugging class: GMRES without a preconditioner passes within the cap
    n, seed = 1024, 3
    A, _ = oracle.generate(n, seed)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    rep = oracle.gmres_ir(A, None, b, restart=30, max_iters=50)
    assert rep["status"] == 0 and rep["eta"] < 16


def test_regenerated_residual_and_norm_follow_the_kind():
    n, seed = 333, 8
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, n)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    for kind, gamma in ((oracle.GEN_DOMINANT, 0.0), (oracle.GEN_SQRTN, 0.7), (oracle.GEN_UNIFORM, 0.0)):
        A, _ = oracle.generate(n, seed, kind, gamma)
        r = oracle.residual_regen(n, seed, x, b, kind, gamma)
        assert np.abs(r - (b - A @ x)).max() <= 4 * n * 2.0 ** -53 * (np.abs(A) @ np.abs(x) + np.abs(b)).max()
        assert oracle.anorm_inf_regen(n, seed, kind, gamma) == np.abs(A).sum(axis=1).max() or \
            kind == oracle.GEN_SQRTN
        assert oracle.anorm_inf_regen(n, seed, kind, gamma) == pytest.approx(np.abs(A).sum(axis=1).max(),
                                                                             rel=2 ** -50)
