"""Pins for the oracle's GMRES-IR and HPL criterion.

Paper, "Algorithmic Framework": GMRES in 64-bit with the LU factors as a
left preconditioner refines x0 to the accuracy of a 64-bit LU solve; more
than 50 iterations make the run invalid; the result is valid when the HPL
scaled residual ||Ax-b||_inf / ((||A||_inf ||x||_inf + ||b||_inf) n eps) is
below 16 with eps = 2^-53.

Pinned by GMRES's defining properties (Arnoldi relation, orthonormal basis,
monotone residual estimate, termination in at most n steps in exact
arithmetic, one step with an exact preconditioner), by a library solve,
and by a hand-worked HPL residual.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

EPS = 2.0 ** -53


def _system(n, seed):
    A, _ = oracle.generate(n, seed)
    b = oracle.generate_rhs(n, 1, seed)[:, 0]
    return A, b


def test_hpl_eta_hand_example():
    # A = 2I (n=2), b = (1, 1), x = (1/2, 1/2 + d): r = (0, -2d)
    d = 2.0 ** -40
    A = np.array([[2.0, 0.0], [0.0, 2.0]], order="F")
    b = np.array([1.0, 1.0])
    x = np.array([0.5, 0.5 + d])
    want = Fraction(2 * d) / ((Fraction(2) * Fraction(0.5 + d) + 1) * 2 * Fraction(EPS))
    assert oracle.hpl_eta(A, x, b) == pytest.approx(float(want), rel=1e-15)
    assert oracle.hpl_eta(A, np.array([0.5, 0.5]), b) == 0.0


def test_eps_is_two_to_minus_53():
    # the paper's eps is 2^-53 (not numpy's 2^-52 spacing)
    A = np.array([[1.0]], order="F")
    eta = oracle.hpl_eta(A, np.array([1.0 + 2.0 ** -52]), np.array([1.0]))
    # r = 2^-52, denominator (1*(1+2^-52) + 1) * 1 * 2^-53  ->  eta ~= 1
    assert eta == pytest.approx(2.0 ** -52 / ((2.0 + 2.0 ** -52) * 2.0 ** -53), rel=1e-15)


def test_exact_preconditioner_converges_immediately():
    A, b = _system(256, 4)
    LU, _ = oracle.lu_nopiv(A)
    rep = oracle.gmres_ir(A, LU, b)
    assert rep["status"] == 0 and rep["eta"] < 16
    assert rep["iters"] <= 2
    xr = np.linalg.solve(A, b)
    assert np.abs(rep["x"] - xr).max() <= 1e-13 * np.abs(xr).max()


def test_identity_preconditioner_terminates_within_n_steps():
    # unpreconditioned GMRES with restart >= n reaches the solution in <= n steps
    n = 24
    rng = np.random.default_rng(0)
    A = np.asfortranarray(rng.uniform(-1, 1, (n, n)) + 3 * np.eye(n))
    b = rng.uniform(-1, 1, n)
    rep = oracle.gmres_ir(A, None, b, restart=n, max_iters=n + 2)
    assert rep["status"] == 0 and rep["eta"] < 16
    assert rep["iters"] <= n + 1


def test_arnoldi_relation_orthogonality_monotone_residual():
    # a system on which the Krylov steps make slow progress, so that the
    # basis stays well conditioned (MGS orthogonality degrades only once
    # the residual has reached rounding level)
    n, m = 180, 12
    rng = np.random.default_rng(11)
    A = np.asfortranarray(rng.uniform(-1, 1, (n, n)) + 6 * np.eye(n))
    b = rng.uniform(-1, 1, n)
    LU, _ = oracle.lu_nopiv(A)
    P = np.asfortranarray(oracle.round_array(oracle.FMT_E4M3, LU * 16.0) / 16.0)  # crude factor
    x0 = np.zeros(n)
    x, k, it, V, H, Hraw, g = oracle.gmres_cycle(A, P, b, x0, m, tau=0.0, max_iters=m)
    assert k == m and it == m
    Vk, Vk1 = V[:, :k], V[:, :k + 1]
    MAV = np.column_stack([oracle.lu_solve(P, A @ Vk[:, j]) for j in range(k)])
    assert np.abs(MAV - Vk1 @ Hraw[:k + 1, :k]).max() <= 1e-13 * np.abs(MAV).max()
    # MGS-GMRES loses orthogonality only in inverse proportion to the
    # residual reduction (Paige, Rozloznik, Strakos 2006)
    r0 = abs(g[0]) if k == 0 else np.linalg.norm(oracle.lu_solve(P, b))
    hist = []
    for j in range(1, k + 1):
        xj, kj, _, _, _, _, gj = oracle.gmres_cycle(A, P, b, x0, j, tau=0.0, max_iters=j)
        assert kj == j
        res = abs(gj[j])                   # rotated residual estimate after j steps
        true = np.linalg.norm(oracle.lu_solve(P, b - A @ xj))
        assert true == pytest.approx(res, rel=1e-6, abs=1e-13 * r0)
        hist.append(res)
        loss = np.abs(V[:, :j + 1].T @ V[:, :j + 1] - np.eye(j + 1)).max()
        assert loss <= 1e-13 * r0 / res
    # minimal-residual property: the residual never grows with the Krylov dimension
    assert np.all(np.diff(hist) <= 1e-12 * r0)
    assert hist[-1] < 1e-3 * r0


def test_low_precision_preconditioner_reaches_fp64_accuracy():
    n = 400
    A, b = _system(n, 12)
    LU, _ = oracle.lu_nopiv(A)
    P = np.asfortranarray(oracle.round_array(oracle.FMT_BF16, LU))  # ~3 digits
    rep = oracle.gmres_ir(A, P, b)
    assert rep["status"] == 0 and rep["eta"] < 16
    assert 2 <= rep["iters"] <= 50
    xr = np.linalg.solve(A, b)
    assert np.abs(rep["x"] - xr).max() <= 1e-12 * np.abs(xr).max()


def test_iteration_cap_failure():
    # a useless preconditioner on a system GMRES cannot finish in 3 steps
    n = 60
    rng = np.random.default_rng(3)
    A = np.asfortranarray(rng.uniform(-1, 1, (n, n)) + 2 * np.eye(n))
    b = rng.uniform(-1, 1, n)
    rep = oracle.gmres_ir(A, None, b, restart=30, max_iters=3)
    assert rep["status"] == 2 and rep["iters"] == 3 and not rep["eta"] < 16


def test_jacobi_regen_matches_lu_and_residual_regen_matches_dense():
    n, seed = 256, 31
    A, b = _system(n, seed)
    LU, _ = oracle.lu_nopiv(A)
    xl = oracle.lu_solve(LU, b)
    xj, sweeps = oracle.jacobi_regen(n, seed, b)
    assert sweeps < 60
    assert np.abs(xj - xl).max() <= 1e-14 * np.abs(xl).max()
    r1 = oracle.residual_regen(n, seed, xl, b)
    r2 = b - A @ xl
    assert np.abs(r1 - r2).max() <= 1e-15 * np.abs(A).max() * np.abs(xl).max() * n
    # at an FP64 LU solution the scaled residual is at rounding level on both paths
    e1, e2 = oracle.hpl_eta_regen(n, seed, xl, b), oracle.hpl_eta(A, xl, b)
    assert e1 < 1.0 and e2 < 1.0
    # and a planted error of 1e-10 relative in x is seen identically by both
    xb = xl * (1 + 1e-10)
    assert oracle.hpl_eta_regen(n, seed, xb, b) == pytest.approx(oracle.hpl_eta(A, xb, b), rel=1e-3)


def test_jacobi_sweep_by_sweep_equals_the_single_call():
    # the sweep-at-a-time form (progress reported) is the same iteration:
    # bit-equal solution and sweep count, and every sweep's largest change
    # is the distance between the iterates it was given and returned
    n, seed = 200, 37
    A, b = _system(n, seed)
    x1, s1 = oracle.jacobi_regen(n, seed, b)
    seen = []
    x2, s2 = oracle.jacobi_regen(n, seed, b, progress=lambda k, dmax: seen.append((k, dmax)))
    assert s1 == s2 == len(seen) and [k for k, _ in seen] == list(range(1, s1 + 1))
    assert np.array_equal(x1, x2)
    # the diagonal the sweeps divide by is the generator's diagonal
    d = np.empty(n)
    oracle.lib().orc_diag_all(n, seed, oracle.GEN_DOMINANT, 0.0, oracle._p(d))
    assert np.array_equal(d, np.diag(A))
    # one sweep from x is x + D^-1 (b - A x), and its reported change is the update's max norm
    x = np.random.default_rng(2).uniform(-1, 1, n)
    y = x.copy()
    dmax = oracle.lib().orc_jacobi_sweep_regen(n, seed, oracle.GEN_DOMINANT, 0.0, oracle._p(d), oracle._p(b),
                                               oracle._p(y))
    want = x + (b - A @ x) / np.diag(A)
    assert np.abs(y - want).max() <= 1e-13 * np.abs(want).max()
    assert dmax == np.abs(y - x).max()


def test_residual_rows_are_the_dense_residual_on_the_sampled_rows():
    # sampled rows of b - A x with A regenerated, against the dense product
    n, seed = 300, 17
    A, b = _system(n, seed)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, n)
    rows = np.array([0, 1, 7, 128, 255, 299] + list(rng.choice(n, 10, replace=False)))
    got = oracle.residual_rows(n, seed, x, b, rows)
    want = (b - A @ x)[rows]
    scale = (np.abs(A) @ np.abs(x) + np.abs(b))[rows]
    assert np.all(np.abs(got - want) <= 4 * n * 2.0 ** -53 * scale)
    # the same values as the full regenerated residual, bit for bit
    assert np.array_equal(got, oracle.residual_regen(n, seed, x, b)[rows])
