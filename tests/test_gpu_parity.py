"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (see the design notes for the derivations):
  * generator: bit-exact (integer and rounding work);
  * residual r = b - A x (FP64, regenerated A): |r_gpu - r_orc| <= 64 n eps |A||x|;
  * factor: low-precision, so only bounded: |M^-1 v - A^-1 v| <= C u_low |A^-1 v|
    (parity unpinned bitwise: MFMA accumulation order is the hardware's);
  * solution: ||x_gpu - x_orc||_inf <= 1e-12 ||x_orc||_inf and eta < 16.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu

STORE_NP = {"f32": np.float32, "f16": np.float16}


def _dev_matrix(prob):
    return mxp.as_matrix(prob.A, prob.n).float().cpu().numpy().astype(np.float64)


def _oracle_stored(A, store):
    if store == "f64":
        return A
    if store == "f32":
        return A.astype(np.float32).astype(np.float64)
    if store == "f16":
        return A.astype(np.float16).astype(np.float64)
    return oracle.round_array(oracle.FMT_BF16, A)


@pytest.mark.parametrize("n", [1, 5, 130, 777])
@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
def test_generator_bit_exact(n, store):
    print("generator", n, store, flush=True)
    prob = mxp.mxp_generate(n, 3, seed=12345, store=store)
    torch.cuda.synchronize()
    A, d, l1 = oracle.generate(n, 12345, row_l1=True)
    got = _dev_matrix(prob)
    want = _oracle_stored(A, store)
    assert np.array_equal(got, want)
    assert np.array_equal(prob.diag.cpu().numpy(), d)
    assert np.array_equal(prob.row_l1.cpu().numpy(), l1)
    assert prob.a_inf.item() == oracle.anorm_inf_regen(n, 12345)
    B = oracle.generate_rhs(n, 3, 12345)
    assert np.array_equal(prob.B.cpu().numpy().T, B)


@pytest.mark.parametrize("n", [1, 6, 333, 1000])
@pytest.mark.parametrize("kind,gamma", [(mxp.GEN_SQRTN, 0.3), (mxp.GEN_SQRTN, 1.7), (mxp.GEN_UNIFORM, 0.0)])
@pytest.mark.parametrize("store", ["f64", "f16", "bf16"])
def test_generator_kinds_bit_exact(n, kind, gamma, store):
    print("generator kind", kind, gamma, n, store, flush=True)
    prob = mxp.mxp_generate(n, 2, seed=77, store=store, kind=kind, gamma=gamma)
    torch.cuda.synchronize()
    A, d, l1 = oracle.generate(n, 77, kind, gamma, row_l1=True)
    got = mxp.as_matrix(prob.A, n).double().cpu().numpy()
    want = A if store == "f64" else _oracle_stored(A, store)
    assert np.array_equal(got, want)
    assert np.array_equal(prob.diag.cpu().numpy(), d)
    assert np.array_equal(prob.row_l1.cpu().numpy(), l1)
    assert prob.a_inf.item() == oracle.anorm_inf_regen(n, 77, kind, gamma)


def test_generator_regen_only_and_large_seed():
    seed = 0xFEDC_BA98_7654_3210
    prob = mxp.mxp_generate(300, 1, seed=seed, store="f16", with_matrix=False)
    A, d = oracle.generate(300, seed)
    assert prob.A is None
    assert np.array_equal(prob.diag.cpu().numpy(), d)


@pytest.mark.parametrize("n,nrhs", [(1, 1), (257, 1), (770, 2), (1000, 3), (1027, 1), (2048, 8)])
def test_residual_regen(n, nrhs):
    print("residual", n, nrhs, flush=True)
    prob = mxp.mxp_generate(n, nrhs, seed=7, store="f16", with_matrix=False)
    rng = np.random.default_rng(n)
    X = rng.uniform(-1, 1, (nrhs, n))
    Xd = torch.from_numpy(X).cuda()
    R = mxp.mxp_residual(prob, Xd, prob.B).cpu().numpy()
    AX = mxp.mxp_residual(prob, Xd, None).cpu().numpy()
    A, _ = oracle.generate(n, 7)
    B = oracle.generate_rhs(n, nrhs, 7)
    for r in range(nrhs):
        want = oracle.residual_regen(n, 7, X[r], B[:, r])
        bound = 64 * n * 2.0 ** -53 * (np.abs(A) @ np.abs(X[r]))
        assert np.all(np.abs(R[r] - want) <= bound + 1e-300)
        assert np.all(np.abs(AX[r] - A @ X[r]) <= bound + 1e-300)


@pytest.mark.parametrize("kind,gamma", [(mxp.GEN_SQRTN, 0.5), (mxp.GEN_UNIFORM, 0.0)])
def test_residual_regen_kinds(kind, gamma):
    n, nrhs = 1027, 3
    print("residual kind", kind, n, flush=True)
    prob = mxp.mxp_generate(n, nrhs, seed=9, store="f16", with_matrix=False, kind=kind, gamma=gamma)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (nrhs, n))
    R = mxp.mxp_residual(prob, torch.from_numpy(X).cuda(), prob.B).cpu().numpy()
    A, _ = oracle.generate(n, 9, kind, gamma)
    B = oracle.generate_rhs(n, nrhs, 9)
    for r in range(nrhs):
        want = oracle.residual_regen(n, 9, X[r], B[:, r], kind, gamma)
        bound = 64 * n * 2.0 ** -53 * (np.abs(A) @ np.abs(X[r]) + np.abs(B[:, r]))
        assert np.all(np.abs(R[r] - want) <= bound)


def test_residual_regen_chunks_meet_row_tiles_in_part():
    # n = 20001: column chunks of 832 columns, not a multiple of the 256-row
    # work-group tiles, so some work-groups' rows meet a chunk's columns (and
    # the diagonal) in part; the last chunk has 33 columns (a ragged quad)
    n, seed = 20001, 11
    print("residual, partial chunk overlaps", n, flush=True)
    prob = mxp.mxp_generate(n, 1, seed=seed, store="f16", with_matrix=False)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, n)
    b = prob.B[0].cpu().numpy()
    R = mxp.mxp_residual(prob, torch.from_numpy(x[None, :]).cuda(), prob.B[:1])[0].cpu().numpy()
    edges = [0, 255, 256, 767, 768, 800, 831, 832, 1023, 1024, 1663, 1664, 19967, 19968, 20000]
    rows = np.unique(np.concatenate([edges, rng.choice(n, 64, replace=False)])).astype(np.int64)
    want = oracle.residual_rows(n, seed, x, b, rows)
    d = prob.diag.cpu().numpy()[rows]
    # sum_j |A_ij| <= 2 A_ii; both sides are FP64 sums of n products
    scale = 2.0 * d * np.abs(x).max() + np.abs(b[rows])
    assert np.all(np.abs(R[rows] - want) <= 2 * n * 2.0 ** -53 * scale)


CASES = [
    # n, nb, update, store
    (256, 64, "f32", "f32"),
    (300, 64, "f16", "f16"),
    (1000, 256, "f16", "f16"),
    (777, 128, "bf16", "bf16"),
    (640, 128, "f8", "f16"),
    (520, 128, "f8", "bf16"),
    (384, 64, "f16", "f32"),
    (390, 64, "bf16", "f32"),
    (64, 64, "f16", "f16"),
    (65, 64, "f32", "f32"),
    (1, 64, "f32", "f32"),
    # the first blocks' strips through the diagonal blocks' inverses
    (2100, 64, "f16", "f16"),
    (2400, 128, "bf16", "bf16"),
]


def _solve(n, nb, update, store, seed=1, nrhs=1, scaling=mxp.SCALE_NONE):
    prob = mxp.mxp_generate(n, nrhs, seed=seed, store=store)
    fac = mxp.mxp_factor(prob, nb, update, scaling=scaling)
    assert fac.info == 0 and fac.status == 0
    res = mxp.mxp_solve_ir(prob, fac)
    return prob, fac, res


@pytest.mark.parametrize("n,nb,update,store", CASES)
def test_solve_matches_oracle(n, nb, update, store):
    print("solve", n, nb, update, store, flush=True)
    prob, fac, res = _solve(n, nb, update, store, seed=11, nrhs=2)
    A, Bo, Xo, reps = oracle.solve(n, 11, nrhs=2)
    X = res.X.cpu().numpy()
    for r in range(2):
        assert res.status[r] == 0 and res.eta[r] < 16, (res.status, res.eta)
        assert res.iters[r] <= 50
        err = np.abs(X[r] - Xo[:, r]).max() / np.abs(Xo[:, r]).max()
        assert err <= 1e-12, err
        assert oracle.hpl_eta(A, X[r], Bo[:, r]) < 16


@pytest.mark.parametrize("n,nb,update,store,gamma", [(1000, 128, "f16", "f16", 0.5), (777, 128, "bf16", "bf16", 0.7),
                                                     (1536, 256, "f32", "f32", 0.3), (1100, 256, "f16", "f32", 0.3)])
def test_solve_sqrtn_kind_matches_oracle(n, nb, update, store, gamma):
    # the diagonal gamma sqrt(n): far from row dominance, GMRES-IR needs the
    # LU preconditioner and more iterations than for the dominant matrices
    print("solve sqrt(n) kind", n, nb, update, store, gamma, flush=True)
    seed = 13
    prob = mxp.mxp_generate(n, 2, seed=seed, store=store, kind=mxp.GEN_SQRTN, gamma=gamma)
    fac = mxp.mxp_factor(prob, nb, update)
    assert fac.info == 0
    res = mxp.mxp_solve_ir(prob, fac)
    A, Bo, Xo, reps = oracle.solve(n, seed, nrhs=2, kind=oracle.GEN_SQRTN, gamma=gamma)
    X = res.X.cpu().numpy()
    print("  iters", res.iters, "eta", res.eta, flush=True)
    for r in range(2):
        assert res.status[r] == 0 and res.eta[r] < 16 and res.iters[r] <= 50
        err = np.abs(X[r] - Xo[:, r]).max() / np.abs(Xo[:, r]).max()
        assert err <= 1e-12, err
        assert oracle.hpl_eta(A, X[r], Bo[:, r]) < 16


def test_plain_method_config_full_size():
    # n = 2048, nb = 256, all-FP32 LU, GMRES-IR restart 30
    print("plain-method 2048", flush=True)
    prob, fac, res = _solve(2048, 256, "f32", "f32", seed=1)
    A, Bo, Xo, reps = oracle.solve(2048, 1)
    x = res.X[0].cpu().numpy()
    assert res.status[0] == 0 and res.eta[0] < 16
    assert np.abs(x - Xo[:, 0]).max() <= 1e-12 * np.abs(Xo[:, 0]).max()
    assert oracle.hpl_eta(A, x, Bo[:, 0]) < 16


@pytest.mark.parametrize("update,store", [("f16", "f16"), ("bf16", "bf16"), ("f8", "f16")])
def test_row_equilibration_solves_the_original_system(update, store):
    n = 1536
    prob, fac, res = _solve(n, 256, update, store, seed=5, scaling=mxp.SCALE_ROW_EQUIL)
    A, Bo, Xo, _ = oracle.solve(n, 5)
    x = res.X[0].cpu().numpy()
    assert res.status[0] == 0 and res.eta[0] < 16
    assert np.abs(x - Xo[:, 0]).max() <= 1e-12 * np.abs(Xo[:, 0]).max()


def test_deterministic_repeat():
    outs = []
    for _ in range(2):
        prob, fac, res = _solve(1100, 256, "f16", "f16", seed=9)
        outs.append((fac.LU[:, :1100].clone(), res.X.clone(), res.iters[0]))  # padding rows of lda are never written
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_hpl_eta_matches_oracle():
    n = 900
    prob = mxp.mxp_generate(n, 1, seed=4, store="f16", with_matrix=False)
    rng = np.random.default_rng(1)
    A, _ = oracle.generate(n, 4)
    b = oracle.generate_rhs(n, 1, 4)[:, 0]
    x = np.linalg.solve(A, b) * (1 + 1e-11 * rng.uniform(-1, 1, n))
    eta = mxp.mxp_hpl_eta(prob, torch.from_numpy(x).cuda(), prob.B[0])
    # the residual's summation order differs: allow its rounding bound
    den = (np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()) * n * 2.0 ** -53
    slack = 2 * n * 2.0 ** -53 * (np.abs(A) @ np.abs(x) + np.abs(b)).max() / den
    assert abs(eta - oracle.hpl_eta(A, x, b)) <= slack
    assert 1.0 < eta < 1e4          # the perturbation is visible


def test_zero_pivot_reported():
    # a matrix whose third pivot is exactly zero: generate, then overwrite A
    n = 128
    prob = mxp.mxp_generate(n, 1, seed=2, store="f32")
    M = torch.eye(n, dtype=torch.float32, device="cuda") * 4
    M[2, 2] = 0.0
    prob.A[:, :n] = M.t()
    fac = mxp.mxp_factor(prob, 64, "f32")
    assert fac.status == mxp.ESINGULAR and fac.info == 3


def test_iteration_cap_reports_enoconv():
    prob = mxp.mxp_generate(512, 1, seed=8, store="f16")
    fac = mxp.mxp_factor(prob, 128, "f8")
    res = mxp.mxp_solve_ir(prob, fac, max_iters=1, tau=0.0)
    assert res.status[0] == mxp.ENOCONV and res.iters[0] == 1
