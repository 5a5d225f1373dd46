"""GPU tests of the low-precision factor itself (not only through GMRES-IR,
which would absorb a wrong factor at the cost of extra iterations).

1. Quantiser, bit-exact: with an identity diagonal block the strip solves
   of the first block step are exact (L21 = A21, U12 = A12 in FP32), so the
   update operands, their power-of-two strip scales and the stored L21 / U12
   must equal the rounding of the known inputs bit for bit: scale 2^(e - c)
   with c = ceil(log2 amax) (e = 15 for FP16, 8 for FP8, no scaling for
   BF16/FP32), q = RNE(s x) (oracle.round_fmt, saturating for e4m3).
2. Backward error of the factor the solve applies (the FP32 diagonal blocks
   kept in aux, the stored panels with their strip scales undone): |L^U^ - A|
   elementwise against the bound derived from the per-step roundings
   (storage u_s, operands u_op, FP32 accumulation); the forward error of L^,
   U^ against the oracle's FP64 unpivoted LU within the first-order
   perturbation bound; the diagonal blocks stored in the matrix equal the
   FP32 blocks rounded to the storage format (in FP16 storage their entries
   below 2^-14 are subnormal: that copy is not what the solve applies).
3. Preconditioner apply: z = M^-1 v against an FP64 substitution with the
   GPU's own factor (FP32 diagonal blocks from aux, panels from the stored
   matrix with their strip scales undone), within the error of the FP32
   inverses of the substitution's diagonal blocks (pairs of factor blocks
   for nb <= 512) that the apply uses.
"""
import threading

import numpy as np
import pytest
import torch

import oracle
import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu

FMT = {"f32": oracle.FMT_F32, "f16": oracle.FMT_F16, "bf16": oracle.FMT_BF16, "f8": oracle.FMT_E4M3}
UNIT = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8, "f8": 2.0 ** -4}
SCALE_EXP = {"f16": 15, "f8": 8}          # amax * s lands in (2^(e-1), 2^e]
TORCH_ST = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
PAIRS = [("f32", "f32"), ("f16", "f16"), ("bf16", "bf16"), ("f8", "f16"), ("f8", "bf16"), ("f16", "f32"),
         ("bf16", "f32")]


def _round(fmt, a):
    return oracle.round_array(FMT[fmt], a)


def _decode_op(raw: torch.Tensor, update: str) -> np.ndarray:
    """operand bytes -> FP64 values"""
    if update == "f8":
        return raw.view(torch.float8_e4m3fn).float().double().numpy()
    if update == "bf16":
        return raw.view(torch.bfloat16).float().double().numpy()
    return raw.view(torch.float16 if update == "f16" else torch.float32).double().numpy()


def _values(rng, rows, cols, store):
    """values exactly representable in the storage format with a different
    range per 32-row strip (one strip's amax a power of two, one strip tiny,
    one all zero) to exercise the strip scales and subnormal rounding"""
    v = np.zeros((rows, cols))
    for s0 in range(0, rows, 32):
        s = s0 // 32
        blk = rng.uniform(-1, 1, (min(32, rows - s0), cols)) * 2.0 ** rng.integers(-6, 1)
        if s % 4 == 1:
            blk *= 2.0 ** -20                      # tiny strip
        if s % 4 == 2:
            blk[0, 0] = 2.0                        # amax exactly a power of two
            blk = np.clip(blk, -2.0, 2.0)
        if s % 4 == 3 and s0 + 32 >= rows:
            blk[:] = 0.0                           # an all-zero (ragged) strip
        v[s0:s0 + blk.shape[0]] = blk
    return _round(store, v)


@pytest.mark.parametrize("update,store", PAIRS)
def test_first_step_quantiser_bit_exact(update, store):
    print("quantiser", update, store, flush=True)
    nb, m = 128, 100
    n = nb + m
    rng = np.random.default_rng(100 + PAIRS.index((update, store)))
    Ah = np.zeros((n, n))
    Ah[:nb, :nb] = np.eye(nb)
    L21 = _values(rng, m, nb, store)                # rows 32-strips
    U12 = _values(rng, m, nb, store).T              # columns in 32-strips
    Ah[nb:, :nb] = L21
    Ah[:nb, nb:] = U12
    Ah[nb:, nb:] = 16384.0 * np.eye(m)               # keeps the second block dominant
    prob = mxp.mxp_generate(n, 1, 1, store=store)   # buffers; A overwritten below
    prob.A[:, :n] = torch.from_numpy(Ah.T.copy()).to(TORCH_ST[store]).cuda()
    fac = mxp.mxp_factor(prob, nb, update)
    torch.cuda.synchronize()
    assert fac.info == 0
    lay = mxp.factor_layout(n, nb, update)
    work = fac.work.cpu()
    aux = fac.aux.cpu()
    esz = {"f32": 4, "f16": 2, "bf16": 2, "f8": 1}[update]
    Lq = _decode_op(work[lay.Lq:lay.Lq + m * nb * esz], update).reshape(m, nb)
    Uq = _decode_op(work[lay.Uq:lay.Uq + m * nb * esz], update).reshape(m, nb)
    isa = work[lay.inv_sa:lay.inv_sa + 4 * 4].view(torch.float32).double().numpy()
    isb = work[lay.inv_sb:lay.inv_sb + 4 * 4].view(torch.float32).double().numpy()
    lsc = aux[lay.lsc:lay.lsc + 4 * lay.strips].view(torch.float32).double().numpy()
    for x, q, inv in ((L21, Lq, isa), (U12.T, Uq, isb)):
        for w in range(4):
            rows = slice(32 * w, min(32 * w + 32, m))
            amax = np.abs(x[rows]).max()
            s = 1.0 / inv[w]
            assert s == 2.0 ** np.round(np.log2(s))                     # a power of two
            if update in SCALE_EXP and amax > 0:
                e = SCALE_EXP[update]
                assert 2.0 ** (e - 1) < amax * s <= 2.0 ** e, (w, amax, s)
            else:
                assert s == 1.0
            want = _round(update, x[rows] * s)                          # RNE, e4m3 saturating
            assert np.array_equal(q[rows], want), (w, np.abs(q[rows] - want).max())
    # the stored L21 (scaled by its strip factor in FP16 storage) and U12 (unscaled)
    got = mxp.as_matrix(prob.A, n).double().cpu().numpy()
    assert np.array_equal(got[:nb, nb:], U12)
    for w in range(4):
        rows = slice(32 * w, min(32 * w + 32, m))
        s = lsc[(nb + 32 * w) // 32]
        amax = np.abs(L21[rows]).max()
        if store == "f16" and amax > 0:
            assert 2.0 ** 14 < amax * s <= 2.0 ** 15
        else:
            assert s == 1.0
        assert np.array_equal(got[nb:, :nb][rows], _round(store, L21[rows] * s))


def _unpack(prob, fac):
    """L^ (unit lower, strip scales undone) and U^ of the stored factor, FP64"""
    n, nb = prob.n, fac.nb
    lay = mxp.factor_layout(n, nb, fac.update)
    F = mxp.as_matrix(fac.LU, n).double().cpu().numpy()
    lsc = fac.aux.cpu()[lay.lsc:lay.lsc + 4 * lay.strips * (-(-n // nb))].view(torch.float32).double().numpy()
    lsc = lsc.reshape(-1, lay.strips)
    L = np.tril(F, -1)
    for blk in range(-(-n // nb)):
        c0, c1 = blk * nb, min(n, blk * nb + nb)
        r = np.arange(c1, n)
        if len(r):
            L[c1:, c0:c1] /= lsc[blk, r // 32][:, None]
    return L + np.eye(n), np.triu(F)


def _backward_bound(A, L, U, nb, update, store):
    n = A.shape[0]
    us, uo = UNIT[store], UNIT[update]
    LU_abs = np.abs(L) @ np.abs(U)
    steps = np.minimum.outer(np.arange(n), np.arange(n)) // nb          # block updates applied to (i, j)
    return 2.0 * ((2 * uo + (steps + 3) * us + 2 * nb * 2.0 ** -24) * LU_abs + (steps + 1) * us * np.abs(A))


CASES = [(1000, 128, p[0], p[1]) for p in PAIRS] + [(4096, 512, "f16", "f16"), (4096, 512, "bf16", "bf16"),
                                                    (4096, 512, "f8", "f16"), (1100, 256, "f8", "bf16")]
# block steps whose trailing part is at least 16 blocks solve their strips
# through the diagonal block's inverses (16-bit storage): these sizes take
# that path for their first blocks (FP16 with 64-row tiles and two idle
# waves at nb = 64, BF16 and FP8 operands with 32-row tiles)
CASES += [(2048, 64, "f16", "f16"), (2600, 128, "bf16", "bf16"), (2600, 128, "f8", "f16"), (2400, 128, "f8", "bf16")]


@pytest.mark.parametrize("n,nb,update,store", CASES)
def test_factor_backward_and_forward_error(n, nb, update, store):
    # the factor the solve applies: the FP32 diagonal blocks kept in aux and
    # the stored panels (strip scales undone)
    print("factor", n, nb, update, store, flush=True)
    seed = 6
    prob = mxp.mxp_generate(n, 1, seed, store=store)
    fac = mxp.mxp_factor(prob, nb, update)
    torch.cuda.synchronize()
    assert fac.info == 0
    L, Uf = _dense_prec(prob, fac)
    A, _ = oracle.generate(n, seed)
    E = L @ Uf - A
    B = _backward_bound(A, L, Uf, nb, update, store)
    R = np.abs(E) / B
    ratio = float(R.max())
    i, j = np.unravel_index(np.argmax(R), R.shape)
    print("  backward error / bound: %.3g at (%d, %d): E %.3g B %.3g A %.4g L %.4g U %.4g (LU)_abs %.4g"
          % (ratio, i, j, E[i, j], B[i, j], A[i, j], L[i, j], Uf[i, j], (np.abs(L[i]) @ np.abs(Uf[:, j]))),
          flush=True)
    assert ratio <= 1.0
    # the diagonal blocks stored in A are the FP32 blocks rounded to the storage format
    Ls, Us = _unpack(prob, fac)
    for blk in range(-(-n // nb)):
        c0, c1 = blk * nb, min(n, blk * nb + nb)
        assert np.array_equal(np.tril(Ls[c0:c1, c0:c1], -1), _round(store, np.tril(L[c0:c1, c0:c1], -1)))
        assert np.array_equal(np.triu(Us[c0:c1, c0:c1]), _round(store, np.triu(Uf[c0:c1, c0:c1])))
    if n <= 1100:
        LU0, info = oracle.lu_nopiv(A)
        assert info == 0
        L0, U0 = np.tril(LU0, -1) + np.eye(n), np.triu(LU0)
        # first order: L^ = L (I + X_low), U^ = (I + X_up) U with X = L^-1 E U^-1
        Li = np.abs(np.linalg.inv(L0)).sum(axis=1).max()
        Ui = np.abs(np.linalg.inv(U0)).sum(axis=1).max()
        xb = Li * np.abs(B).sum(axis=1).max() * Ui
        fu = np.abs(Uf - U0).max() / (4 * xb * np.abs(U0).sum(axis=0).max())
        fl = np.abs(L - L0).max() / (4 * xb * np.abs(L0).sum(axis=1).max())
        print("  forward error / bound: U %.3g L %.3g" % (fu, fl), flush=True)
        assert fu <= 1.0 and fl <= 1.0


def _dense_prec(prob, fac):
    """M with the FP32 diagonal blocks the apply uses (aux T) and the stored panels"""
    n, nb = prob.n, fac.nb
    L, Uf = _unpack(prob, fac)
    lay = mxp.factor_layout(n, nb, fac.update)
    nblk = -(-n // nb)
    T = fac.aux.cpu()[lay.T:lay.T + 4 * nblk * nb * nb].view(torch.float32).double().numpy().reshape(nblk, nb, nb)
    for blk in range(nblk):
        c0, kb = blk * nb, min(nb, n - blk * nb)
        Tb = T[blk].T[:kb, :kb]                          # column-major in aux
        L[c0:c0 + kb, c0:c0 + kb] = np.tril(Tb, -1) + np.eye(kb)
        Uf[c0:c0 + kb, c0:c0 + kb] = np.triu(Tb)
    return L, Uf


PREC_CASES = [(256, 64, "f32", "f32"), (300, 64, "f16", "f16"), (1000, 256, "f16", "f16"), (777, 128, "bf16", "bf16"),
              (640, 128, "f8", "f16"), (520, 128, "f8", "bf16"), (384, 64, "f16", "f32"), (390, 64, "bf16", "f32"),
              (2048, 512, "f8", "f16")]


@pytest.mark.parametrize("n,nb,update,store", PREC_CASES)
def test_preconditioner_apply_against_own_factor(n, nb, update, store):
    print("prec apply", n, nb, update, store, flush=True)
    prob = mxp.mxp_generate(n, 2, 3, store=store)
    fac = mxp.mxp_factor(prob, nb, update)
    assert fac.info == 0
    V = prob.B.clone()
    Z = mxp.mxp_apply_prec(fac, V).cpu().numpy()
    L, Uf = _dense_prec(prob, fac)
    LU = np.array(np.tril(L, -1) + Uf, order="F")
    # FP32 inverses of the substitution's diagonal blocks: pairs of factor
    # blocks (size 2 nb) for nb <= 512, their off-diagonal parts formed by
    # two FP32 products
    D = 2 * nb if nb <= 512 else nb
    bound = 32 * D * 2.0 ** -24
    for r in range(2):
        want = oracle.lu_solve(LU, V[r].cpu().numpy())
        err = np.abs(Z[r] - want).max() / np.abs(want).max()
        print("  rel err %.3g (bound %.3g)" % (err, bound), flush=True)
        assert err <= bound


def test_concurrent_factorisations_from_two_threads():
    # two host threads factor at once on their own streams, without a
    # caller look-ahead context: each takes its own from the library's pool
    print("two threads factoring", flush=True)
    cases = [(1500, 256, "f16", 21), (1300, 256, "bf16", 22)]
    out = {}

    def run(n, nb, up, seed):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            prob = mxp.mxp_generate(n, 1, seed, store=up, stream=s)
            A0 = prob.A.clone()
            for _ in range(3):
                prob.A.copy_(A0)
                fac = mxp.mxp_factor(prob, nb, up, stream=s)
            res = mxp.mxp_solve_ir(prob, fac, stream=s)
            s.synchronize()
            out[seed] = (fac.info, res, prob)

    ths = [threading.Thread(target=run, args=c) for c in cases]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for n, nb, up, seed in cases:
        info, res, prob = out[seed]
        assert info == 0 and res.status[0] == 0
        A, Bo, Xo, _ = oracle.solve(n, seed)
        x = res.X[0].cpu().numpy()
        assert np.abs(x - Xo[:, 0]).max() <= 1e-12 * np.abs(Xo[:, 0]).max()


def test_concurrent_substitutions_from_several_threads():
    # the preconditioner's dataflow kernels of three solves running at once
    # on their own streams, each launch with more work-groups than fit on
    # the device together: every apply completes (a wait that expired would
    # raise) and equals the same apply run alone, bit for bit
    print("three threads applying the preconditioner", flush=True)
    cases = [(16384, 512, "bf16", 8, 31), (12288, 512, "f16", 8, 32), (9000, 512, "bf16", 5, 33)]
    facs = {}
    for n, nb, up, nrhs, seed in cases:
        prob = mxp.mxp_generate(n, nrhs, seed, store=up)
        fac = mxp.mxp_factor(prob, nb, up)
        assert fac.info == 0
        V = prob.B.clone()
        facs[seed] = (fac, V, mxp.mxp_apply_prec(fac, V))
    torch.cuda.synchronize()
    bad = {}

    def run(seed):
        fac, V, Zref = facs[seed]
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                for _ in range(10):
                    Z = mxp.mxp_apply_prec(fac, V, stream=s)
                    s.synchronize()
                    if not torch.equal(Z, Zref):
                        bad[seed] = "result differs from the apply run alone"
                        return
        except Exception as e:          # an expired wait raises MxpError
            bad[seed] = repr(e)

    ths = [threading.Thread(target=run, args=(c[-1],)) for c in cases]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not bad, bad
