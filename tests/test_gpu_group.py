"""GPU tests of the grouped launches of the solve server (mxp_factor_group):
one launch per kernel and block step serves several factorisations of
different sizes and block sizes through descriptor arrays.  Every element of
a factor is computed by the same arithmetic in the same order as by
mxp_factor (which splits the update differently for its look-ahead), so the
grouped factors must equal the individual ones bit for bit, for both
trailing-update tiles, and the solutions must match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu

# (2600, 128): its first blocks solve their strips through the diagonal
# blocks' inverses, the other members' through substitution, in the same launches
GROUP = [(700, 128), (1500, 256), (2100, 256), (513, 128), (3000, 512), (64, 64), (2600, 128)]


@pytest.mark.parametrize("update,store", [("bf16", "bf16"), ("f16", "f16"), ("f8", "f16")])
@pytest.mark.parametrize("tile", [mxp.TILE_256x128, mxp.TILE_128x128])
def test_grouped_factor_equals_individual_factor(update, store, tile):
    print("grouped factor", update, store, "tile", tile, flush=True)
    group = [(n, nb if update != "f8" else max(nb, 128)) for n, nb in GROUP]
    probs = [mxp.mxp_generate(n, 2, 500 + i, store=store) for i, (n, _) in enumerate(group)]
    facs = mxp.mxp_factor_group(probs, [nb for _, nb in group], update, tile=tile)
    torch.cuda.synchronize()
    for i, ((n, nb), prob, fac) in enumerate(zip(group, probs, facs)):
        assert fac.info == 0
        single = mxp.mxp_generate(n, 2, 500 + i, store=store)
        fs = mxp.mxp_factor(single, nb, update)
        torch.cuda.synchronize()
        assert torch.equal(fac.LU[:, :n], fs.LU[:, :n]), (n, nb)
        rg = mxp.mxp_solve_ir(prob, fac)
        rs = mxp.mxp_solve_ir(single, fs)
        assert torch.equal(rg.X, rs.X)
        if n <= 2100:
            A, Bo, Xo, _ = oracle.solve(n, 500 + i, nrhs=2)
            X = rg.X.cpu().numpy()
            for r in range(2):
                assert rg.status[r] == 0 and rg.eta[r] < 16
                assert np.abs(X[r] - Xo[:, r]).max() <= 1e-12 * np.abs(Xo[:, r]).max()


def test_grouped_update_tile_128_matches_definition():
    # the 128 x 128 tile of the trailing update through the group call's
    # single-item path: same result as the 256 x 128 tile, bit for bit
    n, nb = 1900, 256
    p1 = mxp.mxp_generate(n, 1, 77, store="f16")
    p2 = mxp.mxp_generate(n, 1, 77, store="f16")
    f1 = mxp.mxp_factor_group([p1], [nb], "f16", tile=mxp.TILE_128x128)[0]
    f2 = mxp.mxp_factor_group([p2], [nb], "f16", tile=mxp.TILE_256x128)[0]
    torch.cuda.synchronize()
    assert f1.info == 0 and f2.info == 0
    assert torch.equal(f1.LU[:, :n], f2.LU[:, :n])
