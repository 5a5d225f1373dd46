"""GPU tests of the solve server (mxp_server_* through the C ABI).

Each request is generated, factored and refined with the arithmetic of a
direct call (a group's factorisations share their launches, which gives the
same bits); the server only schedules.  The checks: every result meets the HPL
criterion and matches the oracle (small sizes); a request's solution is the
same when it runs alone and when it runs in a mix of concurrent requests;
admission respects the HBM budget; the tuner's block sizes are valid.
"""
import numpy as np
import pytest

import oracle
import paper_2509_19618_amd as mxp

pytestmark = pytest.mark.gpu

REQS = [(512, 1, 1001), (700, 2, 1002), (1500, 1, 1003), (2100, 3, 1004), (3000, 1, 1005), (4096, 2, 1006),
        (5000, 1, 1007), (513, 8, 1008)]


def _arena(reqs, nb, slack=1.25):
    return int(slack * sum(mxp.server_request_bytes(n, r, nb) for n, r, _ in reqs))


def test_alone_and_in_the_mix_agree():
    print("serving: alone vs mix", flush=True)
    with mxp.Server(_arena(REQS, 256), max_slots=4, nb=256) as srv:
        alone = {}
        for n, r, seed in REQS:
            rid = srv.submit(n, r, seed)
            res = srv.wait(rid)
            assert res.status == mxp.OK and res.eta < 16, res
            alone[(n, r, seed)] = srv.solution(rid).copy()
        ids = [(srv.submit(n, r, seed), (n, r, seed)) for n, r, seed in REQS]
        srv.drain()
        st = srv.stats()
        assert st["failed"] == 0 and st["completed"] == 2 * len(REQS)
        assert st["peak_in_flight"] >= 2          # the mix really ran concurrently
        assert st["peak_group"] >= 2              # some requests were factored with shared launches
        assert st["grouped_requests"] == 2 * len(REQS) and 1 <= st["streams"] <= 3
        assert st["peak_bytes_in_use"] <= st["arena_bytes"]
        for rid, key in ids:
            res = srv.wait(rid)
            assert res.status == mxp.OK and res.eta < 16 and res.nb == 256
            xm, xa = srv.solution(rid), alone[key]
            err = np.abs(xm - xa).max() / np.abs(xa).max()
            assert err <= 1e-12, (key, err)


@pytest.mark.parametrize("n,nrhs,seed", [(512, 1, 1001), (700, 2, 1002), (1500, 1, 1003)])
def test_served_solution_matches_oracle(n, nrhs, seed):
    print("serving vs oracle", n, nrhs, seed, flush=True)
    with mxp.Server(_arena([(n, nrhs, seed)], 256, 1.1), max_slots=1, nb=256) as srv:
        rid = srv.submit(n, nrhs, seed)
        res = srv.wait(rid)
        assert res.status == mxp.OK and res.eta < 16
        A, B, X, reps = oracle.solve(n, seed, nrhs=nrhs)
        xg = srv.solution(rid)
        for r in range(nrhs):
            err = np.abs(xg[r] - X[:, r]).max() / np.abs(X[:, r]).max()
            assert err <= 1e-12, (r, err)
            assert oracle.hpl_eta(A, xg[r], B[:, r]) < 16


def test_admission_by_hbm_budget():
    print("serving: budget", flush=True)
    one = mxp.server_request_bytes(4096, 1, 256)
    with mxp.Server(int(1.5 * one), max_slots=4, nb=256) as srv:
        ids = [srv.submit(4096, 1, 2000 + k) for k in range(5)]
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 5 and st["failed"] == 0
        assert st["peak_in_flight"] == 1          # only one fits at a time
        assert st["peak_bytes_in_use"] <= st["arena_bytes"]
        for rid in ids:
            res = srv.wait(rid)
            assert res.status == mxp.OK and res.eta < 16
            assert res.t_start_ns >= res.t_submit_ns and res.t_done_ns > res.t_start_ns
        # a request that can never fit is refused at submission
        with pytest.raises(mxp.MxpError):
            srv.submit(8192, 1, 1)


def test_autotuned_block_sizes():
    print("serving: autotune", flush=True)
    with mxp.Server(2 * mxp.server_request_bytes(16384, 1, 512), max_slots=2, autotune=True) as srv:
        for n in (512, 1024, 2048, 4096, 8192, 16384):
            assert srv.block_size(n) in (128, 256, 512)
            assert srv.tile(n) in (mxp.TILE_256x128, mxp.TILE_128x128)
        ids = [srv.submit(n, 1, 3000 + n) for n in (600, 2500, 9000)]
        for rid in ids:
            res = srv.wait(rid)
            assert res.status == mxp.OK and res.eta < 16
            assert res.nb == srv.block_size(res.n)


def test_saturated_mix_every_request_valid():
    # every request queued at once (eight slots, three worker streams): the
    # groups' factorisations and the requests' refinements overlap on the
    # device the whole time.  Every request must succeed with eta < 16 in
    # the usual few iterations -- an expired wait of a kernel that waits on
    # other work-groups would fail its request (and stall the server)
    print("serving: saturated mix", flush=True)
    rng = np.random.default_rng(11)
    ns = np.floor(np.exp(rng.uniform(np.log(512), np.log(8192), 150))).astype(int)
    rs = rng.integers(1, 9, 150)
    arena = int(1.25 * 8 * mxp.server_request_bytes(8192, 8, 512))
    with mxp.Server(arena, max_slots=8, nb=512) as srv:
        ids = [srv.submit(int(n), int(r), 5000 + k, want_x=False) for k, (n, r) in enumerate(zip(ns, rs))]
        srv.drain()
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    bad = [(x.n, x.nrhs, x.status, x.iters) for x in res if x.status != mxp.OK or not x.eta < 16 or x.iters > 10]
    assert not bad, bad
    assert st["failed"] == 0 and st["completed"] == 150 and st["peak_in_flight"] >= 4
