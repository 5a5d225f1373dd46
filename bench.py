#!/usr/bin/env python3
"""Benchmark of the mixed-precision LU + GMRES-IR solve on one MI355X.

One step = one solve of the HPL-MxP hot path on the same synthetic input:
factor the generated matrix (FP32 panel and strip TRSMs, trailing update on
MFMA with FP16 inputs and FP32 accumulation) and refine the solution with
FP64 GMRES-IR until the HPL scaled residual is below 16.  The matrix is
generated once; before every step the pristine copy is restored into the
working buffer (the factorisation overwrites it), outside the timed region,
which follows the benchmark's timing rule: scaling, LU and refinement are
timed, generation and the final validation are not.

Metric: effective TFLOP/s = (2/3 n^3) / t with t the timed region of a step.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")
GEMM_SRC = os.path.join(ROOT, "paper_2509_19618_amd", "csrc", "gemm.hip")
CALIB_BYTES = 1 << 30   # size of the plain copy that calibrates the HBM byte counters

PEAK = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "f16_tflops": 2500.0,
    "bf16_tflops": 2500.0,
    "f8_tflops": 5000.0,
    "f32_tflops": 157.3,
    "f64_tflops": 78.6,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--update", default="f16")
    ap.add_argument("--store", default="f16")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--scaling", default="none", choices=["none", "row_equil"])
    ap.add_argument("--cpu-n", type=int, default=4608, help="oracle sample size for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--traffic-run", action="store_true",
                    help="one untimed step plus a %d-byte calibration copy, for rocprofv3 --pmc" % CALIB_BYTES)
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv outputs into the traffic summary")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="turn a rocprofv3 --kernel-trace --stats csv output into a kernel-time summary")
    ap.add_argument("--cmd", default="", help="the rocprofv3 command(s) that produced the summarized output")
    ap.add_argument("--serve", action="store_true",
                    help="only the serving stream, full protocol (2000 requests at 0.5x and 0.8x saturation)")
    ap.add_argument("--no-serving", action="store_true", help="leave the serving summary out of the default line")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--no-configs", action="store_true", help="leave the other configurations out of the line")
    ap.add_argument("--no-studies", action="store_true", help="leave the reduced kind and pivoting studies out")
    ap.add_argument("--study", choices=["kinds", "pivoting"],
                    help="only one study at its full sizes (matrix kinds x update precision; FP64 pivoting)")
    return ap.parse_args()


def serving_stream(torch, mxp, n_requests: int, drop: int, loads, sat_requests: int, slots: int) -> dict:
    """Serving stream: n log-uniform in [512, 16384], 1..8 right-hand sides,
    request seed 1000 + id, BF16 update and storage, FP64 refinement.  The
    saturated rate is measured first (all requests queued at once); then
    Poisson arrivals (generator seed 7) at the given fractions of it.
    Latency = completion - arrival; the first `drop` requests are warm-up."""
    import numpy as np
    rng = np.random.default_rng(7)

    def draw(k):
        n = np.floor(np.exp(rng.uniform(np.log(512), np.log(16384), k))).astype(np.int64)
        r = rng.integers(1, 9, k)
        return list(zip(n.tolist(), r.tolist()))

    arena = int(1.25 * slots * mxp.server_request_bytes(16384, 8, 512))
    srv = mxp.Server(arena, max_slots=slots, update="bf16", store="bf16", autotune=True)
    try:
        tuned = {n: {"nb": srv.block_size(n), "tile": "128x128" if srv.tile(n) == mxp.TILE_128x128 else "256x128"}
                 for n in (512, 1024, 2048, 4096, 8192, 16384)}
        sat = draw(sat_requests)
        t0 = time.perf_counter()
        ids = [srv.submit(n, r, 1000 + k, want_x=False) for k, (n, r) in enumerate(sat)]
        srv.drain()
        t_sat = time.perf_counter() - t0
        bad = sum(1 for i in ids if srv.wait(i).status != mxp.OK)
        rate_sat = len(sat) / t_sat
        st = srv.stats()
        out = {"saturated_solves_per_s": round(rate_sat, 2), "saturation_requests": len(sat),
               "saturation_failed": bad, "slots": slots, "streams": st["streams"], "tuned": tuned,
               "saturation_groups": st["groups"], "saturation_mean_group": round(st["grouped_requests"] /
                                                                                 max(st["groups"], 1), 2),
               "peak_group": st["peak_group"], "runs": []}
        for frac in loads:
            lam = frac * rate_sat
            reqs = draw(n_requests)
            gaps = rng.exponential(1.0 / lam, n_requests)
            arrive = np.cumsum(gaps)
            ids = []
            t0 = time.perf_counter()
            for k, (n, r) in enumerate(reqs):
                dt = arrive[k] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                ids.append(srv.submit(n, r, 1000 + k, want_x=False))
            srv.drain()
            res = [srv.wait(i) for i in ids]
            lat = np.array([x.latency_ms for x in res[drop:]])
            ok = all(x.status == mxp.OK and x.eta < 16 for x in res)
            span = (max(x.t_done_ns for x in res[drop:]) - min(x.t_submit_ns for x in res[drop:])) / 1e9
            out["runs"].append({"load": frac, "lambda_per_s": round(lam, 2), "requests": n_requests, "dropped": drop,
                                "solves_per_s": round((n_requests - drop) / span, 2),
                                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                                "mean_ms": round(float(lat.mean()), 3), "all_valid": ok,
                                "max_iters": max(x.iters for x in res), "max_eta": max(x.eta for x in res),
                                "peak_in_flight": srv.stats()["peak_in_flight"],
                                "peak_group": srv.stats()["peak_group"]})
        return out
    finally:
        srv.close()
        del srv
        torch.cuda.empty_cache()


def gemm_source_hash() -> str:
    with open(GEMM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_file(args) -> str:
    return os.path.join(PROFILES, "k_gemm_update_traffic_n%d_nb%d_%s_%s.txt" % (args.n, args.nb, args.update,
                                                                               args.store))


def _csv_rows(d: str, suffix: str):
    rows = []
    for fn in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return rows


def summarize_pmc(args):
    """HBM bytes per trailing-update launch from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    plain copy of CALIB_BYTES at the end of the traffic run."""
    out = {}
    for counter, d in (("FETCH_SIZE", args.summarize_pmc[0]), ("WRITE_SIZE", args.summarize_pmc[1])):
        rows = [r for r in _csv_rows(d, "counter_collection.csv") if r["Counter_Name"] == counter]
        gemm = [float(r["Counter_Value"]) for r in rows if "k_gemm_update" in r["Kernel_Name"]]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower()]
        calib_kib = float(copies[-1]["Counter_Value"])       # the calibration copy is the last copy
        factor = (CALIB_BYTES / 1024.0) / calib_kib
        out[counter] = {"launches": len(gemm), "raw_kib_per_launch": sum(gemm) / len(gemm),
                        "calib_raw_kib": calib_kib, "calib_factor": factor,
                        "bytes_per_launch": sum(gemm) / len(gemm) * 1024.0 * factor}
    rec = {"kernel": "k_gemm_update<%s,%s>" % (args.update, args.store), "gemm_source_sha256_16": gemm_source_hash(),
           "workload": "n=%d nb=%d, one factorisation" % (args.n, args.nb),
           "fetch_bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"],
           "write_bytes_per_launch": out["WRITE_SIZE"]["bytes_per_launch"],
           "traffic_bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"],
           "counters": out}
    os.makedirs(PROFILES, exist_ok=True)
    with open(traffic_file(args), "w") as f:
        f.write("# HBM traffic of the trailing update (rocprofv3 --pmc, one counter per run)\n")
        f.write("# command: %s\n" % args.cmd)
        f.write("# each counter is scaled by the ratio of true to counted bytes of a %d-byte plain copy\n"
                % CALIB_BYTES)
        f.write(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec))


def summarize_stats(args):
    rows = _csv_rows(args.summarize_stats, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    os.makedirs(PROFILES, exist_ok=True)
    fn = os.path.join(PROFILES, "kernel_stats_n%d_nb%d_%s_%s.txt" % (args.n, args.nb, args.update, args.store))
    with open(fn, "w") as f:
        f.write("# rocprofv3 --kernel-trace --stats summary of bench.py --steps 1 --warmup 1 (n=%d nb=%d %s/%s):\n"
                "# three solves: the warm-up step, the timed step and the per-phase timing step\n"
                % (args.n, args.nb, args.update, args.store))
        f.write("# command: %s\n" % args.cmd)
        f.write("%-60s %7s %12s %12s %7s\n" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
        for r in rows[:25]:
            name = r["Name"].split("(")[0].replace("void ", "")[:60]
            f.write("%-60s %7d %12.3f %12.2f %7.2f\n" % (name, int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e3,
                                                        100.0 * float(r["TotalDurationNs"]) / total))
        # the trailing update over both work-group tiles (what bench.py's roofline averages over)
        upd = [r for r in rows if "k_gemm_update<" in r["Name"]]
        if len(upd) > 1:
            calls = sum(int(r["Calls"]) for r in upd)
            tns = sum(float(r["TotalDurationNs"]) for r in upd)
            f.write("%-60s %7d %12.3f %12.2f %7.2f\n" % ("k_gemm_update, all tiles", calls, tns / 1e6,
                                                        tns / calls / 1e3, 100.0 * tns / total))
    print(open(fn).read())


def cpu_baseline(n: int, seed: int) -> dict:
    """The oracle (plain C, FP64) on a bounded sample of the same workload:
    generate, unpivoted LU, GMRES-IR at size n, in a child process pinned to
    one OpenMP thread so that the core count is exact."""
    code = ("import json, sys, time; sys.path.insert(0, %r); import oracle; oracle.build(); "
            "t0 = time.perf_counter(); A, B, X, reps = oracle.solve(%d, %d); t = time.perf_counter() - t0; "
            "print(json.dumps({'t': t, 'status': reps[0]['status'], 'eta': reps[0]['eta']}))" % (ROOT, n, seed))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, check=True, capture_output=True, text=True)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    assert r["status"] == 0 and r["eta"] < 16, r
    t = r["t"]
    return {"value": (2.0 / 3.0) * n ** 3 / t / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "oracle FP64 unpivoted LU + GMRES-IR solve at n=%d (same generator, seed %d), %.1f s on one "
                      "thread (OMP_NUM_THREADS=1), rate by the same 2/3 n^3 formula" % (n, seed, t)}


def fp64_gpu_baselines(torch, mxp, n: int, seed: int, reps: int = 3) -> dict:
    """The FP64 solve on the same GPU and the exact FP64 matrix, timed the
    same way as the mixed-precision solve (HIP events around factor + solve on
    the current stream, one untimed warm-up, the mean of `reps` runs):
      * own:       this library's FP64 LU without pivoting (FP64 matrix-core
                   trailing update) and its FP64 triangular solves;
      * rocsolver: torch.linalg.lu_factor_ex + lu_solve (rocSOLVER getrf /
                   getrs, partial pivoting).
      * own_rocblas: the same LU with rocBLAS dgemm as its trailing update.
    The fastest one is the denominator of the speed-up."""
    prob = mxp.mxp_generate(n, 1, seed, store="f64")
    A0 = prob.A.clone()
    A = mxp.as_matrix(prob.A, n)
    b = prob.B[0].clone().unsqueeze(1)
    work = torch.empty(mxp.lib().mxp_lu64_work_bytes(n), dtype=torch.uint8, device="cuda")
    out = {}

    def timed(fn):
        times, x = [], None
        for it in range(reps + 1):
            prob.A.copy_(A0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            x = fn()
            e1.record()
            torch.cuda.synchronize()
            if it > 0:
                times.append(e0.elapsed_time(e1))
        return statistics.mean(times), x

    def own():
        fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=False, sync_info=False, work=work)
        return mxp.mxp_lu64_solve(fac, prob.B[:1])[0]

    def own_rocblas():
        fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=False, sync_info=False, work=work,
                                  gemm=mxp.GEMM64_ROCBLAS)
        return mxp.mxp_lu64_solve(fac, prob.B[:1])[0]

    def rocsolver():
        LU, piv, info = torch.linalg.lu_factor_ex(A.contiguous())
        return torch.linalg.lu_solve(LU, piv, b)[:, 0]

    mxp.profile_reset()
    mxp.profile_enable(True, classes=[mxp.PROF_GEMM64])
    t_own, x_own = timed(own)
    mxp.profile_enable(False)
    g = mxp.profile_read(mxp.PROF_GEMM64)
    mxp.profile_reset()
    mxp.profile_enable(True, classes=[mxp.PROF_GEMM64])
    t_ob, x_ob = timed(own_rocblas)
    mxp.profile_enable(False)
    gb = mxp.profile_read(mxp.PROF_GEMM64)
    t_roc, x_roc = timed(rocsolver)
    for name, t, x, kind in (("own", t_own, x_own, "libmxp FP64 LU without pivoting (mxp_lu64_factor/solve)"),
                             ("own_rocblas", t_ob, x_ob, "libmxp FP64 LU without pivoting, rocBLAS dgemm update"),
                             ("rocsolver", t_roc, x_roc, "torch.linalg.lu_factor_ex + lu_solve, float64 "
                                                         "(rocSOLVER getrf/getrs)")):
        out[name] = {"value": (2.0 / 3.0) * n ** 3 / (t * 1e-3) / 1e12, "unit": "TFLOP/s", "ms": t,
                     "eta": mxp.mxp_hpl_eta(prob, x.contiguous(), prob.B[0]), "kind": kind}
    out["own"]["gemm64_tflops"] = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else None
    out["own"]["gemm64_frac_of_fp64_peak"] = (out["own"]["gemm64_tflops"] or 0.0) / PEAK["f64_tflops"]
    out["own_rocblas"]["dgemm_tflops"] = gb["flops"] / (gb["ms"] * 1e-3) / 1e12 if gb["ms"] > 0 else None
    best = max(("own", "own_rocblas", "rocsolver"), key=lambda k: out[k]["value"])
    out["faster"] = best
    del prob, A, A0, work
    torch.cuda.empty_cache()
    return out


CONFIGS = [
    # (name, n, nb, update, store, scaling, warmup, steps)
    ("plain method, FP32 LU", 2048, 256, "f32", "f32", "none", 2, 5),
    ("n=131072 BF16, unscaled", 131072, 1024, "bf16", "bf16", "none", 1, 1),
    ("n=131072 BF16, row-equilibrated", 131072, 1024, "bf16", "bf16", "row_equil", 1, 1),
    ("n=131072 FP16, unscaled", 131072, 1024, "f16", "f16", "none", 1, 1),
    ("n=131072 FP16, row-equilibrated", 131072, 1024, "f16", "f16", "row_equil", 1, 1),
    ("n=65536 FP8-E4M3, per-strip scales", 65536, 512, "f8", "f16", "none", 1, 2),
    ("n=65536 FP16 (for the FP8 ratio)", 65536, 512, "f16", "f16", "none", 1, 2),
]


def config_runs(torch, mxp, seed: int) -> list:
    """The other configurations, each timed like the headline (inputs
    generated once and restored before every step, untimed; scaling, LU and
    refinement timed), with the trailing update's own rate from HIP events."""
    out = []
    L = mxp.lib()
    cache = {}
    for name, n, nb, update, store, scaling, warmup, steps in CONFIGS:
        key = (n, store)
        if key not in cache:
            cache.clear()
            torch.cuda.empty_cache()
            prob = mxp.mxp_generate(n, 1, seed, store=store)
            cache[key] = (prob, prob.A.clone())
        prob, A0 = cache[key]
        up = mxp.dtype_code(update)
        aux = torch.empty(L.mxp_factor_aux_bytes(n, nb), dtype=torch.uint8, device="cuda")
        fwork = torch.empty(L.mxp_factor_work_bytes(n, nb, up), dtype=torch.uint8, device="cuda")
        swork = torch.empty(L.mxp_solve_work_bytes(n, 1, 30), dtype=torch.uint8, device="cuda")
        X = torch.empty((1, n), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        sc = mxp.SCALE_ROW_EQUIL if scaling == "row_equil" else mxp.SCALE_NONE
        times, res = [], None
        for it in range(warmup + steps):
            prob.A.copy_(A0)
            timed = it >= warmup
            if timed:
                mxp.profile_reset()
                mxp.profile_enable(True, classes=[mxp.PROF_GEMM])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            fac = mxp.mxp_factor(prob, nb, update, work=fwork, aux=aux, scaling=sc)
            res = mxp.mxp_solve_ir(prob, fac, work=swork, X=X)
            if timed:
                e1.record(stream)
                torch.cuda.synchronize()
                mxp.profile_enable(False)
                times.append(e0.elapsed_time(e1))
                g = mxp.profile_read(mxp.PROF_GEMM)
        ms = statistics.mean(times)
        tflops_upd = g["flops"] / (g["ms"] * 1e-3) / 1e12
        peak = PEAK["%s_tflops" % update]
        intensity = g["flops"] / g["bytes"]
        ridge = peak * 1e12 / (PEAK["hbm_gbs"] * 1e9)
        if intensity >= ridge:
            roof = {"bound": "mfma", "achieved": round(tflops_upd, 1), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(tflops_upd / peak, 4)}
        else:
            gbs = g["bytes"] / (g["ms"] * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                    "frac": round(gbs / PEAK["hbm_gbs"], 4)}
        roof.update({"kernel": "k_gemm_update<%s,%s>" % (update, store), "mfma_tflops": round(tflops_upd, 1),
                     "mfma_frac": round(tflops_upd / peak, 4), "launches": g["launches"]})
        out.append({"config": name, "n": n, "nb": nb, "update": update, "store": store, "scaling": scaling,
                    "value": round((2.0 / 3.0) * n ** 3 / (ms * 1e-3) / 1e12, 2), "unit": "TFLOP/s",
                    "ms": round(ms, 3), "steps": steps, "iters": res.iters[0], "eta": res.eta[0],
                    "valid": res.status[0] == 0 and res.eta[0] < 16, "update_roofline": roof})
        print(json.dumps({"config_done": name, "ms": round(ms, 3)}), file=sys.stderr, flush=True)
        del aux, fwork, swork, X, fac, res
    cache.clear()
    torch.cuda.empty_cache()
    return out


def kinds_study(torch, mxp, n: int, nb: int, seed: int) -> list:
    """Iterations and backward error of the low-precision LU + GMRES-IR
    against the diagonal of the matrix ("Matrix Generation": the dominant
    diagonal is for debugging; a diagonal gamma sqrt(n) departs from
    dominance, and near gamma = 1/sqrt(12) leaves GMRES without a
    preconditioner far from convergence) and the update precision."""
    out = []
    for kind, gamma in ((mxp.GEN_DOMINANT, 0.0), (mxp.GEN_SQRTN, 1.0), (mxp.GEN_SQRTN, 0.5), (mxp.GEN_SQRTN, 0.3)):
        for update, store in (("f16", "f16"), ("bf16", "bf16"), ("f8", "f16")):
            prob = mxp.mxp_generate(n, 1, seed, store=store, kind=kind, gamma=gamma)
            A0 = prob.A.clone()
            rec = {"kind": {mxp.GEN_DOMINANT: "dominant", mxp.GEN_SQRTN: "sqrt(n)"}[kind], "gamma": gamma,
                   "update": update, "store": store, "n": n, "nb": nb}
            for rep in range(2):                                   # the first run warms up
                prob.A.copy_(A0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fac = mxp.mxp_factor(prob, nb, update)
                if fac.info:
                    rec.update({"status": "singular pivot", "info": fac.info})
                    break
                res = mxp.mxp_solve_ir(prob, fac)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                rec.update({"iters": res.iters[0], "eta": res.eta[0], "status": res.status[0], "ms": round(1e3 * t, 2),
                            "tflops": round((2.0 / 3.0) * n ** 3 / t / 1e12, 2)})
            out.append(rec)
            del prob, A0
            torch.cuda.empty_cache()
    return out


def pivot_study(torch, mxp, sizes, seeds) -> list:
    """The FP64 experiments behind Figures 2-4 ("Experimental Results"):
    entries uniform in [-1, 1) without diagonal scaling, LU in FP64 with and
    without partial pivoting; the largest pivot |u_kk| of the pivoted LU and
    where it falls, next to sqrt(n), 5/8 sqrt(n) and n^0.45; the 1-, 2- and
    inf-norms of the residual b - A x of both solves (and the HPL scaled
    residual of each)."""
    out = []
    for n in sizes:
        for seed in seeds:
            rec = {"n": n, "seed": seed, "sqrt_n": n ** 0.5, "five_eighths_sqrt_n": 0.625 * n ** 0.5,
                   "n_pow_045": n ** 0.45}
            prob = mxp.mxp_generate(n, 1, seed, store="f64", kind=mxp.GEN_UNIFORM)
            A0 = prob.A.clone()
            for pivot in (True, False):
                prob.A.copy_(A0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fac = mxp.mxp_lu64_factor(prob.A, n, prob.lda, pivot=pivot)
                x = mxp.mxp_lu64_solve(fac, prob.B[:1])
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                r = mxp.mxp_residual(prob, x, prob.B[:1])[0]
                d = mxp.as_matrix(prob.A, n).diagonal().abs()
                key = "pivoting" if pivot else "no_pivoting"
                rec[key] = {"r_1": float(r.abs().sum()), "r_2": float(r.norm()), "r_inf": float(r.abs().max()),
                            "eta": mxp.mxp_hpl_eta(prob, x[0].contiguous(), prob.B[0]), "info": fac.info,
                            "ms": round(1e3 * t, 2), "max_pivot": float(d.max()),
                            "max_pivot_at_frac": round(float(d.argmax()) / n, 4)}
            out.append(rec)
            del prob, A0
            torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.summarize_pmc:
        return summarize_pmc(args)
    if args.summarize_stats:
        return summarize_stats(args)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU design is described in DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2509_19618_amd as mxp

    if args.study == "kinds":
        print(json.dumps({"study": "kinds", "runs": kinds_study(torch, mxp, 32768, 512, args.seed)}), flush=True)
        return
    if args.study == "pivoting":
        print(json.dumps({"study": "pivoting",
                          "runs": pivot_study(torch, mxp, (1000, 2000, 4000, 8000, 16000, 32000, 46340), (1, 2, 3))}),
              flush=True)
        return
    if args.serve:
        sv = serving_stream(torch, mxp, 2000, 200, (0.5, 0.8), 400, args.serve_slots)
        r8 = sv["runs"][-1]
        print(json.dumps({"metric": "served solves/s (serving stream, n log-uniform 512..16384, 1-8 RHS); p50/p99",
                          "value": r8["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
                          "p50_ms": r8["p50_ms"], "p99_ms": r8["p99_ms"], "dtype": "bf16", "data": "synthetic",
                          "config": {"workload": "serving stream, Poisson arrivals at 0.5x and 0.8x saturation, "
                                                 "2000 requests, first 200 dropped"},
                          "serving": sv}), flush=True)
        return

    n, nb = args.n, args.nb
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    prob = mxp.mxp_generate(n, 1, args.seed, store=args.store)
    A0 = prob.A.clone()                         # pristine input, restored before each step
    L = mxp.lib()
    up = mxp.dtype_code(args.update)
    aux = torch.empty(L.mxp_factor_aux_bytes(n, nb), dtype=torch.uint8, device="cuda")
    fwork = torch.empty(L.mxp_factor_work_bytes(n, nb, up), dtype=torch.uint8, device="cuda")
    swork = torch.empty(L.mxp_solve_work_bytes(n, 1, args.restart), dtype=torch.uint8, device="cuda")
    X = torch.empty((1, n), dtype=torch.float64, device="cuda")

    def step(timed_events=None):
        prob.A.copy_(A0)                        # untimed input restore
        if timed_events:
            timed_events[0].record(stream)
        fac = mxp.mxp_factor(prob, nb, args.update, work=fwork, aux=aux,
                             scaling=mxp.SCALE_ROW_EQUIL if args.scaling == "row_equil" else mxp.SCALE_NONE)
        res = mxp.mxp_solve_ir(prob, fac, restart=args.restart, work=swork, X=X)
        if timed_events:
            timed_events[1].record(stream)
        return fac, res

    if args.traffic_run:
        fac, res = step()
        src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                          # the calibration copy: the run's last copy kernel
        torch.cuda.synchronize()
        print(json.dumps({"traffic_run": True, "info": fac.info, "status": res.status[0]}), flush=True)
        return

    for _ in range(args.warmup):
        fac, res = step()
    torch.cuda.synchronize()

    # the timed steps time only the dominant kernel (the trailing update) with
    # events: its roofline below comes from them; every other class's events
    # would add work to the critical chain of the timed region
    mxp.profile_reset()
    mxp.profile_enable(True, classes=[mxp.PROF_GEMM])
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fac, res = step(evs[k])
        results.append((fac.info, res.status[0], res.iters[0], res.eta[0]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mxp.profile_enable(False)
    step_ms = [a.elapsed_time(b) for a, b in evs]
    prof = {c: mxp.profile_read(c) for c in (mxp.PROF_GEMM, mxp.PROF_TRSM, mxp.PROF_DIAG, mxp.PROF_PREC,
                                              mxp.PROF_REGEN)}
    # the per-phase kernel times: one more, untimed step with every class timed
    mxp.profile_reset()
    mxp.profile_enable(True)
    step()
    torch.cuda.synchronize()
    mxp.profile_enable(False)
    phase = {c: mxp.profile_read(c) for c in (mxp.PROF_GEMM, mxp.PROF_TRSM, mxp.PROF_DIAG, mxp.PROF_PREC,
                                               mxp.PROF_REGEN)}
    valid = all(r[0] == 0 and r[1] == 0 and r[3] < 16 for r in results)
    ms = statistics.mean(step_ms)
    ops = (2.0 / 3.0) * n ** 3
    value = ops / (ms * 1e-3) / 1e12

    # roofline of the dominant kernel: the trailing update
    g = prof[mxp.PROF_GEMM]
    sC = {"f32": 4, "f16": 2, "bf16": 2}[args.store]
    intensity = g["flops"] / g["bytes"]
    peak_fl = PEAK["%s_tflops" % args.update]
    ridge = peak_fl * 1e12 / (PEAK["hbm_gbs"] * 1e9)
    tflops = g["flops"] / (g["ms"] * 1e-3) / 1e12
    gbs = g["bytes"] / (g["ms"] * 1e-3) / 1e9
    if intensity >= ridge:
        roof = {"bound": "mfma", "achieved": round(tflops, 1), "peak": peak_fl, "unit": "TFLOP/s",
                "frac": round(tflops / peak_fl, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": round(gbs / PEAK["hbm_gbs"], 4)}
    traffic = None
    tf = traffic_file(args)
    if os.path.exists(tf):
        rec = json.loads(open(tf).read().split("\n", 3)[3])
        if rec["gemm_source_sha256_16"] == gemm_source_hash():   # counters taken on this kernel
            traffic = round(rec["traffic_bytes_per_launch"])
    roof.update({"traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                 "algorithmic_bytes_per_launch": round(g["bytes"] / max(g["launches"], 1)),
                 "kernel": "k_gemm_update<%s,%s>" % (args.update, args.store),
                 "launches": g["launches"], "avg_launch_us": round(1e3 * g["ms"] / max(g["launches"], 1), 2),
                 "mfma_tflops": round(tflops, 1), "mfma_frac": round(tflops / peak_fl, 4),
                 "intensity_flop_per_byte": round(intensity, 1), "ridge": round(ridge, 1),
                 "attainable_frac_of_mfma_peak": round(min(1.0, intensity / ridge), 3)})

    line = {
        "metric": "effective TFLOP/s (2/3*n^3/time) to FP64 backward error vs FP64 LU; p50/p99",
        "value": round(value, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.update, "data": "synthetic",
        "config": {"workload": "HPL-MxP solve n=%d nb=%d %s update %s storage, FP32 panel/TRSM, FP64 GMRES-IR "
                               "restart %d, seed %d%s" % (n, nb, args.update, args.store, args.restart, args.seed,
                                                      ", row-equilibrated" if args.scaling == "row_equil" else ""),
                   "n": n, "nb": nb, "update": args.update, "store": args.store, "restart": args.restart,
                   "nrhs": 1, "scaling": args.scaling, "parallelism": "single GPU"},
        "p50_ms": round(statistics.median(step_ms), 3),
        "p99_ms": round(sorted(step_ms)[min(len(step_ms) - 1, int(0.99 * len(step_ms)))], 3),
        "wall_ms_per_step_incl_untimed_restore": round(1e3 * wall / args.steps, 3),
        "valid": valid, "iters": results[-1][2], "eta": results[-1][3],
        "value_incl_3_2_n2": round((ops + 1.5 * n * n) / (ms * 1e-3) / 1e12, 2),
        "phase_ms_per_step": {k: round(phase[c]["ms"], 3) for k, c in
                              (("trailing_update", mxp.PROF_GEMM), ("strip_trsm", mxp.PROF_TRSM),
                               ("diag_lu", mxp.PROF_DIAG), ("prec_apply", mxp.PROF_PREC),
                               ("regen_matvec", mxp.PROF_REGEN))},
        "roofline": roof,
    }
    del A0, aux, fwork, swork
    prob = None
    torch.cuda.empty_cache()
    if not args.no_serving:
        sv = serving_stream(torch, mxp, 600, 60, (0.5, 0.8), 200, args.serve_slots)
        r8 = sv["runs"][-1]
        line["p50_ms_served"] = r8["p50_ms"]
        line["p99_ms_served"] = r8["p99_ms"]
        line["serving"] = sv
    if not args.no_configs:
        line["configs"] = config_runs(torch, mxp, args.seed)
    if not args.no_studies:
        line["study_kinds"] = kinds_study(torch, mxp, 16384, 512, args.seed)
        line["study_pivoting"] = pivot_study(torch, mxp, (2000, 8000, 32000), (1,))
    if not args.no_fp64_baseline:
        fb = fp64_gpu_baselines(torch, mxp, n, args.seed)
        line["fp64_baseline"] = {k: ({kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                                     if isinstance(v, dict) else v) for k, v in fb.items()}
        line["speedup_vs_fp64_lu"] = round(value / fb[fb["faster"]]["value"], 2)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, args.seed)
        line["cpu_baseline"]["value"] = round(line["cpu_baseline"]["value"], 6)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
