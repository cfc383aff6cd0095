#!/usr/bin/env python3
"""Benchmark: entropic OT solves per second to a 1e-6 L1 marginal error on
one MI355X, SK-NR(l) with the sequential spectral warm start against plain
log-domain Sinkhorn on the same GPU, with p50/p99 solve latency.

Workload (one "step" = one full solve): n = m = 4096 points in [0,1]^2,
x from a 3-component Gaussian mixture (sigma 0.05), y uniform, weights
Dirichlet(5); squared-Euclidean cost built on the fly in FP32; eps annealed
1e-1 -> 1e-3 by halving (8 stages), each stage run to an L1 marginal error
below 1e-6: intermediate stages stop on the sweeps' FP32 estimate of it, the
last stage is verified in FP64.  Inputs are resident in HBM before timing.

Prints one JSON line (see the fields below).  `--gpus N` with N > 1 exits:
the solver runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "OT solves/s to 1e-6 marginal err (SK-NR vs SK); p50/p99 latency"

# MI355X peaks used for the roofline (public figures; the VALU peak is
# derived from unit counts: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz).
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.32 T lane-instructions/s


def algorithmic_work(kind: str):
    """(bound, work per cost element, unit) of a sweep kind.

    Points sweeps ("alu"): per element the squared distance for d = 2 (2
    sub, 1 mul, 1 fma), the exponent U - C and its scaling by 1/eps, the
    running max, exp2 (issued at half rate: 2 slots) and the accumulation:
    10 VALU slots; a weighted sweep adds one FMA per basis column.
    Stored-cost sweeps ("hbm"): 4 bytes of C read per element."""
    kind = kind.split(":")[0]
    width = int(kind.rsplit("_l", 1)[1]) if "_l" in kind else 0
    if "stored" in kind:
        return "hbm", 4.0, "GB/s"
    if "bf16" in kind:
        # matrix-core cost: the cross term is MFMA work; on the VALU the
        # cost is finished by one add and one fma, then the same exponent,
        # max, exp and accumulation as above; the adds joining the product
        # chains come on top (hi/lo split: 1, hi/mid/lo split: 3)
        join = 3.0 if "bf16x6" in kind else 1.0 if "bf16x3" in kind else 0.0
        return "alu", 8.0 + join + width, "TOP/s"
    return "alu", 10.0 + width, "TOP/s"


# HBM bytes per launch of the main sweep kernels from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the counts of a
# plain 1 GiB device copy (FETCH_SIZE reads 0.5 GiB -> x2.0, WRITE_SIZE 1 GiB
# -> x1.0); see profiles/.  Valid only for the kernel sources they were
# taken with (SHA-1 over sknr_device.h, sknr_kernels.hip, sknr_mfma.hip,
# sknr_fused.hip, sknr_sweep_tail.h).
TRAFFIC_KERNEL_SHA1 = "a8e9d1e12731519ec171961a5e39e5d8818902fe"
TRAFFIC_BYTES = {
    "sweep_stream_points_l0:main": (338.14 * 1.9999 + 2846.24 * 1.0000) * 1024,
    "sweep_stream_stored_l0:main": (518397.07 * 1.9999 + 6067.04 * 1.0000) * 1024,
    "sweep_rows_stored_l0:main": (525961.34 * 1.9999 + 640.09 * 1.0000) * 1024,
    "sk_fused_stored:main": (525314.82 * 1.9999 + 32947.58 * 1.0000) * 1024,
    "sk_fused_stored": ((525314.82 + 16669.98) * 1.9999 + (32947.58 + 159.97) * 1.0000) * 1024,
    "sweep_stream_points_bf16x3_l0:main": (90819.55 * 1.9999 + 6223.96 * 1.0000) * 1024,
    "sweep_stream_points_bf16x6_l0:main": (140137.07 * 1.9999 + 6223.96 * 1.0000) * 1024,
    "sweep_stream_points_bf16_l0:main": (24530.40 * 1.9999 + 6223.96 * 1.0000) * 1024,
}


def kernel_traffic(name):
    import hashlib
    h = hashlib.sha1()
    for f in ("sknr_device.h", "sknr_kernels.hip", "sknr_mfma.hip", "sknr_fused.hip", "sknr_sweep_tail.h"):
        h.update(open(os.path.join(ROOT, "paper_2506_14780_amd", "csrc", f), "rb").read())
    if h.hexdigest() != TRAFFIC_KERNEL_SHA1:
        return None
    return TRAFFIC_BYTES.get(name)


PEAK_MFMA_BF16_TFLOPS = 2500.0  # dense bf16 matrix-core peak


def mfma_sweep_roofline(sk, W, torch, reps=4):
    """The d = 64 point-cloud sweep (20000 x 30000, cost cross term on
    bf16 matrix cores: one, two or three bf16 parts per point coordinate):
    per-kernel HIP event timing of column and row c-transforms, VALU
    fraction against the algorithmic slots per element and matrix-core
    fraction against the bf16 peak."""
    prob = W.gaussian_clouds()
    dev = torch.device("cuda:0")
    x, y = torch.from_numpy(prob.x).to(dev), torch.from_numpy(prob.y).to(dev)
    a, b = torch.from_numpy(prob.a).to(dev), torch.from_numpy(prob.b).to(dev)
    out = {"workload": f"gaussian_clouds {prob.n}x{prob.m} d={prob.d}, one column + one row c-transform per rep"}
    ctx = sk.Context(0)
    f = torch.zeros(prob.n, dtype=torch.float64, device=dev)
    for name, xt in (("bf16x3", sk.XTERM_BF16X3), ("bf16x6", sk.XTERM_BF16X6), ("bf16", sk.XTERM_BF16)):
        gp = sk.Problem(a=a, b=b, x=x, y=y, xterm=xt)
        g, _, _ = sk.c_transform_col(ctx, gp, 0.1, f)  # warm-up
        ctx.profile(True)
        for _ in range(reps):
            g, _, _ = sk.c_transform_col(ctx, gp, 0.1, f)
            sk.c_transform_row(ctx, gp, 0.1, g)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        main = [e for e in prof if e["name"].endswith(":main")][0]
        avg_s = main["total_ms"] / main["launches"] / 1e3
        elems = main["units"] / main["launches"]
        _, slots, _ = algorithmic_work(main["name"])
        dpad = (prob.d + 31) // 32 * 32
        flops = 2.0 * dpad * {"bf16": 1, "bf16x3": 3, "bf16x6": 6}[name] * elems
        out[name] = {"kernel": main["name"], "avg_launch_us": avg_s * 1e6, "elements_per_launch": elems,
                     "bound": "alu", "achieved": slots * elems / avg_s / 1e12, "peak": PEAK_VALU_TOPS,
                     "unit": "TOP/s", "frac": slots * elems / avg_s / 1e12 / PEAK_VALU_TOPS,
                     "work_per_element": slots, "traffic": kernel_traffic(main["name"]),
                     "mfma_tflops": flops / avg_s / 1e12,
                     "mfma_frac": flops / avg_s / 1e12 / PEAK_MFMA_BF16_TFLOPS}
    ctx.close()
    return out


def paper_workloads_bench(sk, W, torch, tol, reps=3):
    """Sec. 5's workloads on the GPU, SK-NR against plain SK (median of
    `reps` solves each, after one warm-up): Fig. 5.1's 200 vs 400 Gaussians
    (eps 1 -> 1/8 by halving, l = 10) and the synthetic stand-ins at the
    single-cell shapes (6507 x 3815 and 3815 x 2982, d = 30, l = 30,
    eps 1 -> 1/16 by halving; plain SK at eps = 1 first)."""
    dev = torch.device("cuda:0")
    ctx = sk.Context(0)
    cases = [("fig5.1 gaussians 200x400 d=2", W.paper_2d_gaussians(200), [1.0, 0.5, 0.25, 0.125], 10),
             ("wot-shaped 6507x3815 d=30", W.wot_shaped(6507, 3815), [1.0, 0.5, 0.25, 0.125, 0.0625], 30),
             ("wot-shaped 3815x2982 d=30", W.wot_shaped(3815, 2982, seed=11), [1.0, 0.5, 0.25, 0.125, 0.0625], 30)]
    out = {}
    for name, prob, ladder, ell in cases:
        gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                        x=torch.from_numpy(prob.x).to(dev), y=torch.from_numpy(prob.y).to(dev))
        row = {"eps_ladder": ladder, "ell": ell}
        for mode, kw in (("sknr", dict(ell=ell, warm_mode=sk.WARM_SEQUENTIAL)), ("sk", {})):
            sk.solve(ctx, gp, ladder, tol=tol, max_iter=100000, **kw)
            torch.cuda.synchronize()
            ts, res = [], None
            for _ in range(reps):
                t0 = time.perf_counter()
                res = sk.solve(ctx, gp, ladder, tol=tol, max_iter=100000, **kw)[2]
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row[mode] = {"ms": 1e3 * float(np.median(ts)), "iters_per_stage": [st["iters"] for st in res["stages"]],
                         "newton_accepted": [st["newton_accepted"] for st in res["stages"]],
                         "marginal_err": res["marginal_err"], "status": res["status"]}
        row["speedup"] = row["sk"]["ms"] / row["sknr"]["ms"]
        out[name] = row
    ctx.close()
    return out


def points_sweep_large(sk, W, torch, n=20000, m=30000, reps=4):
    """The d = 2 points sweep of the benchmark workload's kind at a size
    where the launch and per-workgroup costs no longer dominate (20000 x
    30000: 37x the elements of 4096^2): main-kernel duration of the column
    and row c-transforms against the same VALU roofline."""
    prob = W.gmm_vs_uniform(n, m, seed=1)
    dev = torch.device("cuda:0")
    gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                    x=torch.from_numpy(prob.x).to(dev), y=torch.from_numpy(prob.y).to(dev))
    ctx = sk.Context(0)
    f = torch.zeros(prob.n, dtype=torch.float64, device=dev)
    g, _, _ = sk.c_transform_col(ctx, gp, 1e-2, f)
    ctx.profile(True)
    for _ in range(reps):
        g, _, _ = sk.c_transform_col(ctx, gp, 1e-2, f)
        sk.c_transform_row(ctx, gp, 1e-2, g)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    main = [e for e in prof if e["name"].endswith(":main")][0]
    avg_s = main["total_ms"] / main["launches"] / 1e3
    elems = main["units"] / main["launches"]
    _, slots, _ = algorithmic_work(main["name"])
    ach = slots * elems / avg_s / 1e12
    return {"workload": f"gmm_vs_uniform {n}x{m} d=2, one column + one row c-transform per rep",
            "kernel": main["name"], "avg_launch_us": avg_s * 1e6, "elements_per_launch": elems,
            "bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s", "frac": ach / PEAK_VALU_TOPS}


def serving_bench(sk, W, torch, n_req, lanes, tol, seed=4, switch_iters=10):
    """Mixed-request serving: Poisson arrivals, n, m log-uniform on
    [64, 8192], d in {2, 3, 64}, target eps in {1e-1, 1e-2, 1e-3} reached by
    halving from 1, l = min(30, min(n, m) - 1).  A closed-loop run (all
    requests submitted at once) calibrates the arrival rate to 0.8 x the
    SK-NR capacity; the same arrival trace then runs with SK-NR (every stage
    after the first), with SK-NR switched on after the first stage that
    needs more than `switch_iters` SK iterations, and with plain SK.
    Latency = completion - scheduled arrival."""
    trace = W.serving_trace(n_requests=n_req, rate=1.0, seed=seed)
    dev = torch.device("cuda:0")
    probs = [sk.Problem(a=torch.from_numpy(q.problem.a).to(dev), b=torch.from_numpy(q.problem.b).to(dev),
                        x=torch.from_numpy(q.problem.x).to(dev), y=torch.from_numpy(q.problem.y).to(dev),
                        cost_scale=q.problem.cost_scale) for q in trace]
    torch.cuda.synchronize()
    base = np.array([q.arrival for q in trace])
    base = base - base[0]

    def run(nr, rate, switch=0, batched=True):
        ctx = sk.Context(0)
        sk.serve_config(ctx, max_active=lanes, pool_bytes=8 << 30, batched=batched)
        arr = base / rate if rate else np.zeros(n_req)
        t0 = time.monotonic()
        sub = []
        for q, gp, ta in zip(trace, probs, arr):
            wait_s = ta - (time.monotonic() - t0)
            if wait_s > 0:
                time.sleep(wait_s)
            n, m = q.problem.n, q.problem.m
            tk = sk.submit(ctx, gp, W.request_ladder(q.eps), tol=tol, max_iter=20000,
                           ell=min(30, min(n, m) - 1) if nr else 0, warm_mode=sk.WARM_SEQUENTIAL, seed=q.rid,
                           nr_switch_iters=switch if nr else 0)
            sub.append((tk, ta, time.monotonic() - t0))
        lat, ends, status, iters = [], [], [], []
        for q, (tk, ta, tret) in zip(trace, sub):
            _, _, r = sk.wait(ctx, tk, q.problem.n, q.problem.m, raise_on_error=False)
            l = r["latency_seconds"] + (tret - ta)
            lat.append(l)
            ends.append(ta + l)
            status.append(r["status"])
            iters.append(r["total_iters"])
        st = sk.serve_stats(ctx)
        ctx.close()
        makespan = max(ends) - arr[0]
        out = {"solves_per_s": n_req / makespan, "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
               "makespan_s": makespan, "converged": int(sum(1 for v in status if v == 0)),
               "not_converged": int(sum(1 for v in status if v == 1)),
               "failed": int(sum(1 for v in status if v < 0)), "mean_iters": float(np.mean(iters))}
        if batched:
            out["batches"] = st["batches"]
            out["requests_per_batch"] = st["batched_jobs"] / max(1, st["batches"])
            out["batched_launches"] = st["batched_launches"]
        return out

    closed = run(True, 0.0, batched=False)
    closed_batched = run(True, 0.0, batched=True)
    closed_ad = run(True, 0.0, switch_iters, batched=False)
    rate = 0.8 * closed["solves_per_s"]
    return {"workload": f"serving_trace {n_req} requests, n,m log-uniform [64,8192], d in {{2,3,64}}, "
                        f"eps in {{1e-1,1e-2,1e-3}} by halving from 1, tol {tol:g}, l=min(30,min(n,m)-1)",
            "lanes": lanes, "closed_loop_sknr": closed, "closed_loop_sknr_batched": closed_batched,
            "closed_loop_sknr_adaptive": closed_ad,
            "arrival_rate_per_s": rate, "nr_switch_iters": switch_iters,
            "sknr": run(True, rate, batched=False), "sknr_adaptive": run(True, rate, switch_iters, batched=False),
            "sk": run(False, rate, batched=False)}


def c1_bench(sk, W, torch, reps=5):
    """The 256 x 256 workload (uniform points, uniform weights, eps =
    1e-2): GPU time per SK iteration of a cold plain SK solve (tol 1e-6) and
    the SK-NR(30) solve from eps' = 2e-2 (sequential warm start); this size
    is bound by launch latency (131,072 cost elements per iteration)."""
    prob = W.uniform_square(256, seed=0)
    dev = torch.device("cuda:0")
    gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                    x=torch.from_numpy(prob.x).to(dev), y=torch.from_numpy(prob.y).to(dev))
    ctx = sk.Context(0)
    out = {"workload": "uniform_square 256x256 d=2, eps 1e-2, tol 1e-6"}
    for name, ladder, kw in (("cold_sk", [1e-2], {}),
                             ("sknr30_from_2e-2", [2e-2, 1e-2], dict(ell=30, warm_mode=sk.WARM_SEQUENTIAL))):
        ts, res = [], None
        for rep in range(reps + 1):
            t0 = time.perf_counter()
            res = sk.solve(ctx, gp, ladder, tol=1e-6, max_iter=100000, **kw)[2]
            torch.cuda.synchronize()
            if rep:
                ts.append(time.perf_counter() - t0)
        st = res["stages"][-1]
        out[name] = {"ms": 1e3 * float(np.median(ts)), "iters_per_stage": [x["iters"] for x in res["stages"]],
                     "last_stage_us_per_iter": 1e6 * st["seconds"] / max(1, st["iters"]),
                     "status": res["status"]}
    ctx.close()
    return out


def newton_solvers_bench(sk, gp, ladder, tol, reps=3):
    """The projected Newton system solved by Gauss-Jordan, by conjugate
    gradients and by Newton-Schulz iterative inversion (Sec. 4,
    disadvantages paragraph) inside the benchmark solve, l = 16 and 30."""
    import torch
    ctx = sk.Context(0)
    out = {}
    for ell in (16, 30):
        for name, solver in (("direct", sk.NEWTON_DIRECT), ("cg", sk.NEWTON_CG), ("newton_schulz", sk.NEWTON_SCHULZ)):
            ts, res = [], None
            for rep in range(reps + 1):
                t0 = time.perf_counter()
                res = sk.solve(ctx, gp, ladder, tol=tol, max_iter=200000, ell=ell, warm_mode=sk.WARM_SEQUENTIAL,
                               newton_solver=solver)[2]
                torch.cuda.synchronize()
                if rep:
                    ts.append(time.perf_counter() - t0)
            out[f"l{ell}_{name}"] = {"ms": 1e3 * float(np.median(ts)),
                                     "iters_per_stage": [x["iters"] for x in res["stages"]],
                                     "newton_accepted": sum(x["newton_accepted"] for x in res["stages"]),
                                     "status": res["status"]}
    ctx.close()
    return out


def c4_ladder(sk, W, torch, cap):
    """20000 x 30000 d = 64 Gaussian clouds (matrix-core cost, three bf16
    parts), eps 1e-1 -> 1e-2 -> 2e-3, tol 1e-6, at most `cap` iterations a
    stage: plain SK, SK-NR(16) with the sequential warm start, and SK-NR(16)
    with the Ritz-value gain test (nr_min_gain = 2).  Each stage is its own
    call (ladder [previous eps, eps] from the previous potentials), so the
    run prints as it goes."""
    prob = W.gaussian_clouds()
    dev = torch.device("cuda:0")
    gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                    x=torch.from_numpy(prob.x).to(dev), y=torch.from_numpy(prob.y).to(dev))
    ctx = sk.Context(0)
    ladder = [1e-1, 1e-2, 2e-3]
    out = {"workload": f"gaussian_clouds {prob.n}x{prob.m} d={prob.d}, eps {ladder}, tol 1e-6, cap {cap}/stage"}
    for name, kw in (("sk", {}), ("sknr16", dict(ell=16)), ("sknr16_gain2", dict(ell=16, nr_min_gain=2.0))):
        f, rows = None, []
        for s_, eps in enumerate(ladder):
            lad = [eps] if s_ == 0 else [ladder[s_ - 1], eps]
            kws = dict(kw) if s_ > 0 else {}
            t0 = time.perf_counter()
            f, g, r = sk.solve(ctx, gp, lad, tol=1e-6, max_iter=cap, f0=f, warm_mode=sk.WARM_SEQUENTIAL, **kws)
            torch.cuda.synchronize()
            st = r["stages"][-1]
            rows.append({"eps": eps, "iters": st["iters"], "newton_tried": st["newton_tried"],
                         "newton_accepted": st["newton_accepted"], "rate_gain": st["rate_gain"],
                         "nr_skipped": st["nr_skipped"], "marginal_err": r["marginal_err"],
                         "marginal_err_exact": r["marginal_err_exact"], "status": r["status"],
                         "seconds": time.perf_counter() - t0})
            print(f"c4 {name} eps {eps}: {json.dumps(rows[-1])}", file=sys.stderr, flush=True)
        out[name] = rows
    ctx.close()
    return out


def percentile(xs, q):
    xs = sorted(xs)
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def stored_sweep_roofline(sk, ctx, side=128, reps=10):
    """HBM roofline of the stored-cost sweeps on the 16384 x 16384 grid
    histograms (C stored FP32, 1 GiB): average duration of the column sweep
    (streaming, float4 along the output axis) and of the row sweep, each
    reading C once; algorithmic bytes = 4 per cost element."""
    import torch
    import workloads as W
    prob = W.grid_histograms(side=side, seed=2)
    dev = torch.device("cuda:0")
    gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                    C=torch.from_numpy(prob.C).to(dev))
    del prob.C
    f = torch.zeros(gp.a.shape[0], dtype=torch.float64, device=dev)
    g = torch.zeros(gp.b.shape[0], dtype=torch.float64, device=dev)
    ctx.profile(True)
    for _ in range(reps):
        sk.c_transform_col(ctx, gp, 5e-4, f)
        sk.c_transform_row(ctx, gp, 5e-4, g)
    prof = ctx.profile_read()
    ctx.profile(False)
    out = {}
    n, m = gp.a.shape[0], gp.b.shape[0]
    for e in prof:
        if not e["name"].endswith(":main"):
            continue
        avg_s = e["total_ms"] / e["launches"] / 1e3
        gbs = 4.0 * n * m / avg_s / 1e9
        out[e["name"]] = {"avg_launch_us": avg_s * 1e6, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": gbs / PEAK_HBM_GBS, "bytes_per_launch": 4.0 * n * m,
                          "traffic": kernel_traffic(e["name"])}
    # the workload's solves: cold plain SK at eps' = 1e-3, then eps = 5e-4 with
    # warm SK or warm SK-NR(16) (sequential warm start), tol 1e-6
    solves = {}
    f_conv = None
    for name, ell in (("sk", 0), ("sknr16", 16)):
        ts, res = [], None
        for rep in range(3):
            t0 = time.perf_counter()
            f_out, _, res = sk.solve(ctx, gp, [1e-3, 5e-4], tol=1e-6, max_iter=100000, ell=ell,
                                     warm_mode=sk.WARM_SEQUENTIAL)
            torch.cuda.synchronize()
            if rep:
                ts.append(time.perf_counter() - t0)
        if ell == 0:
            f_conv = f_out
        st = res["stages"]
        solves[name] = {"solves_per_s": 1.0 / float(np.median(ts)), "ms": 1e3 * float(np.median(ts)),
                        "iters_per_stage": [x["iters"] for x in st], "stage_ms": [1e3 * x["seconds"] for x in st],
                        "newton_accepted": [x["newton_accepted"] for x in st], "status": res["status"],
                        "marginal_err": res["marginal_err"],
                        "stage2_iters_per_s": st[1]["iters"] / st[1]["seconds"]}
    solves["speedup_sknr_vs_sk"] = solves["sknr16"]["solves_per_s"] / solves["sk"]["solves_per_s"]
    # the single-read SK pass (one read of C per iteration: f = T_r(g) by rows
    # and the column sums of T_c(f) from the same read, then the column
    # merge), timed over 40 passes from the converged potentials at eps 5e-4;
    # algorithmic bytes = 4 per cost element
    ctx.profile(True)
    sk.solve(ctx, gp, [5e-4], tol=1e-12, max_iter=40, f0=f_conv)
    prof = ctx.profile_read()
    ctx.profile(False)
    for e in prof:
        if e["name"] not in ("sk_fused_stored:main", "sk_fused_stored"):
            continue
        avg_s = e["total_ms"] / e["launches"] / 1e3
        gbs = 4.0 * n * m / avg_s / 1e9
        out[e["name"]] = {"avg_launch_us": avg_s * 1e6, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": gbs / PEAK_HBM_GBS, "bytes_per_launch": 4.0 * n * m,
                          "traffic": kernel_traffic(e["name"])}
        if e["name"] == "sk_fused_stored":
            out[e["name"]]["iters_per_s"] = 1.0 / avg_s
    del gp
    torch.cuda.empty_cache()
    return {"workload": f"grid_histograms {side}x{side} (n=m={side*side}), stored FP32 cost, eps 5e-4",
            "kernels": out, "solves": solves}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_counts(gpu_counts):
    """Per-stage iteration counts of the oracle's own solve of this workload
    (stored by tests/golden/make_c2_oracle.py), else the GPU's."""
    try:
        g = np.load(os.path.join(ROOT, "tests", "golden", "c2_oracle.npz"))
        return [int(v) for v in g["iters_tol1e6"]], "the oracle's own full solve"
    except OSError:
        return list(gpu_counts), "the GPU run"


def cpu_baseline(prob, ladder, tol, ell, gpu_counts, full=False):
    """The FP64 oracle, untuned, on the host cores: the same workload and
    schedule (Algorithm 4.1, sequential spectral warm start, l = ell).

    Default (bounded, about a minute): the schedule's first stage (plain SK
    at eps_1 to tol, 15 iterations) timed on all cores and on one core,
    plus one warm-start eigensolve and one SK-NR(l) iteration at eps_2 on
    one core; a full solve is then estimated from the oracle's own
    per-stage iteration counts.  full=True times the whole 8-stage oracle
    solve on all cores and on one core (several minutes each) and reports
    that."""
    import oracle as O
    from threadpoolctl import threadpool_info, threadpool_limits
    C = O.sqeuclid_cost(prob.x, prob.y)
    a, b = prob.a, prob.b
    np.ones((64, 64)) @ np.ones((64, 64))  # load the BLAS pool
    all_threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    host = {"cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    if full:
        out = {}
        for th in (all_threads, 1):
            with threadpool_limits(limits=th):
                t0 = time.perf_counter()
                _, _, rs = O.solve_schedule(C, a, b, ladder, tol, 100000, ell=ell, mode="sequential")
                out[th] = (time.perf_counter() - t0, [r.iters for r in rs])
        t_all, it_all = out[all_threads]
        t_one, _ = out[1]
        return {"value": 1.0 / t_all, "unit": "solves/s", "cores": all_threads, "kind": "oracle",
                "value_1core": 1.0 / t_one, "seconds_per_solve": t_all, "seconds_per_solve_1core": t_one,
                "oracle_iters_per_stage": it_all, **host,
                "sample": (f"one full FP64 oracle solve of the {prob.n}x{prob.m} workload (8 stages, SK-NR(l={ell}) "
                           f"with the sequential warm start, tol {tol:g}), timed on {all_threads} BLAS threads "
                           f"and on 1")}
    counts, src = _oracle_counts(gpu_counts)
    t0 = time.perf_counter()
    r = O.sinkhorn(C, a, b, ladder[0], tol=tol, max_iter=100000)
    t_stage1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    V, _ = O.spectral_basis(r.f, r.g, C, a, b, ladder[0], ell)
    t_eig = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.sknr(C, a, b, ladder[1], tol=0.0, max_iter=1, V=V, f0=r.f)
    t_nr = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.sinkhorn(C, a, b, ladder[0], tol=0.0, max_iter=3)
        t_sk1 = (time.perf_counter() - t0) / 3
        t0 = time.perf_counter()
        O.spectral_basis(r.f, r.g, C, a, b, ladder[0], ell)
        t_eig1 = time.perf_counter() - t0
    per_sk = t_stage1 / max(1, r.iters)
    est = per_sk * counts[0] + t_nr * sum(counts[1:]) + t_eig * (len(ladder) - 1)
    est1 = t_sk1 * counts[0] + t_nr * (t_sk1 / per_sk) * sum(counts[1:]) + t_eig1 * (len(ladder) - 1)
    return {"value": 1.0 / est, "unit": "solves/s", "cores": all_threads, "kind": "oracle",
            "value_1core": 1.0 / est1, **host,
            "measured": {"stage1_seconds": t_stage1, "stage1_iters": r.iters, "eigensolve_s": t_eig,
                         "sknr_iteration_s": t_nr, "sk_iteration_s_1core": t_sk1, "eigensolve_s_1core": t_eig1},
            "sample": (f"FP64 oracle on the {prob.n}x{prob.m} workload, {all_threads} BLAS threads: stage 1 "
                       f"(plain SK, eps {ladder[0]:g}, {r.iters} iterations to tol {tol:g}), one ARPACK warm-start "
                       f"eigensolve and one SK-NR(l={ell}) iteration; one core: 3 SK iterations and the "
                       f"eigensolve; a solve estimated with the per-stage counts {counts} of {src}; "
                       f"bench.py --cpu-full times a whole solve")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sk-steps", type=int, default=3, help="timed plain-SK solves for the comparison")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--ell", type=int, default=30, help="low-frequency modes l (30: the paper's printed value)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=200000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="cpu_baseline: time one whole oracle solve on all cores and on one core (slow)")
    ap.add_argument("--c4", action="store_true",
                    help="run the 20000 x 30000 d = 64 eps ladder (SK, SK-NR(16), SK-NR(16) with the gain test)")
    ap.add_argument("--c4-cap", type=int, default=20000, help="iteration cap per stage of --c4")
    ap.add_argument("--no-sk", action="store_true")
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-cost HBM sweep measurement")
    ap.add_argument("--no-mfma", action="store_true", help="skip the d = 64 matrix-core sweep measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the mixed-request serving run")
    ap.add_argument("--no-paper", action="store_true", help="skip the Sec. 5 workloads (Fig. 5.1, single-cell shapes)")
    ap.add_argument("--no-gradient", action="store_true", help="skip the W_eps gradient timing")
    ap.add_argument("--serve-requests", type=int, default=2048)
    ap.add_argument("--serve-lanes", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(how the path would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_14780_amd as sk
    import workloads as W

    prob = W.gmm_vs_uniform(args.n, seed=1)
    ladder = list(W.EPS_LADDER_C2)
    dev = torch.device("cuda:0")
    gp = sk.Problem(a=torch.from_numpy(prob.a).to(dev), b=torch.from_numpy(prob.b).to(dev),
                    x=torch.from_numpy(prob.x).to(dev), y=torch.from_numpy(prob.y).to(dev))
    ctx = sk.Context(0)
    f_out = torch.empty(prob.n, dtype=torch.float64, device=dev)
    g_out = torch.empty(prob.m, dtype=torch.float64, device=dev)

    def one(ell):
        return sk.solve(ctx, gp, ladder, tol=args.tol, max_iter=args.max_iter, ell=ell,
                        warm_mode=sk.WARM_SEQUENTIAL, f_out=f_out, g_out=g_out)[2]

    def timed(ell, steps, warmup):
        for _ in range(warmup):
            one(ell)
        torch.cuda.synchronize()
        lat = []
        res = None
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            res = one(ell)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        return total, lat, res

    total, lat, res = timed(args.ell, args.steps, args.warmup)
    iters_nr = [s["iters"] for s in res["stages"]]
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"gmm_vs_uniform n=m={args.n} d=2, cost built on the fly, eps 1e-1->1e-3 halving "
                         f"({len(ladder)} stages), tol {args.tol:g} L1 (last stage FP64-verified), SK-NR(l={args.ell}) "
                         f"sequential spectral warm start"),
            "n": prob.n, "m": prob.m, "d": 2, "eps_ladder": ladder, "tol": args.tol, "ell": args.ell,
        },
        "p50_ms": 1e3 * percentile(lat, 50),
        "p99_ms": 1e3 * percentile(lat, 99),
        "iters_per_stage": iters_nr,
        "eig_iters_per_stage": [s["eig_iters"] for s in res["stages"]],
        "newton_accepted_per_stage": [s["newton_accepted"] for s in res["stages"]],
        "marginal_err": res["marginal_err"],
        "status": res["status"],
    }
    if not args.no_sk:
        tsk, latsk, rsk = timed(0, args.sk_steps, 1)
        out["sk"] = {
            "value": args.sk_steps / tsk, "unit": "solves/s",
            "p50_ms": 1e3 * percentile(latsk, 50), "p99_ms": 1e3 * percentile(latsk, 99),
            "iters_per_stage": [s["iters"] for s in rsk["stages"]],
            "marginal_err": rsk["marginal_err"], "status": rsk["status"],
        }
        out["speedup_vs_sk"] = out["value"] / out["sk"]["value"]

    # roofline of the dominant kernel: one more solve with per-kernel HIP
    # events on the solve's stream
    ctx.profile(True)
    one(args.ell)
    prof = ctx.profile_read()
    ctx.profile(False)
    mains = [e for e in prof if e["name"].endswith(":main")]
    dom = max(mains, key=lambda e: e["total_ms"])
    whole = next(e for e in prof if e["name"] == dom["name"].split(":")[0])
    bound, per_unit, unit = algorithmic_work(dom["name"])
    avg_s = dom["total_ms"] / dom["launches"] / 1e3
    per_launch = per_unit * dom["units"] / dom["launches"]
    if bound == "hbm":
        achieved, peak = per_launch / avg_s / 1e9, PEAK_HBM_GBS
    else:
        achieved, peak = per_launch / avg_s / 1e12, PEAK_VALU_TOPS
    out["roofline"] = {
        "bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
        "traffic": kernel_traffic(dom["name"]), "kernel": dom["name"], "avg_launch_us": avg_s * 1e6,
        "launches_per_solve": dom["launches"], "elements_per_launch": dom["units"] / dom["launches"],
        "work_per_element": per_unit,
        "with_merge_and_finish": {"avg_us": 1e3 * whole["total_ms"] / whole["launches"],
                                  "frac": per_launch / (whole["total_ms"] / whole["launches"] / 1e3)
                                  / (1e12 if bound != "hbm" else 1e9) / peak},
        "share_of_sweep_time": dom["total_ms"] / sum(e["total_ms"] for e in prof if e["name"].endswith(":main")),
    }
    out["kernel_profile"] = [{"name": e["name"], "launches": e["launches"],
                              "avg_us": 1e3 * e["total_ms"] / max(1, e["launches"]),
                              "total_ms": e["total_ms"]} for e in sorted(prof, key=lambda e: -e["total_ms"])]
    # gradients of W_eps at the solution (x, y, a, b): the envelope gradients
    # cost two weighted sweeps
    if not args.no_gradient:
        sk.gradient(ctx, gp, ladder[-1], f_out, g_out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            sk.gradient(ctx, gp, ladder[-1], f_out, g_out)
        torch.cuda.synchronize()
        out["gradient"] = {"ms": 1e3 * (time.perf_counter() - t0) / 10,
                           "what": "sknr_gradient of W_eps with respect to x, y, a, b at the solution"}
    if not args.no_stored:
        print("bench: stored-cost leg", file=sys.stderr, flush=True)
        out["roofline_stored_cost"] = stored_sweep_roofline(sk, ctx)
    if not args.no_mfma:
        print("bench: matrix-core cost leg", file=sys.stderr, flush=True)
        out["roofline_mfma_cost"] = mfma_sweep_roofline(sk, W, torch)
    if not args.no_stored:
        out["roofline_points_large"] = points_sweep_large(sk, W, torch)
    if not args.no_serve:
        print("bench: serving leg", file=sys.stderr, flush=True)
        out["serving"] = serving_bench(sk, W, torch, args.serve_requests, args.serve_lanes, args.tol)
    if not args.no_paper:
        print("bench: Sec. 5 workloads leg", file=sys.stderr, flush=True)
        out["paper_workloads"] = paper_workloads_bench(sk, W, torch, args.tol)
    if not args.no_paper:
        out["c1"] = c1_bench(sk, W, torch)
        out["newton_solvers"] = newton_solvers_bench(sk, gp, ladder, args.tol)
    if args.c4:
        out["c4"] = c4_ladder(sk, W, torch, args.c4_cap)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, ladder, args.tol, args.ell, iters_nr, full=args.cpu_full)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
