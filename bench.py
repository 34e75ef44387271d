"""Benchmark: linear-memory DTW alignment (arXiv 2008.02734) on one MI355X.

Default workload (the headline): a single 20000 x 16000 pair, d = 12, FP64,
chroma-like frames, cutoff m = 500, exact FP64 path.  One step = one complete
dtw_align call: every wavefront sweep, split-cost + argmin, recursion level,
leaf solve and path assembly, with the inputs already resident in HBM.

Prints one JSON line.  `value` is textbook-equivalent throughput M*N / step
time (GCUPS).  The roofline entry is for the dominant kernel, the wavefront
sweep: cells evaluated by the sweeps / summed sweep-kernel time (HIP events on
the launch stream around the sweep launches of the timed steps), against the
VALU peak divided by the algorithmic VALU slots one cell needs.  kernel_ms is
the per-class breakdown from untimed runs with events around every launch.  The CPU baseline is the oracle's textbook full-table
DTW timed single-threaded on this host.

The default run also measures, in the same process, the two other targets
of the method's AI-systems forms, and the tie-exact mode (unless --no-extras):
  long_pair  the 200000 x 160000, d = 128 pair in the BF16 and FP16 Gram
             forms, each against the all-FP64 path on the same input (time,
             relative cost error, frame deviation of the path);
  serving    a Poisson stream of 96 requests, M log-uniform in [2000, 400000],
             through the serving loop in the BF16 and FP16 mixes, against every
             request one at a time through the plain FP64 path (throughput
             ratio, p50/p99 latency, largest relative cost error);
  tie_exact  the headline pair with tie-exact splits beside the default ones.

  edit_distance  the config-6 edit-distance workload (below).

Other workloads (--config): 1 = 500 x 400 FP64 latency; 3 = 200000 x 160000,
d = 128, BF16 Gram cost on the matrix cores; 4 = 512 pairs in one batched
call, d = 24, FP32; 5 = the serving stream alone (also an all-FP32 mix);
6 = edit distance of two 200000 x 160000 byte strings (dtw_edit_align), with
its own roofline (the integer sweep) and CPU baseline (the oracle's
recursion on a leading block).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector peaks: FP64 78.6 TFLOP/s = 256 CUs x 4 SIMD x 16 FMA lanes x
# 2.4 GHz x 2 flop; FP32 157.3 TFLOP/s = 32 lanes per SIMD per cycle (the FP32
# batch sweep retires 4.7e13 VALU lane-instructions/s, above the 16-lane rate,
# so unpacked FP32 runs at that rate too).  Lane-slots/s per arithmetic type:
VALU_SLOTS_PER_S = {"f64": 256 * 4 * 16 * 2.4e9, "f32": 256 * 4 * 32 * 2.4e9}
# Algorithmic VALU slots per DP cell (from the gfx950 ISA of the sweep kernel):
#  FP64, d = 12: 12 subtract + 12 fma, 21 for the correctly rounded square root
#    (18 instructions, v_rsq_f64 counted 4 as a quarter-rate transcendental),
#    2 min + 1 add for the recurrence;
#  FP32, d: d subtract + d fma + 4 (v_sqrt_f32, quarter rate) + 3;
#  BF16 Gram form: the dot product is on the matrix cores; VALU epilogue add,
#    fma, max, v_sqrt_f32 (4) and the recurrence's 3 = 10.
SLOTS_FP64_D12 = 48


def slots_per_cell(precision, d):
    if precision == "fp64":
        return SLOTS_FP64_D12 if d == 12 else 2 * d + 24
    if precision == "fp32":
        return 2 * d + 7
    return 10


WORKLOADS = {
    2: dict(name="single pair 20000x16000, d=12 f64 chroma-like, exact FP64 linmdtw (m=500)", M=20000, N=16000,
            d=12, family="chroma", m=500, precision="fp64"),
    1: dict(name="single pair 500x400, d=12 f64 Gaussian walk, exact FP64 (one leaf at m=500)", M=500, N=400,
            d=12, family="gaussian_walk", m=500, precision="fp64"),
    3: dict(name="single pair 200000x160000, d=128 embedding-like, BF16 Gram cost on MFMA, FP32 DP, FP64 split "
                 "(m=500)", M=200000, N=160000, d=128, family="embedding", m=500, precision="bf16"),
}

TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "pass_kernel_f64_d12_20000x16000_hbm_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2008_02734_amd", "csrc", "dtw_wave.hip")


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter record
    (FETCH_SIZE and WRITE_SIZE scaled by a calibrating copy), or None when the
    sweep kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_RECORD).read()
        rec = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and " " not in line.split(": ")[0])
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if not sha.startswith(rec["kernel_source_sha256_prefix"].strip()):
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def base_record(args, value, ms_per_step, dtype, config):
    return {
        "metric": "DP cells/sec (GCUPS) + fraction of VALU roofline; p50/p99 align latency",
        "value": value, "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic", "config": config,
    }


def roofline(stats, precision, d, kernel, traffic=None):
    sweep_ms = float(np.mean([s["ms_sweep"] for s in stats]))
    st = stats[-1]
    achieved = st["sweep_cells"] / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    peak = VALU_SLOTS_PER_S["f64" if precision == "fp64" else "f32"] / slots_per_cell(precision, d) / 1e9
    return {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak, "unit": "Gcells/s",
            "frac": (achieved / peak) if achieved else None, "traffic": traffic,
            "launches_per_step": st["levels"], "sweep_cells_per_step": st["sweep_cells"],
            "avg_sweep_launch_ms": sweep_ms / max(1, st["levels"])}


def timed_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        stats.append(fn())  # each call synchronises its stream
        lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, lat, stats


def bench_single(args, cfg):
    import torch

    from paper_2008_02734_amd import dtw, synth

    W = dict(WORKLOADS[cfg])
    if args.precision:
        W["precision"] = args.precision
        W["name"] = W["name"].replace("BF16 Gram", args.precision.upper() + " Gram")
    M, N, d, prec = W["M"], W["N"], W["d"], W["precision"]
    X, Y = synth.make_pair(cfg, 0, M, N, d, W["family"])
    tdt = torch.float64 if prec == "fp64" else torch.float32
    Xd = torch.from_numpy(X).to("cuda:0", dtype=tdt)
    Yd = torch.from_numpy(Y).to("cuda:0", dtype=tdt)
    al = dtw.Aligner(M, N, d, tdt, prec, W["m"], device="cuda:0")
    al.opts.profile = 2  # HIP events around the sweep launches only, inside the timed region
    stream = torch.cuda.current_stream()
    ms, lat, stats = timed_steps(lambda: al.run(Xd, Yd, stats=True, stream=stream), args.steps, args.warmup)
    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), st
    al.opts.profile = 1  # every kernel class, outside the timed region
    breakdown = [al.run(Xd, Yd, stats=True, stream=stream) for _ in range(2)]
    kname = {"fp64": f"pass_kernel<double,{d}>", "fp32": f"pass_kernel<float,{d}>",
             "bf16": "pass_kernel<float,128,Gram>", "fp16": "pass_kernel<float,128,GramF16>"}[prec] + " (wavefront sweep)"
    out = base_record(args, M * N / (ms * 1e-3) / 1e9, ms, {"fp64": "f64", "fp32": "f32", "bf16": "bf16/f32", "fp16": "f16/f32"}[prec],
                      {"workload": W["name"], "M": M, "N": N, "d": d, "min_block": W["m"], "precision": prec,
                       "seed": [cfg, 0]})
    out.update({
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "cells_processed": st["cells_processed"], "cells_ratio_to_MN": st["cells_processed"] / (M * N),
        "processed_gcups": st["cells_processed"] / (ms * 1e-3) / 1e9,
        "kernel_ms": {k: float(np.mean([s[k] for s in breakdown])) for k in
                      ("ms_sweep", "ms_split", "ms_plan", "ms_leaf", "ms_other")},
        "levels": st["levels"], "leaves": st["leaves"],
        "roofline": roofline(stats, prec, d, kname, measured_traffic() if cfg == 2 else None),
    })
    if cfg == 3 and not args.no_fp64_comparison:
        out["fp64_same_input"] = fp64_comparison_single(Xd, Yd, W, al)
        del out["fp64_same_input"]["_aligner"]
        out["fp64_same_input"]["speedup_of_reduced_precision"] = out["fp64_same_input"]["ms"] / ms
    if not args.no_cpu_baseline:
        import oracle
        # the oracle's full table on the pair (cfg 1, 2) or on its leading
        # sub-block (cfg 3, whose full table does not fit a host)
        Ms, Ns = (M, N) if cfg != 3 else (8000, 6400)
        Xs, Ys = X[:Ms], Y[:Ns]
        t = time.perf_counter()
        c_ref, p_ref = oracle.full(Xs, Ys)
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = cpu_record(
            Ms * Ns, cpu_s,
            (f"the full {M}x{N} pair" if cfg != 3 else
             f"the leading {Ms}x{Ns} block of the pair (its rate taken as the whole pair's)")
            + f": textbook FP64 full table + backtrace, single thread, {cpu_s:.1f} s", cfg != 3)
        if cfg != 3:
            path = al.path[: int(al.plen.item())].cpu().numpy()
            out["parity"] = {"path_equal_to_oracle": bool(path.tolist() == p_ref.tolist()),
                             "cost_rel_err": abs(float(al.cost.item()) - c_ref) / c_ref}
        else:
            cs, ps, _ = dtw.align(Xd[:Ms].contiguous(), Yd[:Ns].contiguous(), precision=prec, min_block=W["m"])
            out["parity"] = {"block": [Ms, Ns], "cost_rel_err_vs_fp64_oracle": (cs - c_ref) / c_ref}
    return out


def fp64_comparison_single(Xd, Yd, W, al, prev=None):
    """The same input through the exact all-FP64 path (identical to the
    oracle's path by the parity tests): its time, and the reduced-precision
    result's cost error and frame deviation against it.  `prev` (the
    "_aligner" entry of an earlier result on the same input) is reused
    instead of running the FP64 path again."""
    import torch

    from paper_2008_02734_amd import dtw, metrics
    M, N, d = Xd.shape[0], Yd.shape[0], Xd.shape[1]
    if prev is None:
        X64, Y64 = Xd.to(torch.float64), Yd.to(torch.float64)
        al64 = dtw.Aligner(M, N, d, torch.float64, "fp64", W["m"], device="cuda:0")
        al64.run(X64, Y64)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = al64.run(X64, Y64, stats=True)
        s64 = time.perf_counter() - t
        prev = {"ms": s64 * 1e3, "cost": float(al64.cost.item()), "device_error": st["device_error"],
                "path": al64.path[: int(al64.plen.item())].cpu().numpy()}
    c64, p64 = prev["cost"], prev["path"]
    plo = al.path[: int(al.plen.item())].cpu().numpy()
    dv = metrics.summary(plo, p64)
    return {"ms": prev["ms"], "gcups": M * N / (prev["ms"] * 1e-3) / 1e9, "cost": c64,
            "device_error": prev["device_error"], "rel_cost_err": (float(al.cost.item()) - c64) / c64,
            "path_dev_mean_frames": dv["mean_frames"], "path_dev_max_frames": int(dv["max_frames"]),
            "frac_within_1_frame": dv["frac_le_1"], "_aligner": prev}


def bench_batched(args):
    """cfg 4: 512 independent pairs, M and N log-uniform in [1000, 30000] with
    N/M in [0.7, 1.4], d = 24 chroma-like FP32 frames, one batched call."""
    import torch

    from paper_2008_02734_amd import dtw, synth

    shapes = synth.batch_shapes(args.batch)
    d = args.batch_d
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(4, p, M, N, d, "chroma")
        Xs.append(X.astype(np.float32))
        Ys.append(Y.astype(np.float32))
    prec = args.precision or "fp32"
    tdt = torch.float64 if prec == "fp64" else torch.float32
    Xp = torch.from_numpy(np.concatenate(Xs)).to("cuda:0", tdt)
    Yp = torch.from_numpy(np.concatenate(Ys)).to("cuda:0", tdt)
    xo = np.concatenate([[0], np.cumsum([s[0] for s in shapes])]).astype(np.int64)
    yo = np.concatenate([[0], np.cumsum([s[1] for s in shapes])]).astype(np.int64)
    Xl = [Xp[xo[i]:xo[i + 1]] for i in range(len(shapes))]
    Yl = [Yp[yo[i]:yo[i + 1]] for i in range(len(shapes))]
    runner = dtw.BatchAligner(Xl, Yl, precision=prec, min_block=500, profile=2)
    ms, lat, stats = timed_steps(runner.run, args.steps, args.warmup)
    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), st
    runner.opts.profile = 1
    breakdown = [runner.run()]
    cells = sum(M * N for M, N in shapes)
    form = "FP32 DP, FP64 split" if prec == "fp32" else prec.upper() + " DP and split"
    out = base_record(args, cells / (ms * 1e-3) / 1e9, ms, {"fp32": "f32", "fp64": "f64"}[prec],
                      {"workload": f"batch of {len(shapes)} pairs, M,N log-uniform in [1000, 30000], N/M in "
                                   f"[0.7, 1.4], d={d} f32 chroma-like, {form} (m=500)",
                       "pairs": len(shapes), "d": d, "min_block": 500, "precision": prec, "seed": [4, "p"]})
    out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "cells_processed": st["cells_processed"],
                "processed_gcups": st["cells_processed"] / (ms * 1e-3) / 1e9,
                "kernel_ms": {k: float(np.mean([s[k] for s in breakdown])) for k in
                              ("ms_sweep", "ms_split", "ms_plan", "ms_leaf", "ms_other")},
                "levels": st["levels"], "leaves": st["leaves"],
                "roofline": roofline(stats, prec, d, f"pass_kernel<{'double' if prec == 'fp64' else 'float'},{d}> (wavefront sweep)")})
    if not args.no_fp64_comparison and prec != "fp64":
        from paper_2008_02734_amd import metrics
        r64 = dtw.BatchAligner([x.to(torch.float64) for x in Xl], [y.to(torch.float64) for y in Yl],
                               precision="fp64", min_block=500)
        r64.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st64 = r64.run()
        s64 = time.perf_counter() - t
        c32, c64 = runner.costs.cpu().numpy(), r64.costs.cpu().numpy()
        rel = (c32 - c64) / c64
        devs = [metrics.summary(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(runner.path_list(), r64.path_list())]
        out["fp64_same_input"] = {
            "ms": s64 * 1e3, "gcups": cells / s64 / 1e9, "device_error": st64["device_error"],
            "speedup_of_reduced_precision": s64 * 1e3 / ms, "max_rel_cost_err": float(np.max(np.abs(rel))),
            "mean_rel_cost_err": float(np.mean(np.abs(rel))),
            "path_dev_mean_frames": float(np.mean([v["mean_frames"] for v in devs])),
            "path_dev_max_frames": int(max(v["max_frames"] for v in devs)),
            "pairs_with_identical_path": int(sum(v["max_frames"] == 0 for v in devs))}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        done = 0
        for p in range(len(shapes)):  # pairs in order until ~15 s of single-thread CPU work
            oracle.full(Xs[p].astype(np.float64), Ys[p].astype(np.float64))
            done += shapes[p][0] * shapes[p][1]
            if time.perf_counter() - t > 15:
                break
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = cpu_record(
            done, cpu_s, f"the batch's first {p + 1} of {len(shapes)} pairs ({done / 1e6:.0f} M cells; their rate "
                         f"taken as the batch's): textbook FP64 full table + backtrace, single thread, {cpu_s:.1f} s",
            p + 1 == len(shapes))
    return out


def run_stream(dtw, reqs, precs, rng, frac=0.7):
    """One pass of the request list through a fresh server: a pilot with every
    request submitted at once (the saturated rate), then a Poisson stream at
    `frac` of that rate.  Returns throughput, latencies and the results."""
    cells = sum(q[0].shape[0] * q[1].shape[0] for q in reqs)
    srv = dtw.Server(pool_bytes=16 << 30, max_slots=8, max_batch=16)
    try:
        t0 = time.perf_counter()
        tk = [srv.submit(q[0], q[1], precision=p) for q, p in zip(reqs, precs)]
        for t in tk:
            srv.wait(t)
        pilot_s = time.perf_counter() - t0
        lam = frac * len(reqs) / pilot_s
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
        t0 = time.perf_counter()
        tickets = []
        for (X, Y, *_), p, at in zip(reqs, precs, arrivals):
            while time.perf_counter() - t0 < at:
                time.sleep(50e-6)
            tickets.append(srv.submit(X, Y, precision=p))
        res = [srv.wait(t) for t in tickets]
        makespan = time.perf_counter() - t0
    finally:
        srv.close()
    assert all(r["status"] == 0 and r["device_error"] == 0 for r in res), [r for r in res if r["status"]][:1]
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) / 1e6 for r in res])
    return {"gcups": cells / makespan / 1e9, "saturated_gcups": cells / pilot_s / 1e9, "lambda_per_s": lam,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "makespan_ms": makespan * 1e3, "max_batch_seen": int(max(r["batch_size"] for r in res)),
            "costs": [r["cost"] for r in res]}


def serving_requests(n_requests, m_hi):
    """The request list of the serving workload: M log-uniform in [2000, m_hi],
    N = M x U[0.75, 1.3] (within the warp generator's slope range), half d = 12
    chroma-like, half d = 128 embedding-like, seeds [5, r]; FP32 device copies
    plus the FP64 host arrays."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    from paper_2008_02734_amd import synth

    rng = np.random.default_rng([5, 999])
    specs = []
    for r in range(n_requests):
        M = int(np.exp(rng.uniform(np.log(2000), np.log(m_hi))))
        N = int(M * rng.uniform(0.75, 1.3))
        d, fam = (12, "chroma") if r % 2 == 0 else (128, "embedding")
        specs.append((r, M, N, d, fam))
    with ThreadPoolExecutor(8) as ex:
        pairs = list(ex.map(lambda q: synth.make_pair(5, q[0], q[1], q[2], q[3], q[4]), specs))
    reqs = []
    for (r, M, N, d, fam), (X, Y) in zip(specs, pairs):
        reqs.append((torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(Y.astype(np.float32)).cuda(),
                     d, X, Y))
    torch.cuda.synchronize()
    return reqs, rng


def fp64_one_at_a_time(dtw, reqs):
    """Every request alone through the plain FP64 path: each request's
    buffers are allocated before its timed call (an Aligner of its shape),
    so the time is the alignment alone.  Returns (seconds, FP64 costs)."""
    import torch
    c64, bt = [], 0.0
    for X, Y, d, Xh, Yh in reqs:
        Xd, Yd = torch.from_numpy(Xh).cuda(), torch.from_numpy(Yh).cuda()
        al = dtw.Aligner(Xh.shape[0], Yh.shape[0], d, torch.float64, "fp64", 500, device="cuda")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        st = al.run(Xd, Yd, stats=True)
        bt += time.perf_counter() - s0
        assert st["device_error"] == 0
        c64.append(float(al.cost.item()))
        del al, Xd, Yd
    return bt, np.array(c64)


def serving_summary(args, n_requests, m_hi, mixes):
    """The serving workload: a Poisson stream of requests through the serving
    loop (each mix: a pilot with every request at once gives the saturated
    rate, then arrivals at 0.7 of it), against every request one at a time
    through the plain FP64 path, which also gives the FP64 costs that the
    reduced-precision results are measured against."""
    from paper_2008_02734_amd import dtw

    reqs, rng = serving_requests(n_requests, m_hi)
    cells = sum(q[0].shape[0] * q[1].shape[0] for q in reqs)
    streams = {name: run_stream(dtw, reqs, [("fp32" if q[2] == 12 else big) for q in reqs], rng)
               for name, big in mixes}
    bt, c64 = fp64_one_at_a_time(dtw, reqs)
    base = cells / bt / 1e9
    is12 = np.array([q[2] == 12 for q in reqs])
    for st in streams.values():
        rel = np.abs((np.array(st.pop("costs")) - c64) / c64)
        st["max_rel_cost_err"] = float(np.max(rel))
        st["max_rel_cost_err_d12"] = float(np.max(rel[is12]))
        st["max_rel_cost_err_d128"] = float(np.max(rel[~is12]))
        st["meets_1e-5"] = bool(np.max(rel) <= 1e-5)
        st["vs_fp64_one_at_a_time"] = st["gcups"] / base
        st["saturated_vs_fp64_one_at_a_time"] = st["saturated_gcups"] / base
    return {"workload": f"Poisson stream of {len(reqs)} requests, M log-uniform in [2000, {m_hi}], N = M x "
                        "U[0.75, 1.3], half d=12 (FP32), half d=128 (Gram cost), at 0.7x the saturated rate",
            "requests": len(reqs), "textbook_cells": cells, "seed": [5, "r"],
            "fp64_one_at_a_time_gcups": base, "fp64_one_at_a_time_s": bt, "streams": streams}, reqs


def bench_serving(args):
    """cfg 5: a Poisson stream of requests through the serving loop: the
    configuration's mix (d = 12 in FP32, d = 128 in the BF16 Gram form), the
    same mix with the FP16 Gram form, and every request in FP32."""
    summ, reqs = serving_summary(args, args.requests, args.serving_m_hi,
                                 [("bf16_mix", "bf16"), ("fp16_mix", "fp16"), ("fp32_all", "fp32")])
    mixed = summ["streams"]["bf16_mix"]
    out = base_record(args, mixed["gcups"], mixed["makespan_ms"], "f32+bf16",
                      {"workload": summ["workload"], "requests": summ["requests"], "seed": [5, "r"]})
    out.update({"p50_ms": mixed["p50_ms"], "p99_ms": mixed["p99_ms"], "serving": summ})
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_sample_serving(reqs)
    return out


def long_pair_summary(args):
    """The long pair (200000 x 160000, d = 128, embedding-like) in the BF16
    and FP16 Gram forms, each against the all-FP64 path on the same input."""
    import torch

    from paper_2008_02734_amd import dtw, synth

    W = WORKLOADS[3]
    M, N, d = W["M"], W["N"], W["d"]
    X, Y = synth.make_pair(3, 0, M, N, d, W["family"])
    Xd = torch.from_numpy(X).to("cuda:0", torch.float32)
    Yd = torch.from_numpy(Y).to("cuda:0", torch.float32)
    out = {"workload": "single pair 200000x160000, d=128 embedding-like (m=500)", "M": M, "N": N, "d": d}
    fp64 = None
    for prec in ("bf16", "fp16"):
        al = dtw.Aligner(M, N, d, torch.float32, prec, W["m"], device="cuda:0")
        al.opts.profile = 2
        ms, lat, stats = timed_steps(lambda: al.run(Xd, Yd, stats=True), 2, 1)
        r = {"ms": ms, "gcups": M * N / (ms * 1e-3) / 1e9, "sweep_ms": float(np.mean([s["ms_sweep"] for s in stats])),
             "roofline": roofline(stats, prec, d, f"pass_kernel<float,128,{'Gram' if prec == 'bf16' else 'GramF16'}>")}
        cmp = fp64_comparison_single(Xd, Yd, W, al, fp64)
        fp64 = cmp.pop("_aligner")
        r.update({k: cmp[k] for k in ("rel_cost_err", "path_dev_mean_frames", "path_dev_max_frames",
                                      "frac_within_1_frame")})
        r["speedup_vs_fp64"] = cmp["ms"] / ms
        out[prec] = r
        out["fp64"] = {k: cmp[k] for k in ("ms", "gcups", "cost")}
        del al
    return out


def tie_exact_summary(args):
    """The headline pair in tie-exact mode (FP64; the split read from labels of
    a forward sweep over each whole block): its time beside the default
    split's, and whether the two paths agree (the chroma-like frames are
    continuous, so no exact tie separates them)."""
    import torch

    from paper_2008_02734_amd import dtw, synth

    W = WORKLOADS[2]
    M, N, d = W["M"], W["N"], W["d"]
    X, Y = synth.make_pair(2, 0, M, N, d, W["family"])
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = {"workload": W["name"] + ", tie-exact splits"}
    paths = {}
    for tie in (False, True):
        al = dtw.Aligner(M, N, d, torch.float64, "fp64", W["m"], device="cuda:0", tie_exact=tie)
        al.opts.profile = 2
        ms, lat, stats = timed_steps(lambda: al.run(Xd, Yd, stats=True), 5, 1)
        key = "tie_exact" if tie else "default"
        out[key] = {"ms": ms, "gcups": M * N / (ms * 1e-3) / 1e9, "sweep_ms": float(np.mean([q["ms_sweep"] for q in stats])),
                    "sweep_cells": int(stats[-1]["sweep_cells"]), "levels": int(stats[-1]["levels"])}
        paths[key] = al.path[: int(al.plen.item())].cpu().numpy()
    out["same_path"] = bool(paths["default"].tolist() == paths["tie_exact"].tolist())
    out["slowdown"] = out["tie_exact"]["ms"] / out["default"]["ms"]
    return out


# Edit distance (config 6): two byte strings over 4 letters, b from a
# through a 10% mutation channel (substitutions, deletions, insertions),
# unit costs, leaves of 64 rows.  The sweep is pure 32-bit integer VALU work
# (no packed form of 32-bit integer add or min: 16 lanes per SIMD per cycle)
# at 6 slots per cell: letter compare, cost select, two adds, two mins.
EDIT = dict(name="edit distance, 200000x160000 byte strings over 4 letters (b = a through 10% substitutions/"
                 "deletions/insertions), unit costs, linear-memory row-split recursion with 64-row leaves",
            M=200000, N=160000, k=4, p=0.1, sub=1, gap=1, leaf_rows=64, seed=6)
EDIT_SLOTS_PER_CELL = 6
INT32_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


def edit_roofline(stats, traffic=None):
    sweep_ms = float(np.mean([s["sweep_ms"] for s in stats]))
    st = stats[-1]
    achieved = st["sweep_cells"] / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    peak = INT32_SLOTS_PER_S / EDIT_SLOTS_PER_CELL / 1e9
    return {"bound": "alu", "kernel": "ed_sweep_kernel (edit-distance wavefront sweep)", "achieved": achieved,
            "peak": peak, "unit": "Gcells/s", "frac": (achieved / peak) if achieved else None, "traffic": traffic,
            "launches_per_step": st["levels"], "sweep_cells_per_step": st["sweep_cells"],
            "avg_sweep_launch_ms": sweep_ms / max(1, st["levels"])}


def edit_run(steps, warmup):
    """Time dtw_edit_align on the config-6 strings; returns the record body and
    the host strings (for the parity check and the CPU sample)."""
    import torch

    from paper_2008_02734_amd import dtw, synth
    E = EDIT
    M, N = E["M"], E["N"]
    a, b = synth.string_pair(E["seed"], M, N, k=E["k"], p=E["p"])
    da, db = torch.from_numpy(a).to("cuda:0"), torch.from_numpy(b).to("cuda:0")
    al = dtw.EditAligner(M, N, E["leaf_rows"], device="cuda:0")
    stream = torch.cuda.current_stream()
    ms, lat, stats = timed_steps(lambda: al.run(da, db, E["sub"], E["gap"], stream=stream, stats=True), steps, warmup)
    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), st
    n = int(al.plen.item())
    body = {"ms": ms, "gcups": M * N / (ms * 1e-3) / 1e9, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "distance": int(al.dist.item()), "path_nodes": n,
            "sweep_ms": float(np.mean([s["sweep_ms"] for s in stats])),
            "cells_processed": st["sweep_cells"] + st["leaf_cells"],
            "processed_gcups": (st["sweep_cells"] + st["leaf_cells"]) / (ms * 1e-3) / 1e9,
            "levels": st["levels"], "roofline": edit_roofline(stats, measured_edit_traffic())}
    return body, a, b, al.path[:n].cpu().numpy()


def edit_checks(a, b, dist, path, with_cpu=True):
    """Parity of the returned path and the CPU baseline: the path's cost (the
    oracle's, move by move) equals the distance; the oracle's recursion on the
    leading 40000 x 32000 block gives that block's distance and is the CPU
    sample (single thread; its rate taken as the workload's)."""
    from oracle import edit
    E = EDIT
    out = {"path_cost_equals_distance": edit.path_cost(a, b, path, E["sub"], E["gap"]) == dist}
    if with_cpu:
        Ms, Ns = 40000, 32000
        t = time.perf_counter()
        r = edit.linear(a[:Ms], b[:Ns], E["sub"], E["gap"], E["leaf_rows"])
        cpu_s = time.perf_counter() - t
        flags = [f for f in edit.GCC_CMD if f.startswith(("-O", "-std"))]
        out["cpu_baseline"] = {"value": Ms * Ns / cpu_s / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's linear-memory recursion (edo_linear) on the leading "
                                         f"{Ms}x{Ns} block, single thread, {cpu_s:.1f} s; its rate taken as "
                                         f"the workload's", "sample_s": cpu_s, "extrapolated": True,
                               "oracle_build": "gcc " + " ".join(flags) + " (oracle/edit_oracle.c, untuned)"}
        out["_block"] = (Ms, Ns, r)
    return out


def edit_summary(args):
    """Default-run sub-object: the config-6 edit-distance workload."""
    body, a, b, path = edit_run(5, 1)
    chk = edit_checks(a, b, body["distance"], path, with_cpu=False)
    body["workload"] = EDIT["name"]
    body["path_cost_equals_distance"] = chk["path_cost_equals_distance"]
    return body


def bench_edit(args):
    import torch

    from paper_2008_02734_amd import dtw
    E = EDIT
    body, a, b, path = edit_run(args.steps, args.warmup)
    out = base_record(args, body["gcups"], body["ms"], "int32",
                      {"workload": E["name"], "M": E["M"], "N": E["N"], "alphabet": E["k"], "mutation": E["p"],
                       "sub": E["sub"], "gap": E["gap"], "leaf_rows": E["leaf_rows"], "seed": [7, E["seed"]]})
    out["metric"] = "edit-distance DP cells/sec (GCUPS, M*N per alignment) + fraction of VALU roofline"
    out.update({k: v for k, v in body.items() if k not in ("ms", "gcups")})
    chk = edit_checks(a, b, body["distance"], path, with_cpu=not args.no_cpu_baseline)
    out["parity"] = {"path_cost_equals_distance": chk["path_cost_equals_distance"]}
    if "_block" in chk:
        # the GPU on the same leading block: distance and path equal the oracle's
        Ms, Ns, r = chk["_block"]
        da = torch.from_numpy(a[:Ms].copy()).cuda()
        db = torch.from_numpy(b[:Ns].copy()).cuda()
        d, p = dtw.edit_align(da, db, E["sub"], E["gap"], E["leaf_rows"])
        out["parity"]["leading_block"] = f"{Ms}x{Ns}"
        out["parity"]["block_distance_equal"] = d == r["dist"]
        out["parity"]["block_path_equal"] = p.cpu().numpy().tolist() == r["path"].tolist()
        out["cpu_baseline"] = chk["cpu_baseline"]
    return out


EDIT_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "ed_sweep_kernel_200000x160000_hbm_traffic.txt")
EDIT_SOURCE = os.path.join(ROOT, "paper_2008_02734_amd", "csrc", "dtw_edit.hip")


def measured_edit_traffic():
    """HBM bytes per edit sweep launch from the committed counter record, or
    None when there is none or dtw_edit.hip has changed since it was taken."""
    import hashlib
    try:
        txt = open(EDIT_TRAFFIC_RECORD).read()
        rec = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and " " not in line.split(": ")[0])
        sha = hashlib.sha256(open(EDIT_SOURCE, "rb").read()).hexdigest()
        if not sha.startswith(rec["kernel_source_sha256_prefix"].strip()):
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_record(cells, cpu_s, sample, whole):
    """The cpu_baseline object: the oracle's rate on `sample`.  `whole` says
    whether the sample is the entire workload; if not, the rate is the
    sample's, taken as the workload's (an extrapolation, marked so)."""
    import oracle
    flags = [a for a in oracle.GCC_CMD if a.startswith(("-O", "-std", "-f")) and a != "-fPIC"]
    return {"value": cells / cpu_s / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle", "sample": sample,
            "sample_s": cpu_s, "extrapolated": not whole,
            "oracle_build": "gcc " + " ".join(flags) + " (oracle/dtw_oracle.c, untuned)"}


def cpu_sample_serving(reqs):
    import oracle
    t = time.perf_counter()
    done = 0
    for X, Y, d, Xh, Yh in reqs:
        if Xh.shape[0] > 6000:
            continue
        oracle.full(Xh, Yh)
        done += Xh.shape[0] * Yh.shape[0]
        if time.perf_counter() - t > 15:
            break
    cpu_s = time.perf_counter() - t
    return cpu_record(done, cpu_s, f"requests with M <= 6000 in stream order ({done / 1e6:.0f} M cells; their rate "
                                   f"taken as the stream's): textbook FP64 full table, single thread, {cpu_s:.1f} s",
                      False)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--batch", type=int, default=512, help="pairs of the batched workload (config 4)")
    ap.add_argument("--batch-d", type=int, default=24, help="frame width of the batched workload (config 4)")
    ap.add_argument("--requests", type=int, default=96, help="requests of the serving stream (config 5)")
    ap.add_argument("--serving-m-hi", type=int, default=400000,
                    help="upper end of the serving requests' lengths (config 5 and the default run)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default run: skip the long-pair and serving summaries (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16", "fp16"], default=None,
                    help="override the single-pair workload's arithmetic (e.g. fp16 for config 3)")
    ap.add_argument("--no-fp64-comparison", action="store_true",
                    help="skip the all-FP64 run of the same input (configs 3 and 4)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (calibration of HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe << 17, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8, "dispatches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method is measured on one "
              f"MI355X, and splitting a batch or a pair over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.config in WORKLOADS:
        out = bench_single(args, args.config)
        if args.config == 2 and not args.no_extras:
            # the two other targets, measured in the same run: the long pair in
            # the reduced-precision Gram forms against FP64, and the serving loop
            out["long_pair"] = long_pair_summary(args)
            out["serving"], _ = serving_summary(args, args.requests, args.serving_m_hi,
                                                [("bf16_mix", "bf16"), ("fp16_mix", "fp16")])
            out["tie_exact"] = tie_exact_summary(args)
            out["edit_distance"] = edit_summary(args)
    elif args.config == 6:
        out = bench_edit(args)
    elif args.config == 4:
        out = bench_batched(args)
    elif args.config == 5:
        out = bench_serving(args)
    else:
        print(f"unknown config {args.config}", file=sys.stderr)
        sys.exit(2)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
