"""Benchmark: linear-memory DTW alignment (arXiv 2008.02734) on one MI355X.

Default workload (the headline): a single 20000 x 16000 pair, d = 12, FP64,
chroma-like frames, cutoff m = 500, exact FP64 path.  One step = one complete
dtw_align call: every wavefront sweep, split-cost + argmin, recursion level,
leaf solve and path assembly, with the inputs already resident in HBM.

Prints one JSON line.  `value` is textbook-equivalent throughput M*N / step
time (GCUPS).  The roofline entry is for the dominant kernel, the wavefront
sweep: cells evaluated by the sweeps / summed sweep-kernel time (HIP events on
the launch stream), against the VALU peak divided by the algorithmic VALU
slots one cell needs.  The CPU baseline is the oracle's textbook full-table
DTW timed single-threaded on this host.

Other workloads (--config): 1 = 500 x 400 FP64 latency; 3 = 200000 x 160000,
d = 128, BF16 Gram cost on the matrix cores; 4 = 512 pairs in one batched
call, d = 24, FP32; 5 = a Poisson stream of requests through the serving loop.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = full-rate VALU lane-slots/s
# (FP64 and unpacked FP32 alike).
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
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
    peak = VALU_SLOTS_PER_S / slots_per_cell(precision, d) / 1e9
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

    W = WORKLOADS[cfg]
    M, N, d, prec = W["M"], W["N"], W["d"], W["precision"]
    X, Y = synth.make_pair(cfg, 0, M, N, d, W["family"])
    tdt = torch.float64 if prec == "fp64" else torch.float32
    Xd = torch.from_numpy(X).to("cuda:0", dtype=tdt)
    Yd = torch.from_numpy(Y).to("cuda:0", dtype=tdt)
    al = dtw.Aligner(M, N, d, tdt, prec, W["m"], device="cuda:0")
    al.opts.profile = 1
    stream = torch.cuda.current_stream()
    ms, lat, stats = timed_steps(lambda: al.run(Xd, Yd, stats=True, stream=stream), args.steps, args.warmup)
    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), st
    kname = {"fp64": f"pass_kernel<double,{d}>", "fp32": f"pass_kernel<float,{d}>",
             "bf16": "pass_kernel<float,128,Gram>"}[prec] + " (wavefront sweep)"
    out = base_record(args, M * N / (ms * 1e-3) / 1e9, ms, {"fp64": "f64", "fp32": "f32", "bf16": "bf16/f32"}[prec],
                      {"workload": W["name"], "M": M, "N": N, "d": d, "min_block": W["m"], "precision": prec,
                       "seed": [cfg, 0]})
    out.update({
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "cells_processed": st["cells_processed"], "cells_ratio_to_MN": st["cells_processed"] / (M * N),
        "processed_gcups": st["cells_processed"] / (ms * 1e-3) / 1e9,
        "kernel_ms": {k: float(np.mean([s[k] for s in stats])) for k in
                      ("ms_sweep", "ms_split", "ms_plan", "ms_leaf", "ms_other")},
        "levels": st["levels"], "leaves": st["leaves"],
        "roofline": roofline(stats, prec, d, kname, measured_traffic() if cfg == 2 else None),
    })
    if not args.no_cpu_baseline:
        import oracle
        # the oracle's full table on the pair (cfg 1, 2) or on its leading
        # sub-block (cfg 3, whose full table does not fit a host)
        Ms, Ns = (M, N) if cfg != 3 else (8000, 6400)
        Xs, Ys = X[:Ms], Y[:Ns]
        t = time.perf_counter()
        c_ref, p_ref = oracle.full(Xs, Ys)
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": Ms * Ns / cpu_s / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": (f"the full {M}x{N} pair" if cfg != 3 else f"the leading {Ms}x{Ns} block of the pair")
                      + f": textbook FP64 full table + backtrace, single thread, {cpu_s:.1f} s"}
        if cfg != 3:
            path = al.path[: int(al.plen.item())].cpu().numpy()
            out["parity"] = {"path_equal_to_oracle": bool(path.tolist() == p_ref.tolist()),
                             "cost_rel_err": abs(float(al.cost.item()) - c_ref) / c_ref}
        else:
            cs, ps, _ = dtw.align(Xd[:Ms].contiguous(), Yd[:Ns].contiguous(), precision=prec, min_block=W["m"])
            out["parity"] = {"block": [Ms, Ns], "cost_rel_err_vs_fp64_oracle": (cs - c_ref) / c_ref}
    return out


def bench_batched(args):
    """cfg 4: 512 independent pairs, M and N log-uniform in [1000, 30000] with
    N/M in [0.7, 1.4], d = 24 chroma-like FP32 frames, one batched call."""
    import torch

    from paper_2008_02734_amd import dtw, synth

    shapes = synth.batch_shapes(args.batch)
    d = 24
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(4, p, M, N, d, "chroma")
        Xs.append(X.astype(np.float32))
        Ys.append(Y.astype(np.float32))
    Xp = torch.from_numpy(np.concatenate(Xs)).to("cuda:0")
    Yp = torch.from_numpy(np.concatenate(Ys)).to("cuda:0")
    xo = np.concatenate([[0], np.cumsum([s[0] for s in shapes])]).astype(np.int64)
    yo = np.concatenate([[0], np.cumsum([s[1] for s in shapes])]).astype(np.int64)
    Xl = [Xp[xo[i]:xo[i + 1]] for i in range(len(shapes))]
    Yl = [Yp[yo[i]:yo[i + 1]] for i in range(len(shapes))]
    runner = dtw.BatchAligner(Xl, Yl, precision="fp32", min_block=500, profile=True)
    ms, lat, stats = timed_steps(runner.run, args.steps, args.warmup)
    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), st
    cells = sum(M * N for M, N in shapes)
    out = base_record(args, cells / (ms * 1e-3) / 1e9, ms, "f32",
                      {"workload": f"batch of {len(shapes)} pairs, M,N log-uniform in [1000, 30000], N/M in "
                                   "[0.7, 1.4], d=24 f32 chroma-like, FP32 DP, FP64 split (m=500)",
                       "pairs": len(shapes), "d": d, "min_block": 500, "precision": "fp32", "seed": [4, "p"]})
    out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "cells_processed": st["cells_processed"],
                "processed_gcups": st["cells_processed"] / (ms * 1e-3) / 1e9,
                "kernel_ms": {k: float(np.mean([s[k] for s in stats])) for k in
                              ("ms_sweep", "ms_split", "ms_plan", "ms_leaf", "ms_other")},
                "levels": st["levels"], "leaves": st["leaves"],
                "roofline": roofline(stats, "fp32", d, "pass_kernel<float,24> (wavefront sweep)")})
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
        out["cpu_baseline"] = {"value": done / cpu_s / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
                               "sample": f"the batch's first {p + 1} pairs ({done / 1e6:.0f} M cells): textbook "
                                         f"FP64 full table + backtrace, single thread, {cpu_s:.1f} s"}
    return out


def bench_serving(args):
    """cfg 5, scaled: a Poisson stream of requests through the serving loop.
    M log-uniform in [2000, 40000] (the configuration's upper end, 400000, is
    scaled down so the stream finishes in seconds), N = M x U[0.75, 1.3],
    half d = 12 chroma-like in FP32, half d = 128 embedding-like in the BF16
    Gram form.  A pilot run (all requests at once) gives the saturated rate;
    the stream then arrives at 0.7 of it.  Baseline: the d = 12 requests one
    at a time through the plain FP64 path."""
    import torch

    from paper_2008_02734_amd import dtw, synth

    rng = np.random.default_rng([5, 999])
    reqs = []
    for r in range(args.requests):
        M = int(np.exp(rng.uniform(np.log(2000), np.log(40000))))
        N = int(M * rng.uniform(0.75, 1.3))
        if r % 2 == 0:
            X, Y = synth.make_pair(5, r, M, N, 12, "chroma")
            reqs.append((torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(Y.astype(np.float32)).cuda(),
                         "fp32", X, Y))
        else:
            X, Y = synth.make_pair(5, r, M, N, 128, "embedding")
            reqs.append((torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(Y.astype(np.float32)).cuda(),
                         "bf16", None, None))
    torch.cuda.synchronize()
    cells = sum(q[0].shape[0] * q[1].shape[0] for q in reqs)
    srv = dtw.Server(pool_bytes=16 << 30, max_slots=8, max_batch=16)
    try:
        # pilot: everything at once
        t0 = time.perf_counter()
        tk = [srv.submit(X, Y, precision=p) for X, Y, p, _, _ in reqs]
        for t in tk:
            srv.wait(t)
        pilot_s = time.perf_counter() - t0
        rate = len(reqs) / pilot_s
        lam = 0.7 * rate
        gaps = rng.exponential(1.0 / lam, size=len(reqs))
        arrivals = np.cumsum(gaps)
        t0 = time.perf_counter()
        tickets = []
        for (X, Y, p, _, _), at in zip(reqs, arrivals):
            while time.perf_counter() - t0 < at:
                time.sleep(50e-6)
            tickets.append(srv.submit(X, Y, precision=p))
        res = [srv.wait(t) for t in tickets]
        makespan = time.perf_counter() - t0
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res), [r for r in res if r["status"] != 0][:1]
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) / 1e6 for r in res])
    out = base_record(args, cells / makespan / 1e9, makespan * 1e3, "f32+bf16",
                      {"workload": f"Poisson stream of {len(reqs)} requests, M log-uniform in [2000, 40000], half "
                                   "d=12 FP32, half d=128 BF16 Gram cost, at 0.7x the saturated rate",
                       "requests": len(reqs), "seed": [5, "r"]})
    out.update({"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "lambda_per_s": lam, "saturated_gcups": cells / pilot_s / 1e9,
                "max_batch_seen": int(max(r["batch_size"] for r in res))})
    # baseline: the d = 12 requests one at a time in FP64
    import torch as _t
    bcells, bt = 0, 0.0
    for X, Y, p, Xh, Yh in reqs:
        if Xh is None:
            continue
        Xd, Yd = _t.from_numpy(Xh).cuda(), _t.from_numpy(Yh).cuda()
        _t.cuda.synchronize()
        s0 = time.perf_counter()
        dtw.align(Xd, Yd)
        bt += time.perf_counter() - s0
        bcells += Xh.shape[0] * Yh.shape[0]
    served_d12 = sum(q[0].shape[0] * q[1].shape[0] for q in reqs if q[2] == "fp32")
    out["baseline_fp64_one_at_a_time"] = {"gcups": bcells / bt / 1e9, "requests": "the d=12 half"}
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_sample_serving(reqs)
    return out


def cpu_sample_serving(reqs):
    import oracle
    t = time.perf_counter()
    done = 0
    for X, Y, p, Xh, Yh in reqs:
        if Xh is None or Xh.shape[0] > 6000:
            continue
        oracle.full(Xh, Yh)
        done += Xh.shape[0] * Yh.shape[0]
        if time.perf_counter() - t > 15:
            break
    cpu_s = time.perf_counter() - t
    return {"value": done / cpu_s / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"d=12 requests with M <= 6000 ({done / 1e6:.0f} M cells): textbook FP64 full table, "
                      f"single thread, {cpu_s:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--batch", type=int, default=512, help="pairs of the batched workload (config 4)")
    ap.add_argument("--requests", type=int, default=96, help="requests of the serving stream (config 5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
              f"MI355X and the multi-GPU sharding is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.config in WORKLOADS:
        out = bench_single(args, args.config)
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
