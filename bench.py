"""Benchmark: exact FP64 linear-memory DTW alignment on one MI355X.

One step = one complete dtw_align call on one pair: every wavefront sweep,
split-cost + argmin, recursion level, leaf solve and path assembly, with the
inputs already resident in HBM.  Default workload: a single 20000 x 16000
pair, d = 12, FP64, chroma-like frames (seeded synthetic stand-in for the
paper's audio features), cutoff m = 500.

Prints one JSON line.  `value` is textbook-equivalent throughput M*N / step
time (GCUPS).  The roofline entry is for the dominant kernel, the wavefront
sweep: cells evaluated by the sweeps / summed sweep-kernel time (HIP events on
the launch stream), against the FP64 VALU peak divided by the algorithmic
VALU slots one cell needs.  The CPU baseline is the oracle's textbook
full-table DTW on the same pair, single-threaded, timed on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = full-rate FP64 VALU lane-slots/s.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU slots per DP cell, FP64, d = 12 (from the gfx950 ISA of the
# sweep kernel): 12 subtract + 12 fma for the squared distance, 21 for the
# correctly rounded square root (18 instructions, the reciprocal square root
# counting 4 as a quarter-rate transcendental), 2 min + 1 add for the
# recurrence.
SLOTS_PER_CELL = {12: 48}

WORKLOADS = {
    2: dict(name="single pair 20000x16000, d=12 f64 chroma-like, exact FP64 linmdtw (m=500)", M=20000, N=16000,
            d=12, family="chroma", m=500),
    1: dict(name="single pair 500x400, d=12 f64 Gaussian walk, exact FP64 (one leaf at m=500)", M=500, N=400,
            d=12, family="gaussian_walk", m=500),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
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

    import torch

    from paper_2008_02734_amd import dtw, synth

    W = WORKLOADS[args.config]
    M, N, d = W["M"], W["N"], W["d"]
    X, Y = synth.make_pair(args.config, 0, M, N, d, W["family"])
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.from_numpy(Y).to("cuda:0")
    al = dtw.Aligner(M, N, d, torch.float64, "fp64", W["m"], device="cuda:0")
    al.opts.profile = 1
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        al.run(Xd, Yd, stats=True)
    torch.cuda.synchronize()

    lat = []
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        st = al.run(Xd, Yd, stats=True, stream=stream)  # synchronises the stream
        lat.append((time.perf_counter() - s0) * 1e3)
        stats.append(st)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = total * 1e3 / args.steps

    st = stats[-1]
    assert all(s["device_error"] == 0 for s in stats), stats[-1]
    cells_mn = M * N
    sweep_ms = float(np.mean([s["ms_sweep"] for s in stats]))
    sweep_launches = st["levels"]
    achieved = st["sweep_cells"] / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    peak = VALU_SLOTS_PER_S / SLOTS_PER_CELL.get(d, 48) / 1e9
    out = {
        "metric": "DP cells/sec (GCUPS) + fraction of VALU roofline; p50/p99 align latency",
        "value": cells_mn / (ms_per_step * 1e-3) / 1e9,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W["name"], "M": M, "N": N, "d": d, "min_block": W["m"], "seed": [args.config, 0]},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "cells_processed": st["cells_processed"],
        "cells_ratio_to_MN": st["cells_processed"] / cells_mn,
        "processed_gcups": st["cells_processed"] / (ms_per_step * 1e-3) / 1e9,
        "kernel_ms": {k: float(np.mean([s[k] for s in stats])) for k in
                      ("ms_sweep", "ms_split", "ms_plan", "ms_leaf", "ms_other")},
        "levels": st["levels"],
        "leaves": st["leaves"],
        "roofline": {
            "bound": "alu",
            "kernel": "pass_kernel<double,12> (wavefront sweep)",
            "achieved": achieved,
            "peak": peak,
            "unit": "Gcells/s",
            "frac": (achieved / peak) if achieved else None,
            "traffic": measured_traffic() if args.config == 2 else None,
            "launches_per_step": sweep_launches,
            "sweep_cells_per_step": st["sweep_cells"],
            "avg_sweep_launch_ms": sweep_ms / max(1, sweep_launches),
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        c_ref, p_ref = oracle.full(X, Y)
        cpu_s = time.perf_counter() - t
        path = al.path[: int(al.plen.item())].cpu().numpy()
        cost = float(al.cost.item())
        out["cpu_baseline"] = {
            "value": cells_mn / cpu_s / 1e9,
            "unit": "GCUPS",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the full {M}x{N} pair: textbook FP64 full table + backtrace, single thread, {cpu_s:.1f} s",
        }
        out["parity"] = {"path_equal_to_oracle": bool(path.tolist() == p_ref.tolist()),
                         "cost_rel_err": abs(cost - c_ref) / c_ref}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
