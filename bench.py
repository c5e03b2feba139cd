"""Benchmark: useful GFLOP/s of batched low-rank products on one MI355X.

Default workload (the uneven grouped batch): 20 000 instances, block size b
uniform in {64,128,256,512,1024}, rank r uniform over {8,...,128} with
r <= b/2, each instance carrying a dense x skinny product C = A U and an
inner product T = V1^T U2 (40 000 FP64 products, N(0,1) entries, device
resident).  One step = one replay of the plan's hipGraph (one grouped
kernel over every tile).  Printed: one JSON line with the throughput, the
roofline of the grouped kernel and the CPU oracle's rate on a bounded,
stratified sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--config grouped|dense|chain|chain-bf16x3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "useful GFLOP/s + % of roofline on uneven batches; p50/p99 latency at fixed load"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_plan(plan, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        plan.execute(stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for s in range(steps):
        plan.execute(stream)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[s].elapsed_time(ev[s + 1]) for s in range(steps)]
    total = ev[0].elapsed_time(ev[steps])
    return total / steps, per


def cpu_baseline_grouped(w, seconds_budget=30.0, per_bucket=40):
    """Oracle on a stratified sample: the first `per_bucket` instances of every
    (b, r) bucket, both products, all host threads."""
    import numpy as np
    import oracle
    from paper_2311_07602_amd import workloads
    shapes = w.meta["shapes"]
    chosen, seen = [], {}
    for i, br in enumerate(shapes):
        if seen.get(br, 0) < per_bucket:
            seen[br] = seen.get(br, 0) + 1
            chosen.append(i)
    As, Us, Vs, U2s = [], [], [], []
    flops = 0.0
    for i in chosen:
        o = workloads.grouped_operands(w, i)
        As.append(o["A"]); Us.append(o["U"]); Vs.append(o["V1"]); U2s.append(o["U2"])
        b, r = shapes[i]
        flops += 2.0 * b * b * r + 2.0 * b * r * r
    nthreads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.dense_ts(As, Us, nthreads=nthreads)
    oracle.inner(Vs, U2s, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {per_bucket} instances of each of the {len(seen)} (b,r) buckets "
                      f"({len(chosen)} instances, both products, {flops / 1e9:.2f} GFLOP) in {dt:.1f} s"}


def run_grouped(args):
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    w = workloads.grouped(args.count, seed=3)
    torch.cuda.synchronize()
    log(f"[bench] workload built: {len(w.descs)} products in {time.perf_counter() - t0:.1f} s")
    flags = 0
    if args.persistent:
        flags |= lrbg.LRBG_PLAN_PERSISTENT
    if args.mix:
        flags |= lrbg.LRBG_PLAN_SCHED_MIX
    plan = lrbg.Plan(w.descs, tune_cache=args.tune_cache, flags=flags)
    st = plan.stats()
    log(f"[bench] plan: {st}")
    ms, per = time_plan(plan, args.steps, args.warmup, stream)
    flops, bytes_ = st["useful_flops"], st["hbm_bytes"]
    achieved_tf = flops / (ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": round(flops / (ms * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"uneven grouped batch: {args.count} instances, b~U{{64..1024}}, "
                               f"r~U{{8..128}} with r<=b/2, C=A*U and T=V1^T*U2 per instance, FP64, N(0,1)",
                   "instances": args.count, "products": len(w.descs), "tiles": st["tiles"],
                   "plan_flags": flags, "launch": "hipGraph replay, one grouped kernel"},
        "roofline": {"bound": "mfma", "achieved": round(achieved_tf, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "lrbg_grouped_kernel",
                     "algorithmic_flops": flops, "algorithmic_bytes": bytes_,
                     "hbm_GBs": round(bytes_ / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(bytes_ / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "roofline_ms": round(max(flops / (PEAK_FP64_TFLOPS * 1e12), bytes_ / (PEAK_HBM_GBS * 1e9)) * 1e3, 4),
                     "frac_of_roofline_time": round(max(flops / (PEAK_FP64_TFLOPS * 1e12),
                                                        bytes_ / (PEAK_HBM_GBS * 1e9)) * 1e3 / ms, 4)},
        "step_ms_min": round(min(per), 4), "step_ms_max": round(max(per), 4),
    }
    plan.close()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline_grouped(w)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="grouped", choices=["grouped"])
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2311_07602_amd", "tune", "mi355x.tune"))
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--mix", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the batched products are "
              f"independent per instance and shard across GPUs without communication, but this build "
              f"measures one GPU's share.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_07602_amd import lrbg
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lrbg.load()
    line = run_grouped(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
