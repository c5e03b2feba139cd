"""Benchmark: useful GFLOP/s of batched low-rank products on one MI355X.

Default workload (the uneven grouped batch): 20 000 instances, block size b
uniform in {64,128,256,512,1024}, rank r uniform over {8,...,128} with
r <= b/2, each instance carrying a dense x skinny product C = A U and an
inner product T = V1^T U2 (40 000 FP64 products, N(0,1) entries, device
resident).  One step = one replay of the plan's hipGraph (one grouped
kernel over every tile).  Printed: one JSON line with the throughput, the
roofline of the grouped kernel and the CPU oracle's rate on a bounded,
stratified sample of the same workload.

Extra fields measure the other workloads on the same GPU: a uniform dense x
skinny batch (64 x 256x256 . 256x16, buffer sets rotated so the 38 MB batch
does not sit in the 256 MB last-level cache) and the low-rank x low-rank
chain (4096 instances, b = 512, r = 32: inner products, then recompression),
the paper's fused low-rank product G = X_A (V_A^T U_B) X_B at batch 20 000
for b in {512, 1024, 2048} and r in {8, 16, 32, 96, 128}, a weakly admissible
BLR matrix times 8 right-hand sides, and the serving loop.

  python bench.py [--steps K] [--warmup W] [--extras/--no-extras]
  python bench.py --calibrate-copy      # plain 1 GiB device copy (counter scaling)
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
PROFILE = os.path.join(ROOT, "profiles", "lrbg_grouped_kernel.uneven_batch_20000.md")
DEFAULT_TUNE = os.path.join(ROOT, "paper_2311_07602_amd", "tune", "mi355x.tune")
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


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_HOST_THREADS = None


def host_threads() -> int:
    """Threads the oracle may use: the process's CPU affinity, capped by the
    OpenMP limit the environment sets.  Read once, before any oracle call:
    a call with an explicit thread count changes the OpenMP default that
    later queries would see."""
    global _HOST_THREADS
    if _HOST_THREADS is None:
        import oracle
        _HOST_THREADS = max(1, min(len(os.sched_getaffinity(0)), oracle.max_threads()))
    return _HOST_THREADS


def _timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def cpu_baseline_grouped(w, per_bucket=40, per_bucket_1t=2):
    """Oracle on stratified samples of the uneven batch: the first
    `per_bucket` instances of every (b, r) bucket on all host threads, the
    first `per_bucket_1t` on one thread; both products."""
    import oracle
    from paper_2311_07602_amd import workloads
    shapes = w.meta["shapes"]

    def sample(k):
        chosen, seen = [], {}
        for i, br in enumerate(shapes):
            if seen.get(br, 0) < k:
                seen[br] = seen.get(br, 0) + 1
                chosen.append(i)
        ops = [workloads.grouped_operands(w, i) for i in chosen]
        flops = sum(2.0 * b * b * r + 2.0 * b * r * r for b, r in (shapes[i] for i in chosen))
        return chosen, len(seen), ops, flops

    nthreads = host_threads()
    chosen, nb, ops, flops = sample(per_bucket)
    dt = _timed(lambda: (oracle.dense_ts([o["A"] for o in ops], [o["U"] for o in ops], nthreads=nthreads),
                         oracle.inner([o["V1"] for o in ops], [o["U2"] for o in ops], nthreads=nthreads)))
    chosen1, _, ops1, flops1 = sample(per_bucket_1t)
    dt1 = _timed(lambda: (oracle.dense_ts([o["A"] for o in ops1], [o["U"] for o in ops1], nthreads=1),
                          oracle.inner([o["V1"] for o in ops1], [o["U2"] for o in ops1], nthreads=1)))
    return {"value": round(flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first {per_bucket} instances of each of the {nb} (b,r) buckets "
                      f"({len(chosen)} instances, both products, {flops / 1e9:.2f} GFLOP) in {dt:.1f} s "
                      f"on {nthreads} threads",
            "cpu_model": cpu_model(),
            "one_thread": {"value": round(flops1 / dt1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                           "sample": f"first {per_bucket_1t} instances of each bucket ({len(chosen1)} instances, "
                                     f"{flops1 / 1e9:.2f} GFLOP) in {dt1:.1f} s"}}


def cpu_baseline_small_configs(chain_1t_instances=256):
    """The oracle on the uniform dense batch (64 x 256x256 . 256x16, in full,
    one thread and all threads) and on the chain (4096 x b=512, r=32, in full
    on all threads; its first `chain_1t_instances` instances on one thread),
    with the same flop counts as the GPU lines."""
    import numpy as np
    import oracle
    from paper_2311_07602_amd import inputs
    nthreads = host_threads()
    out = {}
    As, Us = zip(*(inputs.dense_ts_instance(1, i, 256, 16) for i in range(64)))
    f1 = 64 * 2.0 * 256 * 256 * 16
    t_all = min(_timed(lambda: oracle.dense_ts(list(As), list(Us), nthreads=nthreads)) for _ in range(3))
    t_one = min(_timed(lambda: oracle.dense_ts(list(As), list(Us), nthreads=1)) for _ in range(2))
    out["dense_uniform"] = {"workload": "64 x (A 256x256 . U 256x16), in full",
                            "all_threads": {"GFLOP/s": round(f1 / t_all / 1e9, 3), "cores": nthreads,
                                            "ms": round(t_all * 1e3, 2)},
                            "one_thread": {"GFLOP/s": round(f1 / t_one / 1e9, 3), "cores": 1,
                                           "ms": round(t_one * 1e3, 2)}}
    count, b, r = 4096, 512, 32
    host = inputs.chain_instances(2, count, b, r)
    ops = [[np.asfortranarray(host[i, t].T) for i in range(count)] for t in range(4)]   # U1, V1, U2, V2
    fch = count * (2.0 * b * r * r + 2.0 * b * b * r + 2.0 * b * r * r)
    t_all = _timed(lambda: oracle.chain(ops[1], ops[2], ops[0], ops[3], nthreads=nthreads))
    n1 = chain_1t_instances
    t_one = _timed(lambda: oracle.chain(ops[1][:n1], ops[2][:n1], ops[0][:n1], ops[3][:n1], nthreads=1))
    out["chain"] = {"workload": f"{count} x chain b={b} r={r} (T = V1^T U2, W = U1 (T V2^T))",
                    "all_threads": {"GFLOP/s": round(fch / t_all / 1e9, 3), "cores": nthreads,
                                    "s": round(t_all, 2), "sample": "in full"},
                    "one_thread": {"GFLOP/s": round(fch / count * n1 / t_one / 1e9, 3), "cores": 1,
                                   "s": round(t_one, 2), "sample": f"first {n1} instances"}}
    del host, ops
    return out


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
    if args.dual:
        flags |= lrbg.LRBG_PLAN_DUAL
    if not args.lpt:
        flags |= lrbg.LRBG_PLAN_SCHED_MIX
    plan = lrbg.Plan(w.descs, tune_cache=args.tune_cache, flags=flags)
    st = plan.stats()
    log(f"[bench] plan: {st}")
    ms, per = time_plan(plan, args.steps, args.warmup, stream)
    flops, bytes_ = st["useful_flops"], st["hbm_bytes"]
    achieved_tf = flops / (ms * 1e-3) / 1e12
    from paper_2311_07602_amd import profiling
    traffic = profiling.current_traffic(PROFILE) if (args.count == 20000 and flags == lrbg.LRBG_PLAN_SCHED_MIX) else None
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
                     "unit": "TFLOP/s", "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
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
        if not args.no_extras:
            log("[bench] timing the CPU oracle on the uniform dense batch and the chain ...")
            line["cpu_baseline"]["configs"] = cpu_baseline_small_configs()
    return line


def run_grouped_bf16x3(count=20000, steps=10, warmup=2):
    """The uneven batch with every product in the BF16x3 split precision
    (FP32 operands, three bf16 terms, FP64 outputs), planned and replayed as
    the headline FP64 batch; useful flops counted as FP64 (2 per
    multiply-add), bytes at 4 per input element."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    w = workloads.grouped(count, seed=3, prec="bf16x3")
    plan = lrbg.Plan(w.descs, tune_cache=DEFAULT_TUNE, flags=lrbg.LRBG_PLAN_SCHED_MIX)
    st = plan.stats()
    ms, _ = time_plan(plan, steps, warmup, stream)
    plan.close()
    del w
    torch.cuda.empty_cache()
    f, by = st["useful_flops"], st["hbm_bytes"]
    return {"workload": f"uneven grouped batch, {count} instances, BF16x3 split precision (FP32 in, FP64 out)",
            "ms_per_step": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1), "GB/s": round(by / ms / 1e6, 1),
            "hbm_frac": round(by / ms / 1e6 / PEAK_HBM_GBS, 4), "algorithmic_flops": f, "algorithmic_bytes": by}


def run_dense_uniform(steps=200, warmup=20, sets=16):
    """64 x (256x256 . 256x16); `sets` independent buffer sets (> 2x the
    last-level cache in total) replayed round-robin."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    ws = [workloads.dense_uniform(64, 256, 16, seed=11 + i) for i in range(sets)]
    plans = [lrbg.Plan(w.descs, flags=lrbg.LRBG_PLAN_UNTIMED) for w in ws]
    st = plans[0].stats()
    for i in range(warmup):
        plans[i % sets].execute(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sp = stream.cuda_stream
    e0.record(stream)
    for i in range(steps):
        plans[i % sets].execute(sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for p in plans:
        p.close()
    roof = max(st["useful_flops"] / (PEAK_FP64_TFLOPS * 1e12), st["hbm_bytes"] / (PEAK_HBM_GBS * 1e9)) * 1e3
    return {"workload": "64 x (A 256x256 . U 256x16), FP64, N(0,1), 16 rotated buffer sets",
            "ms_per_step": round(ms, 5), "GFLOP/s": round(st["useful_flops"] / ms / 1e6, 1),
            "GB/s": round(st["hbm_bytes"] / ms / 1e6, 1), "roofline_ms": round(roof, 5),
            "frac_of_roofline_time": round(roof / ms, 4),
            "note": "launch-inclusive (one plan replay per step: a single small launch, issued directly)"}


def run_chain(count=4096, b=512, r=32, steps=20, warmup=3, prec="fp64", tune_cache=None):
    """Low-rank x low-rank chain: T = V1^T U2 (level 1), W = U1 (T V2^T)
    (level 2), both levels in one captured graph, tile variants from the
    tuning cache (the package's MI355X cache by default)."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    w = workloads.chain(count, b, r, prec=prec)
    torch.cuda.synchronize()
    log(f"[bench] chain workload ({prec}) built in {time.perf_counter() - t0:.1f} s")
    plan = lrbg.Plan(w.descs, tune_cache=tune_cache or DEFAULT_TUNE)
    st = plan.stats()
    ms, _ = time_plan(plan, steps, warmup, stream)
    plan.close()
    f, by = st["useful_flops"], st["hbm_bytes"]
    roof = max(f / (PEAK_FP64_TFLOPS * 1e12), by / (PEAK_HBM_GBS * 1e9)) * 1e3
    return {"workload": f"{count} x chain b={b} r={r} ({prec} inner, FP64 recompression)",
            "levels": st["levels"], "ms_per_step": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1),
            "GB/s": round(by / ms / 1e6, 1), "roofline_ms": round(roof, 4),
            "frac_of_roofline_time": round(roof / ms, 4), "bound": "hbm"}


def run_lrmult_config(args):
    """One (b, r) of the paper's fused low-rank product as the timed workload
    (``--config lrmult``): batch ``--count`` of G = X_A (V_A^T U_B) X_B."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    b, r = args.lr_b, args.lr_r
    w = workloads.lrmult(args.count, b, r)
    plan = lrbg.Plan(w.descs, tune_cache=args.tune_cache)
    st = plan.stats()
    kernel = {"lrm": "lrbg_lrmult_kernel", "lrm4": "lrbg_lrmult4_kernel", "lrmb": "lrbg_lrmultb_kernel",
              "lrm96": "lrbg_lrmult96_kernel"}[lrbg.lrbg_schedule_variants(w.descs[:1], args.tune_cache)[0].split("_")[0]]
    ms, per = time_plan(plan, args.steps, args.warmup, stream)
    plan.close()
    f, by = st["useful_flops"], st["hbm_bytes"]
    t_f, t_b = f / (PEAK_FP64_TFLOPS * 1e12), by / (PEAK_HBM_GBS * 1e9)
    if t_f >= t_b:
        roof = {"bound": "mfma", "achieved": round(f / ms / 1e9, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(f / ms / 1e9 / PEAK_FP64_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(by / ms / 1e6, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(by / ms / 1e6 / PEAK_HBM_GBS, 4)}
    from paper_2311_07602_amd import profiling
    prof = os.path.join(ROOT, "profiles", f"{kernel}.lrmult_b{b}_r{r}_{args.count}.md")
    traffic = profiling.current_traffic(prof, profiling.LRMULT_SOURCES) if os.path.exists(prof) else None
    roof.update({"traffic": traffic, "kernel": kernel, "algorithmic_flops": f, "algorithmic_bytes": by,
                 "roofline_ms": round(max(t_f, t_b) * 1e3, 4), "frac_of_roofline_time": round(max(t_f, t_b) * 1e3 / ms, 4)})
    return {"metric": METRIC, "value": round(f / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{args.count} x G = X_A (V_A^T U_B) X_B, b={b}, r={r}, FP64, N(0,1) "
                                   f"(the paper's fused low-rank product)", "instances": args.count,
                       "tiles": st["tiles"], "launch": "hipGraph replay, one fused kernel"},
            "roofline": roof, "step_ms_min": round(min(per), 4), "step_ms_max": round(max(per), 4)}


def run_chain_recomp_config(args):
    """The recompression level of the low-rank chain alone (``--config
    chain_recomp``): 4096 x W = U1 (T V2^T), b = 512, r = 32, with T from one
    run of the whole chain; the plan holds only the recompression products,
    so every timed launch is the HBM-write-bound RECOMP kernel."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    count, b, r = 4096, 512, 32
    w = workloads.chain(count, b, r)
    full = lrbg.Plan(w.descs, tune_cache=args.tune_cache)
    full.execute(stream)
    torch.cuda.synchronize()
    full.close()
    plan = lrbg.Plan(w.descs[count:], tune_cache=args.tune_cache)
    st = plan.stats()
    ms, per = time_plan(plan, args.steps, args.warmup, stream)
    plan.close()
    f, by = st["useful_flops"], st["hbm_bytes"]
    t_f, t_b = f / (PEAK_FP64_TFLOPS * 1e12), by / (PEAK_HBM_GBS * 1e9)
    from paper_2311_07602_amd import profiling
    prof = os.path.join(ROOT, "profiles", "lrbg_grouped_kernel.chain_recomp_4096.md")
    traffic = profiling.current_traffic(prof) if os.path.exists(prof) else None
    return {"metric": METRIC, "value": round(f / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{count} x W = U1 (T V2^T), b={b}, r={r}, FP64 (the recompression level of "
                                   f"the low-rank chain)", "instances": count, "tiles": st["tiles"],
                       "launch": "hipGraph replay, one grouped kernel"},
            "roofline": {"bound": "hbm", "achieved": round(by / ms / 1e6, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(by / ms / 1e6 / PEAK_HBM_GBS, 4), "traffic": traffic,
                         "kernel": "lrbg_grouped_kernel", "algorithmic_flops": f, "algorithmic_bytes": by,
                         "roofline_ms": round(max(t_f, t_b) * 1e3, 4),
                         "frac_of_roofline_time": round(max(t_f, t_b) * 1e3 / ms, 4)},
            "step_ms_min": round(min(per), 4), "step_ms_max": round(max(per), 4)}


def time_calls(fn, steps, warmup, stream):
    """Average time of fn() (device work enqueued on `stream`), HIP events."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def vendor_lrmult(w, steps, warmup, stream):
    """The same batch as three vendor strided-batched DGEMMs (torch.bmm on
    ROCm: rocBLAS / hipBLASLt), C and E through HBM, on the operands in place.
    Returns (ms, max |G_vendor - G| / max |G|) on the first instances."""
    import torch
    pin, pout = w.pools
    n, b, r, per, per_g = w.meta["count"], w.meta["b"], w.meta["r"], w.meta["per"], w.meta["per_g"]
    oV, oU, oXA, oXB = w.meta["offs"]
    VAt = pin.as_strided((n, r, b), (per, b, 1), oV)     # V_A^T (V_A stored b x r column-major)
    UB = pin.as_strided((n, b, r), (per, 1, b), oU)
    XA = pin.as_strided((n, r, r), (per, 1, r), oXA)
    XB = pin.as_strided((n, r, r), (per, 1, r), oXB)
    C = torch.empty(n, r, r, dtype=torch.float64, device=pin.device)
    E, G = torch.empty_like(C), torch.empty_like(C)

    def chain():
        torch.bmm(VAt, UB, out=C)
        torch.bmm(XA, C, out=E)
        torch.bmm(E, XB, out=G)
    ms = time_calls(chain, steps, warmup, stream)
    ours = pout.as_strided((min(n, 64), r, r), (per_g, 1, r), 0)
    diff = float((G[:ours.shape[0]] - ours).abs().max() / ours.abs().max())
    return ms, diff


def paper_rates(b, r):
    """The CPU rates the paper tabulates at this (b, r), batch 20 000 (its
    rank-96 and rank-128 tables, Sec. 7): context beside the MI355X rate,
    not a target."""
    path = os.path.join(ROOT, "tests", "golden", "paper_tables.json")
    if not os.path.exists(path):
        return {}
    rows = []
    for t in json.load(open(path))["tables"]:
        if t["rank"] == r and b in t["block_size"]:
            j = t["block_size"].index(b)
            rows.append({"cpu": t["cpu"], "GFLOP/s": t["ours"][j], "vendor": t["vendor"],
                         "vendor_GFLOP/s": t["vendor_gflops"][j], "cite": t["cite"]})
    return {"paper_cpu": rows} if rows else {}


def run_lrmult_paper(count=20000, bs=(512, 1024, 2048), rs=(8, 16, 32, 96, 128), steps=10, warmup=2):
    """The paper's batched low-rank product G = X_A (V_A^T U_B) X_B at its
    measured shapes (batch 20 000 per (b, r)); GFLOP/s by the paper's count
    4 r^3 + 2 r^2 b per instance.  Beside each: the vendor library's
    batched DGEMM on the same operands (three calls), as context."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    out = []
    for b in bs:
        for r in rs:
            w = workloads.lrmult(count, b, r)
            plan = lrbg.Plan(w.descs)
            st = plan.stats()
            ms, _ = time_plan(plan, steps, warmup, stream)
            plan.close()
            vms, vdiff = vendor_lrmult(w, steps, warmup, stream)
            del w
            torch.cuda.empty_cache()
            f, by = st["useful_flops"], st["hbm_bytes"]
            roof = max(f / (PEAK_FP64_TFLOPS * 1e12), by / (PEAK_HBM_GBS * 1e9)) * 1e3
            out.append({"b": b, "r": r, "ms_per_step": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1),
                        "GB/s": round(by / ms / 1e6, 1), "frac_of_roofline_time": round(roof / ms, 4),
                        "vendor_ms": round(vms, 4), "speedup_vs_vendor": round(vms / ms, 2),
                        "vendor_rel_diff": vdiff, **paper_rates(b, r)})
            log(f"[bench] lrmult b={b} r={r}: {ms:.4f} ms, {f / ms / 1e6:.0f} GFLOP/s, {by / ms / 1e6:.0f} GB/s; "
                f"vendor {vms:.4f} ms")
    return {"workload": f"{count} x G = X_A (V_A^T U_B) X_B per (b, r), FP64, N(0,1), fused (one tile per "
                        f"instance)", "flops_per_instance": "4 r^3 + 2 r^2 b",
            "bound": "hbm for r <= 32, mfma for r >= 96",
            "vendor": "torch.bmm (rocBLAS/hipBLASLt strided-batched DGEMM), three calls per step, C and E in HBM",
            "shapes": out}


def run_vendor_grouped(w, steps=5, warmup=2):
    """The uneven batch through the vendor library: one strided-batched DGEMM
    per (op, b, r) bucket (torch.bmm), on contiguous per-bucket copies of the
    operands made before timing (the copies are not timed)."""
    import torch
    from collections import defaultdict
    from paper_2311_07602_amd import workloads
    stream = torch.cuda.current_stream()
    pin = w.pools[0]
    groups = defaultdict(list)
    for i, (b, r) in enumerate(w.meta["shapes"]):
        groups[(b, r)].append(i)
    calls = []
    for (b, r), ids in sorted(groups.items()):
        cm = lambda off, rows, cols: pin[off:off + rows * cols].view(cols, rows)   # [col, row]
        A = torch.stack([cm(w.index[i][2], b, b) for i in ids]).transpose(1, 2)     # n x b x b
        U = torch.stack([cm(w.index[i][3], b, r) for i in ids]).transpose(1, 2)     # n x b x r
        V1t = torch.stack([cm(w.index[i][4], b, r) for i in ids])                   # n x r x b = V1^T
        U2 = torch.stack([cm(w.index[i][5], b, r) for i in ids]).transpose(1, 2)    # n x b x r
        C = torch.empty(len(ids), b, r, dtype=torch.float64, device=pin.device)
        T = torch.empty(len(ids), r, r, dtype=torch.float64, device=pin.device)
        calls.append((A, U, C, V1t, U2, T))
    torch.cuda.synchronize()

    def all_calls():
        for A, U, C, V1t, U2, T in calls:
            torch.bmm(A, U, out=C)
            torch.bmm(V1t, U2, out=T)
    ms = time_calls(all_calls, steps, warmup, stream)
    del calls
    torch.cuda.empty_cache()
    return {"workload": "the uneven batch, one torch.bmm (rocBLAS/hipBLASLt strided-batched DGEMM) per (op, b, r) "
                        f"bucket, {2 * len(groups)} calls per step on contiguous per-bucket copies",
            "ms_per_step": round(ms, 4)}


def round_args(pin, per, count, b, r, kmax, tol, U, V, sigma, kout):
    """Host arrays (numpy: the binding passes them without conversion) of the
    pointer-array entry points of the recompressed product and the rounded
    addition, for `count` instances laid out in `pin` as A_U, A_V, B_U, B_V
    (b x r each), then A_X, B_X (r x r), `per` doubles apart; outputs U, V
    are (count, kmax, b) tensors."""
    import numpy as np
    t = np.arange(count, dtype=np.uint64)
    base = np.uint64(pin.data_ptr())
    off = lambda j: base + np.uint64(8) * (t * np.uint64(per) + np.uint64(j * b * r))
    offs = lambda j: base + np.uint64(8) * (t * np.uint64(per) + np.uint64(4 * b * r + j * r * r))
    full = lambda v: np.full(count, v, dtype=np.int32)
    uo = np.uint64(U.data_ptr()) + np.uint64(8 * kmax * b) * t
    vo = np.uint64(V.data_ptr()) + np.uint64(8 * kmax * b) * t
    return (full(b), full(r), full(r), off(0), full(b), off(1), full(b), offs(0), full(r), off(2), full(b),
            offs(1), full(r), off(3), full(b), kmax, tol, uo, full(b), vo, full(b), sigma.data_ptr(), kout.data_ptr())


def run_round(count=20000, b=1024, rs=(8, 16, 32), tol=1e-8, steps=10, warmup=2):
    """The product of two low-rank blocks recompressed to rank <= r / 2 (fused
    core, batched truncated SVD, new bases) on device-resident N(0,1)
    operands: one-shot calls (host scheduling included), their device time,
    and replays of the plan form."""
    import torch
    from paper_2311_07602_amd import inputs, lrbg
    stream = torch.cuda.current_stream()
    out = []
    for r in rs:
        kmax = max(r // 2, 1)
        per = 4 * b * r + 2 * r * r
        pin = inputs.device_normal(count * per, seed=17 + r)
        U = torch.empty(count, kmax, b, dtype=torch.float64, device="cuda")
        V = torch.empty_like(U)
        sigma = torch.empty(count * kmax, dtype=torch.float64, device="cuda")
        kout = torch.empty(count, dtype=torch.int32, device="cuda")
        args = round_args(pin, per, count, b, r, kmax, tol, U, V, sigma, kout)
        call = lambda: lrbg.lr_batched_lrmult_round(*args, stream=stream)
        ms = time_calls(call, steps, warmup, stream)        # host-inclusive: schedules built per call
        # device time: hold the stream in a device-side sleep while the host enqueues, then
        # bracket only the enqueued work with events
        dev = []
        for _ in range(3):
            torch.cuda._sleep(int(2e8))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            dev.append(e0.elapsed_time(e1))
        # plan form: scheduled once, each call one graph replay
        plan = lrbg.RoundPlan(*args)
        pms = time_calls(lambda: plan.execute(stream), steps, warmup, stream)
        plan.close()
        out.append({"b": b, "r": r, "kmax": kmax, "ms_per_call": round(ms, 4), "device_ms": round(min(dev), 4),
                    "plan_ms_per_call": round(pms, 4)})
        log(f"[bench] recompressed product b={b} r={r}: {ms:.4f} ms per call, {min(dev):.4f} ms on the device, "
            f"{pms:.4f} ms per plan replay")
        del pin, U, V
        torch.cuda.empty_cache()
    return {"workload": f"{count} x (A_U A_X A_V^T)(B_U B_X B_V^T) recompressed to rank <= r/2 (tol {tol}), FP64, "
                        f"lr_batched_lrmult_round calls (fused core, batched SVD, two basis updates) and replays of its plan form",
            "sizes": out}


def lradd_work(b, ra, rb, k):
    """Useful FP64 flops and compulsory HBM bytes of one rounded addition:
    Householder QR of both b x s stacked bases (2 b s^2 - 2 s^3 / 3 each),
    the core (E = R_U diag(A_X, B_X): 2 s (ra^2 + rb^2); M = E R_V^T: 2 s^3),
    and the two new bases Q [X_k; 0] (4 k (b s - s^2 / 2) each; the SVD's
    iterations are not counted); bytes: the four bases and two cores read
    once, U, V, sigma and kout written once."""
    s = ra + rb
    flops = 2 * (2.0 * b * s * s - 2.0 * s ** 3 / 3) + 2.0 * s * (ra * ra + rb * rb) + 2.0 * s ** 3 \
        + 2 * 4.0 * k * (b * s - s * s / 2.0)
    bytes_ = 8.0 * (2 * b * ra + 2 * b * rb + ra * ra + rb * rb + 2 * b * k + k) + 4.0
    return flops, bytes_


def run_add(count=20000, b=1024, rs=(8, 16, 32), tol=1e-8, steps=5, warmup=2):
    """The rounded addition of two rank-r blocks (stacked rank 2r) recompressed
    to rank <= r on device-resident N(0,1) operands: QR of both stacked bases,
    the core, its truncated SVD and the new bases; one-shot calls (host
    scheduling included) and their device time."""
    import torch
    from paper_2311_07602_amd import inputs, lrbg
    stream = torch.cuda.current_stream()
    out = []
    for r in rs:
        kmax = r
        per = 4 * b * r + 2 * r * r
        pin = inputs.device_normal(count * per, seed=27 + r)
        U = torch.empty(count, kmax, b, dtype=torch.float64, device="cuda")
        V = torch.empty_like(U)
        sigma = torch.empty(count * kmax, dtype=torch.float64, device="cuda")
        kout = torch.empty(count, dtype=torch.int32, device="cuda")
        args = round_args(pin, per, count, b, r, kmax, tol, U, V, sigma, kout)
        call = lambda: lrbg.lr_batched_lradd_round(*args, stream=stream)
        ms = time_calls(call, steps, warmup, stream)
        dev = []
        for _ in range(3):
            torch.cuda._sleep(int(2e8))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            dev.append(e0.elapsed_time(e1))
        f1, b1 = lradd_work(b, r, r, kmax)
        dms = min(dev)
        roof = max(f1 * count / (PEAK_FP64_TFLOPS * 1e12), b1 * count / (PEAK_HBM_GBS * 1e9)) * 1e3
        out.append({"b": b, "r": r, "kmax": kmax, "ms_per_call": round(ms, 4), "device_ms": round(dms, 4),
                    "GFLOP/s": round(f1 * count / dms / 1e6, 1), "GB/s": round(b1 * count / dms / 1e6, 1),
                    "roofline_ms": round(roof, 4), "frac_of_roofline_time": round(roof / dms, 4),
                    "kept_rank_mean": round(float(kout.double().mean()), 2)})
        log(f"[bench] rounded addition b={b} r={r}: {ms:.4f} ms per call, {dms:.4f} ms on the device")
        del pin, U, V
        torch.cuda.empty_cache()
    return {"workload": f"{count} x (A_U A_X A_V^T + B_U B_X B_V^T), both of rank r, recompressed to rank <= r "
                        f"(tol {tol}), FP64, lr_batched_lradd_round calls (QR of both stacked bases, core, batched "
                        f"SVD, new bases)", "bound": "fp64 vector ALU (78.6 TFLOP/s) for r >= 16",
            "sizes": out}


def run_blr(nbs=(32, 64, 128), b=512, r=8, nrhs=8, steps=20, warmup=3):
    """Weakly admissible BLR matrix times 8 right-hand sides (rank 8), the
    application of the paper's evaluation; one captured two-level plan per
    size (INNER products into the stacked right-hand sides, then one
    DENSE_TS per block row over [A_ii | U_i])."""
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    stream = torch.cuda.current_stream()
    out = []
    for nb in nbs:
        m = workloads.blr(nb, b, r, nrhs)
        f, by = m.work()
        plan = m.plan(flags=lrbg.LRBG_PLAN_UNTIMED)
        ms, _ = time_plan(plan, steps, warmup, stream)
        m.close()
        del m
        torch.cuda.empty_cache()
        roof = max(f / (PEAK_FP64_TFLOPS * 1e12), by / (PEAK_HBM_GBS * 1e9)) * 1e3
        out.append({"N": nb * b, "blocks": nb, "ms_per_step": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1),
                    "GB/s": round(by / ms / 1e6, 1), "frac_of_roofline_time": round(roof / ms, 4)})
        log(f"[bench] blr N={nb * b}: {ms:.4f} ms, {by / ms / 1e6:.0f} GB/s")
    return {"workload": f"Y = A X, A weakly admissible BLR (blocks of {b}, rank {r}, dense diagonal), X with "
                        f"{nrhs} columns, FP64, N(0,1) blocks", "bound": "hbm", "sizes": out}


def run_serving(budget=64e9, slots=8, sat_requests=400, warm=200, measured=2000, rhos=(0.5, 0.7, 0.9),
                per_bucket=128, grouped_gflops=None, mix_gflops=None):
    """Continuous-batching loop over a device-resident operand pool: the
    saturated request rate first (all requests queued at t=0), then Poisson
    arrivals at rho x that rate for each rho; latency is arrival ->
    completion, over the `measured` requests after `warm` warm-up ones."""
    import torch
    from paper_2311_07602_amd import serve
    t0 = time.perf_counter()
    pool = serve.ResidentPool(per_bucket=per_bucket)
    torch.cuda.synchronize()
    log(f"[bench] serving pool: {pool.nbytes / 1e9:.1f} GB resident in {time.perf_counter() - t0:.1f} s")
    ex = serve.GpuExecutor(pool, slots=slots)
    serve.Scheduler(ex, budget, slots).run(serve.make_requests(50, float("inf"), seed=100))   # warm-up
    torch.cuda.synchronize()
    sat = serve.summarize(serve.Scheduler(ex, budget, slots).run(
        serve.make_requests(sat_requests, float("inf"), seed=101)))
    if grouped_gflops:
        sat["of_grouped_kernel_rate"] = round(sat["GFLOP/s"] / grouped_gflops, 3)
    if mix_gflops:
        sat["of_grouped_rate_same_mix"] = round(sat["GFLOP/s"] / mix_gflops, 3)
    mu = sat["requests_per_s"]
    loads = []
    for j, rho in enumerate(rhos):
        reqs = serve.make_requests(warm + measured, rho * mu, seed=102 + j)
        sch = serve.Scheduler(ex, budget, slots)
        recs = sch.run(reqs)
        loads.append({"rho": rho, "rate_per_s": round(rho * mu, 2), "warmup_requests": warm,
                      **serve.summarize(recs, skip=warm), "max_resident_GB": round(sch.max_resident / 1e9, 2)})
        log(f"[bench] serving rho={rho}: {loads[-1]}")
    del ex, pool
    torch.cuda.empty_cache()
    return {"workload": "Poisson arrivals, requests of 16..2048 instances (A.U and V1^T.U2 each, (b,r) as the "
                        "uneven batch), FP64 or BF16x3 with p=0.5, operands from a device-resident pool of "
                        f"{per_bucket} blocks per (b,r) bucket, HBM budget {budget / 1e9:.0f} GB, {slots} streams",
            "saturated": sat, "offered_load": loads}


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM
    traffic counters (FETCH_SIZE / WRITE_SIZE) of the profiled kernels."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="grouped", choices=["grouped", "lrmult", "chain_recomp", "grouped_bf16x3",
                                                            "lrmult_round", "lradd"],
                    help="grouped: the uneven batch (default); lrmult: one (b, r) of the paper's fused product; "
                         "chain_recomp: the recompression level of the low-rank chain alone; grouped_bf16x3, "
                         "lrmult_round, lradd: one workload of the extras (the last two at --lr-b, --lr-r)")
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--lr-b", type=int, default=2048)
    ap.add_argument("--lr-r", type=int, default=32)
    ap.add_argument("--tune-cache", default=DEFAULT_TUNE)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--dual", action="store_true", help="dual-role persistent workgroups (one matrix-core-bound "
                    "and one memory-bound workgroup per CU)")
    ap.add_argument("--lpt", action="store_true", help="longest-first tile order instead of the mixed "
                    "compute-/memory-bound order")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the batched products are "
              f"independent per instance and shard across GPUs without communication; the benchmark "
              f"measures one GPU's share.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_07602_amd import lrbg
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lrbg.load()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.config == "lrmult":
        print(json.dumps(run_lrmult_config(args)), flush=True)
        return
    if args.config == "chain_recomp":
        print(json.dumps(run_chain_recomp_config(args)), flush=True)
        return
    # single workloads of the extras, for profiling one at a time
    if args.config == "grouped_bf16x3":
        print(json.dumps(run_grouped_bf16x3(args.count, args.steps, args.warmup)), flush=True)
        return
    if args.config == "lrmult_round":
        print(json.dumps(run_round(args.count, args.lr_b, (args.lr_r,), steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.config == "lradd":
        print(json.dumps(run_add(args.count, args.lr_b, (args.lr_r,), steps=args.steps, warmup=args.warmup)), flush=True)
        return
    line = run_grouped(args)
    if not args.no_extras:
        log("[bench] extra workloads ...")
        line["extra"] = {"dense_uniform": run_dense_uniform(), "chain_fp64": run_chain(),
                         "chain_bf16x3": run_chain(prec="bf16x3"), "uneven_batch_bf16x3": run_grouped_bf16x3()}
        # the serving loop allocates each request's outputs: run it before the large workloads
        # below so that the allocator's cache, not fresh device allocations, serves them
        log("[bench] serving ...")
        g3 = line["extra"]["uneven_batch_bf16x3"]["GFLOP/s"]
        # requests are FP64 or BF16x3 with equal probability: the batch rate of
        # that mix, by time, is the harmonic mean of the two batch rates
        line["extra"]["serving"] = run_serving(grouped_gflops=line["value"],
                                               mix_gflops=2.0 / (1.0 / line["value"] + 1.0 / g3))
        log("[bench] vendor batched DGEMM on the uneven batch ...")
        wv = None
        try:
            from paper_2311_07602_amd import workloads
            wv = workloads.grouped(args.count, seed=3)
            vg = run_vendor_grouped(wv)
            vg["speedup_of_grouped_kernel"] = round(vg["ms_per_step"] / line["ms_per_step"], 2)
            line["extra"]["vendor_uneven_batch"] = vg
        finally:
            del wv
            import torch
            torch.cuda.empty_cache()
        log("[bench] paper-shape low-rank products ...")
        line["extra"]["lrmult_paper_shapes"] = run_lrmult_paper()
        log("[bench] recompressed low-rank products ...")
        line["extra"]["lrmult_round"] = run_round()
        log("[bench] rounded additions of low-rank blocks ...")
        line["extra"]["lradd_round"] = run_add()
        log("[bench] BLR matrix x 8 right-hand sides ...")
        line["extra"]["blr_matvec"] = run_blr()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
