"""Summaries of rocprofv3 runs of the grouped kernel.

A summary (markdown, committed under profiles/) holds the kernel-trace
statistics of the benchmark command and the HBM traffic per launch from two
counter runs (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled
by what the same counter reads for a plain device copy of known size.  It is
tagged with a digest of the kernel sources and the tuning cache, so a
benchmark can tell whether the counters still describe the kernel it runs.

    python -m paper_2311_07602_amd.profiling summarize --kt DIR --fetch DIR \\
        --write DIR --cal-fetch DIR --cal-write DIR --out FILE.md \\
        --kernel lrbg_grouped_kernel --flops F --bytes B --cmd "..." ...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/lrbg_kernels.hip", "csrc/lrbg_tiles.h", "csrc/lrbg_internal.h", "tune/mi355x.tune"]


def source_digest(sources=None) -> str:
    h = hashlib.sha256()
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _csv(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(kt_dir: str, kernel: str) -> dict:
    for row in csv.DictReader(open(_csv(kt_dir, "kernel_stats.csv"))):
        if kernel in row["Name"]:
            return {"calls": int(row["Calls"]), "avg_ns": float(row["AverageNs"]),
                    "min_ns": float(row["MinNs"]), "max_ns": float(row["MaxNs"])}
    raise KeyError(kernel)


def dispatch_durations_ns(kt_dir: str, kernel: str) -> List[float]:
    """Duration of every dispatch of `kernel`, in dispatch order, from the
    kernel trace (end minus start timestamp, ns)."""
    rows = list(csv.DictReader(open(_csv(kt_dir, "kernel_trace.csv"))))
    if not rows:
        raise KeyError(kernel)
    cols = rows[0].keys()
    start = next(c for c in cols if c.lower().startswith("start_timestamp"))
    end = next(c for c in cols if c.lower().startswith("end_timestamp"))
    name = next(c for c in cols if c.lower() == "kernel_name")
    hits = sorted((int(r[start]), int(r[end])) for r in rows if kernel in r[name])
    if not hits:
        raise KeyError(kernel)
    return [float(e - s) for s, e in hits]


def counter_per_dispatch(pmc_dir: str, kernel: str, counter: Optional[str] = None) -> List[float]:
    """Per-dispatch value of a counter (summed over its instances), in
    dispatch order; `counter` selects one counter of a multi-counter run."""
    per: Dict[str, float] = {}
    for row in csv.DictReader(open(_csv(pmc_dir, "counter_collection.csv"))):
        if counter is not None and row.get("Counter_Name") != counter:
            continue
        if kernel in row["Kernel_Name"]:
            per[row["Dispatch_Id"]] = per.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    if not per:
        raise KeyError(kernel)
    return [per[k] for k in sorted(per, key=int)]


def summarize(args) -> str:
    st = kernel_stats(args.kt, args.kernel)
    durs = dispatch_durations_ns(args.kt, args.kernel)
    if args.skip >= len(durs):
        raise ValueError(f"--skip {args.skip} leaves no dispatch of {len(durs)}")
    timed = durs[args.skip:]
    med_ms = statistics.median(timed) * 1e-6
    fetch = counter_per_dispatch(args.fetch, args.kernel)
    write = counter_per_dispatch(args.write, args.kernel)
    cal_f = statistics.median(counter_per_dispatch(args.cal_fetch, args.cal_kernel))
    cal_w = statistics.median(counter_per_dispatch(args.cal_write, args.cal_kernel))
    fs = args.cal_bytes / (cal_f * 1024.0)
    ws = args.cal_bytes / (cal_w * 1024.0)
    f_b = statistics.median(fetch) * 1024.0 * fs
    w_b = statistics.median(write) * 1024.0 * ws
    avg_ms = st["avg_ns"] * 1e-6
    timed_avg_ms = statistics.fmean(timed) * 1e-6
    mfma = None
    if args.mfma:
        # executed FP64 matrix-core flops (the counter is in units of 512 flops) and the share of
        # SIMD-cycles the matrix cores were busy (busy cycles summed over SIMDs / (active cycles x SIMDs))
        mops = statistics.median(counter_per_dispatch(args.mfma, args.kernel, "SQ_INSTS_VALU_MFMA_MOPS_F64"))
        busy = statistics.median(counter_per_dispatch(args.mfma, args.kernel, "SQ_VALU_MFMA_BUSY_CYCLES"))
        active = statistics.median(counter_per_dispatch(args.mfma, args.kernel, "GRBM_GUI_ACTIVE"))
        # GRBM_GUI_ACTIVE is summed over the accelerator dies: per die it is the
        # kernel's duration in shader-clock cycles, which also gives the clock
        per_die = active / args.xcds
        mfma = {"flops": mops * 512.0, "util": busy / (per_die * args.simds) if active else float("nan"),
                "clock_ghz": per_die / (med_ms * 1e-3) / 1e9}
    lines = [
        f"# {args.kernel}: {args.workload}",
        "",
        f"rocprofv3 summaries of {args.kernel} in the benchmark command below (one launch per step).",
        "",
        "## Commands",
        "",
    ]
    for c in args.cmd:
        lines.append(f"    {c}")
    lines += [
        "",
        "## Kernel trace (--kernel-trace --stats)",
        "",
        f"| kernel | calls | average ms | min ms | max ms |",
        f"|---|---|---|---|---|",
        f"| {args.kernel} | {st['calls']} | {avg_ms:.4f} | {st['min_ns'] * 1e-6:.4f} | {st['max_ns'] * 1e-6:.4f} |",
        "",
        f"Timed dispatches (the {len(timed)} after the first {args.skip}, which are the benchmark's warm-up "
        f"launches; from the per-dispatch kernel trace): median {med_ms:.4f} ms, mean {timed_avg_ms:.4f} ms, "
        f"min {min(timed) * 1e-6:.4f} ms, max {max(timed) * 1e-6:.4f} ms.",
        "",
        "## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE; KiB per dispatch)",
        "",
        f"| counter | kernel (median of {len(fetch)}) | copy of {args.cal_bytes / 2**30:.0f} GiB | scale |",
        f"|---|---|---|---|",
        f"| FETCH_SIZE | {statistics.median(fetch):.0f} | {cal_f:.0f} | {fs:.4f} |",
        f"| WRITE_SIZE | {statistics.median(write):.0f} | {cal_w:.0f} | {ws:.4f} |",
        "",
        f"Scaled traffic per launch: read {f_b / 1e9:.3f} GB + write {w_b / 1e9:.3f} GB = "
        f"{(f_b + w_b) / 1e9:.3f} GB; algorithmic (compulsory) bytes {args.bytes / 1e9:.3f} GB "
        f"(ratio {(f_b + w_b) / args.bytes:.3f}).",
        f"Achieved (median timed dispatch): {args.flops / (med_ms * 1e-3) / 1e12:.2f} TFLOP/s useful "
        f"({args.flops / (med_ms * 1e-3) / 78.6e12 * 100:.1f}% of 78.6), "
        f"{args.bytes / (med_ms * 1e-3) / 1e9:.0f} GB/s algorithmic "
        f"({args.bytes / (med_ms * 1e-3) / 8.0e12 * 100:.1f}% of 8000).",
        "",
    ]
    if mfma:
        lines += [
            "## FP64 matrix-core work (--pmc SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE)",
            "",
            f"Executed FP64 MFMA flops per launch: {mfma['flops'] / 1e9:.2f} GFLOP (counter x 512) against "
            f"{args.flops / 1e9:.2f} GFLOP useful (ratio {mfma['flops'] / args.flops:.3f}: the excess is padding "
            f"of partial tiles); executed rate {mfma['flops'] / (med_ms * 1e-3) / 1e12:.2f} TFLOP/s at the median "
            f"timed dispatch.  Shader clock during the kernel {mfma['clock_ghz']:.2f} GHz (GRBM_GUI_ACTIVE / "
            f"{args.xcds} dies / duration), so the FP64 matrix-core peak at that clock is "
            f"{78.6 * mfma['clock_ghz'] / 2.4:.1f} TFLOP/s; matrix cores busy {mfma['util'] * 100:.1f}% of "
            f"SIMD-cycles (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / {args.xcds} x {args.simds} SIMDs)).",
            "",
        ]
    lines += [
        "## Machine-readable",
        "",
        "```",
        f"kernel: {args.kernel}",
        f"source_digest: {args.digest or source_digest(args.sources.split(',') if args.sources else None)}",
        f"avg_duration_ms: {avg_ms:.6f}",
        f"median_timed_duration_ms: {med_ms:.6f}",
        f"timed_dispatches: {len(timed)}",
        f"algorithmic_flops: {args.flops:.6g}",
        f"algorithmic_bytes: {args.bytes:.6g}",
        f"fetch_bytes_per_launch: {f_b:.6g}",
        f"write_bytes_per_launch: {w_b:.6g}",
        f"traffic_bytes_per_launch: {f_b + w_b:.6g}",
    ]
    if mfma:
        lines += [f"mfma_f64_flops_per_launch: {mfma['flops']:.6g}", f"mfma_busy_frac: {mfma['util']:.4f}",
                  f"shader_clock_ghz: {mfma['clock_ghz']:.3f}"]
    lines += [
        "```",
        "",
    ]
    text = "\n".join(lines)
    with open(args.out, "w") as f:
        f.write(text)
    return text


def kernels_table(args) -> str:
    """A pipeline of several kernels (one call = several launches): per
    kernel, the dispatches in the kernel trace, their average duration and
    share of the traced kernel time, and the median scaled HBM traffic per
    dispatch from the two counter runs."""
    rows = []
    for row in csv.DictReader(open(_csv(args.kt, "kernel_stats.csv"))):
        if args.prefix in row["Name"]:
            rows.append((row["Name"], int(row["Calls"]), float(row["AverageNs"]), float(row["TotalDurationNs"])))
    total = sum(r[3] for r in rows) or 1.0
    cal_f = statistics.median(counter_per_dispatch(args.cal_fetch, args.cal_kernel))
    cal_w = statistics.median(counter_per_dispatch(args.cal_write, args.cal_kernel))
    fs, ws = args.cal_bytes / (cal_f * 1024.0), args.cal_bytes / (cal_w * 1024.0)
    lines = [f"# {args.title}", "", "rocprofv3 summaries of the kernels one call launches, in the benchmark "
             "command below.", "", "## Commands", ""] + [f"    {c}" for c in args.cmd] + [
        "", "## Kernels (--kernel-trace --stats; --pmc FETCH_SIZE, then WRITE_SIZE, scaled by a 1 GiB copy)", "",
        "| kernel | dispatches | average ms | share of kernel time | read GB per dispatch | written GB per dispatch |",
        "|---|---|---|---|---|---|"]
    for name, calls, avg, tot in sorted(rows, key=lambda r: -r[3]):
        short = name.split("(")[0].replace("void ", "")
        try:
            f = statistics.median(counter_per_dispatch(args.fetch, name)) * 1024.0 * fs
            w = statistics.median(counter_per_dispatch(args.write, name)) * 1024.0 * ws
            tr = f"| {f / 1e9:.4f} | {w / 1e9:.4f} |"
        except (KeyError, statistics.StatisticsError):
            tr = "| - | - |"
        lines.append(f"| {short} | {calls} | {avg * 1e-6:.4f} | {tot / total * 100:.1f}% {tr}")
    lines += ["", "```", f"source_digest: {source_digest(args.sources.split(',') if args.sources else None)}", "```", ""]
    text = "\n".join(lines)
    with open(args.out, "w") as fh:
        fh.write(text)
    return text


def read_summary(path: str) -> Optional[dict]:
    if not os.path.exists(path):
        return None
    out, inside = {}, False
    for ln in open(path):
        ln = ln.rstrip("\n")
        if ln.strip() == "```":
            inside = not inside
            continue
        if inside and ":" in ln:
            k, v = ln.split(":", 1)
            out[k.strip()] = v.strip()
    return out or None


# Sources behind the fused low-rank product kernels (their own translation unit).
LRMULT_SOURCES = ["csrc/lrbg_lrmult.hip", "csrc/lrbg_tiles.h", "csrc/lrbg_internal.h", "tune/mi355x.tune"]


def current_traffic(path: str, sources=None) -> Optional[float]:
    """Traffic per launch from a summary, or None once the kernel sources or
    tuning cache have changed since the counters were taken."""
    s = read_summary(path)
    if not s or s.get("source_digest") != source_digest(sources):
        return None
    return float(s["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    sm = sub.add_parser("summarize")
    sm.add_argument("--kt", required=True)
    sm.add_argument("--fetch", required=True)
    sm.add_argument("--write", required=True)
    sm.add_argument("--cal-fetch", required=True)
    sm.add_argument("--cal-write", required=True)
    sm.add_argument("--cal-kernel", default="copyBuffer")
    sm.add_argument("--cal-bytes", type=float, default=float(1 << 30))
    sm.add_argument("--kernel", default="lrbg_grouped_kernel")
    sm.add_argument("--workload", default="")
    sm.add_argument("--flops", type=float, required=True)
    sm.add_argument("--bytes", type=float, required=True)
    sm.add_argument("--digest", default=None)
    sm.add_argument("--sources", default=None, help="comma list of sources (relative to the package) the digest covers")
    sm.add_argument("--mfma", default=None, help="counter run with SQ_INSTS_VALU_MFMA_MOPS_F64, "
                    "SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE")
    sm.add_argument("--simds", type=int, default=1024, help="SIMDs on the chip (MI355X: 256 CUs x 4)")
    sm.add_argument("--xcds", type=int, default=8, help="accelerator dies GRBM_GUI_ACTIVE is summed over")
    sm.add_argument("--skip", type=int, default=0, help="warm-up dispatches to leave out of the timed statistics")
    sm.add_argument("--cmd", action="append", default=[])
    sm.add_argument("--out", required=True)
    kt = sub.add_parser("kernels")
    for opt in ("--kt", "--fetch", "--write", "--cal-fetch", "--cal-write", "--out", "--title"):
        kt.add_argument(opt, required=True)
    kt.add_argument("--prefix", default="lrbg_")
    kt.add_argument("--cal-kernel", default="copyBuffer")
    kt.add_argument("--cal-bytes", type=float, default=float(1 << 30))
    kt.add_argument("--sources", default=None)
    kt.add_argument("--cmd", action="append", default=[])
    sub.add_parser("digest")
    a = ap.parse_args()
    if a.what == "digest":
        print(source_digest())
    elif a.what == "kernels":
        print(kernels_table(a))
    else:
        print(summarize(a))


if __name__ == "__main__":
    main()
