"""Regenerate the MI355X tuning cache (mi355x.tune) with the library's
autotuners, on a GPU:

    python -m paper_2311_07602_amd.tune.autotune [out_path]

1. In isolation (lrbg_autotune): every (op, prec, b, r) bucket of the uneven
   grouped batch in FP64 and in split BF16x3 precision, and the
   recompression bucket of the low-rank chain; every compatible tile variant
   of a bucket is timed on that bucket's own products.
2. In the mix (lrbg_autotune_mix): starting from those picks, a coordinate
   search over the FP64 uneven batch as the benchmark plans it (mixed tile
   order, one captured graph): one bucket's variant changed at a time, kept
   only if the whole batch replays faster.  The BF16x3 and recompression
   buckets keep their isolation picks (the FP64 batch does not contain them).

The written cache holds only what the tools produced: the isolated time of
every candidate, the whole-batch times of every mix trial, and each bucket's
pick with its own isolated time.
"""
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "mi355x.tune")


def main(out=DEFAULT, count=20000, reps=3, mix_reps=5, passes=3):
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    lrbg.load()
    w = workloads.grouped(count, seed=3)
    w3 = workloads.grouped(count, seed=4, prec="bf16x3")
    c = workloads.chain(1024, 512, 32)
    iso_descs = list(w.descs) + list(w3.descs) + list(c.descs[len(c.descs) // 2:])
    torch.cuda.synchronize()
    fd, iso = tempfile.mkstemp(suffix=".tune")
    os.close(fd)
    try:
        print(f"isolation: {len(iso_descs)} products", flush=True)
        lrbg.lrbg_autotune(iso_descs, iso, reps=reps)
        del w3, c, iso_descs
        torch.cuda.empty_cache()
        print("in the mix: the FP64 uneven batch", flush=True)
        lrbg.lrbg_autotune_mix(list(w.descs), iso, out, reps=mix_reps, passes=passes,
                               flags=lrbg.LRBG_PLAN_SCHED_MIX)
    finally:
        os.unlink(iso)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else DEFAULT)
