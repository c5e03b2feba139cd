"""Regenerate the MI355X tuning cache (mi355x.tune) with the library's
autotuner: every (op, prec, b, r) bucket of the uneven grouped batch, every
compatible tile variant, timed on the device.  Run on a GPU:

    python -m paper_2311_07602_amd.tune.autotune [out_path]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "mi355x.tune")


def main(out=DEFAULT, count=20000, reps=3):
    import torch
    from paper_2311_07602_amd import lrbg, workloads
    lrbg.load()
    w = workloads.grouped(count, seed=3)
    descs = list(w.descs)
    try:
        c = workloads.chain(1024, 512, 32)          # recompression buckets
        descs += c.descs[len(c.descs) // 2:]
    except Exception as e:                          # pragma: no cover - memory-limited hosts
        print("chain buckets skipped:", e, file=sys.stderr)
    torch.cuda.synchronize()
    lrbg.lrbg_autotune(descs, out, reps=reps)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else DEFAULT)
