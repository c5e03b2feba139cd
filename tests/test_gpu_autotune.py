"""The autotuners on a small mixed sample: the isolation tuner
(lrbg_autotune) over FP64 and split-precision buckets, then the in-mix
search (lrbg_autotune_mix) over the FP64 part.  Checks that each cache
parses, that every pick's time is that variant's own isolated time, that a
plan built from the cache runs exactly the picked variants, and that its
results pass the oracle bar."""
import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import lrbg, workloads

from gpu_util import ref_dense_ts, ref_inner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


def _parse(path):
    picks, cands, mix = {}, {}, []
    for line in open(path):
        f = line.split()
        if not f:
            continue
        if f[0] == "#cand":
            key = tuple(int(x) for x in f[1:5])
            cands.setdefault(key, {})[f[5]] = float(f[6])
        elif f[0] == "#mix":
            mix.append(f)
        elif not f[0].startswith("#"):
            key = tuple(int(x) for x in f[:4])
            assert key not in picks, key
            picks[key] = (f[4], float(f[5]))
    return picks, cands, mix


def _bucket(op, prec, b, r):
    rb = lambda x, lo: max(lo, 1 << (x - 1).bit_length())
    return (op, prec, rb(b, 64), rb(r, 8))


def test_isolation_then_mix_tuning(tmp_path):
    import torch
    w = workloads.grouped(240, seed=21)
    w3 = workloads.grouped(120, seed=22, prec="bf16x3")
    names = set(lrbg.lrbg_variant_names())
    iso = str(tmp_path / "iso.tune")
    lrbg.lrbg_autotune(list(w.descs) + list(w3.descs), iso, reps=1)
    picks, cands, _ = _parse(iso)
    want = {_bucket(0, p, b, r) for p, ww in ((0, w), (1, w3)) for b, r in ww.meta["shapes"]} | \
           {_bucket(1, p, b, r) for p, ww in ((0, w), (1, w3)) for b, r in ww.meta["shapes"]}
    assert set(picks) == want
    assert any(k[1] == 1 for k in picks)                  # split-precision buckets tuned
    for key, (name, ms) in picks.items():
        assert name in names
        assert ms == min(cands[key].values()) == cands[key][name]

    mixed = str(tmp_path / "mix.tune")
    lrbg.lrbg_autotune_mix(list(w.descs), iso, mixed, reps=2, passes=1, flags=lrbg.LRBG_PLAN_SCHED_MIX)
    mpicks, mcands, mix = _parse(mixed)
    assert mcands == cands                                # isolated times carried over
    assert set(mpicks) == set(picks)                      # split-precision picks kept
    for key, (name, ms) in mpicks.items():
        assert name in names
        assert ms == mcands[key][name]                    # every time belongs to its own variant
        if key[1] == 1:
            assert name == picks[key][0]
    for f in mix:
        assert f[6] == "->" and f[7] in names and f[8] == "batch_ms"
    print(f"{len(mix)} mix trials, {sum(f[-1] == 'kept' for f in mix)} kept", flush=True)

    # a plan from the refined cache runs exactly its picks, and passes the oracle bar
    descs = list(w.descs) + list(w3.descs)
    ran = lrbg.lrbg_schedule_variants(descs, mixed)
    for d, name in zip(descs, ran):
        shape = (d.m, d.n, d.k)
        b, r = (shape[0], shape[1]) if d.op == 0 else (shape[2], max(shape[0], shape[1]))
        assert name == mpicks[_bucket(d.op, d.prec, b, r)][0]
    plan = lrbg.Plan(descs, tune_cache=mixed, flags=lrbg.LRBG_PLAN_SCHED_MIX)
    plan.execute(torch.cuda.current_stream())
    torch.cuda.synchronize()
    plan.close()
    for ww, tol in ((w, 1e-13), (w3, 1e-6)):
        worst = 0.0
        for i in range(0, len(ww.meta["shapes"]), 7):
            o = workloads.grouped_operands(ww, i)
            Cref, Dc = ref_dense_ts(o["A"], o["U"])
            Tref, Dt = ref_inner(o["V1"], o["U2"])
            worst = max(worst, oracle.normalized_error(o["C"], Cref, Dc), oracle.normalized_error(o["T"], Tref, Dt))
        assert worst <= tol, (ww.meta["prec"], worst)
