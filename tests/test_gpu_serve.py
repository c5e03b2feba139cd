"""Serving on the GPU: a request's result is the same alone and in the mix,
and every instance of the watched requests matches the oracle (FP64 and
split-precision requests, on the resident FP64 originals)."""
import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import lrbg, serve

from gpu_util import ref_dense_ts, ref_inner

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "bf16x3": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


@pytest.fixture(scope="module")
def pool():
    return serve.ResidentPool(per_bucket=3, seed=5)


def _check_against_oracle(pool, req, flat):
    worst = 0.0
    slots = req.slots(pool.per_bucket)
    for (b, r), slot, (C, T) in zip(req.shapes, slots, serve.request_outputs(req, flat)):
        A, U, V1, U2 = pool.host_operands(int(b), int(r), int(slot))
        Cref, Dc = ref_dense_ts(A, U)
        Tref, Dt = ref_inner(V1, U2)
        worst = max(worst, oracle.normalized_error(np.asfortranarray(C), Cref, Dc),
                    oracle.normalized_error(np.asfortranarray(T), Tref, Dt))
    return worst


def test_alone_equals_in_mix_and_oracle(pool):
    reqs = serve.make_requests(16, float("inf"), seed=11, nmin=4, nmax=40)
    watch = [r.rid for r in reqs if r.prec == "fp64"][:2] + [r.rid for r in reqs if r.prec == "bf16x3"][:2]
    assert {reqs[i].prec for i in watch} == {"fp64", "bf16x3"}
    ex = serve.GpuExecutor(pool, slots=4, keep_outputs=watch)
    recs = serve.Scheduler(ex, budget_bytes=64e9, slots=4).run(reqs)
    assert all(r.status == "ok" for r in recs)
    mixed = {k: v.copy() for k, v in ex.outputs.items()}
    assert set(mixed) == set(watch)
    for rid in watch:
        req = reqs[rid]
        print(f"request {rid}: {req.prec}, {req.n} instances", flush=True)
        alone = serve.GpuExecutor(pool, slots=1, keep_outputs=[rid])
        one = serve.Request(req.rid, 0.0, req.shapes, req.prec, req.seed)
        r = serve.Scheduler(alone, budget_bytes=64e9, slots=1).run([one])
        assert r[0].status == "ok"
        assert np.array_equal(alone.outputs[rid], mixed[rid]), rid
        worst = _check_against_oracle(pool, req, mixed[rid])
        print(f"  worst normalised error against the oracle: {worst:.3e}", flush=True)
        assert worst <= TOL[req.prec], (rid, req.prec, worst)


def test_short_poisson_run_reports_latency(pool):
    reqs = serve.make_requests(40, 400.0, seed=12, nmax=256)
    ex = serve.GpuExecutor(pool, slots=4)
    recs = serve.Scheduler(ex, budget_bytes=16e9, slots=4).run(reqs)
    s = serve.summarize(recs)
    assert s["completed"] == 40 and s["p99_ms"] >= s["p50_ms"] > 0
