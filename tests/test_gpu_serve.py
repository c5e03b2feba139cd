"""Serving on the GPU: a request's result is the same alone and in the mix."""
import numpy as np
import pytest

from paper_2311_07602_amd import lrbg, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


def test_alone_equals_in_mix_bitwise():
    reqs = serve.make_requests(16, float("inf"), seed=11, nmax=96)
    watch = [2, 5, 9]
    ex = serve.GpuExecutor(slots=4, keep_outputs=watch)
    recs = serve.Scheduler(ex, budget_bytes=64e9, slots=4).run(reqs)
    assert all(r.status == "ok" for r in recs)
    mixed = {k: v.copy() for k, v in ex.outputs.items()}
    assert set(mixed) == set(watch)
    for rid in watch:
        alone = serve.GpuExecutor(slots=1, keep_outputs=[rid])
        req = reqs[rid]
        one = serve.Request(req.rid, 0.0, req.shapes, req.prec, req.seed)
        r = serve.Scheduler(alone, budget_bytes=64e9, slots=1).run([one])
        assert r[0].status == "ok"
        assert np.array_equal(alone.outputs[rid], mixed[rid]), rid
        assert np.all(np.isfinite(mixed[rid]))


def test_short_poisson_run_reports_latency():
    reqs = serve.make_requests(40, 400.0, seed=12, nmax=256)
    ex = serve.GpuExecutor(slots=4)
    recs = serve.Scheduler(ex, budget_bytes=16e9, slots=4).run(reqs)
    s = serve.summarize(recs)
    assert s["completed"] == 40 and s["p99_ms"] >= s["p50_ms"] > 0
