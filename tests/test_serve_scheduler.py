"""Serving-loop policy on the CPU: a simulated executor and clock stand in
for the GPU (they exist only in this test)."""
import numpy as np
import pytest

from paper_2311_07602_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def idle(self, next_arrival, ex):
        cands = [x for x in (next_arrival, ex.next_completion()) if x is not None]
        self.t = max(self.t, min(cands)) if cands else self.t + 1e-3


class FakeExecutor:
    """Each request takes flops / rate seconds; checks the limits at launch."""

    def __init__(self, clock, budget, slots, rate=40e12, fail_ids=(), fail_on_release=()):
        self.clock, self.budget, self.slots, self.rate = clock, budget, slots, rate
        self.fail_ids, self.fail_on_release = set(fail_ids), set(fail_on_release)
        self.running = {}
        self.max_conc = 0
        self.order = []

    def launch(self, req):
        if req.rid in self.fail_ids:
            raise RuntimeError("injected launch failure")
        assert len(self.running) < self.slots
        assert sum(r.nbytes for r, _ in self.running.values()) + req.nbytes <= self.budget
        h = object()
        self.running[h] = (req, self.clock.now() + req.flops / self.rate)
        self.max_conc = max(self.max_conc, len(self.running))
        self.order.append(req.rid)
        return h

    def query(self, h):
        return self.clock.now() >= self.running[h][1]

    def release(self, h):
        req, _ = self.running.pop(h)
        if req.rid in self.fail_on_release:
            raise RuntimeError("injected device error")

    def next_completion(self):
        return min((t for _, t in self.running.values()), default=None)


def run(reqs, budget=64e9, slots=8, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, budget, slots, **kw)
    sch = serve.Scheduler(ex, budget_bytes=budget, slots=slots, clock=clock)
    return sch.run(reqs), ex, sch


def test_requests_reproducible():
    a = serve.make_requests(50, 100.0, seed=3)
    b = serve.make_requests(50, 100.0, seed=3)
    c = serve.make_requests(50, 100.0, seed=4)
    assert all(x.arrival == y.arrival and np.array_equal(x.shapes, y.shapes) and x.prec == y.prec
               and x.seed == y.seed for x, y in zip(a, b))
    assert any(not np.array_equal(x.shapes, y.shapes) for x, y in zip(a, c))
    for r in a:
        assert 16 <= r.n <= 2048
        assert np.all(r.shapes[:, 1] <= r.shapes[:, 0] // 2)
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) >= 0)


def test_all_complete_fifo_and_latency():
    reqs = serve.make_requests(200, 2000.0, seed=1)
    recs, ex, sch = run(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.order == sorted(ex.order)                        # FIFO admission
    for r in recs:
        assert r.admitted >= r.arrival and r.done >= r.admitted
        assert r.latency >= r.flops / 40e12 - 1e-12
    s = serve.summarize(recs)
    assert s["completed"] == 200 and s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_and_slots_never_exceeded():
    reqs = serve.make_requests(150, float("inf"), seed=2)      # all at once
    budget = 12e9
    recs, ex, sch = run([r for r in reqs if r.nbytes <= budget], budget=budget, slots=3)
    assert sch.max_resident <= budget
    assert ex.max_conc <= 3
    assert ex.max_conc >= 2                                    # work overlaps
    assert all(r.status == "ok" for r in recs)


def test_oversized_request_rejected_others_served():
    reqs = serve.make_requests(40, 500.0, seed=5)
    budget = 2e9
    recs, ex, sch = run(reqs, budget=budget, slots=4)
    for req, rec in zip(reqs, recs):
        if req.nbytes > budget:
            assert rec.status == "rejected"
        else:
            assert rec.status == "ok"
    assert any(r.status == "rejected" for r in recs) and any(r.status == "ok" for r in recs)


def test_launch_failure_frees_budget_and_continues():
    reqs = serve.make_requests(60, float("inf"), seed=6, nmax=200)
    recs, ex, sch = run(reqs, budget=64e9, slots=2, fail_ids={3, 10}, fail_on_release={20})
    assert recs[3].status == "failed" and recs[10].status == "failed" and recs[20].status == "failed"
    assert sum(r.status == "ok" for r in recs) == 57
    assert sch.resident == 0


def test_budget_waits_then_admits():
    reqs = serve.make_requests(30, float("inf"), seed=7, nmin=500, nmax=600)
    biggest = max(r.nbytes for r in reqs)
    recs, ex, sch = run(reqs, budget=biggest * 1.5, slots=8)
    assert all(r.status == "ok" for r in recs)
    assert ex.max_conc == 1 or sch.max_resident <= biggest * 1.5
    waited = [r for r in recs if r.admitted > r.arrival]
    assert waited, "a tight budget must make requests wait"


def test_layout_offsets_aligned_and_disjoint():
    reqs = serve.make_requests(5, 10.0, seed=8)
    for r in reqs:
        off_in, off_out, nin, es, nout = serve.request_layout(r.shapes, r.prec)
        assert np.all(off_in % 256 == 0) and np.all(off_out % 256 == 0)
        assert np.all(np.diff(off_in) > 0) and off_in[-1] < nin
        assert r.nbytes == nin + nout


def test_resident_pool_descriptors_validate_on_host():
    """The descriptors a request is served with (built over a resident pool,
    here on the host) pass the library's validation as one level, and the
    library's accounting equals the request's own flop count."""
    from paper_2311_07602_amd import lrbg
    pool = serve.ResidentPool(per_bucket=2, seed=3, device="cpu")
    assert len(pool.buckets) == 22
    for req in serve.make_requests(6, float("inf"), seed=21, nmax=300):
        off_out, nout = serve.output_layout(req.shapes)
        slots = req.slots(pool.per_bucket)
        assert slots.min() >= 0 and slots.max() < pool.per_bucket
        assert np.array_equal(slots, req.slots(pool.per_bucket))           # fixed by the request's seed
        src = pool.f64 if req.prec == "fp64" else pool.f32
        ops = pool.operand_offsets(req.shapes, slots)
        # every operand lies inside the pool
        b = req.shapes[:, 0]; r = req.shapes[:, 1]
        ends = ops + np.stack([b * b, b * r, b * r, b * r], axis=1)
        assert ops.min() >= 0 and ends.max() <= src.numel()
        arr = serve.GpuExecutor._descs(req, src.data_ptr(), src.element_size(), ops, 1 << 44, off_out)
        descs = [lrbg.lrbg_desc.from_buffer_copy(arr[i].tobytes()) for i in range(len(arr))]
        st = lrbg.lrbg_schedule_stats(descs)
        assert st["levels"] == 1 and st["products"] == 2 * req.n
        assert st["useful_flops"] == pytest.approx(req.flops, rel=1e-12)
