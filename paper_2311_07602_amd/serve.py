"""Continuous-batching request loop for batched low-rank products.

A request is a batch of n low-rank instances (n uniform in 16..2048), each
with a block size b and rank r drawn like the uneven grouped batch and two
products, C = A U and T = V1^T U2, in FP64 or in the BF16x3 split precision
(per-request flag).  Requests arrive as a Poisson process.  The scheduler
keeps a FIFO queue and admits the head request as soon as a slot (a HIP
stream) is free and its device memory fits in the HBM budget; admitted
requests run concurrently on their streams, so work that arrives while
others are on the GPU overlaps with them on the device.  A request whose
memory alone exceeds the budget is rejected.  When a request completes its
memory returns to the budget and its latency (arrival to completion) is
recorded.

The scheduler core is independent of the GPU: it drives an executor
(``launch``/``query``/``release``) under a clock (``now``/``idle``), so its
policy is tested on the CPU with a simulated executor and clock.  The GPU
executor serves from a :class:`ResidentPool`: the low-rank blocks live in
device memory before any request arrives (FP64, and their FP32 roundings for
split-precision requests), and a request names, for each of its instances,
one resident block of its (b, r) bucket (drawn from the request's own seed,
so a request's operands never depend on the mix).  Admission allocates the
request's outputs, builds its descriptors and issues one grouped call on the
request's stream, then records a completion event; no operand is copied or
generated per request.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import inputs

SEED0 = (2311, 7602, 5)


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    shapes: np.ndarray             # (n, 2) int64: b, r per instance
    prec: str                      # "fp64" | "bf16x3"
    seed: int

    @property
    def n(self) -> int:
        return int(self.shapes.shape[0])

    @property
    def nbytes(self) -> int:
        lay = request_layout(self.shapes, self.prec)
        return lay[2] + lay[4]

    def slots(self, per_bucket: int) -> np.ndarray:
        """Resident block index (within its (b, r) bucket) of every instance."""
        rng = np.random.default_rng([*SEED0, 1, self.seed])
        return rng.integers(0, per_bucket, self.n)

    @property
    def flops(self) -> float:
        b = self.shapes[:, 0].astype(np.float64); r = self.shapes[:, 1].astype(np.float64)
        return float(np.sum(2.0 * b * b * r + 2.0 * b * r * r))


def request_layout(shapes: np.ndarray, prec: str, align: int = 256):
    """Byte offsets of each instance's operands (A, U, V1, U2) and outputs
    (C, T) inside one operand buffer and one output buffer."""
    es = 8 if prec == "fp64" else 4
    b = shapes[:, 0].astype(np.int64); r = shapes[:, 1].astype(np.int64)
    sizes_in = np.stack([b * b, b * r, b * r, b * r], axis=1).reshape(-1) * es
    sizes_out = np.stack([b * r, r * r], axis=1).reshape(-1) * 8
    pin = (sizes_in + align - 1) // align * align
    pout = (sizes_out + align - 1) // align * align
    off_in = np.concatenate([[0], np.cumsum(pin)[:-1]]) if len(pin) else np.zeros(0, np.int64)
    off_out = np.concatenate([[0], np.cumsum(pout)[:-1]]) if len(pout) else np.zeros(0, np.int64)
    return off_in, off_out, int(pin.sum()), es, int(pout.sum())


def make_requests(count: int, rate: float, seed: int = 0, nmin: int = 16, nmax: int = 2048,
                  p_bf16x3: float = 0.5, t0: float = 0.0) -> List[Request]:
    """Poisson arrivals at `rate` requests/s (rate=inf: all at t0)."""
    rng = np.random.default_rng([*SEED0, seed])
    gaps = np.zeros(count) if not np.isfinite(rate) else rng.exponential(1.0 / rate, count)
    arrivals = t0 + np.cumsum(gaps) - (gaps[0] if count else 0.0)
    ns = rng.integers(nmin, nmax + 1, count)
    flags = rng.random(count) < p_bf16x3
    B = np.array(inputs.GROUPED_B); R = np.array(inputs.GROUPED_R)
    out = []
    for i in range(count):
        bi = rng.integers(0, len(B), ns[i])
        b = B[bi]
        nallowed = np.array([np.sum(R <= bb // 2) for bb in B])[bi]
        ri = np.minimum((rng.random(ns[i]) * nallowed).astype(np.int64), nallowed - 1)
        shapes = np.stack([b, R[ri]], axis=1).astype(np.int64)
        out.append(Request(i, float(arrivals[i]), shapes, "bf16x3" if flags[i] else "fp64",
                           seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


@dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    status: str = "pending"        # ok | rejected | failed
    flops: float = 0.0
    nbytes: int = 0
    prec: str = "fp64"
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, next_arrival: Optional[float], executor) -> None:
        # short poll: completions are observed within tens of microseconds
        if next_arrival is not None:
            dt = next_arrival - self.now()
            if dt > 200e-6:
                time.sleep(min(dt - 100e-6, 100e-6))
        else:
            time.sleep(20e-6)


class Scheduler:
    """FIFO admission under an HBM budget and a slot limit."""

    def __init__(self, executor, budget_bytes: float = 64e9, slots: int = 8, clock=None):
        self.ex = executor
        self.budget = float(budget_bytes)
        self.slots = int(slots)
        self.clock = clock or RealClock()
        self.resident = 0
        self.max_resident = 0
        self.occupancy_integral = 0.0

    def run(self, requests: List[Request]) -> List[Record]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        running: Dict[object, tuple] = {}
        recs = {r.rid: Record(r.rid, r.arrival, flops=r.flops, nbytes=r.nbytes, prec=r.prec) for r in requests}
        last_t = self.clock.now()
        while pending or queue or running:
            now = self.clock.now()
            self.occupancy_integral += self.resident * max(now - last_t, 0.0)
            last_t = now
            progressed = False
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
                progressed = True
            for h in list(running):
                if self.ex.query(h):
                    req, _ = running.pop(h)
                    rec = recs[req.rid]
                    try:
                        self.ex.release(h)
                        rec.status = "ok"
                    except Exception as e:           # device error surfaced at completion
                        rec.status, rec.error = "failed", str(e)
                    rec.done = self.clock.now()
                    self.resident -= req.nbytes
                    progressed = True
            while queue and len(running) < self.slots:
                req = queue[0]
                rec = recs[req.rid]
                if req.nbytes > self.budget:
                    queue.popleft()
                    rec.status, rec.error, rec.done = "rejected", "exceeds the HBM budget", now
                    progressed = True
                    continue
                if self.resident + req.nbytes > self.budget:
                    break
                queue.popleft()
                rec.admitted = self.clock.now()
                try:
                    h = self.ex.launch(req)
                except Exception as e:
                    rec.status, rec.error, rec.done = "failed", str(e), self.clock.now()
                    progressed = True
                    continue
                running[h] = (req, rec.admitted)
                self.resident += req.nbytes
                self.max_resident = max(self.max_resident, self.resident)
                progressed = True
            if not progressed:
                self.clock.idle(pending[0].arrival if pending else None, self.ex)
        return [recs[r.rid] for r in requests]


def summarize(recs: List[Record], skip: int = 0) -> dict:
    ok = [r for r in recs if r.status == "ok" and r.rid >= skip]
    if not ok:
        return {"completed": 0}
    lat = np.array([r.latency for r in ok]) * 1e3
    t_first = min(r.arrival for r in ok)
    t_last = max(r.done for r in ok)
    flops = sum(r.flops for r in ok)
    return {"completed": len(ok), "rejected": sum(r.status == "rejected" for r in recs),
            "failed": sum(r.status == "failed" for r in recs),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "GFLOP/s": round(flops / (t_last - t_first) / 1e9, 1),
            "requests_per_s": round(len(ok) / (t_last - t_first), 2)}


def bucket_list():
    """The (b, r) buckets a request can draw: b over the uneven batch's block
    sizes, r over its ranks with r <= b/2."""
    return [(b, r) for b in inputs.GROUPED_B for r in inputs.GROUPED_R if r <= b // 2]


class ResidentPool:
    """Device-resident low-rank blocks, `per_bucket` instances of each (b, r)
    bucket: A (b x b), U, V1, U2 (b x r), column-major, N(0,1) from a seeded
    device generator, 256-byte aligned.  `f32` holds the same values rounded
    to FP32 (round to nearest even), the operands of split-precision
    requests, so their results can be judged against the FP64 originals."""

    def __init__(self, per_bucket: int = 256, seed: int = 77, device="cuda"):
        import torch
        self.per_bucket = int(per_bucket)
        self.buckets = bucket_list()
        self.index = {br: i for i, br in enumerate(self.buckets)}
        sizes = []
        for b, r in self.buckets:
            sizes += [b * b, b * r, b * r, b * r] * self.per_bucket
        off, total = inputs.pool_layout(sizes)
        # off[((bucket * per_bucket) + slot) * 4 + operand], elements
        self.offsets = off.reshape(len(self.buckets), self.per_bucket, 4)
        self.f64 = inputs.device_normal(total, seed=seed, device=device)
        self.f32 = self.f64.float()
        self.nbytes = total * 12

    def operand_offsets(self, shapes: np.ndarray, slots: np.ndarray) -> np.ndarray:
        """[n, 4] element offsets of A, U, V1, U2 for each (b, r) and slot."""
        if getattr(self, "_lut", None) is None:   # (b, r) -> bucket, one vectorised lookup per request
            bmax = max(b for b, _ in self.buckets); rmax = max(r for _, r in self.buckets)
            self._lut = np.full((bmax + 1, rmax + 1), -1, dtype=np.int64)
            for (b, r), i in self.index.items():
                self._lut[b, r] = i
        bi = self._lut[shapes[:, 0], shapes[:, 1]]
        if np.any(bi < 0):
            raise KeyError("a (b, r) outside the pool's buckets")
        return self.offsets[bi, slots]

    def host_operands(self, b: int, r: int, slot: int):
        """FP64 host copies (column-major) of one resident block's A, U, V1, U2."""
        o = self.offsets[self.index[(b, r)], slot]
        def cm(off, rows, cols):
            t = self.f64[int(off):int(off) + rows * cols].view(cols, rows).T
            return np.asfortranarray(t.cpu().numpy())
        return cm(o[0], b, b), cm(o[1], b, r), cm(o[2], b, r), cm(o[3], b, r)


def output_layout(shapes: np.ndarray, align: int = 256):
    """Byte offsets of each instance's outputs (C, T) in one FP64 buffer."""
    b = shapes[:, 0].astype(np.int64); r = shapes[:, 1].astype(np.int64)
    sizes = np.stack([b * r, r * r], axis=1).reshape(-1) * 8
    pad = (sizes + align - 1) // align * align
    off = np.concatenate([[0], np.cumsum(pad)[:-1]]) if len(pad) else np.zeros(0, np.int64)
    return off, int(pad.sum())


class _Launch:
    """In-flight request on the GPU (hashable by identity)."""
    __slots__ = ("slot", "event", "out", "req")

    def __init__(self, slot, event, out, req):
        self.slot, self.event, self.out, self.req = slot, event, out, req


class GpuExecutor:
    """Runs each request as one grouped call on its own HIP stream, over the
    operands of a resident pool."""

    def __init__(self, pool: ResidentPool, slots: int = 8, keep_outputs=(), device="cuda"):
        import torch
        self.torch = torch
        self.pool = pool
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]   # default priority
        self.free = list(range(slots))
        self.keep = set(keep_outputs)
        self.outputs: Dict[int, np.ndarray] = {}
        self.device = device

    def launch(self, req: Request):
        from . import lrbg
        torch = self.torch
        if not self.free:
            raise RuntimeError("no free slot")
        slot = self.free.pop()
        s = self.streams[slot]
        try:
            off_out, nout = output_layout(req.shapes)
            ops = self.pool.operand_offsets(req.shapes, req.slots(self.pool.per_bucket))
            with torch.cuda.stream(s):
                out = torch.empty(max(nout // 8, 1), dtype=torch.float64, device=self.device)
            src = self.pool.f64 if req.prec == "fp64" else self.pool.f32
            arr = self._descs(req, src.data_ptr(), src.element_size(), ops, out.data_ptr(), off_out)
            lrbg.lrbg_grouped_array(arr, s)
            ev = torch.cuda.Event()
            ev.record(s)
        except Exception:
            self.free.append(slot)
            raise
        return _Launch(slot, ev, out, req)

    @staticmethod
    def _descs(req, pin, es, ops, pout, off_out):
        from . import lrbg
        n = req.n
        b = req.shapes[:, 0].astype(np.int64); r = req.shapes[:, 1].astype(np.int64)
        arr = np.zeros(2 * n, dtype=lrbg.desc_dtype())
        oi = ops.astype(np.uint64) * np.uint64(es) + np.uint64(pin)
        oo = off_out.reshape(n, 2).astype(np.uint64) + np.uint64(pout)
        prec = lrbg.PRECS[req.prec]
        d = arr[0::2]   # C = A U
        d["op"] = lrbg.LRBG_OP_DENSE_TS; d["prec"] = prec
        d["m"] = b; d["n"] = r; d["k"] = b; d["lda"] = b; d["ldb"] = b; d["lds"] = 1; d["ldc"] = b
        d["a"] = oi[:, 0]; d["b"] = oi[:, 1]; d["c"] = oo[:, 0]
        t = arr[1::2]   # T = V1^T U2
        t["op"] = lrbg.LRBG_OP_INNER; t["prec"] = prec
        t["m"] = r; t["n"] = r; t["k"] = b; t["lda"] = b; t["ldb"] = b; t["lds"] = 1; t["ldc"] = r
        t["a"] = oi[:, 2]; t["b"] = oi[:, 3]; t["c"] = oo[:, 1]
        return arr

    def query(self, h) -> bool:
        return h.event.query()

    def release(self, h):
        if h.req.rid in self.keep:
            h.event.synchronize()
            self.outputs[h.req.rid] = h.out.cpu().numpy()
        h.out = None
        self.free.append(h.slot)


def request_outputs(req: Request, flat: np.ndarray):
    """(C, T) of every instance of a request from its flat output buffer."""
    off, _ = output_layout(req.shapes)
    off = off.reshape(req.n, 2) // 8
    out = []
    for i, (b, r) in enumerate(req.shapes):
        b, r = int(b), int(r)
        C = flat[off[i, 0]:off[i, 0] + b * r].reshape(r, b).T
        T = flat[off[i, 1]:off[i, 1] + r * r].reshape(r, r).T
        out.append((C, T))
    return out
