"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (plan with the committed tuning cache and the mixed tile order, replayed
from its hipGraph): sampled instances against the oracle, and replay
determinism of the whole output."""
import os

import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import lrbg, workloads

from gpu_util import ref_dense_ts, ref_inner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_2311_07602_amd", "tune", "mi355x.tune")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


def _replay(plan, n=2):
    import torch
    s = torch.cuda.current_stream()
    for _ in range(n):
        plan.execute(s)
    torch.cuda.synchronize()


def test_uneven_batch_full_size_sampled():
    import torch
    w = workloads.grouped(20000, seed=3)
    plan = lrbg.Plan(w.descs, tune_cache=TUNE, flags=lrbg.LRBG_PLAN_SCHED_MIX)
    _replay(plan)
    digest1 = torch.sum(w.pools[1].view(torch.int64) * 0x9E3779B1).item()
    # two instances of every (b, r) bucket
    seen, picks = {}, []
    for i, br in enumerate(w.meta["shapes"]):
        if seen.get(br, 0) < 2:
            seen[br] = seen.get(br, 0) + 1
            picks.append(i)
    assert len(seen) == 22
    worst = 0.0
    for i in picks:
        o = workloads.grouped_operands(w, i)
        Cref, Dc = ref_dense_ts(o["A"], o["U"])
        Tref, Dt = ref_inner(o["V1"], o["U2"])
        worst = max(worst, oracle.normalized_error(o["C"], Cref, Dc), oracle.normalized_error(o["T"], Tref, Dt))
    assert worst <= 1e-13, worst
    w.pools[1].fill_(float("nan"))
    _replay(plan, 1)
    digest2 = torch.sum(w.pools[1].view(torch.int64) * 0x9E3779B1).item()
    assert digest1 == digest2, "replays differ"
    plan.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("bf16x3", 1e-6)])
def test_chain_full_size_sampled(prec, tol):
    w = workloads.chain(4096, 512, 32, prec=prec)
    plan = lrbg.Plan(w.descs)
    assert plan.stats()["levels"] == 2
    _replay(plan)
    for i in (0, 1, 777, 2048, 4095):
        o = workloads.chain_host_instance(w, i)
        Tref, Wref = oracle.chain([o["V1"]], [o["U2"]], [o["U1"]], [o["V2"]])
        Dt = oracle.inner([np.abs(o["V1"])], [np.abs(o["U2"])])[0]
        Dw = oracle.recomp([np.abs(o["U1"])], [Dt], [np.abs(o["V2"])])[0]
        assert oracle.normalized_error(o["T"], Tref[0], Dt) <= tol
        assert oracle.normalized_error(o["W"], Wref[0], Dw) <= tol
    plan.close()


def test_dense_uniform_every_instance():
    w = workloads.dense_uniform(64, 256, 16, seed=11)
    plan = lrbg.Plan(w.descs, tune_cache=TUNE)
    _replay(plan)
    pin, pout = w.pools
    for i, (b, r, oA, oU, oC) in enumerate(w.index):
        A = np.asfortranarray(workloads._cm(pin, oA, b, b).cpu().numpy())
        U = np.asfortranarray(workloads._cm(pin, oU, b, r).cpu().numpy())
        C = workloads._cm(pout, oC, b, r).cpu().numpy()
        Cref, D = ref_dense_ts(A, U)
        assert oracle.normalized_error(C, Cref, D) <= 1e-13, i
    plan.close()
