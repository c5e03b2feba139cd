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
    """The chain as the benchmark times it: the committed tuning cache picks
    the inner and recompression variants at 4096 x (512, 32)."""
    w = workloads.chain(4096, 512, 32, prec=prec)
    names = lrbg.lrbg_schedule_variants(w.descs[:1] + w.descs[-1:], TUNE)
    plan = lrbg.Plan(w.descs, tune_cache=TUNE)
    assert plan.stats()["levels"] == 2
    print("chain variants:", names, flush=True)
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


@pytest.mark.parametrize("b,r", [(2048, 32), (2048, 128), (512, 8), (2048, 96), (512, 96)])
def test_lrmult_paper_shape_sampled(b, r):
    """The paper's fused product at its batch of 20 000 (the bench's
    lrmult_paper_shapes configuration): sampled instances against Alg. 1 in
    the oracle, replays bitwise identical."""
    import torch
    from gpu_util import ref_lrmult
    w = workloads.lrmult(20000, b, r)
    plan = lrbg.Plan(w.descs)
    _replay(plan)
    g = w.pools[1].clone()
    worst = 0.0
    for i in (0, 1, 4999, 10001, 19999):
        o = workloads.lrmult_operands(w, i)
        Gref, D = ref_lrmult(o["AV"], o["BU"], o["AX"], o["BX"])
        worst = max(worst, oracle.normalized_error(o["G"], Gref, D))
    assert worst <= 1e-13, worst
    w.pools[1].fill_(float("nan"))
    _replay(plan, 1)
    assert torch.equal(g.view(torch.int64), w.pools[1].view(torch.int64)), "replays differ"
    plan.close()


def test_blr_large_sampled_rows():
    """BLR matrix x 8 right-hand sides at N = 65 536 (128 block rows of 512,
    rank 8): sampled block rows against the oracle's BLR evaluation."""
    from paper_2311_07602_amd import blr as _blr  # noqa: F401
    m = workloads.blr(128, 512)
    _replay(m.plan())
    nb = m.nb
    X = [np.asfortranarray(m.x(j).cpu().numpy()) for j in range(nb)]
    worst = 0.0
    for i in (0, 63, 127):
        D = np.asfortranarray(m.diag(i).cpu().numpy())
        U = [[None] * nb for _ in range(nb)]
        V = [[None] * nb for _ in range(nb)]
        for j in range(nb):
            if j != i:
                U[i][j] = np.asfortranarray(m.u(i, j).cpu().numpy())
                V[i][j] = np.asfortranarray(m.v(i, j).cpu().numpy())
        Dl = [None] * nb
        Dl[i] = D
        Y = oracle.blr_matvec(Dl, U, V, X, rows=[i])[0]
        ab = lambda a: None if a is None else np.asfortranarray(np.abs(a))
        Dy = oracle.blr_matvec([ab(d) for d in Dl], [[ab(u) for u in row] for row in U],
                               [[ab(v) for v in row] for row in V], [ab(x) for x in X], rows=[i])[0]
        worst = max(worst, oracle.normalized_error(m.y(i).cpu().numpy(), Y, Dy))
    m.close()
    assert worst <= 1e-13, worst


def test_round_at_scale_sampled():
    """The recompressed product over 2000 instances (b = 1024, r = 32, rank
    <= 16): sampled instances' singular values against the oracle (within
    1e-12 sigma_1) and orthonormal kept bases."""
    import torch
    from paper_2311_07602_amd import inputs
    count, b, r, kmax, tol = 2000, 1024, 32, 16, 1e-8
    per = 4 * b * r + 2 * r * r
    pin = inputs.device_normal(count * per, seed=71)
    U = torch.empty(count, kmax, b, dtype=torch.float64, device="cuda")
    V = torch.empty_like(U)
    sigma = torch.empty(count * kmax, dtype=torch.float64, device="cuda")
    kout = torch.empty(count, dtype=torch.int32, device="cuda")
    base = pin.data_ptr()
    off = lambda t, j: base + 8 * (t * per + j * b * r)
    offs = lambda t, j: base + 8 * (t * per + 4 * b * r + j * r * r)
    ts = range(count)
    lrbg.lr_batched_lrmult_round([b] * count, [r] * count, [r] * count,
                                 [off(t, 0) for t in ts], [b] * count, [off(t, 1) for t in ts], [b] * count,
                                 [offs(t, 0) for t in ts], [r] * count, [off(t, 2) for t in ts], [b] * count,
                                 [offs(t, 1) for t in ts], [r] * count, [off(t, 3) for t in ts], [b] * count,
                                 kmax, tol, [U[t].data_ptr() for t in ts], [b] * count,
                                 [V[t].data_ptr() for t in ts], [b] * count, sigma.data_ptr(), kout.data_ptr(),
                                 torch.cuda.current_stream())
    torch.cuda.synchronize()
    host = pin.cpu().numpy()
    sig = sigma.cpu().numpy().reshape(count, kmax)
    ks = kout.cpu().numpy()
    cm = lambda o, rows, cols: np.asfortranarray(host[o:o + rows * cols].reshape(cols, rows).T)
    for t in (0, 777, 1999):
        o = t * per
        AU, AV, BU, BV = (cm(o + j * b * r, b, r) for j in range(4))
        AX, BX = cm(o + 4 * b * r, r, r), cm(o + 4 * b * r + r * r, r, r)
        Uo, so, Vo, ko = oracle.lr_mult_round(AU, AV, AX, BU, BX, BV, kmax, tol)
        assert ks[t] == ko
        assert np.all(np.abs(sig[t] - so) <= 1e-12 * so[0])
        # kept columns equal the oracle's up to sign (the random cores have distinct singular values)
        Ut = U[t].cpu().numpy().T
        for j in range(ko):
            d = min(np.max(np.abs(Ut[:, j] - Uo[:, j])), np.max(np.abs(Ut[:, j] + Uo[:, j])))
            assert d <= 1e-8 * np.max(np.abs(Uo[:, j])), (t, j, d)


@pytest.mark.parametrize("r", [8, 32])
def test_round_plan_at_bench_scale_matches_one_shot(r):
    """The plan form at the bench's size (20000 instances, b = 1024) gives
    the one-shot call's outputs bit for bit (same kernels, same schedules)."""
    import torch
    from paper_2311_07602_amd import inputs
    count, b, kmax, tol = 20000, 1024, r // 2, 1e-8
    per = 4 * b * r + 2 * r * r
    pin = inputs.device_normal(count * per, seed=90 + r)
    outs = []
    for _ in range(2):
        U = torch.full((count, kmax, b), np.nan, dtype=torch.float64, device="cuda")
        V = torch.full_like(U, np.nan)
        sigma = torch.full((count * kmax,), np.nan, dtype=torch.float64, device="cuda")
        kout = torch.full((count,), -1, dtype=torch.int32, device="cuda")
        outs.append((U, V, sigma, kout))
    base = pin.data_ptr()
    off = lambda t, j: base + 8 * (t * per + j * b * r)
    offs = lambda t, j: base + 8 * (t * per + 4 * b * r + j * r * r)
    ts = range(count)
    def args(o):
        U, V, sigma, kout = o
        return ([b] * count, [r] * count, [r] * count,
                [off(t, 0) for t in ts], [b] * count, [off(t, 1) for t in ts], [b] * count,
                [offs(t, 0) for t in ts], [r] * count, [off(t, 2) for t in ts], [b] * count,
                [offs(t, 1) for t in ts], [r] * count, [off(t, 3) for t in ts], [b] * count,
                kmax, tol, [U[t].data_ptr() for t in ts], [b] * count,
                [V[t].data_ptr() for t in ts], [b] * count, sigma.data_ptr(), kout.data_ptr())
    stream = torch.cuda.current_stream()
    lrbg.lr_batched_lrmult_round(*args(outs[0]), stream=stream)
    with lrbg.RoundPlan(*args(outs[1])) as plan:
        plan.execute(stream)
        plan.execute(stream)
        torch.cuda.synchronize()
    for x, y in zip(outs[0], outs[1]):
        assert torch.equal(x, y)
    assert int(outs[0][3].min()) == kmax


@pytest.mark.parametrize("r", [8, 16, 32])
def test_lradd_at_bench_scale_sampled(r):
    """The rounded addition at the benchmark's size (20000 instances, b =
    1024, both ranks r, kept rank <= r, N(0,1) factors): sampled instances
    against the oracle -- kept rank, singular values within 1e-12 sigma_1,
    the kept sum, and orthonormal new bases."""
    import torch
    from paper_2311_07602_amd import inputs
    count, b, kmax, tol = 20000, 1024, r, 1e-8
    per = 4 * b * r + 2 * r * r
    pin = inputs.device_normal(count * per, seed=27 + r)
    U = torch.full((count, kmax, b), np.nan, dtype=torch.float64, device="cuda")
    V = torch.full_like(U, np.nan)
    sigma = torch.full((count * kmax,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    base = pin.data_ptr()
    off = lambda t, j: base + 8 * (t * per + j * b * r)
    offs = lambda t, j: base + 8 * (t * per + 4 * b * r + j * r * r)
    ts = range(count)
    lrbg.lr_batched_lradd_round([b] * count, [r] * count, [r] * count,
                                [off(t, 0) for t in ts], [b] * count, [off(t, 1) for t in ts], [b] * count,
                                [offs(t, 0) for t in ts], [r] * count, [off(t, 2) for t in ts], [b] * count,
                                [offs(t, 1) for t in ts], [r] * count, [off(t, 3) for t in ts], [b] * count,
                                kmax, tol, [U[t].data_ptr() for t in ts], [b] * count,
                                [V[t].data_ptr() for t in ts], [b] * count, sigma.data_ptr(), kout.data_ptr(),
                                torch.cuda.current_stream())
    torch.cuda.synchronize()
    sig = sigma.cpu().numpy().reshape(count, kmax)
    ks = kout.cpu().numpy()
    assert np.all(ks == kmax)
    cm = lambda t0, o, rows, cols: np.asfortranarray(
        pin[t0 * per + o:t0 * per + o + rows * cols].cpu().numpy().reshape(cols, rows).T)
    for t in (0, 4321, 19999):
        AU, AV, BU, BV = (cm(t, j * b * r, b, r) for j in range(4))
        AX, BX = cm(t, 4 * b * r, r, r), cm(t, 4 * b * r + r * r, r, r)
        Uo, so, Vo, ko = oracle.lr_add_round(AU, AV, AX, BU, BX, BV, kmax, tol)
        assert ks[t] == ko
        assert np.all(np.abs(sig[t] - so) <= 1e-12 * so[0])
        Ut, Vt = U[t].cpu().numpy().T, V[t].cpu().numpy().T
        assert np.max(np.abs(Ut.T @ Ut - np.eye(kmax))) <= 1e-12
        assert np.max(np.abs(Vt.T @ Vt - np.eye(kmax))) <= 1e-12
        P = Ut @ np.diag(sig[t]) @ Vt.T
        Po = Uo @ np.diag(so) @ Vo.T
        assert np.max(np.abs(P - Po)) <= 1e-11 * so[0], t
