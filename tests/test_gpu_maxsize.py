"""The largest block the boundary accepts (65 536, the limit the C ABI
checks): DENSE_TS over a 65 536 x 65 536 block (32 GiB of A) and RECOMP to a
65 536 x 65 536 output, checked on sampled rows against the oracle (a row of
the output depends on that row of the left operand only, so the oracle runs
on the sampled rows); INNER and the fused product with a contraction of
65 536, checked in full.  The plans use the committed tuning cache (whose
buckets stop at 2048, so these take the built-in choices).  One above the
limit is rejected by the host checks (tests/test_abi.py)."""
import os

import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import inputs, lrbg, workloads

from gpu_util import ref_dense_ts, ref_inner, ref_lrmult, ref_recomp

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_2311_07602_amd", "tune", "mi355x.tune")
B = 65536
TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


def _run(descs):
    import torch
    p = lrbg.Plan(descs, tune_cache=TUNE)
    p.execute(torch.cuda.current_stream())
    torch.cuda.synchronize()
    p.close()


def _host(t):
    return np.asfortranarray(t.double().cpu().numpy())


def _rows():
    # the first and last rows of the block, every tile boundary class, and random rows
    rng = np.random.default_rng(7)
    fixed = [0, 1, 63, 64, 127, 255, 256, B // 2 - 1, B // 2, B - 257, B - 256, B - 65, B - 2, B - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, B, 50)])).astype(np.int64)


@pytest.mark.parametrize("r", [16, 128])
def test_dense_ts_at_block_limit(r):
    import torch
    pool = inputs.device_normal(B * B + B * r, seed=70 + r)
    A = workloads._cm(pool, 0, B, B)
    U = workloads._cm(pool, B * B, B, r)
    C = torch.full((r, B), float("nan"), dtype=torch.float64, device="cuda").T
    _run([lrbg.desc("dense_ts", A, U, C)])
    rows = _rows()
    idx = torch.from_numpy(rows).cuda()
    Cref, D = ref_dense_ts(_host(A[idx, :]), _host(U))
    err = oracle.normalized_error(_host(C[idx, :]), Cref, D)
    assert err <= TOL, err
    assert not torch.isnan(C).any().item()
    del pool, A, U, C
    torch.cuda.empty_cache()


def test_recomp_at_block_limit():
    import torch
    r = 32
    pool = inputs.device_normal(2 * B * r + r * r, seed=80)
    U1 = workloads._cm(pool, 0, B, r)
    V2 = workloads._cm(pool, B * r, B, r)
    S = workloads._cm(pool, 2 * B * r, r, r)
    W = torch.full((B, B), float("nan"), dtype=torch.float64, device="cuda").T
    _run([lrbg.desc("recomp", U1, V2, W, s=S)])
    rows = _rows()
    idx = torch.from_numpy(rows).cuda()
    Wref, D = ref_recomp(_host(U1[idx, :]), _host(S), _host(V2))
    err = oracle.normalized_error(_host(W[idx, :]), Wref, D)
    assert err <= TOL, err
    assert not torch.isnan(W).any().item()
    del pool, U1, V2, S, W
    torch.cuda.empty_cache()


@pytest.mark.parametrize("r", [8, 64, 128])
def test_inner_at_block_limit(r):
    import torch
    pool = inputs.device_normal(2 * B * r, seed=90 + r)
    V1 = workloads._cm(pool, 0, B, r)
    U2 = workloads._cm(pool, B * r, B, r)
    T = torch.full((r, r), float("nan"), dtype=torch.float64, device="cuda").T
    _run([lrbg.desc("inner", V1, U2, T)])
    Tref, D = ref_inner(_host(V1), _host(U2))
    assert oracle.normalized_error(_host(T), Tref, D) <= TOL


@pytest.mark.parametrize("r", [16, 64, 96, 128])
def test_lrmult_at_block_limit(r):
    import torch
    pool = inputs.device_normal(2 * B * r + 2 * r * r, seed=100 + r)
    AV = workloads._cm(pool, 0, B, r)
    BU = workloads._cm(pool, B * r, B, r)
    AX = workloads._cm(pool, 2 * B * r, r, r)
    BX = workloads._cm(pool, 2 * B * r + r * r, r, r)
    G = torch.full((r, r), float("nan"), dtype=torch.float64, device="cuda").T
    _run([lrbg.desc("lrmult", AV, BU, G, s=AX, e=BX)])
    Gref, D = ref_lrmult(_host(AV), _host(BU), _host(AX), _host(BX))
    assert oracle.normalized_error(_host(G), Gref, D) <= TOL


def test_bf16x3_at_block_limit():
    """The split-precision products over a contraction of 65 536: FP32
    operands (RNE-rounded from the FP64 draw), within 1e-6 of the FP64
    oracle on the FP64 originals; the FP32 accumulation within each split
    term does not grow the normalised error with k (7e-8 at k = 512 and
    65 536 alike)."""
    import torch
    r = 16
    p64 = inputs.device_normal(B * B + B * r, seed=110)
    p32 = p64.float()
    A = workloads._cm(p32, 0, B, B)
    U = workloads._cm(p32, B * B, B, r)
    C = torch.full((r, B), float("nan"), dtype=torch.float64, device="cuda").T
    V1 = workloads._cm(p32, 0, B, 64)
    U2 = workloads._cm(p32, B * 64, B, 64)
    T = torch.full((64, 64), float("nan"), dtype=torch.float64, device="cuda").T
    _run([lrbg.desc("dense_ts", A, U, C, prec="bf16x3"), lrbg.desc("inner", V1, U2, T, prec="bf16x3")])
    rows = _rows()
    idx = torch.from_numpy(rows).cuda()
    Cref, D = ref_dense_ts(_host(workloads._cm(p64, 0, B, B)[idx, :]), _host(workloads._cm(p64, B * B, B, r)))
    assert oracle.normalized_error(_host(C[idx, :]), Cref, D) <= 1e-6
    Tref, Dt = ref_inner(_host(workloads._cm(p64, 0, B, 64)), _host(workloads._cm(p64, B * 64, B, 64)))
    assert oracle.normalized_error(_host(T), Tref, Dt) <= 1e-6
    del p64, p32, A, U, C, V1, U2, T
    torch.cuda.empty_cache()
