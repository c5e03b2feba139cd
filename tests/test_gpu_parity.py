"""GPU parity: every product kind and tile variant against the FP64 oracle.

Integer-valued inputs must give bitwise-identical results (every partial
sum is exact, so summation order cannot matter); N(0,1) inputs must be
within 1e-13 componentwise normalised error |C - Cref| / (|A||B|).  Outputs
live inside guard bands (padding rows of ld > rows and a guard column on
each side) that must be untouched, and input padding holds NaN so that a
read outside the matrix poisons the result.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import inputs, lrbg

from gpu_util import DevMat, ref_dense_ts, ref_inner, ref_recomp

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()
    oracle.load()


def sync():
    import torch
    torch.cuda.synchronize()


def stream():
    import torch
    return torch.cuda.current_stream()


def cache_for(variant_name, op, prec, b, r):
    f = tempfile.NamedTemporaryFile("w", suffix=".tune", delete=False)
    f.write(f"{op} {prec} {b} {r} {variant_name} 0\n")
    f.close()
    return f.name


def bucket(x, lo):
    v = lo
    while v < x:
        v *= 2
    return v


def run_plan(descs, tune=None, flags=0, reps=1):
    p = lrbg.Plan(descs, tune_cache=tune, flags=flags)
    for _ in range(reps):
        p.execute(stream())
    sync()
    st = p.stats()
    p.close()
    return st


# ------------------------------------------------------------------ DENSE_TS

DTS_SHAPES = [(64, 64, 8), (64, 64, 16), (128, 128, 32), (256, 256, 16), (96, 96, 12), (100, 100, 7),
              (1024, 1024, 128), (512, 512, 64), (200, 130, 50), (33, 70, 1), (300, 37, 128), (17, 5, 3)]


def _dts_case(m, k, n, integer, seed, lds_pad=(0, 0, 0), tune=None):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    A = f(rng, m, k); U = f(rng, k, n)
    dA = DevMat.from_numpy(A, ld=m + lds_pad[0]); dU = DevMat.from_numpy(U, ld=k + lds_pad[1])
    dC = DevMat(m, n, ld=m + lds_pad[2])
    run_plan([lrbg.desc("dense_ts", dA.view, dU.view, dC.view)], tune=tune)
    C = dC.numpy()
    Cref, D = ref_dense_ts(A, U)
    assert dC.guards_intact(), "write outside the output matrix"
    return C, Cref, D


@pytest.mark.parametrize("m,k,n", DTS_SHAPES)
def test_dense_ts_integer_bitwise(m, k, n):
    C, Cref, _ = _dts_case(m, k, n, True, 100 + m + n, lds_pad=(3, 1, 5))
    assert np.array_equal(C, Cref)


@pytest.mark.parametrize("m,k,n", DTS_SHAPES)
def test_dense_ts_normal(m, k, n):
    C, Cref, D = _dts_case(m, k, n, False, 200 + m + n, lds_pad=(2, 0, 1))
    assert oracle.normalized_error(C, Cref, D) <= TOL


# ------------------------------------------------------------------ INNER

INN_SHAPES = [(512, 32, 32), (64, 8, 8), (1024, 128, 128), (256, 16, 16), (512, 64, 64), (100, 7, 9),
              (1000, 50, 70), (37, 128, 3), (5, 16, 16), (2048, 32, 32)]


def _inner_case(k, m, n, integer, seed, pad=(0, 0, 0), tune=None):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    V1 = f(rng, k, m); U2 = f(rng, k, n)
    dV = DevMat.from_numpy(V1, ld=k + pad[0]); dU = DevMat.from_numpy(U2, ld=k + pad[1])
    dT = DevMat(m, n, ld=m + pad[2])
    run_plan([lrbg.desc("inner", dV.view, dU.view, dT.view)], tune=tune)
    T = dT.numpy()
    Tref, D = ref_inner(V1, U2)
    assert dT.guards_intact()
    return T, Tref, D


@pytest.mark.parametrize("k,m,n", INN_SHAPES)
def test_inner_integer_bitwise(k, m, n):
    T, Tref, _ = _inner_case(k, m, n, True, 300 + k + m, pad=(1, 3, 2))
    assert np.array_equal(T, Tref)


@pytest.mark.parametrize("k,m,n", INN_SHAPES)
def test_inner_normal(k, m, n):
    T, Tref, D = _inner_case(k, m, n, False, 400 + k + m, pad=(0, 2, 0))
    assert oracle.normalized_error(T, Tref, D) <= TOL


# ------------------------------------------------------------------ RECOMP

REC_SHAPES = [(512, 512, 32), (64, 64, 8), (128, 96, 16), (1024, 1024, 128), (256, 256, 64), (100, 70, 7),
              (33, 200, 50), (7, 5, 3)]


def _recomp_case(m, n, k, integer, seed, pad=(0, 0, 0, 0), tune=None):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    U1 = f(rng, m, k); S = f(rng, k, k); V2 = f(rng, n, k)
    dU = DevMat.from_numpy(U1, ld=m + pad[0]); dS = DevMat.from_numpy(S, ld=k + pad[1])
    dV = DevMat.from_numpy(V2, ld=n + pad[2]); dW = DevMat(m, n, ld=m + pad[3])
    run_plan([lrbg.desc("recomp", dU.view, dV.view, dW.view, s=dS.view)], tune=tune)
    W = dW.numpy()
    Wref, D = ref_recomp(U1, S, V2)
    assert dW.guards_intact()
    return W, Wref, D


@pytest.mark.parametrize("m,n,k", REC_SHAPES)
def test_recomp_integer_bitwise(m, n, k):
    W, Wref, _ = _recomp_case(m, n, k, True, 500 + m + k, pad=(2, 1, 3, 4))
    assert np.array_equal(W, Wref)


@pytest.mark.parametrize("m,n,k", REC_SHAPES)
def test_recomp_normal(m, n, k):
    W, Wref, D = _recomp_case(m, n, k, False, 600 + m + k, pad=(0, 0, 1, 0))
    assert oracle.normalized_error(W, Wref, D) <= TOL


# ---------------------------------------------------- every variant, forced

def _variants():
    lrbg.load()
    return [(i, n) for i, n in enumerate(lrbg.lrbg_variant_names())
            if n != "nop" and not n.startswith(("dts3", "inn3"))]


def _variant_params():
    try:
        return _variants()
    except Exception:
        return []


@pytest.mark.parametrize("vid,name", _variant_params())
def test_every_variant_forced(vid, name):
    if name.startswith("dtss"):
        # short contraction: one k chunk, a ragged one, several chunks
        rn = int(name.split("_rn")[1].split("_")[0])
        n = 16 * rn - 3
        m = 300
        for k in (8, 37, 64):
            tune = cache_for(name, 0, 0, bucket(max(m, k), 64), bucket(n, 8))
            C, Cref, _ = _dts_case(m, k, n, True, vid + k, lds_pad=(1, 2, 3), tune=tune)
            assert np.array_equal(C, Cref)
            C, Cref, D = _dts_case(m, k, n, False, vid + k, tune=tune)
            assert oracle.normalized_error(C, Cref, D) <= TOL
    elif name.startswith(("dts64", "dtsl")):
        rn = int(name.split("_rn")[1].split("_")[0])
        n = min(16 * rn, 128) - 3
        m = k = 300
        tune = cache_for(name, 0, 0, bucket(max(m, k), 64), bucket(n, 8))
        C, Cref, _ = _dts_case(m, k, n, True, vid, lds_pad=(1, 2, 3), tune=tune)
        assert np.array_equal(C, Cref)
        C, Cref, D = _dts_case(m, k, n, False, vid, tune=tune)
        assert oracle.normalized_error(C, Cref, D) <= TOL
    elif name.startswith(("inn64", "innl")):
        rj = int(name.split("_rj")[1].split("_")[0])
        wc = 4 // int(name.split("_wr")[1].split("_")[0]) if "_wr" in name else 1
        n = min(16 * rj * wc, 128) - 1
        m = 45
        k = 333
        tune = cache_for(name, 1, 0, bucket(k, 64), bucket(max(m, n), 8))
        T, Tref, _ = _inner_case(k, m, n, True, vid, pad=(1, 1, 1), tune=tune)
        assert np.array_equal(T, Tref)
        T, Tref, D = _inner_case(k, m, n, False, vid, tune=tune)
        assert oracle.normalized_error(T, Tref, D) <= TOL
    elif name.startswith("rec64"):
        bn = int(name.split("_bn")[1].split("_")[0])
        k = min(4096 // (16 * bn) - 5, 128)
        m, n = 150, 170
        tune = cache_for(name, 2, 0, bucket(max(m, n), 64), bucket(k, 8))
        W, Wref, _ = _recomp_case(m, n, k, True, vid, pad=(1, 1, 1, 1), tune=tune)
        assert np.array_equal(W, Wref)
        W, Wref, D = _recomp_case(m, n, k, False, vid, tune=tune)
        assert oracle.normalized_error(W, Wref, D) <= TOL


# ------------------------------------------------------------ edge cases

def test_zero_contraction_gives_zeros():
    dC = DevMat(64, 16)
    dA = DevMat(64, 0); dU = DevMat(0, 16)
    d = lrbg.desc("dense_ts", dA.view, dU.view, dC.view)
    d.a = None; d.b = None
    run_plan([d])
    assert np.all(dC.numpy() == 0) and dC.guards_intact()


def test_empty_products_are_noops():
    dU = DevMat.from_numpy(np.ones((64, 16), order="F"))
    d = lrbg.lrbg_desc(op=0, prec=0, m=0, n=16, k=64, lda=1, ldb=64, lds=1, ldc=1, flags=0,
                       a=None, b=dU.view.data_ptr(), s=None, c=None)
    lrbg.lrbg_grouped([d], stream())
    sync()
    assert lrbg.lrbg_schedule_stats([d])["tiles"] == 0


# ------------------------------------------------------- grouped / chain / plan

def _mixed_batch(seed, count=60):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        kind = i % 3
        b = int(rng.choice([64, 128, 256, 512, 100, 77]))
        r = int(rng.choice([8, 16, 32, 64, 5, 20]))
        r = min(r, max(b // 2, 1))
        if kind == 0:
            A = inputs.normal_f(rng, b, b); U = inputs.normal_f(rng, b, r)
            cases.append(("dense_ts", (A, U)))
        elif kind == 1:
            V1 = inputs.normal_f(rng, b, r); U2 = inputs.normal_f(rng, b, r)
            cases.append(("inner", (V1, U2)))
        else:
            U1 = inputs.normal_f(rng, b, r); S = inputs.normal_f(rng, r, r); V2 = inputs.normal_f(rng, b, r)
            cases.append(("recomp", (U1, S, V2)))
    return cases


def _descs_for(cases):
    descs, outs, keep = [], [], []
    for op, ops in cases:
        if op == "dense_ts":
            A, U = ops
            dA, dU, dC = DevMat.from_numpy(A), DevMat.from_numpy(U), DevMat(A.shape[0], U.shape[1])
            descs.append(lrbg.desc(op, dA.view, dU.view, dC.view)); keep += [dA, dU]; outs.append(dC)
        elif op == "inner":
            V1, U2 = ops
            dV, dU, dT = DevMat.from_numpy(V1), DevMat.from_numpy(U2), DevMat(V1.shape[1], U2.shape[1])
            descs.append(lrbg.desc(op, dV.view, dU.view, dT.view)); keep += [dV, dU]; outs.append(dT)
        else:
            U1, S, V2 = ops
            dU, dS, dV = DevMat.from_numpy(U1), DevMat.from_numpy(S), DevMat.from_numpy(V2)
            dW = DevMat(U1.shape[0], V2.shape[0])
            descs.append(lrbg.desc(op, dU.view, dV.view, dW.view, s=dS.view)); keep += [dU, dS, dV]; outs.append(dW)
    return descs, outs, keep


def _check_cases(cases, outs, bitwise_to=None):
    for idx, ((op, ops), o) in enumerate(zip(cases, outs)):
        got = o.numpy()
        ref, D = {"dense_ts": ref_dense_ts, "inner": ref_inner, "recomp": ref_recomp}[op](*ops)
        assert o.guards_intact()
        e = oracle.normalized_error(got, ref, D)
        assert e <= TOL, (idx, op, e)
        if bitwise_to is not None:
            assert np.array_equal(got, bitwise_to[idx]), idx


@pytest.mark.parametrize("flags", [0, lrbg.LRBG_PLAN_NO_GRAPH, lrbg.LRBG_PLAN_SCHED_MIX,
                                   lrbg.LRBG_PLAN_PERSISTENT, lrbg.LRBG_PLAN_DUAL,
                                   lrbg.LRBG_PLAN_DUAL | lrbg.LRBG_PLAN_NO_GRAPH, lrbg.LRBG_PLAN_UNTIMED,
                                   lrbg.LRBG_PLAN_UNTIMED | lrbg.LRBG_PLAN_SCHED_MIX])
def test_grouped_mixed_plan(flags):
    cases = _mixed_batch(7)
    descs, outs, keep = _descs_for(cases)
    p = lrbg.Plan(descs, flags=flags)
    first = None
    for rep in range(3):
        for o in outs:
            o.view.fill_(np.nan)       # eager work between replays
        p.execute(stream())
        sync()
        _check_cases(cases, outs, bitwise_to=first)
        first = [o.numpy() for o in outs]
        if flags & lrbg.LRBG_PLAN_UNTIMED:
            assert p.last_ms() < 0
        else:
            assert p.last_ms() >= 0
    p.close()


def test_grouped_one_shot_and_batched_api():
    cases = _mixed_batch(8, count=30)
    descs, outs, keep = _descs_for(cases)
    lrbg.lrbg_grouped(descs, stream())
    sync()
    _check_cases(cases, outs)
    # lr_batched_gemm over the DENSE_TS subset
    sub = [(c, d, o) for c, d, o in zip(cases, descs, outs) if c[0] == "dense_ts"]
    for _, _, o in sub:
        o.view.fill_(np.nan)
    ds = [d for _, d, _ in sub]
    lrbg.lr_batched_gemm(0, 0, [d.m for d in ds], [d.n for d in ds], [d.k for d in ds],
                         [d.a for d in ds], [d.lda for d in ds], [d.b for d in ds], [d.ldb for d in ds],
                         None, None, [d.c for d in ds], [d.ldc for d in ds], stream())
    sync()
    _check_cases([c for c, _, _ in sub], [o for _, _, o in sub])


def test_chain_in_one_grouped_call():
    b, r = 512, 32
    cis = [inputs.chain_instance(2, i, b, r) for i in range(8)]
    descs, keep, Ts, Ws = [], [], [], []
    for ci in cis:
        dV1, dU2, dU1, dV2 = (DevMat.from_numpy(x) for x in (ci.V1, ci.U2, ci.U1, ci.V2))
        dT, dW = DevMat(r, r), DevMat(b, b)
        descs += [lrbg.desc("recomp", dU1.view, dV2.view, dW.view, s=dT.view),   # listed first on purpose
                  lrbg.desc("inner", dV1.view, dU2.view, dT.view)]
        keep += [dV1, dU2, dU1, dV2]; Ts.append(dT); Ws.append(dW)
    st = lrbg.lrbg_schedule_stats(descs)
    assert st["levels"] == 2
    lrbg.lrbg_grouped(descs, stream())
    sync()
    for ci, dT, dW in zip(cis, Ts, Ws):
        Tref, Wref = oracle.chain([ci.V1], [ci.U2], [ci.U1], [ci.V2])
        Dt = oracle.inner([np.abs(ci.V1)], [np.abs(ci.U2)])[0]
        Dw = oracle.recomp([np.abs(ci.U1)], [Dt], [np.abs(ci.V2)])[0]
        assert oracle.normalized_error(dT.numpy(), Tref[0], Dt) <= TOL
        assert oracle.normalized_error(dW.numpy(), Wref[0], Dw) <= TOL


def test_alone_equals_in_mix_bitwise():
    cases = _mixed_batch(9, count=45)
    descs, outs, keep = _descs_for(cases)
    run_plan(descs)
    mixed = [o.numpy() for o in outs]
    for i in (0, 1, 2, 10, 44):
        outs[i].view.fill_(np.nan)
        run_plan([descs[i]])
        assert np.array_equal(outs[i].numpy(), mixed[i]), i
