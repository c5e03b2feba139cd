"""GPU parity of the BF16x3 split-precision path (FP32 operands, FP64 output).

Integer inputs with |x| <= 8 are exact in bfloat16 (the second and third
split terms are zero) and every FP32 partial sum stays below 2^24, so the
result must equal the FP64 oracle bitwise.  On N(0,1) inputs the error is
measured against the FP64 oracle on the original FP64 inputs, so the FP32
rounding of the inputs is included, and must stay within 1e-6 componentwise
normalised error; against the oracle on the FP32-rounded inputs it measures
the split arithmetic alone.
"""
import tempfile

import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import inputs, lrbg

from gpu_util import DevMat, ref_dense_ts, ref_inner

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()


def f32dev(x, ld=None):
    import torch
    return DevMat.from_numpy(x, ld=ld, dtype=torch.float32)


def run(descs, tune=None):
    import torch
    p = lrbg.Plan(descs, tune_cache=tune)
    p.execute(torch.cuda.current_stream())
    torch.cuda.synchronize()
    p.close()


def f32(x):
    return np.asfortranarray(x.astype(np.float32).astype(np.float64))


def bucket(x, lo):
    v = lo
    while v < x:
        v *= 2
    return v


def tune_file(line):
    f = tempfile.NamedTemporaryFile("w", suffix=".tune", delete=False)
    f.write(line + "\n")
    f.close()
    return f.name


INN = [(512, 32, 32), (64, 8, 8), (1024, 128, 128), (300, 20, 7), (77, 64, 64), (1000, 16, 16)]
DTS = [(256, 256, 16), (64, 64, 8), (1024, 1024, 128), (130, 130, 33), (512, 512, 64), (100, 37, 5)]


def _inner(k, m, n, integer, seed, tune=None, pad=(0, 0, 0)):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    V1 = f(rng, k, m); U2 = f(rng, k, n)
    dV, dU = f32dev(V1, ld=k + pad[0]), f32dev(U2, ld=k + pad[1])
    dT = DevMat(m, n, ld=m + pad[2])
    run([lrbg.desc("inner", dV.view, dU.view, dT.view, prec="bf16x3")], tune)
    assert dT.guards_intact()
    return V1, U2, dT.numpy()


def _dense(m, k, n, integer, seed, tune=None, pad=(0, 0, 0)):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    A = f(rng, m, k); U = f(rng, k, n)
    dA, dU = f32dev(A, ld=m + pad[0]), f32dev(U, ld=k + pad[1])
    dC = DevMat(m, n, ld=m + pad[2])
    run([lrbg.desc("dense_ts", dA.view, dU.view, dC.view, prec="bf16x3")], tune)
    assert dC.guards_intact()
    return A, U, dC.numpy()


@pytest.mark.parametrize("k,m,n", INN)
def test_inner_bf16x3_integer_bitwise(k, m, n):
    V1, U2, T = _inner(k, m, n, True, 10 + k, pad=(3, 1, 2))
    assert np.array_equal(T, ref_inner(V1, U2)[0])


@pytest.mark.parametrize("k,m,n", INN)
def test_inner_bf16x3_normal(k, m, n):
    V1, U2, T = _inner(k, m, n, False, 20 + k)
    Tref, D = ref_inner(V1, U2)
    assert oracle.normalized_error(T, Tref, D) <= TOL
    T32, D32 = ref_inner(f32(V1), f32(U2))
    assert oracle.normalized_error(T, T32, D32) <= 1e-6


@pytest.mark.parametrize("m,k,n", DTS)
def test_dense_bf16x3_integer_bitwise(m, k, n):
    A, U, C = _dense(m, k, n, True, 30 + m, pad=(1, 2, 3))
    assert np.array_equal(C, ref_dense_ts(A, U)[0])


@pytest.mark.parametrize("m,k,n", DTS)
def test_dense_bf16x3_normal(m, k, n):
    A, U, C = _dense(m, k, n, False, 40 + m)
    Cref, D = ref_dense_ts(A, U)
    assert oracle.normalized_error(C, Cref, D) <= TOL


def _bf_variants():
    try:
        lrbg.load()
        return [(i, n) for i, n in enumerate(lrbg.lrbg_variant_names()) if n.startswith(("dts3", "inn3"))]
    except Exception:
        return []


@pytest.mark.parametrize("vid,name", _bf_variants())
def test_every_bf16x3_variant(vid, name):
    if name.startswith("dts3"):
        rn = int(name.split("_rn")[1].split("_")[0])
        n = min(16 * rn, 128) - 3
        m = k = 200
        tune = tune_file(f"0 1 {bucket(max(m, k), 64)} {bucket(n, 8)} {name} 0")
        A, U, C = _dense(m, k, n, True, vid, tune=tune, pad=(1, 1, 1))
        assert np.array_equal(C, ref_dense_ts(A, U)[0])
        A, U, C = _dense(m, k, n, False, vid, tune=tune)
        Cref, D = ref_dense_ts(A, U)
        assert oracle.normalized_error(C, Cref, D) <= TOL
    else:
        rj = int(name.split("_rj")[1].split("_")[0])
        n = min(16 * rj, 128) - 1
        m, k = 40, 333
        tune = tune_file(f"1 1 {bucket(k, 64)} {bucket(max(m, n), 8)} {name} 0")
        V1, U2, T = _inner(k, m, n, True, vid, tune=tune, pad=(1, 1, 1))
        assert np.array_equal(T, ref_inner(V1, U2)[0])
        V1, U2, T = _inner(k, m, n, False, vid, tune=tune)
        Tref, D = ref_inner(V1, U2)
        assert oracle.normalized_error(T, Tref, D) <= TOL


def test_chain_bf16x3_inner_fp64_recomp():
    """Precision variant of the chain: the inner product on the split path,
    the recompression in FP64, error stated against the FP64 oracle."""
    import torch
    b, r = 512, 32
    errs = []
    for i in range(4):
        ci = inputs.chain_instance(4, i, b, r)
        dV1, dU2 = f32dev(ci.V1), f32dev(ci.U2)
        dU1, dV2 = DevMat.from_numpy(ci.U1), DevMat.from_numpy(ci.V2)
        dT, dW = DevMat(r, r), DevMat(b, b)
        lrbg.lrbg_grouped([lrbg.desc("inner", dV1.view, dU2.view, dT.view, prec="bf16x3"),
                           lrbg.desc("recomp", dU1.view, dV2.view, dW.view, s=dT.view)],
                          torch.cuda.current_stream())
        torch.cuda.synchronize()
        Tref, Wref = oracle.chain([ci.V1], [ci.U2], [ci.U1], [ci.V2])
        Dt = oracle.inner([np.abs(ci.V1)], [np.abs(ci.U2)])[0]
        Dw = oracle.recomp([np.abs(ci.U1)], [Dt], [np.abs(ci.V2)])[0]
        errs.append((oracle.normalized_error(dT.numpy(), Tref[0], Dt),
                     oracle.normalized_error(dW.numpy(), Wref[0], Dw)))
    assert max(e[0] for e in errs) <= TOL, errs
    assert max(e[1] for e in errs) <= TOL, errs


def test_error_table_every_bucket():
    """BF16x3 error against the FP64 oracle on the FP64 originals, for both
    products on every (b, r) bucket of the uneven batch; printed, and written
    to the file LRBG_ERROR_TABLE names when that variable is set."""
    import os
    rows = []
    for b in inputs.GROUPED_B:
        for r in [x for x in inputs.GROUPED_R if x <= b // 2]:
            e_d = e_i = 0.0
            for i in range(2):
                A, U = inputs.dense_ts_instance(9, 1000 * b + 10 * r + i, b, r)
                dA, dU, dC = f32dev(A), f32dev(U), DevMat(b, r)
                V1, U2 = inputs.inner_instance(9, 2000 * b + 10 * r + i, b, r)
                dV, dU2, dT = f32dev(V1), f32dev(U2), DevMat(r, r)
                run([lrbg.desc("dense_ts", dA.view, dU.view, dC.view, prec="bf16x3"),
                     lrbg.desc("inner", dV.view, dU2.view, dT.view, prec="bf16x3")])
                Cref, Dc = ref_dense_ts(A, U)
                Tref, Dt = ref_inner(V1, U2)
                e_d = max(e_d, oracle.normalized_error(dC.numpy(), Cref, Dc))
                e_i = max(e_i, oracle.normalized_error(dT.numpy(), Tref, Dt))
            rows.append((b, r, e_d, e_i))
    text = "b r dense_ts_err inner_err\n" + "\n".join(f"{b} {r} {d:.3e} {i:.3e}" for b, r, d, i in rows)
    if os.environ.get("LRBG_ERROR_TABLE"):
        with open(os.environ["LRBG_ERROR_TABLE"], "w") as f:
            f.write(text + "\n")
    print(text)
    assert max(max(d, i) for _, _, d, i in rows) <= TOL
