"""GPU parity of the fused low-rank product G = X_A (V_A^T U_B) X_B (Alg. 1)
against the FP64 oracle.

Integer inputs give bitwise-identical results (every partial sum is exact);
N(0,1) inputs stay within 1e-13 of the oracle, componentwise normalised by
|X_A| |V_A|^T |U_B| |X_B|.  Outputs sit inside guard bands; input padding
holds NaN so that a read outside an operand poisons the result.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import inputs, lrbg

from gpu_util import DevMat, ref_inner, ref_lrmult

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


def _operands(k, ra, rb, integer, seed):
    rng = np.random.default_rng(seed)
    f = inputs.integer_f if integer else inputs.normal_f
    return f(rng, k, ra), f(rng, k, rb), f(rng, ra, ra), f(rng, rb, rb)


def _dev(AV, BU, AX, BX, pad):
    k, ra = AV.shape
    rb = BU.shape[1]
    return (DevMat.from_numpy(AV, ld=k + pad[0]), DevMat.from_numpy(BU, ld=k + pad[1]),
            DevMat.from_numpy(AX, ld=ra + pad[2]), DevMat.from_numpy(BX, ld=rb + pad[3]),
            DevMat(ra, rb, ld=ra + pad[4]))


def _plan_case(k, ra, rb, integer, seed, pad=(0, 0, 0, 0, 0), tune=None, expect=None):
    ops = _operands(k, ra, rb, integer, seed)
    dAV, dBU, dAX, dBX, dG = _dev(*ops, pad)
    d = lrbg.desc("lrmult", dAV.view, dBU.view, dG.view, s=dAX.view, e=dBX.view)
    if expect is not None:   # the forced variant is the one scheduled
        assert lrbg.lrbg_schedule_variants([d], tune_cache=tune) == [expect]
    p = lrbg.Plan([d], tune_cache=tune)
    p.execute(stream())
    sync()
    p.close()
    Gref, D = ref_lrmult(*ops)
    assert dG.guards_intact(), "write outside G"
    return dG.numpy(), Gref, D


# (k = b, ra, rb): square paper shapes, ragged ranks, tails of every tile
SHAPES = [(512, 8, 8), (512, 16, 16), (512, 32, 32), (1024, 32, 32), (2048, 16, 16), (512, 64, 64),
          (100, 7, 9), (333, 17, 31), (65, 33, 12), (1000, 64, 47), (3, 5, 5), (1, 1, 1), (37, 2, 64),
          (600, 48, 48), (129, 20, 3), (512, 128, 128), (1024, 96, 96), (1000, 100, 77), (300, 65, 128),
          (129, 128, 1), (77, 70, 120), (512, 96, 96), (2048, 96, 96), (333, 65, 96), (129, 96, 70),
          (1000, 80, 81), (95, 66, 90)]


@pytest.mark.parametrize("k,ra,rb", SHAPES)
def test_lrmult_integer_bitwise(k, ra, rb):
    G, Gref, _ = _plan_case(k, ra, rb, True, 700 + k + ra + 3 * rb, pad=(1, 2, 3, 1, 2))
    assert np.array_equal(G, Gref)


@pytest.mark.parametrize("k,ra,rb", SHAPES)
def test_lrmult_normal(k, ra, rb):
    G, Gref, D = _plan_case(k, ra, rb, False, 800 + k + ra + 3 * rb, pad=(0, 3, 0, 2, 1))
    assert oracle.normalized_error(G, Gref, D) <= TOL


def _forced_cache(name, b, r):
    def bucket(x, lo):
        v = lo
        while v < x:
            v *= 2
        return v
    f = tempfile.NamedTemporaryFile("w", suffix=".tune", delete=False)
    f.write(f"3 0 {bucket(b, 64)} {bucket(r, 8)} {name} 0\n")
    f.close()
    return f.name


def _lrm_variants():
    try:
        lrbg.load()
        return [n for n in lrbg.lrbg_variant_names() if n.startswith("lrm")]
    except Exception:
        return []


@pytest.mark.parametrize("name", _lrm_variants())
def test_every_lrmult_variant_forced(name):
    """Each fused tile at a rank below its limit (ragged), with a k tail."""
    rj = int(name.split("_rj")[1].split("_")[0])
    r = 128 if name.startswith("lrmb") else 96 if name.startswith("lrm96") else 16 * rj
    for ra, rb in ((r - 1, r - 3), (max(r // 2 - 1, 1), r)):
        k = 301
        tune = _forced_cache(name, k, max(ra, rb))
        try:
            G, Gref, _ = _plan_case(k, ra, rb, True, 900 + r + ra, pad=(1, 0, 2, 0, 1), tune=tune, expect=name)
            assert np.array_equal(G, Gref)
            G, Gref, D = _plan_case(k, ra, rb, False, 950 + r + ra, tune=tune, expect=name)
            assert oracle.normalized_error(G, Gref, D) <= TOL
        finally:
            os.unlink(tune)


def test_lr_batched_lrmult_entry_mixed_sizes():
    """The Alg. 2-style entry point over arrays: uneven (b, ra, rb) per instance."""
    rng_shapes = [(512, 8, 8), (77, 13, 5), (1024, 32, 16), (200, 64, 64), (0, 4, 4), (5, 0, 3), (300, 128, 90),
                  (0, 100, 100)]
    ops, devs = [], []
    for t, (k, ra, rb) in enumerate(rng_shapes):
        o = _operands(k, ra, rb, False, 1000 + t)
        ops.append(o)
        devs.append(_dev(*o, (t % 2, 1, 0, t % 3, 2)))
    def ptr(m):
        return m.view.data_ptr() if m.rows * m.cols else 0
    lrbg.lr_batched_lrmult([s[0] for s in rng_shapes], [s[1] for s in rng_shapes], [s[2] for s in rng_shapes],
                           [ptr(d[0]) for d in devs], [d[0].ld for d in devs],
                           [ptr(d[1]) for d in devs], [d[1].ld for d in devs],
                           [ptr(d[2]) for d in devs], [d[2].ld for d in devs],
                           [ptr(d[3]) for d in devs], [d[3].ld for d in devs],
                           [ptr(d[4]) for d in devs], [d[4].ld for d in devs], stream())
    sync()
    for (k, ra, rb), o, d in zip(rng_shapes, ops, devs):
        G = d[4].numpy()
        assert d[4].guards_intact()
        if ra == 0 or rb == 0:
            continue
        Gref, D = ref_lrmult(*o)
        if k == 0:
            assert np.all(G == 0)
        else:
            assert oracle.normalized_error(G, Gref, D) <= TOL


def test_lrmult_in_grouped_call_with_dependency():
    """LRMULT beside other products in one grouped call, its X_A being the
    output of an INNER product of the same call (runs one level later)."""
    rng = np.random.default_rng(1234)
    k, r = 384, 24
    V1 = inputs.normal_f(rng, 256, r); U2 = inputs.normal_f(rng, 256, r)
    AV, BU, _, BX = _operands(k, r, r, False, 1235)
    dV1, dU2 = DevMat.from_numpy(V1), DevMat.from_numpy(U2)
    dT = DevMat(r, r)
    dAV, dBU, _, dBX, dG = _dev(AV, BU, np.zeros((r, r), order="F"), BX, (0, 0, 0, 0, 0))
    descs = [lrbg.desc("lrmult", dAV.view, dBU.view, dG.view, s=dT.view, e=dBX.view),
             lrbg.desc("inner", dV1.view, dU2.view, dT.view)]
    p = lrbg.Plan(descs)
    assert p.stats()["levels"] == 2
    for _ in range(3):
        p.execute(stream())
    sync()
    p.close()
    T = dT.numpy()
    Tref, DT = ref_inner(V1, U2)
    assert oracle.normalized_error(T, Tref, DT) <= TOL
    Gref, D = ref_lrmult(AV, BU, np.asfortranarray(T), BX)
    assert oracle.normalized_error(dG.numpy(), Gref, D) <= TOL


def test_lrmult_one_shot_matches_plan_bitwise():
    ops = _operands(700, 30, 30, False, 77)
    outs = []
    for mode in ("plan", "grouped"):
        dAV, dBU, dAX, dBX, dG = _dev(*ops, (0, 0, 0, 0, 0))
        d = lrbg.desc("lrmult", dAV.view, dBU.view, dG.view, s=dAX.view, e=dBX.view)
        if mode == "plan":
            p = lrbg.Plan([d])
            p.execute(stream())
            sync()
            p.close()
        else:
            lrbg.lrbg_grouped([d], stream())
            sync()
        outs.append(dG.numpy())
    assert np.array_equal(outs[0], outs[1])
