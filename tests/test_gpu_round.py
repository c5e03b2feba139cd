"""GPU parity of the recompressed low-rank product (fused core G, batched
truncated SVD, new bases) against the oracle (Alg. 1 loops + LAPACK SVD).

Singular vectors are unique up to sign, so the checks compare what is
unique: the kept rank, the singular values (within 1e-12 sigma_1: G itself
agrees to ~1e-15 relative, and Weyl's inequality moves each singular value by
at most |dG|_2), the truncated product U diag(sigma) V^T where the spectrum
has a gap at the truncation, and orthonormality of the kept U and V columns.
"""
import numpy as np
import pytest

import oracle
from paper_2311_07602_amd import inputs, lrbg

from gpu_util import DevMat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lrbg.load()
    oracle.load()


def _instance(rng, b, ra, rb, spectrum=None):
    AU = inputs.orthonormal_f(rng, b, ra) if b >= ra else inputs.normal_f(rng, b, ra)
    BV = inputs.orthonormal_f(rng, b, rb) if b >= rb else inputs.normal_f(rng, b, rb)
    AV = inputs.normal_f(rng, b, ra)
    BU = inputs.normal_f(rng, b, rb)
    AX = inputs.normal_f(rng, ra, ra)
    BX = inputs.normal_f(rng, rb, rb)
    if spectrum is not None:   # planted: A_V^T B_U = I (shared orthonormal W), B_X = I
        r = ra
        W = inputs.orthonormal_f(rng, b, r)
        P = inputs.orthonormal_f(rng, r, r); Q = inputs.orthonormal_f(rng, r, r)
        AX = np.asfortranarray(P @ np.diag(spectrum) @ Q.T)
        AV = BU = W
        BX = np.asfortranarray(np.eye(r))
    return AU, AV, AX, BU, BX, BV


def _run(insts, bs, kmax, tol):
    import torch
    n = len(insts)
    dev = [[DevMat.from_numpy(m) for m in ins] for ins in insts]
    outs = [(DevMat(b, kmax), DevMat(b, kmax)) for b in bs]
    sigma = torch.full((n * kmax,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ptr = lambda m: m.view.data_ptr() if m.rows * m.cols else 0
    col = lambda j: [ptr(d[j]) for d in dev]
    ld = lambda j: [d[j].ld for d in dev]
    lrbg.lr_batched_lrmult_round(bs, [ins[0].shape[1] for ins in insts], [ins[3].shape[1] for ins in insts],
                                 col(0), ld(0), col(1), ld(1), col(2), ld(2), col(3), ld(3), col(4), ld(4),
                                 col(5), ld(5), kmax, tol, [ptr(u) for u, _ in outs], [u.ld for u, _ in outs],
                                 [ptr(v) for _, v in outs], [v.ld for _, v in outs],
                                 sigma.data_ptr(), kout.data_ptr(), torch.cuda.current_stream())
    torch.cuda.synchronize()
    for u, v in outs:
        assert u.guards_intact() and v.guards_intact()
    sig = sigma.cpu().numpy().reshape(n, kmax)
    return [(outs[t][0].numpy(), sig[t], outs[t][1].numpy(), int(kout[t].item())) for t in range(n)]


def _check(got, ref, smax_ref, gap=True):
    U, s, V, k = got
    Uo, so, Vo, ko = ref
    assert k == ko
    assert np.all(np.abs(s - so) <= 1e-12 * max(smax_ref, 1e-300))
    assert np.all(s[k:] == 0) and np.all(U[:, k:] == 0) and np.all(V[:, k:] == 0)
    if k:
        assert np.allclose(U[:, :k].T @ U[:, :k], np.eye(k), atol=1e-12)
        assert np.allclose(V[:, :k].T @ V[:, :k], np.eye(k), atol=1e-12)
        if gap:
            P = U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T
            Po = Uo[:, :k] @ np.diag(so[:k]) @ Vo[:, :k].T
            assert np.max(np.abs(P - Po)) <= 1e-11 * smax_ref


@pytest.mark.parametrize("b,r,kmax,tol", [(128, 8, 8, 1e-6), (512, 16, 12, 1e-6), (300, 32, 32, 1e-10),
                                          (1024, 64, 40, 1e-12), (64, 5, 8, 0.0), (100, 20, 3, 0.0)])
def test_round_planted_spectrum(b, r, kmax, tol):
    rng = np.random.default_rng(b + r)
    spec = np.sort(10.0 ** rng.uniform(-14, 0, r))[::-1].copy()
    spec[: r // 2] = np.linspace(4.0, 2.0, r // 2) if r >= 2 else spec[: r // 2]
    insts = [_instance(rng, b, r, r, spectrum=spec) for _ in range(3)]
    got = _run(insts, [b] * 3, kmax, tol)
    for ins, g in zip(insts, got):
        ref = oracle.lr_mult_round(*ins, kmax, tol)
        # a gap at the cut: the planted values are distinct, so the kept product is unique
        _check(g, ref, ref[1][0])


@pytest.mark.parametrize("b,ra,rb,kmax", [(256, 8, 8, 8), (512, 16, 24, 16), (333, 32, 17, 32), (64, 1, 7, 4),
                                          (200, 64, 64, 64), (5, 3, 2, 2)])
def test_round_random_full_rank(b, ra, rb, kmax):
    """N(0,1) cores kept to kmax >= min(ra, rb) with tol = 0: nothing is cut
    beyond the exact rank, so U diag(sigma) V^T is the whole product."""
    rng = np.random.default_rng(7 * b + ra + rb)
    insts = [_instance(rng, b, ra, rb) for _ in range(4)]
    kk = max(kmax, min(ra, rb))
    got = _run(insts, [b] * 4, kk, 0.0)
    for ins, g in zip(insts, got):
        ref = oracle.lr_mult_round(*ins, kk, 0.0)
        _check(g, ref, ref[1][0])
        AU, AV, AX, BU, BX, BV = ins
        full = AU @ (oracle.lr_mult([AV], [BU], [AX], [BX])[0]) @ BV.T
        U, s, V, k = g
        assert np.max(np.abs(U @ np.diag(s) @ V.T - full)) <= 1e-11 * ref[1][0]


def test_round_mixed_shapes_and_degenerate_cases():
    rng = np.random.default_rng(99)
    shapes = [(256, 8, 8), (0, 4, 4), (128, 16, 8), (64, 1, 1), (300, 32, 32)]
    insts = [_instance(rng, b, ra, rb) for b, ra, rb in shapes]
    insts[2] = (insts[2][0], insts[2][1], np.zeros((16, 16), order="F"), insts[2][3], insts[2][4], insts[2][5])
    got = _run(insts, [s[0] for s in shapes], 8, 1e-8)
    for (b, ra, rb), ins, g in zip(shapes, insts, got):
        ref = oracle.lr_mult_round(*ins, 8, 1e-8)
        if b == 0 or not np.any(ins[2]):      # zero core: nothing kept
            assert g[3] == 0 and np.all(g[1] == 0) and np.all(g[0] == 0) and np.all(g[2] == 0)
            continue
        _check(g, ref, ref[1][0], gap=False)


def test_round_plan_matches_one_shot_and_tracks_inputs():
    """The plan form runs the same kernels on the same schedules, so it
    reproduces the one-shot call bit for bit; a replay after the inputs
    changed in place computes from the new contents."""
    import torch
    rng = np.random.default_rng(2024)
    shapes = [(256, 8, 8), (512, 16, 12), (300, 32, 32), (0, 4, 4), (128, 40, 24)]
    kmax, tol = 12, 1e-8
    insts = [_instance(rng, b, ra, rb) for b, ra, rb in shapes]
    n = len(insts)
    dev = [[DevMat.from_numpy(m) for m in ins] for ins in insts]
    outs = [(DevMat(b, kmax), DevMat(b, kmax)) for b, _, _ in shapes]
    sigma = torch.full((n * kmax,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ptr = lambda m: m.view.data_ptr() if m.rows * m.cols else 0
    col = lambda j: [ptr(d[j]) for d in dev]
    ld = lambda j: [d[j].ld for d in dev]
    args = ([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes],
            col(0), ld(0), col(1), ld(1), col(2), ld(2), col(3), ld(3), col(4), ld(4), col(5), ld(5),
            kmax, tol, [ptr(u) for u, _ in outs], [u.ld for u, _ in outs], [ptr(v) for _, v in outs],
            [v.ld for _, v in outs], sigma.data_ptr(), kout.data_ptr())
    stream = torch.cuda.current_stream()

    def snapshot():
        torch.cuda.synchronize()
        for u, v in outs:
            assert u.guards_intact() and v.guards_intact()
        return ([u.numpy().copy() for u, _ in outs], [v.numpy().copy() for _, v in outs],
                sigma.cpu().numpy().copy(), kout.cpu().numpy().copy())

    def same(x, y):
        for a, b in zip(x, y):
            if isinstance(a, list):
                assert all(np.array_equal(p, q) for p, q in zip(a, b))
            else:
                assert np.array_equal(a, b)

    lrbg.lr_batched_lrmult_round(*args, stream=stream)
    one = snapshot()
    sigma.fill_(np.nan); kout.fill_(-1)
    with lrbg.RoundPlan(*args) as plan:
        plan.execute(stream)
        same(snapshot(), one)
        for t, (b, ra, rb) in enumerate(shapes):       # new A_X in place
            if b:
                dev[t][2].copy_from(inputs.normal_f(rng, ra, ra))
        plan.execute(stream)
        second = snapshot()
        plan.execute(stream)
        same(snapshot(), second)
    lrbg.lr_batched_lrmult_round(*args, stream=stream)
    same(snapshot(), second)
    for t, (b, ra, rb) in enumerate(shapes):
        if b == 0:
            continue
        ins = tuple(d.numpy() for d in dev[t])
        ref = oracle.lr_mult_round(*ins, kmax, tol)
        got = (second[0][t], second[2][t * kmax:(t + 1) * kmax], second[1][t], int(second[3][t]))
        _check(got, ref, ref[1][0], gap=False)


def test_round_plan_empty():
    import torch
    with lrbg.RoundPlan([], [], [], [], [], [], [], [], [], [], [], [], [], [], [], 4, 0.0, [], [], [], [],
                        8, 8) as plan:
        plan.execute(torch.cuda.current_stream())
