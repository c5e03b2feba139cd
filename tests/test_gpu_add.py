"""GPU parity of the rounded addition of two low-rank blocks (batched QR of
the stacked bases, the small core, batched truncated SVD, new bases)
against the oracle (plain-loop Householder QR, recompression loops, LAPACK
SVD).

The GPU QR (LAPACK sign convention, blocked top to bottom) and the
oracle's (non-negative diagonal, one pass) differ in signs and rounding, and
singular vectors are unique up to sign, so the checks compare what is
unique: the kept rank, the singular values (within 1e-12 sigma_1), the
truncated sum U diag(sigma) V^T where the spectrum has a gap at the cut,
the full sum A + B when nothing is cut, and orthonormality of the kept U
and V columns.
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


def _instance(rng, b, ra, rb, orth=False):
    f = (lambda r, c: inputs.orthonormal_f(rng, r, c) if r >= c else inputs.normal_f(rng, r, c)) if orth \
        else (lambda r, c: inputs.normal_f(rng, r, c))
    return (f(b, ra), f(b, ra), inputs.normal_f(rng, ra, ra), f(b, rb), inputs.normal_f(rng, rb, rb), f(b, rb))


def _run(insts, kmax, tol, ld_pad=0):
    import torch
    n = len(insts)
    bs = [ins[0].shape[0] for ins in insts]
    dev = [[DevMat.from_numpy(m, ld=m.shape[0] + ld_pad) for m in ins] for ins in insts]
    outs = [(DevMat(b, kmax, ld=b + ld_pad), DevMat(b, kmax, ld=b + ld_pad)) for b in bs]
    sigma = torch.full((n * kmax,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ptr = lambda m: m.view.data_ptr() if m.rows * m.cols else 0
    col = lambda j: [ptr(d[j]) for d in dev]
    ld = lambda j: [d[j].ld for d in dev]
    print(f"lradd: {n} instances, b {sorted(set(bs))}, kmax {kmax}", flush=True)
    lrbg.lr_batched_lradd_round(bs, [ins[0].shape[1] for ins in insts], [ins[3].shape[1] for ins in insts],
                                col(0), ld(0), col(1), ld(1), col(2), ld(2), col(3), ld(3), col(4), ld(4),
                                col(5), ld(5), kmax, tol, [ptr(u) for u, _ in outs], [u.ld for u, _ in outs],
                                [ptr(v) for _, v in outs], [v.ld for _, v in outs],
                                sigma.data_ptr(), kout.data_ptr(), torch.cuda.current_stream())
    torch.cuda.synchronize()
    for u, v in outs:
        assert u.guards_intact() and v.guards_intact()
    sig = sigma.cpu().numpy().reshape(n, kmax)
    return [(outs[t][0].numpy(), sig[t], outs[t][1].numpy(), int(kout[t].item())) for t in range(n)]


def _full_sum(ins):
    AU, AV, AX, BU, BX, BV = ins
    return AU @ AX @ AV.T + BU @ BX @ BV.T


def _check(got, ref, smax, gap=True, orth_tol=1e-12):
    U, s, V, k = got
    Uo, so, Vo, ko = ref
    assert k == ko
    assert np.all(np.abs(s - so) <= 1e-12 * max(smax, 1e-300))
    assert np.all(s[k:] == 0) and np.all(U[:, k:] == 0) and np.all(V[:, k:] == 0)
    if k:
        assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= orth_tol
        assert np.max(np.abs(V[:, :k].T @ V[:, :k] - np.eye(k))) <= orth_tol
        if gap:
            P = U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T
            Po = Uo[:, :k] @ np.diag(so[:k]) @ Vo[:, :k].T
            assert np.max(np.abs(P - Po)) <= 1e-11 * smax


@pytest.mark.parametrize("b,ra,rb,orth", [(256, 8, 8, True), (512, 16, 16, False), (333, 32, 17, True),
                                          (64, 1, 7, False), (200, 32, 32, True), (1024, 24, 40, False),
                                          (130, 5, 11, True), (2048, 16, 16, True)])
def test_lradd_nothing_cut_is_the_sum(b, ra, rb, orth):
    """tol = 0 and kmax >= ra + rb: the result is the whole sum A + B."""
    rng = np.random.default_rng(11 * b + ra + rb)
    insts = [_instance(rng, b, ra, rb, orth) for _ in range(3)]
    kmax = min(64, ra + rb)
    got = _run(insts, kmax, 0.0)
    for ins, g in zip(insts, got):
        ref = oracle.lr_add_round(*ins, kmax, 0.0)
        _check(g, ref, ref[1][0])
        U, s, V, k = g
        full = _full_sum(ins)
        assert np.max(np.abs(U @ np.diag(s) @ V.T - full)) <= 1e-11 * ref[1][0]


@pytest.mark.parametrize("b,ra,rb", [(128, 4, 4), (700, 16, 16), (64, 32, 32), (1000, 20, 12)])
def test_lradd_planted_spectrum(b, ra, rb):
    """Complementary blocks of orthonormal P and Q with diagonal cores: the
    sum is P diag(s) Q^T, so the tolerance decides k exactly."""
    rng = np.random.default_rng(b + 3 * ra)
    s_ = ra + rb
    spec = 10.0 ** rng.uniform(-14, 0.5, s_)
    spec[: s_ // 3] = np.linspace(5.0, 3.0, s_ // 3)
    insts = []
    for _ in range(3):
        P = inputs.orthonormal_f(rng, b, s_)
        Q = inputs.orthonormal_f(rng, b, s_)
        perm = rng.permutation(s_)
        Pp, Qp, sp = P[:, perm], Q[:, perm], spec[perm]
        insts.append((np.asfortranarray(Pp[:, :ra]), np.asfortranarray(Qp[:, :ra]),
                      np.asfortranarray(np.diag(sp[:ra])), np.asfortranarray(Pp[:, ra:]),
                      np.asfortranarray(np.diag(sp[ra:])), np.asfortranarray(Qp[:, ra:])))
    for kmax, tol in ((s_, 1e-6), (s_ // 2, 1e-12), (max(1, s_ // 4), 0.0)):
        got = _run(insts, kmax, tol)
        for ins, g in zip(insts, got):
            ref = oracle.lr_add_round(*ins, kmax, tol)
            want = min(kmax, int(np.sum(spec > tol * spec.max())))
            assert ref[3] == want
            _check(g, ref, ref[1][0])


@pytest.mark.parametrize("b,ra,rb,kmax", [(1000, 24, 40, 32), (777, 20, 30, 16), (2047, 32, 32, 32),
                                           (96, 17, 47, 20), (33, 40, 24, 32)])
def test_lradd_wide_stack_rounded_to_at_most_half(b, ra, rb, kmax):
    """Stacks wider than 32 rounded to at most 32 columns (adding two rank-r
    blocks and keeping rank r), with ragged last row blocks and b below the
    stack width: a planted spectrum with a clear gap after kmax, tol = 0."""
    rng = np.random.default_rng(5 * b + ra + kmax)
    s_ = ra + rb
    if b < s_:
        # at most b directions: N(0,1) factors; singular values and orthonormality only
        insts = [_instance(rng, b, ra, rb) for _ in range(3)]
        for ins, g in zip(insts, _run(insts, kmax, 0.0)):
            ref = oracle.lr_add_round(*ins, kmax, 0.0)
            _check(g, ref, ref[1][0], gap=False)
        return
    spec = np.concatenate([np.linspace(5.0, 3.0, kmax), 10.0 ** rng.uniform(-3, -1, s_ - kmax)])
    insts = []
    for _ in range(3):
        P = inputs.orthonormal_f(rng, b, s_)
        Q = inputs.orthonormal_f(rng, b, s_)
        perm = rng.permutation(s_)
        Pp, Qp, sp = P[:, perm], Q[:, perm], spec[perm]
        insts.append((np.asfortranarray(Pp[:, :ra]), np.asfortranarray(Qp[:, :ra]),
                      np.asfortranarray(np.diag(sp[:ra])), np.asfortranarray(Pp[:, ra:]),
                      np.asfortranarray(np.diag(sp[ra:])), np.asfortranarray(Qp[:, ra:])))
    for ins, g in zip(insts, _run(insts, kmax, 0.0)):
        ref = oracle.lr_add_round(*ins, kmax, 0.0)
        _check(g, ref, ref[1][0])


def test_lradd_kmax_beyond_the_stack_width():
    """kmax above the stacked width of 16-, 32- and 64-wide classes (the
    general application kernels at their full top-part width, the output
    columns past the width zero-filled): everything is kept, so the result is
    the whole sum."""
    rng = np.random.default_rng(25)
    shapes = [(300, 5, 9), (257, 12, 13), (200, 20, 25), (96, 3, 2)]
    insts = [_instance(rng, b, ra, rb) for b, ra, rb in shapes]
    kmax = 40
    got = _run(insts, kmax, 0.0)
    for (b, ra, rb), ins, g in zip(shapes, insts, got):
        ref = oracle.lr_add_round(*ins, kmax, 0.0)
        _check(g, ref, ref[1][0], gap=False)
        U, s, V, k = g
        assert k == min(ra + rb, kmax)
        if ra + rb <= kmax:
            assert np.max(np.abs(U @ np.diag(s) @ V.T - _full_sum(ins))) <= 1e-11 * ref[1][0]


def test_lradd_shared_bases_rank_deficient_stack():
    """B on the same orthonormal bases as A: each stacked basis is exactly
    rank deficient (two copies of one basis); the sum is A_U (A_X + B_X)
    A_V^T and the new bases stay orthonormal."""
    rng = np.random.default_rng(21)
    b, r = 512, 16
    insts = []
    for _ in range(4):
        AU = inputs.orthonormal_f(rng, b, r); AV = inputs.orthonormal_f(rng, b, r)
        insts.append((AU, AV, inputs.normal_f(rng, r, r), AU, inputs.normal_f(rng, r, r), AV))
    got = _run(insts, 2 * r, 1e-10)
    for ins, g in zip(insts, got):
        U, s, V, k = g
        sx = np.linalg.svd(ins[2] + ins[4], compute_uv=False)
        assert k == r
        assert np.max(np.abs(s[:r] - sx)) <= 1e-12 * sx[0]
        assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-12
        assert np.max(np.abs(V[:, :k].T @ V[:, :k] - np.eye(k))) <= 1e-12
        full = ins[0] @ (ins[2] + ins[4]) @ ins[1].T
        assert np.max(np.abs(U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T - full)) <= 1e-12 * sx[0]


def test_lradd_ill_conditioned_bases_keep_orthonormal_outputs():
    """Bases with condition number 1e10 (N(0,1) times a graded diagonal): a
    Gram-matrix QR would lose orthogonality; the Householder one keeps the
    new bases orthonormal to working precision."""
    rng = np.random.default_rng(22)
    b, ra, rb = 640, 12, 12
    insts = []
    for _ in range(3):
        ins = list(_instance(rng, b, ra, rb))
        for j in (0, 1, 3, 5):
            ins[j] = np.asfortranarray(ins[j] * np.logspace(0, -10, ins[j].shape[1]))
        insts.append(tuple(ins))
    got = _run(insts, 24, 0.0)
    for ins, g in zip(insts, got):
        ref = oracle.lr_add_round(*ins, 24, 0.0)
        U, s, V, k = g
        assert k == ref[3]
        assert np.all(np.abs(s - ref[1]) <= 1e-12 * ref[1][0])
        assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-12
        assert np.max(np.abs(V[:, :k].T @ V[:, :k] - np.eye(k))) <= 1e-12


def test_lradd_mixed_shapes_degenerate_cases_and_ld_gaps():
    """One call over every width class, ragged last row blocks, fewer rows
    than stacked columns, empty blocks and zero ranks, with leading
    dimensions beyond the row counts."""
    rng = np.random.default_rng(23)
    shapes = [(256, 8, 8), (0, 4, 4), (5, 4, 3), (64, 0, 6), (100, 32, 32), (77, 1, 1), (1, 2, 2),
              (129, 16, 9), (64, 0, 0), (300, 30, 34)]
    insts = [_instance(rng, b, ra, rb, orth=(i % 2 == 0)) for i, (b, ra, rb) in enumerate(shapes)]
    kmax = 12
    got = _run(insts, kmax, 1e-9, ld_pad=3)
    for (b, ra, rb), ins, g in zip(shapes, insts, got):
        ref = oracle.lr_add_round(*ins, kmax, 1e-9)
        if b == 0 or ra + rb == 0:
            assert g[3] == 0 and np.all(g[1] == 0) and np.all(g[0] == 0) and np.all(g[2] == 0)
            continue
        _check(g, ref, ref[1][0], gap=False)


def test_lradd_cancellation_is_noise():
    """B = -A: the sum is zero; every singular value the GPU reports is at
    the rounding level of A's."""
    rng = np.random.default_rng(24)
    b, r = 256, 8
    insts = []
    for _ in range(2):
        AU, AV, AX = inputs.orthonormal_f(rng, b, r), inputs.orthonormal_f(rng, b, r), inputs.normal_f(rng, r, r)
        insts.append((AU, AV, AX, AU, np.asfortranarray(-AX), AV))
    got = _run(insts, 2 * r, 0.0)
    for ins, (U, s, V, k) in zip(insts, got):
        sa = np.linalg.svd(ins[2], compute_uv=False)[0]
        assert np.all(s <= 64 * r * 2.0 ** -52 * sa)
        if k:
            assert np.max(np.abs(U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T)) <= 64 * r * 2.0 ** -52 * sa


def test_lradd_rejects_bad_arguments():
    import torch
    rng = np.random.default_rng(25)
    ins = _instance(rng, 64, 40, 30)
    dev = [DevMat.from_numpy(m) for m in ins]
    u, v = DevMat(64, 8), DevMat(64, 8)
    sigma = torch.zeros(8, dtype=torch.float64, device="cuda")
    kout = torch.zeros(1, dtype=torch.int32, device="cuda")
    args = [[64], [40], [30]]
    for d in dev:
        args += [[d.view.data_ptr()], [d.ld]]
    with pytest.raises(RuntimeError, match="exceeds 64"):
        lrbg.lr_batched_lradd_round(*args, 8, 0.0, [u.view.data_ptr()], [u.ld], [v.view.data_ptr()], [v.ld],
                                    sigma.data_ptr(), kout.data_ptr())
    # U aliasing an input
    ins = _instance(rng, 64, 8, 8)
    dev = [DevMat.from_numpy(m) for m in ins]
    args = [[64], [8], [8]]
    for d in dev:
        args += [[d.view.data_ptr()], [d.ld]]
    with pytest.raises(RuntimeError, match="overlaps"):
        lrbg.lr_batched_lradd_round(*args, 8, 0.0, [dev[0].view.data_ptr()], [64], [v.view.data_ptr()], [v.ld],
                                    sigma.data_ptr(), kout.data_ptr())
