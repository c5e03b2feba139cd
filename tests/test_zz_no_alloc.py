"""The allocation-free recompressed product (lr_batched_lrmult_round_noalloc)
against the allocating entry point (lr_batched_lrmult_round): the same
kernels and schedules, so the same bits, on two calls in a row -- the second
smaller, so it runs over what the first left in the fixed scratch array --
and both within the recompressed product's oracle bar."""
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


def _instance(rng, b, ra, rb):
    AU = inputs.orthonormal_f(rng, b, ra) if b >= ra else inputs.normal_f(rng, b, ra)
    BV = inputs.orthonormal_f(rng, b, rb) if b >= rb else inputs.normal_f(rng, b, rb)
    return (AU, inputs.normal_f(rng, b, ra), inputs.normal_f(rng, ra, ra), inputs.normal_f(rng, b, rb),
            inputs.normal_f(rng, rb, rb), BV)


def _call(fn, insts, bs, kmax, tol):
    import torch
    n = len(insts)
    dev = [[DevMat.from_numpy(m) for m in ins] for ins in insts]
    outs = [(DevMat(b, kmax), DevMat(b, kmax)) for b in bs]
    sigma = torch.full((n * kmax,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ptr = lambda m: m.view.data_ptr() if m.rows * m.cols else 0
    col = lambda j: [ptr(d[j]) for d in dev]
    ld = lambda j: [d[j].ld for d in dev]
    fn(bs, [ins[0].shape[1] for ins in insts], [ins[3].shape[1] for ins in insts],
       col(0), ld(0), col(1), ld(1), col(2), ld(2), col(3), ld(3), col(4), ld(4), col(5), ld(5),
       kmax, tol, [ptr(u) for u, _ in outs], [u.ld for u, _ in outs], [ptr(v) for _, v in outs],
       [v.ld for _, v in outs], sigma.data_ptr(), kout.data_ptr(), torch.cuda.current_stream())
    torch.cuda.synchronize()
    for u, v in outs:
        assert u.guards_intact() and v.guards_intact()
    return ([u.numpy().copy() for u, _ in outs], [v.numpy().copy() for _, v in outs],
            sigma.cpu().numpy().reshape(n, kmax), kout.cpu().numpy())


def _oracle_bar(insts, got, kmax, tol):
    Us, Vs, sig, kk = got
    for t, ins in enumerate(insts):
        Uo, so, Vo, ko = oracle.lr_mult_round(*ins, kmax, tol)
        k = int(kk[t])
        assert k == ko
        smax = max(so[0], 1e-300)
        assert np.all(np.abs(sig[t] - so) <= 1e-12 * smax)
        if k:
            P = Us[t][:, :k] @ np.diag(sig[t][:k]) @ Vs[t][:, :k].T
            Po = Uo[:, :k] @ np.diag(so[:k]) @ Vo[:, :k].T
            assert np.max(np.abs(P - Po)) <= 1e-11 * smax
            assert np.allclose(Us[t][:, :k].T @ Us[t][:, :k], np.eye(k), atol=1e-12)


@pytest.mark.parametrize("first,second", [
    ([(256, 16, 16), (512, 32, 24), (300, 8, 8), (1024, 64, 40), (0, 4, 4), (128, 20, 12)] * 6,
     [(128, 8, 8), (64, 5, 3), (200, 16, 16)]),
])
def test_noalloc_matches_allocating_entry_point_twice(first, second):
    rng = np.random.default_rng(77)
    for shapes, kmax, tol in ((first, 16, 1e-10), (second, 8, 0.0)):
        print(f"noalloc call: {len(shapes)} products, kmax {kmax}", flush=True)
        insts = [_instance(rng, b, ra, rb) for b, ra, rb in shapes]
        bs = [s[0] for s in shapes]
        ref = _call(lrbg.lr_batched_lrmult_round, insts, bs, kmax, tol)
        got = _call(lrbg.lr_batched_lrmult_round_noalloc, insts, bs, kmax, tol)
        for a, b in zip(ref[0] + ref[1], got[0] + got[1]):
            assert np.array_equal(a, b)
        assert np.array_equal(ref[2], got[2]) and np.array_equal(ref[3], got[3])
        _oracle_bar(insts, got, kmax, tol)


def test_noalloc_rejects_oversize_batch_without_side_effects():
    """A batch beyond the fixed array is refused before any launch: the
    outputs keep their sentinel values."""
    import torch
    n, b, r = 2000, 64, 64
    rng = np.random.default_rng(5)
    small = _instance(rng, b, r, r)
    dev = [DevMat.from_numpy(m) for m in small]
    outs = [(DevMat(b, 64), DevMat(b, 64)) for _ in range(n)]
    sigma = torch.full((n * 64,), np.nan, dtype=torch.float64, device="cuda")
    kout = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ins = []
    for d in dev:
        ins += [[d.view.data_ptr()] * n, [d.ld] * n]
    with pytest.raises(RuntimeError, match="scratch"):
        lrbg.lr_batched_lrmult_round_noalloc([b] * n, [r] * n, [r] * n, *ins, 64, 0.0,
                                             [u.view.data_ptr() for u, _ in outs], [u.ld for u, _ in outs],
                                             [v.view.data_ptr() for _, v in outs], [v.ld for _, v in outs],
                                             sigma.data_ptr(), kout.data_ptr(), torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert torch.all(kout == -1) and torch.all(torch.isnan(sigma))
