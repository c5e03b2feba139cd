"""Seeded synthetic inputs for the batched low-rank products.

This module only draws numbers: it contains none of the products' arithmetic,
and both the GPU path and the oracle's tests take their inputs from it.

Recipe (the paper runs on normally distributed random entries in double
precision, Sec. 7; it uses no dataset):
  * host instances: ``numpy.random.default_rng([2311, 7602, cfg, i])`` per
    instance ``i``, so an instance's data never depends on which other
    instances share its batch; operands are drawn in the order listed and
    each matrix is filled in column-major order with ``standard_normal``;
  * low-rank chain bases: reduced QR of an N(0,1) matrix with the column signs
    fixed so that diag(R) > 0, singular scalings sigma_k = 10^(-8k/(r-1))
    folded into the V factors (V = Q diag(sigma));
  * large device-resident pools: ``torch.randn`` on the GPU from a seeded
    ``torch.Generator`` (a counter-based Philox stream), sliced per instance;
  * integer-valued inputs in {-8..8} (every partial sum of a product is then
    exact in binary64, so any summation order gives the same bits).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

SEED0 = (2311, 7602)

#: block sizes and ranks of the uneven grouped batch
GROUPED_B = (64, 128, 256, 512, 1024)
GROUPED_R = (8, 16, 32, 64, 128)


def instance_rng(cfg: int, i: int) -> np.random.Generator:
    return np.random.default_rng([SEED0[0], SEED0[1], int(cfg), int(i)])


def normal_f(rng: np.random.Generator, rows: int, cols: int, ld: int | None = None) -> np.ndarray:
    """rows x cols N(0,1) matrix, column-major, drawn column by column.

    With ld > rows the padding rows of the backing buffer hold NaN, so that a
    read of the gap would poison the result.
    """
    vals = rng.standard_normal(rows * cols).reshape(cols, rows).T
    if ld is None or ld == rows:
        return np.asfortranarray(vals)
    buf = np.full((cols, ld), np.nan)
    out = buf.T[:rows, :cols]
    out[...] = vals
    return out


def integer_f(rng: np.random.Generator, rows: int, cols: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    return np.asfortranarray(rng.integers(lo, hi + 1, size=(cols, rows)).T.astype(np.float64))


def sigma_profile(r: int, lo_exp: float = -8.0) -> np.ndarray:
    """Log-spaced singular scalings 1 .. 10^lo_exp (r values)."""
    if r == 1:
        return np.ones(1)
    return 10.0 ** (lo_exp * np.arange(r) / (r - 1))


def orthonormal_f(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Orthonormal columns: reduced QR of an N(0,1) matrix, diag(R) > 0."""
    g = normal_f(rng, rows, cols)
    q, rr = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return np.asfortranarray(q * s[None, :])


# ---------------------------------------------------------------- configs

def dense_ts_instance(cfg: int, i: int, b: int, r: int, integer: bool = False):
    """A (b x b) and U (b x r) for one dense x tall-skinny instance."""
    rng = instance_rng(cfg, i)
    f = integer_f if integer else normal_f
    return f(rng, b, b), f(rng, b, r)


def inner_instance(cfg: int, i: int, b: int, r: int, integer: bool = False):
    """V1 (b x r), U2 (b x r) for one inner-product instance."""
    rng = instance_rng(cfg, i)
    f = integer_f if integer else normal_f
    return f(rng, b, r), f(rng, b, r)


@dataclass
class ChainInstance:
    U1: np.ndarray
    V1: np.ndarray
    U2: np.ndarray
    V2: np.ndarray


def chain_instance(cfg: int, i: int, b: int, r: int) -> ChainInstance:
    """Two rank-r operands U1 V1^T and U2 V2^T with orthonormal U, V bases
    and log-spaced singular values folded into V."""
    rng = instance_rng(cfg, i)
    sig = sigma_profile(r)
    U1 = orthonormal_f(rng, b, r)
    V1 = np.asfortranarray(orthonormal_f(rng, b, r) * sig[None, :])
    U2 = orthonormal_f(rng, b, r)
    V2 = np.asfortranarray(orthonormal_f(rng, b, r) * sig[None, :])
    return ChainInstance(U1, V1, U2, V2)


def _chain_chunk(cfg: int, lo: int, hi: int, b: int, r: int, scale: np.ndarray, out: np.ndarray) -> None:
    g = np.empty((hi - lo, 4, b, r))
    for i in range(lo, hi):
        rng = instance_rng(cfg, i)
        for t in range(4):
            g[i - lo, t] = normal_f(rng, b, r)
    q, rr = np.linalg.qr(g, mode="reduced")                      # [n, 4, b, r], [n, 4, r, r]
    s = np.sign(np.diagonal(rr, axis1=-2, axis2=-1)).copy()     # [n, 4, r]
    s[s == 0] = 1.0
    q = q * s[..., None, :]
    q = q * scale[None, :, None, :]
    out[lo:hi] = np.swapaxes(q, -1, -2)


def chain_instances(cfg: int, count: int, b: int, r: int, chunk: int = 64, threads: int = 8) -> np.ndarray:
    """[count, 4, r, b] array: instance i's U1, V1, U2, V2, each stored
    column-major (row j of the last two axes is column j of the operand).

    Generated in this process: each instance draws its four N(0,1) matrices
    from its own seed in the order of :func:`chain_instance`, then one
    stacked reduced QR per chunk of instances orthonormalises them, with the
    same column-sign fix (diag(R) > 0) and the same scalings folded into V,
    so the values are those of :func:`chain_instance` instance by instance.
    Chunks run on a few threads of this process (each QR on one BLAS
    thread); no worker process is started."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((count, 4, r, b))
    sig = sigma_profile(r)
    scale = np.stack([np.ones(r), sig, np.ones(r), sig])          # [operand, col]
    jobs = [(lo, min(lo + chunk, count)) for lo in range(0, count, chunk)]
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except ImportError:
        limit = None
    try:
        with ThreadPoolExecutor(max(1, min(threads, len(jobs)))) as ex:
            for f in [ex.submit(_chain_chunk, cfg, lo, hi, b, r, scale, out) for lo, hi in jobs]:
                f.result()
    finally:
        if limit is not None:
            limit.restore_original_limits()
    return out


def grouped_shapes(count: int, seed: int = 3) -> List[Tuple[int, int]]:
    """(b, r) for each instance of the uneven grouped batch.

    b is uniform over {64,128,256,512,1024}; r is then uniform over the
    ranks in {8,16,32,64,128} with r <= b/2.
    """
    rng = np.random.default_rng([SEED0[0], SEED0[1], 1000 + seed])
    bs = rng.integers(0, len(GROUPED_B), size=count)
    u = rng.random(count)
    out = []
    for bi, uu in zip(bs, u):
        b = GROUPED_B[int(bi)]
        allowed = [r for r in GROUPED_R if r <= b // 2]
        out.append((b, allowed[min(int(uu * len(allowed)), len(allowed) - 1)]))
    return out


# ------------------------------------------------- device-resident pools

def device_normal(numel: int, seed: int, device="cuda", dtype=None):
    """``numel`` N(0,1) values on the device from a seeded torch Generator."""
    import torch
    dtype = dtype or torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(int(numel), generator=g, device=device, dtype=dtype)


def pool_layout(sizes: Sequence[int], align: int = 32) -> Tuple[np.ndarray, int]:
    """Element offsets of consecutive blocks (each rounded up to ``align``
    elements, 256 B for FP64) and the total element count."""
    sizes = np.asarray(sizes, dtype=np.int64)
    padded = (sizes + align - 1) // align * align
    offs = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes):
        offs[1:] = np.cumsum(padded)[:-1]
    return offs, int(padded.sum())
