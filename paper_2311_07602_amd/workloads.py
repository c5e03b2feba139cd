"""Device-resident synthetic workloads shaped like the paper's batches.

Allocates operand pools on the GPU, fills them from the seeded generators of
:mod:`.inputs`, and returns lrbg descriptors over them.  No product
arithmetic happens here.

  grouped(count)   uneven batch: per instance b ~ U{64,...,1024}, r ~ U{ranks
                   <= b/2}; two products per instance, C = A U (b x b . b x r)
                   and T = V1^T U2 (r x b . b x r); N(0,1) entries.
  dense_uniform()  count x (A b x b . U b x r), N(0,1).
  chain(count)     low-rank x low-rank chain: T = V1^T U2, W = U1 (T V2^T)
                   with orthonormal bases and log-spaced singular values
                   folded into V (generated on the host per instance).
  lrmult(count)    the paper's batched low-rank product at one (b, r):
                   G = X_A (V_A^T U_B) X_B, all four operands N(0,1).
  blr(nb, b)       a weakly admissible BLR matrix (dense diagonal blocks,
                   rank-r off-diagonal blocks U V^T with the log-spaced
                   scalings of the chain folded into V) and nrhs N(0,1)
                   right-hand sides, in the device layout of blr.BlrMatvec.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from . import inputs, lrbg


@dataclass
class Workload:
    name: str
    descs: list
    pools: list = field(default_factory=list)       # tensors kept alive
    meta: dict = field(default_factory=dict)
    # per instance: (b, r, offsets ...) used to read operands back for checks
    index: list = field(default_factory=list)


def _cm(pool, off, rows, cols):
    """rows x cols column-major view (ld = rows) of a flat pool at `off`."""
    return pool[off:off + rows * cols].view(cols, rows).T


def grouped(count: int = 20000, seed: int = 3, device="cuda", dtype=None, prec: str = "fp64") -> Workload:
    import torch
    dtype = dtype or (torch.float64 if prec == "fp64" else torch.float32)
    shapes = inputs.grouped_shapes(count, seed)
    in_sizes, out_sizes = [], []
    for b, r in shapes:
        in_sizes += [b * b, b * r, b * r, b * r]          # A, U, V1, U2
        out_sizes += [b * r, r * r]                      # C, T
    in_off, in_total = inputs.pool_layout(in_sizes)
    out_off, out_total = inputs.pool_layout(out_sizes)
    pin = inputs.device_normal(in_total, seed=1000 * seed + 1, device=device, dtype=dtype)
    pout = torch.empty(out_total, dtype=torch.float64, device=device)
    descs, index = [], []
    for i, (b, r) in enumerate(shapes):
        oA, oU, oV, oU2 = (int(x) for x in in_off[4 * i:4 * i + 4])
        oC, oT = (int(x) for x in out_off[2 * i:2 * i + 2])
        A = _cm(pin, oA, b, b); U = _cm(pin, oU, b, r); V1 = _cm(pin, oV, b, r); U2 = _cm(pin, oU2, b, r)
        C = _cm(pout, oC, b, r); T = _cm(pout, oT, r, r)
        descs.append(lrbg.desc("dense_ts", A, U, C, prec=prec))
        descs.append(lrbg.desc("inner", V1, U2, T, prec=prec))
        index.append((b, r, oA, oU, oV, oU2, oC, oT))
    return Workload("grouped", descs, [pin, pout], {"count": count, "seed": seed, "shapes": shapes,
                                                    "prec": prec}, index)


def grouped_operands(w: Workload, i: int):
    """Host copies (float64, column-major) of instance i's operands/outputs."""
    pin, pout = w.pools
    b, r, oA, oU, oV, oU2, oC, oT = w.index[i]
    def host(pool, off, rows, cols):
        return np.asfortranarray(_cm(pool, off, rows, cols).double().cpu().numpy())
    return dict(A=host(pin, oA, b, b), U=host(pin, oU, b, r), V1=host(pin, oV, b, r), U2=host(pin, oU2, b, r),
                C=host(pout, oC, b, r), T=host(pout, oT, r, r))


def dense_uniform(count: int = 64, b: int = 256, r: int = 16, seed: int = 1, device="cuda") -> Workload:
    import torch
    sizes = []
    for _ in range(count):
        sizes += [b * b, b * r]
    off, total = inputs.pool_layout(sizes)
    pin = inputs.device_normal(total, seed=seed, device=device)
    oo, ototal = inputs.pool_layout([b * r] * count)
    pout = torch.empty(ototal, dtype=torch.float64, device=device)
    descs, index = [], []
    for i in range(count):
        oA, oU = int(off[2 * i]), int(off[2 * i + 1])
        descs.append(lrbg.desc("dense_ts", _cm(pin, oA, b, b), _cm(pin, oU, b, r), _cm(pout, int(oo[i]), b, r)))
        index.append((b, r, oA, oU, int(oo[i])))
    return Workload("dense_uniform", descs, [pin, pout], {"count": count, "b": b, "r": r}, index)


def chain(count: int = 4096, b: int = 512, r: int = 32, cfg: int = 2, device="cuda",
          operand_dtype=None, prec: str = "fp64") -> Workload:
    """Chain instances generated on the host (QR per basis), uploaded once.

    prec="bf16x3" stores V1, U2 in FP32 (RNE-rounded from the FP64 draw) and
    runs the inner product on the split-bf16 path; U1, V2, T, W stay FP64.
    """
    import torch
    per = 4 * b * r
    host = inputs.chain_instances(cfg, count, b, r)      # [i, operand, col, row]
    pin = torch.from_numpy(host.reshape(-1)).to(device)
    del host
    small = None
    if prec == "bf16x3":
        small = pin.view(count, 4, r * b)[:, 1:3].float().contiguous().reshape(-1)   # V1, U2 as FP32
    T = torch.empty(count * r * r, dtype=torch.float64, device=device)
    W = torch.empty(count * b * b, dtype=torch.float64, device=device)
    descs_inner, descs_rec, index = [], [], []
    for i in range(count):
        base = i * per
        U1 = _cm(pin, base, b, r); V1 = _cm(pin, base + b * r, b, r)
        U2 = _cm(pin, base + 2 * b * r, b, r); V2 = _cm(pin, base + 3 * b * r, b, r)
        Ti = _cm(T, i * r * r, r, r); Wi = _cm(W, i * b * b, b, b)
        if small is not None:
            V1 = _cm(small, i * 2 * b * r, b, r); U2 = _cm(small, i * 2 * b * r + b * r, b, r)
        descs_inner.append(lrbg.desc("inner", V1, U2, Ti, prec=prec))
        descs_rec.append(lrbg.desc("recomp", U1, V2, Wi, s=Ti))
        index.append(i)
    pools = [pin, T, W] + ([small] if small is not None else [])
    return Workload("chain", descs_inner + descs_rec, pools,
                    {"count": count, "b": b, "r": r, "cfg": cfg, "prec": prec}, index)


def chain_host_instance(w: Workload, i: int):
    """Host operands (FP64 originals) and device outputs of chain instance i."""
    import torch  # noqa: F401
    pin, T, W = w.pools[:3]
    b, r = w.meta["b"], w.meta["r"]
    base = i * 4 * b * r
    ops = [np.asfortranarray(_cm(pin, base + t * b * r, b, r).cpu().numpy()) for t in range(4)]
    return dict(U1=ops[0], V1=ops[1], U2=ops[2], V2=ops[3],
                T=np.asfortranarray(_cm(T, i * r * r, r, r).cpu().numpy()),
                W=np.asfortranarray(_cm(W, i * b * b, b, b).cpu().numpy()))


def lrmult(count: int = 20000, b: int = 1024, r: int = 16, seed: int = 5, device="cuda") -> Workload:
    """`count` instances of G = X_A (V_A^T U_B) X_B with V_A, U_B b x r and
    X_A, X_B, G r x r, the operands of one instance adjacent in one pool."""
    import torch
    sizes = [b * r, b * r, r * r, r * r]
    off1, per = inputs.pool_layout(sizes)
    pin = inputs.device_normal(count * per, seed=seed, device=device)
    offg, per_g = inputs.pool_layout([r * r])
    pout = torch.empty(count * per_g, dtype=torch.float64, device=device)
    descs, index = [], []
    for i in range(count):
        base = i * per
        oV, oU, oXA, oXB = (base + int(o) for o in off1)
        oG = i * per_g
        descs.append(lrbg.desc("lrmult", _cm(pin, oV, b, r), _cm(pin, oU, b, r), _cm(pout, oG, r, r),
                               s=_cm(pin, oXA, r, r), e=_cm(pin, oXB, r, r)))
        index.append((oV, oU, oXA, oXB, oG))
    return Workload("lrmult", descs, [pin, pout], {"count": count, "b": b, "r": r, "seed": seed, "per": per,
                                                  "offs": [int(o) for o in off1], "per_g": per_g}, index)


def lrmult_operands(w: Workload, i: int):
    """Host copies (float64, column-major) of lrmult instance i."""
    pin, pout = w.pools
    b, r = w.meta["b"], w.meta["r"]
    oV, oU, oXA, oXB, oG = w.index[i]
    def host(pool, off, rows, cols):
        return np.asfortranarray(_cm(pool, off, rows, cols).cpu().numpy())
    return dict(AV=host(pin, oV, b, r), BU=host(pin, oU, b, r), AX=host(pin, oXA, r, r),
                BX=host(pin, oXB, r, r), G=host(pout, oG, r, r))


def blr(nb: int = 64, b: int = 512, r: int = 8, nrhs: int = 8, seed: int = 9, device="cuda"):
    """A BlrMatvec filled with seeded synthetic blocks (all on the device)."""
    import torch
    from .blr import BlrMatvec
    m = BlrMatvec(nb, b, r, nrhs, device=device)
    m.rows.copy_(inputs.device_normal(m.rows.numel(), seed=seed, device=device).view_as(m.rows))
    sig = torch.from_numpy(inputs.sigma_profile(r)).to(device)
    m.vs.copy_(inputs.device_normal(m.vs.numel(), seed=seed + 1, device=device).view_as(m.vs))
    m.vs.mul_(sig.view(1, 1, r, 1))
    m.xs[:, :, :b].copy_(inputs.device_normal(nb * nrhs * b, seed=seed + 2, device=device).view(nb, nrhs, b))
    return m


def work_totals(descs) -> Tuple[float, float]:
    """Useful flops and compulsory bytes of a descriptor list (host accounting,
    the same formulas as the library's plan statistics)."""
    st = lrbg.lrbg_schedule_stats(descs)
    return st["useful_flops"], st["hbm_bytes"]
