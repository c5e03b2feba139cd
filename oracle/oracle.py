"""Python front end of the C oracle -- TEST INFRASTRUCTURE ONLY.

Plain FP64 definitions of the batched low-rank products, evaluated by the
triple loops in ``lrbg_oracle.c`` (see that file for the conventions).  This
module marshals numpy arrays into pointer arrays and adds the error metric
the GPU results are judged by.

Matrices are 2-D numpy float64 arrays in column-major layout: either
Fortran-contiguous, or a column-major view into a larger buffer (leading
dimension = column stride / 8, which may exceed the row count).

Nothing here is used by the GPU library; only tests, the smoke check and the
CPU-baseline leg of the benchmark import it.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblrbg_oracle.so")
_lib = None

__all__ = [
    "load", "dense_ts", "inner", "recomp", "chain", "lr_mult", "lr_mult_round", "householder_qr", "lr_add_round",
    "blr_matvec", "dot2",
    "max_threads", "normalized_error", "normwise_error", "col_major",
]


def load():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LRBG_ORACLE_LIB") or _LIB_PATH   # mutation tests load a planted copy
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(path)
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    for name in ("orc_dense_ts", "orc_inner"):
        f = getattr(lib, name)
        f.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
        f.restype = None
    lib.orc_recomp.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
    lib.orc_recomp.restype = ctypes.c_int
    lib.orc_lr_mult.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
    lib.orc_lr_mult.restype = ctypes.c_int
    lib.orc_householder_qr.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
    lib.orc_householder_qr.restype = ctypes.c_int
    lib.orc_dot2.argtypes = [i64, vp, i64, vp, i64]
    lib.orc_dot2.restype = ctypes.c_double
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(load().orc_max_threads())


def col_major(rows: int, cols: int, ld: int | None = None, fill=np.nan) -> np.ndarray:
    """A rows x cols column-major float64 matrix with leading dimension ld."""
    ld = rows if ld is None else ld
    buf = np.full((max(cols, 1), max(ld, 1)), fill, dtype=np.float64)
    return buf.T[:rows, :cols]


def _ld(x: np.ndarray) -> int:
    if x.dtype != np.float64 or x.ndim != 2:
        raise TypeError("oracle operands are 2-D float64 arrays")
    if x.size == 0 or (x.shape[0] <= 1 and x.shape[1] <= 1):
        return max(x.shape[0], 1)
    if x.shape[0] > 1 and x.strides[0] != 8:
        raise ValueError("oracle operands must be column-major (unit row stride)")
    if x.shape[1] <= 1:
        return max(x.shape[0], 1)
    ld, rem = divmod(x.strides[1], 8)
    if rem or ld < x.shape[0]:
        raise ValueError("bad column stride")
    return ld


def _arrays(mats: Sequence[np.ndarray]):
    ptrs = np.array([m.ctypes.data for m in mats], dtype=np.uintp)
    lds = np.array([_ld(m) for m in mats], dtype=np.int32)
    return ptrs, lds


def _i32(vals):
    return np.ascontiguousarray(np.asarray(vals, dtype=np.int32))


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def dense_ts(As, Us, nthreads: int = 0, out=None):
    """C_t = A_t U_t for each instance t (A m x k, U k x n)."""
    cnt = len(As)
    m = _i32([a.shape[0] for a in As]); k = _i32([a.shape[1] for a in As])
    n = _i32([u.shape[1] for u in Us])
    for a, u in zip(As, Us):
        if u.shape[0] != a.shape[1]:
            raise ValueError("inner dimensions differ")
    Cs = out if out is not None else [col_major(int(m[t]), int(n[t])) for t in range(cnt)]
    pa, la = _arrays(As); pu, lu = _arrays(Us); pc, lc = _arrays(Cs)
    load().orc_dense_ts(cnt, _p(m), _p(n), _p(k), _p(pa), _p(la), _p(pu), _p(lu), _p(pc), _p(lc), nthreads)
    return Cs


def inner(V1s, U2s, nthreads: int = 0, out=None):
    """T_t = V1_t^T U2_t for each instance t (V1 k x m, U2 k x n)."""
    cnt = len(V1s)
    k = _i32([v.shape[0] for v in V1s]); m = _i32([v.shape[1] for v in V1s])
    n = _i32([u.shape[1] for u in U2s])
    for v, u in zip(V1s, U2s):
        if u.shape[0] != v.shape[0]:
            raise ValueError("contraction lengths differ")
    Ts = out if out is not None else [col_major(int(m[t]), int(n[t])) for t in range(cnt)]
    pv, lv = _arrays(V1s); pu, lu = _arrays(U2s); pt, lt = _arrays(Ts)
    load().orc_inner(cnt, _p(m), _p(n), _p(k), _p(pv), _p(lv), _p(pu), _p(lu), _p(pt), _p(lt), nthreads)
    return Ts


def recomp(U1s, Ss, V2s, nthreads: int = 0, out=None):
    """W_t = U1_t (S_t V2_t^T) (U1 m x k, S k x k, V2 n x k)."""
    cnt = len(U1s)
    m = _i32([u.shape[0] for u in U1s]); k = _i32([u.shape[1] for u in U1s])
    n = _i32([v.shape[0] for v in V2s])
    for u, s, v in zip(U1s, Ss, V2s):
        if s.shape != (u.shape[1], u.shape[1]) or v.shape[1] != u.shape[1]:
            raise ValueError("core / basis shapes differ")
    Ws = out if out is not None else [col_major(int(m[t]), int(n[t])) for t in range(cnt)]
    pu, lu = _arrays(U1s); ps, ls = _arrays(Ss); pv, lv = _arrays(V2s); pw, lw = _arrays(Ws)
    rc = load().orc_recomp(cnt, _p(m), _p(n), _p(k), _p(pu), _p(lu), _p(ps), _p(ls),
                           _p(pv), _p(lv), _p(pw), _p(lw), nthreads)
    if rc:
        raise MemoryError("oracle recomp: allocation failed")
    return Ws


def chain(V1s, U2s, U1s, V2s, nthreads: int = 0):
    """Low-rank x low-rank chain: T = V1^T U2, then W = U1 (T V2^T)."""
    Ts = inner(V1s, U2s, nthreads)
    Ws = recomp(U1s, Ts, V2s, nthreads)
    return Ts, Ws


def lr_mult(AVs, BUs, AXs, BXs, nthreads: int = 0):
    """The paper's low-rank product G = A_X (A_{V^T} B_U) B_X, in Alg. 1 order."""
    cnt = len(AVs)
    kk = _i32([a.shape[0] for a in AVs]); ra = _i32([a.shape[1] for a in AVs])
    rb = _i32([b.shape[1] for b in BUs])
    Gs = [col_major(int(ra[t]), int(rb[t])) for t in range(cnt)]
    p1, l1 = _arrays(AVs); p2, l2 = _arrays(BUs); p3, l3 = _arrays(AXs); p4, l4 = _arrays(BXs)
    pg, lg = _arrays(Gs)
    rc = load().orc_lr_mult(cnt, _p(ra), _p(rb), _p(kk), _p(p1), _p(l1), _p(p2), _p(l2),
                            _p(p3), _p(l3), _p(p4), _p(l4), _p(pg), _p(lg), nthreads)
    if rc:
        raise MemoryError("oracle lr_mult: allocation failed")
    return Gs


def lr_mult_round(AU, AV, AX, BU, BX, BV, kmax: int, tol: float):
    """The product of two low-rank blocks recompressed to rank <= kmax:
    G = A_X (A_V^T B_U) B_X (Alg. 1, the oracle's loops), its singular value
    decomposition (LAPACK through numpy, a library step), truncation to the
    k largest singular values above tol * sigma_1, and the new bases A_U X_k,
    B_V Y_k (the oracle's loops).  Returns (U, sigma, V, k) with U, V
    b x kmax and sigma of length kmax, zero beyond k."""
    G = lr_mult([AV], [BU], [AX], [BX])[0]
    Xk, sig, Yk, k = _truncate(G, kmax, tol)
    U = dense_ts([AU], [Xk])[0]
    V = dense_ts([BV], [Yk])[0]
    return U, sig, V, k


def householder_qr(Ws, nthreads: int = 0):
    """Thin QR W_t = Q_t R_t of each W_t (m x n) by Householder reflections,
    Q m x p with orthonormal columns and R p x n upper trapezoidal with a
    non-negative diagonal, p = min(m, n) (the oracle's loops).  Returns a
    list of (Q, R)."""
    cnt = len(Ws)
    m = _i32([w.shape[0] for w in Ws]); n = _i32([w.shape[1] for w in Ws])
    Qs = [col_major(int(m[t]), int(min(m[t], n[t]))) for t in range(cnt)]
    Rs = [col_major(int(min(m[t], n[t])), int(n[t])) for t in range(cnt)]
    pw, lw = _arrays(Ws); pq, lq = _arrays(Qs); pr, lr = _arrays(Rs)
    rc = load().orc_householder_qr(cnt, _p(m), _p(n), _p(pw), _p(lw), _p(pq), _p(lq), _p(pr), _p(lr), nthreads)
    if rc:
        raise MemoryError("oracle householder_qr: allocation failed")
    return list(zip(Qs, Rs))


def _truncate(M, kmax: int, tol: float):
    """SVD of the small core M (LAPACK through numpy, a library step) and
    the truncation rule shared by the recompressed product and the rounded
    addition: keep the k <= kmax largest singular values above tol * sigma_1
    (none if sigma_1 = 0).  Returns (X_k, sigma, Y_k, k) with X_k, Y_k padded
    with zero columns to kmax and sigma of length kmax, zero beyond k."""
    ra, rb = M.shape
    if M.size == 0:
        s = np.zeros(0); X = np.zeros((ra, 0)); Yt = np.zeros((0, rb))
    else:
        X, s, Yt = np.linalg.svd(M, full_matrices=False)
    k = 0
    while k < len(s) and k < kmax and s[0] > 0 and s[k] > tol * s[0]:
        k += 1
    Xk = col_major(ra, kmax, fill=0.0); Yk = col_major(rb, kmax, fill=0.0)
    Xk[:, :k] = X[:, :k]; Yk[:, :k] = Yt[:k, :].T
    sig = np.zeros(kmax); sig[:k] = s[:k]
    return Xk, sig, Yk, k


def lr_add_round(AU, AV, AX, BU, BX, BV, kmax: int, tol: float):
    """Rounded addition of two low-rank blocks A = A_U A_X A_V^T and
    B = B_U B_X B_V^T (b x b, ranks ra and rb, bases of any conditioning):
    A + B = [A_U | B_U] diag(A_X, B_X) [A_V | B_V]^T; Householder QR of both
    stacked bases (the oracle's loops), the small core
    M = R_U diag(A_X, B_X) R_V^T (the oracle's recompression loops), its
    SVD and truncation (as in ``lr_mult_round``), and the new bases Q_U X_k
    and Q_V Y_k (the oracle's loops).  Returns (U, sigma, V, k) with U, V
    b x kmax and sigma of length kmax, zero beyond k."""
    b, ra = AU.shape
    rb = BU.shape[1]
    WU = col_major(b, ra + rb); WU[:, :ra] = AU; WU[:, ra:] = BU
    WV = col_major(b, ra + rb); WV[:, :ra] = AV; WV[:, ra:] = BV
    (QU, RU), (QV, RV) = householder_qr([WU, WV])
    D = col_major(ra + rb, ra + rb, fill=0.0)
    D[:ra, :ra] = AX; D[ra:, ra:] = BX
    M = recomp([RU], [D], [RV])[0]
    Xk, sig, Yk, k = _truncate(M, kmax, tol)
    U = dense_ts([QU], [Xk])[0]
    V = dense_ts([QV], [Yk])[0]
    return U, sig, V, k


def blr_matvec(diag, U, V, X, nthreads: int = 0, rows=None):
    """Block low-rank matrix times multiple right-hand sides (the application
    of Sec. 7): Y_i = A_ii X_i + sum over j != i of U_ij (V_ij^T X_j), each
    low-rank block applied as the paper's low-rank product does, rank-sized
    factor first.  diag[i]: b x b; U[i][j], V[i][j]: b x r (None on the
    diagonal); X[j]: b x nrhs.  The terms of a block row are added in order
    of j, after the diagonal term.  Returns the list of Y_i (only the block
    rows listed in `rows`, in that order, when given; blocks of other rows
    are not read)."""
    nb = len(X)
    rows = list(range(nb)) if rows is None else list(rows)
    Ys = dense_ts([diag[i] for i in rows], [X[i] for i in rows], nthreads=nthreads)
    pos = {i: t for t, i in enumerate(rows)}
    pairs = [(i, j) for i in rows for j in range(nb) if i != j]
    if not pairs:
        return Ys
    Ps = inner([V[i][j] for i, j in pairs], [X[j] for i, j in pairs], nthreads=nthreads)
    Zs = dense_ts([U[i][j] for i, j in pairs], Ps, nthreads=nthreads)
    for (i, j), Z in zip(pairs, Zs):
        Ys[pos[i]] += Z
    return Ys


def dot2(x: np.ndarray, y: np.ndarray) -> float:
    """Compensated dot product (Ogita-Rump-Oishi Dot2) of two 1-D vectors."""
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("dot2 takes two 1-D vectors of equal length")
    x = np.asarray(x, dtype=np.float64); y = np.asarray(y, dtype=np.float64)
    return float(load().orc_dot2(x.shape[0], ctypes.c_void_p(x.ctypes.data), x.strides[0] // 8,
                                 ctypes.c_void_p(y.ctypes.data), y.strides[0] // 8))


def normalized_error(C: np.ndarray, Cref: np.ndarray, D: np.ndarray) -> float:
    """Componentwise normalised error max_ij |C - Cref| / D_ij.

    D is |A||B| (the product of elementwise absolute values, evaluated by the
    oracle in FP64); the standard forward error bound of a product reads
    |C_hat - C| <= gamma_k |A||B|, so this is the natural scale.  Where
    D_ij == 0 the exact result is 0 and C_ij must be exactly zero (sign of
    zero ignored); a non-zero value there returns +inf.  NaN anywhere in C
    returns +inf.
    """
    C = np.asarray(C, dtype=np.float64); Cref = np.asarray(Cref, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    if C.shape != Cref.shape or C.shape != D.shape:
        raise ValueError("shape mismatch")
    if C.size == 0:
        return 0.0
    if not np.all(np.isfinite(C)):
        return float("inf")
    diff = np.abs(C - Cref)
    zero = D == 0
    if np.any(C[zero] != 0):
        return float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(zero, 0.0, diff / np.where(zero, 1.0, D))
    return float(e.max())


def normwise_error(C: np.ndarray, Cref: np.ndarray, a_fro: float, b_fro: float) -> float:
    """max_ij |C - Cref| / (||A||_F ||B||_F)."""
    if C.size == 0:
        return 0.0
    den = a_fro * b_fro
    d = float(np.max(np.abs(np.asarray(C) - np.asarray(Cref))))
    return d / den if den > 0 else (0.0 if d == 0 else float("inf"))
