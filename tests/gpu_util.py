"""Helpers for the GPU parity tests: column-major device buffers with guard
bands, and the oracle-side reference + normalised error of each op."""
import numpy as np

import oracle

SENTINEL = -1.2345e300


def dev():
    import torch
    return torch.device("cuda:0")


class DevMat:
    """rows x cols column-major device matrix with leading dimension ld,
    inside a buffer with one guard column before and after; the padding
    rows and guard columns hold `fill`."""

    def __init__(self, rows, cols, ld=None, fill=SENTINEL, dtype=None):
        import torch
        self.rows, self.cols = rows, cols
        self.ld = max(ld if ld is not None else rows, 1)
        dtype = dtype or torch.float64
        self.buf = torch.full((cols + 2, self.ld), fill, dtype=dtype, device=dev())
        self.view = self.buf[1:cols + 1].T[:rows] if cols > 0 else self.buf[1:1].T[:rows]
        self.fill = fill

    @classmethod
    def from_numpy(cls, x, ld=None, gap=np.nan, dtype=None):
        import torch
        m = cls(x.shape[0], x.shape[1], ld, fill=gap, dtype=dtype)
        if x.size:
            m.buf[1:x.shape[1] + 1, :x.shape[0]] = torch.from_numpy(np.ascontiguousarray(x.T)).to(m.buf.dtype).to(dev())
        return m

    def copy_from(self, x):
        """Overwrite the matrix in place (same shape) from a host array."""
        import torch
        assert x.shape == (self.rows, self.cols)
        if x.size:
            self.buf[1:self.cols + 1, :self.rows] = torch.from_numpy(np.ascontiguousarray(x.T)).to(self.buf.dtype).to(dev())

    def numpy(self):
        b = self.buf.cpu().numpy()
        return np.asfortranarray(b[1:self.cols + 1, :self.rows].T.astype(np.float64))

    def guards_intact(self):
        b = self.buf.cpu().numpy()
        def same(x):
            return np.all(x == self.fill) if not np.isnan(self.fill) else np.all(np.isnan(x))
        ok = same(b[0]) and same(b[-1])
        if self.ld > self.rows:
            ok = ok and same(b[1:self.cols + 1, self.rows:])
        return bool(ok)


def ref_dense_ts(A, U):
    C = oracle.dense_ts([A], [U])[0]
    D = oracle.dense_ts([np.asfortranarray(np.abs(A))], [np.asfortranarray(np.abs(U))])[0]
    return C, D


def ref_inner(V1, U2):
    T = oracle.inner([V1], [U2])[0]
    D = oracle.inner([np.asfortranarray(np.abs(V1))], [np.asfortranarray(np.abs(U2))])[0]
    return T, D


def ref_recomp(U1, S, V2):
    W = oracle.recomp([U1], [S], [V2])[0]
    D = oracle.recomp([np.asfortranarray(np.abs(U1))], [np.asfortranarray(np.abs(S))],
                      [np.asfortranarray(np.abs(V2))])[0]
    return W, D


def ref_lrmult(AV, BU, AX, BX):
    G = oracle.lr_mult([AV], [BU], [AX], [BX])[0]
    ab = [np.asfortranarray(np.abs(x)) for x in (AV, BU, AX, BX)]
    D = oracle.lr_mult([ab[0]], [ab[1]], [ab[2]], [ab[3]])[0]
    return G, D
