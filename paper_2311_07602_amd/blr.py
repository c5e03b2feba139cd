"""Block low-rank (BLR) matrix times multiple right-hand sides on the batched
products (the application of the paper's evaluation, Sec. 7: a weakly
admissible BLR matrix, rank 8, 8 right-hand sides).

A is nb x nb blocks of size b: dense diagonal blocks A_ii and low-rank
off-diagonal blocks A_ij = U_ij V_ij^T (rank r; a middle factor is folded into
V).  Y = A X is

    Y_i = A_ii X_i + sum_{j != i} U_ij (V_ij^T X_j),

the low-rank blocks applied in the paper's order (the rank-sized product
first).  On the device the sum over j never materialises: block row i is
stored as one b x (b + (nb - 1) r) column-major matrix [A_ii | U_i,0 | U_i,1 |
...] and its right-hand side as the stacked (b + (nb - 1) r) x nrhs matrix
Xs_i = [X_i; P_i,0; P_i,1; ...] with P_ij = V_ij^T X_j.  Then

    level 1: nb (nb - 1) INNER products  P_ij = V_ij^T X_j  -> rows of Xs_i
    level 2: nb DENSE_TS products         Y_i = [A_ii | U_i] Xs_i

and the segmented sum of the paper's implementation is part of the level-2
contraction.  The plan's dependency analysis is element-exact, so the level-1
outputs written into rows of Xs_i do not conflict with the X_j they read.
"""
from __future__ import annotations

from typing import Optional

from . import lrbg


class BlrMatvec:
    """Device storage of a BLR matrix and of a block of right-hand sides, and
    the captured two-level plan computing Y = A X.  Fill the blocks through
    the views (``diag``, ``u``, ``v``, ``x``), then ``run``; read ``y``."""

    def __init__(self, nb: int, b: int, r: int = 8, nrhs: int = 8, device="cuda"):
        import torch
        if nb < 1 or b < 1 or r < 1 or nrhs < 1:
            raise ValueError("nb, b, r, nrhs must be positive")
        self.nb, self.b, self.r, self.nrhs = nb, b, r, nrhs
        self.kw = b + (nb - 1) * r                  # width of a stored block row / height of Xs_i
        f64 = torch.float64
        self.rows = torch.empty(nb, self.kw, b, dtype=f64, device=device)          # [i, col, row]
        self.vs = torch.empty(nb, max(nb - 1, 1), r, b, dtype=f64, device=device)  # [i, jj, col, row]
        self.xs = torch.zeros(nb, nrhs, self.kw, dtype=f64, device=device)         # [i, col, row]
        self.ys = torch.empty(nb, nrhs, b, dtype=f64, device=device)
        self._plan: Optional[lrbg.Plan] = None

    # column-major views ---------------------------------------------------
    def _jj(self, i: int, j: int) -> int:
        if i == j or not (0 <= i < self.nb and 0 <= j < self.nb):
            raise IndexError("off-diagonal block index expected")
        return j if j < i else j - 1

    def diag(self, i: int):
        return self.rows[i, :self.b].T                                    # b x b, ld b

    def u(self, i: int, j: int):
        c0 = self.b + self._jj(i, j) * self.r
        return self.rows[i, c0:c0 + self.r].T                             # b x r, ld b

    def v(self, i: int, j: int):
        return self.vs[i, self._jj(i, j)].T                               # b x r, ld b

    def x(self, i: int):
        return self.xs[i, :, :self.b].T                                   # b x nrhs, ld kw

    def p(self, i: int, j: int):
        r0 = self.b + self._jj(i, j) * self.r
        return self.xs[i, :, r0:r0 + self.r].T                            # r x nrhs, ld kw

    def y(self, i: int):
        return self.ys[i].T                                               # b x nrhs, ld b

    # products -------------------------------------------------------------
    def descriptors(self):
        ds = []
        for i in range(self.nb):
            for j in range(self.nb):
                if i != j:
                    ds.append(lrbg.desc("inner", self.v(i, j), self.x(j), self.p(i, j)))
        for i in range(self.nb):
            ds.append(lrbg.desc("dense_ts", self.rows[i].T, self.xs[i].T, self.y(i)))
        return ds

    def work(self):
        """(useful flops, compulsory bytes) of one Y = A X."""
        st = lrbg.lrbg_schedule_stats(self.descriptors())
        return st["useful_flops"], st["hbm_bytes"]

    def plan(self, tune_cache: Optional[str] = None, flags: int = 0) -> lrbg.Plan:
        if self._plan is None:
            self._plan = lrbg.Plan(self.descriptors(), tune_cache=tune_cache, flags=flags,
                                   keepalive=(self.rows, self.vs, self.xs, self.ys))
        return self._plan

    def run(self, stream=None):
        self.plan().execute(stream)

    def close(self):
        if self._plan is not None:
            self._plan.close()
            self._plan = None
