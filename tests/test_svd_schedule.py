"""Host checks of the batched SVD kernel's index arithmetic (no GPU).

The kernel keeps a core's columns in LDS by tournament position: the pair
that owns positions pr and N-1-pr reads the same two slots every step and
writes the rotated columns to the slots their positions take next
(position 0 stays, x >= 2 moves to x - 1, 1 moves to N - 1).  One-sided
Jacobi needs every pair of columns rotated once per sweep; the layout needs
the LPP lanes of the pairs in one half-wave to hit distinct banks.  These
tests restate the kernel's two formulas and check both properties for every
core width and size class the library launches.
"""
import itertools

import pytest


def nxt(x, N):
    return 0 if x == 0 else (N - 1 if x == 1 else x - 1)


@pytest.mark.parametrize("n", list(range(1, 65)))
def test_every_pair_meets_once_per_sweep(n):
    N = (n + 1) & ~1                     # a zero column pads odd n
    if N < 2:
        return
    slot_of = list(range(N))             # column c sits in slot slot_of[c]
    for sweep in range(3):
        met = set()
        for step in range(N - 1):
            col_in = {s: c for c, s in enumerate(slot_of)}
            for pr in range(N // 2):
                a, b = col_in[pr], col_in[N - 1 - pr]
                pair = (min(a, b), max(a, b))
                assert pair not in met
                met.add(pair)
            slot_of = [nxt(s, N) for s in slot_of]
            assert sorted(slot_of) == list(range(N))     # a permutation of the slots
        assert met == set(itertools.combinations(range(N), 2))


def slot_index(x, i, NMAX, LPP):
    """Element (slot x, row i) as the kernel lays it out."""
    RPL = NMAX // LPP
    swz = 32 // LPP <= RPL
    ld = NMAX if swz else NMAX + LPP
    return x * ld + ((i ^ (LPP * (x & (32 // LPP - 1)))) if swz else i), ld


@pytest.mark.parametrize("NMAX,LPP", [(16, 4), (16, 8), (32, 4), (64, 8)])
def test_slot_layout_in_bounds_and_conflict_free(NMAX, LPP):
    RPL = NMAX // LPP
    # a bijection of (slot, row) onto the slot's storage, inside the array
    for x in range(NMAX):
        idx = sorted(slot_index(x, i, NMAX, LPP)[0] for i in range(NMAX))
        ld = slot_index(x, 0, NMAX, LPP)[1]
        assert idx[0] >= x * ld and idx[-1] < x * ld + ld and len(set(idx)) == NMAX
    # every step, for every row step j: lanes 32h..32h+31 of the workgroup
    # read their slots in distinct banks (32 banks of 8 bytes), whatever N
    # is; the slots those positions move to are consecutive too except for
    # the wrap-around (position 1 -> N - 1), so a write meets at most one
    # other pair's lanes in a bank
    NT = NMAX // 2 * LPP
    for n in range(2, NMAX + 1):
        N = (n + 1) & ~1
        for side in (0, 1):
            for write in (False, True):
                for j in range(RPL):
                    for half in range(NT // 32):
                        banks = []
                        for lane in range(32 * half, 32 * half + 32):
                            pr, ll = lane // LPP, lane % LPP
                            if pr >= N // 2:
                                continue
                            slot = pr if side == 0 else N - 1 - pr
                            if write:
                                slot = nxt(slot, N)
                            banks.append(slot_index(slot, ll + LPP * j, NMAX, LPP)[0] % 32)
                        worst = max(banks.count(b) for b in banks) if banks else 0
                        assert worst <= (2 if write else 1), (n, side, write, j, half)
