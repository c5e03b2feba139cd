"""Thin ctypes binding of the lrbg C ABI (include/lrbg.h).

Argument marshalling only: every product is computed by the HIP kernels of
``liblrbg.so``.  The entry points keep the C names (``lr_batched_gemm``,
``lrbg_grouped``, ``lrbg_plan_create`` ...); they take raw device pointers and
host sequences and return the C status code, raising :class:`LrbgError` on a
non-zero status.  :func:`desc` and :class:`Plan` are conveniences over them
for column-major torch tensors (``x.stride(0) == 1``, leading dimension
``x.stride(1)``).

The library is loaded on first use; if it has not been built this raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrbg.so")

LRBG_OK, LRBG_EINVAL, LRBG_EUNSUPPORTED, LRBG_ENOMEM, LRBG_EDEVICE, LRBG_EBUDGET = range(6)
LRBG_OP_DENSE_TS, LRBG_OP_INNER, LRBG_OP_RECOMP, LRBG_OP_LRMULT = 0, 1, 2, 3
LRBG_FP64, LRBG_BF16X3 = 0, 1
LRBG_PLAN_PERSISTENT, LRBG_PLAN_NO_GRAPH, LRBG_PLAN_SCHED_MIX, LRBG_PLAN_DUAL = 0x1, 0x2, 0x4, 0x8
LRBG_PLAN_UNTIMED = 0x10

OPS = {"dense_ts": LRBG_OP_DENSE_TS, "inner": LRBG_OP_INNER, "recomp": LRBG_OP_RECOMP,
       "lrmult": LRBG_OP_LRMULT}
PRECS = {"fp64": LRBG_FP64, "bf16x3": LRBG_BF16X3}


class LrbgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class lrbg_desc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("lda", ctypes.c_int32), ("ldb", ctypes.c_int32), ("lds", ctypes.c_int32),
                ("ldc", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("lde", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("e", ctypes.c_void_p)]


class lrbg_plan_stats(ctypes.Structure):
    _fields_ = [("products", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("useful_flops", ctypes.c_double), ("hbm_bytes", ctypes.c_double)]


_lib = None

# numpy view of lrbg_desc (same field offsets), for building large
# descriptor arrays without per-descriptor Python objects
DESC_NP = None


def desc_dtype():
    global DESC_NP
    if DESC_NP is None:
        import numpy as np
        names = [f for f, _ in lrbg_desc._fields_]
        fmts = ["<i4" if t is ctypes.c_int32 else "<u8" for _, t in lrbg_desc._fields_]
        offs = [getattr(lrbg_desc, f).offset for f in names]
        DESC_NP = np.dtype({"names": names, "formats": fmts, "offsets": offs,
                            "itemsize": ctypes.sizeof(lrbg_desc)})
    return DESC_NP


def load(path: Optional[str] = None):
    """Load liblrbg.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or os.environ.get("LRBG_LIB") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"liblrbg.so not built ({p}); run `python -c 'import __graft_entry__ as g; g.build()'`")
    try:
        # Bind to the HIP runtime PyTorch ships (same SONAME) rather than
        # loading a second copy of the runtime into the process.
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    i32, i64, vp, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint32
    P = ctypes.POINTER
    lib.lr_batched_gemm.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lr_batched_gemm.restype = ctypes.c_int
    lib.lr_batched_lrmult.argtypes = [i64] + [vp] * 13 + [vp]
    lib.lr_batched_lrmult.restype = ctypes.c_int
    lib.lr_batched_lrmult_round.argtypes = [i64] + [vp] * 15 + [i32, ctypes.c_double] + [vp] * 6 + [vp]
    lib.lr_batched_lrmult_round.restype = ctypes.c_int
    lib.lr_batched_lradd_round.argtypes = [i64] + [vp] * 15 + [i32, ctypes.c_double] + [vp] * 6 + [vp]
    lib.lr_batched_lradd_round.restype = ctypes.c_int
    lib.lr_batched_lrmult_round_noalloc.argtypes = [i64] + [vp] * 15 + [i32, ctypes.c_double] + [vp] * 6 + [vp]
    lib.lr_batched_lrmult_round_noalloc.restype = ctypes.c_int
    lib.lrbg_round_plan_create.argtypes = [P(vp), i64] + [vp] * 15 + [i32, ctypes.c_double] + [vp] * 6
    lib.lrbg_round_plan_create.restype = ctypes.c_int
    lib.lrbg_round_plan_execute.argtypes = [vp, vp]
    lib.lrbg_round_plan_execute.restype = ctypes.c_int
    lib.lrbg_round_plan_destroy.argtypes = [vp]
    lib.lrbg_round_plan_destroy.restype = ctypes.c_int
    lib.lrbg_grouped.argtypes = [P(lrbg_desc), i64, vp]
    lib.lrbg_grouped.restype = ctypes.c_int
    lib.lrbg_plan_create.argtypes = [P(vp), P(lrbg_desc), i64, ctypes.c_char_p, u32]
    lib.lrbg_plan_create.restype = ctypes.c_int
    lib.lrbg_plan_execute.argtypes = [vp, vp]
    lib.lrbg_plan_execute.restype = ctypes.c_int
    lib.lrbg_plan_destroy.argtypes = [vp]
    lib.lrbg_plan_destroy.restype = ctypes.c_int
    lib.lrbg_plan_get_stats.argtypes = [vp, P(lrbg_plan_stats)]
    lib.lrbg_plan_get_stats.restype = ctypes.c_int
    lib.lrbg_schedule_stats.argtypes = [P(lrbg_desc), i64, ctypes.c_char_p, u32, P(lrbg_plan_stats)]
    lib.lrbg_schedule_stats.restype = ctypes.c_int
    lib.lrbg_schedule_variants.argtypes = [P(lrbg_desc), i64, ctypes.c_char_p, u32, P(i32)]
    lib.lrbg_schedule_variants.restype = ctypes.c_int
    lib.lrbg_plan_last_ms.argtypes = [vp]
    lib.lrbg_plan_last_ms.restype = ctypes.c_double
    lib.lrbg_autotune.argtypes = [P(lrbg_desc), i64, ctypes.c_char_p, i32]
    lib.lrbg_autotune.restype = ctypes.c_int
    lib.lrbg_autotune_mix.argtypes = [P(lrbg_desc), i64, ctypes.c_char_p, ctypes.c_char_p, i32, i32, u32]
    lib.lrbg_autotune_mix.restype = ctypes.c_int
    lib.lrbg_variant_count.argtypes = []
    lib.lrbg_variant_count.restype = i32
    lib.lrbg_variant_name.argtypes = [i32]
    lib.lrbg_variant_name.restype = ctypes.c_char_p
    lib.lrbg_status_string.argtypes = [ctypes.c_int]
    lib.lrbg_status_string.restype = ctypes.c_char_p
    lib.lrbg_last_error.argtypes = []
    lib.lrbg_last_error.restype = ctypes.c_char_p
    lib.lrbg_version.argtypes = []
    lib.lrbg_version.restype = i32
    _lib = lib
    return lib


def _check(st: int, where: str) -> int:
    if st != LRBG_OK:
        raise LrbgError(st, where, load().lrbg_last_error().decode(errors="replace"))
    return st


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)   # torch.cuda.Stream


def _arr(ctype, vals):
    """vals (a sequence, or a numpy array used in place when it already has
    the C type's width and is contiguous) as a host array; returns its
    address as a c_void_p that keeps the array alive."""
    import numpy as np
    dt = np.int32 if ctype is ctypes.c_int32 else np.uint64
    try:
        a = np.ascontiguousarray(vals, dtype=dt)
    except TypeError:   # null pointers given as None
        a = np.ascontiguousarray([0 if v is None else v for v in vals], dtype=dt)
    if a.size == 0:
        a = np.zeros(1, dtype=dt)
    p = ctypes.c_void_p(a.ctypes.data)
    p._keep = a
    return p


# ------------------------------------------------------------ raw entry points

def lr_batched_gemm(op: int, prec: int, m: Sequence[int], n: Sequence[int], k: Sequence[int],
                    A: Sequence[int], lda: Sequence[int], B: Sequence[int], ldb: Sequence[int],
                    S: Optional[Sequence[int]], lds: Optional[Sequence[int]],
                    C: Sequence[int], ldc: Sequence[int], stream=None) -> int:
    count = len(m)
    i32, vp = ctypes.c_int32, ctypes.c_void_p
    args = [_arr(i32, m), _arr(i32, n), _arr(i32, k), _arr(vp, A), _arr(i32, lda), _arr(vp, B), _arr(i32, ldb),
            _arr(vp, S) if S is not None else None, _arr(i32, lds) if lds is not None else None,
            _arr(vp, C), _arr(i32, ldc)]
    st = load().lr_batched_gemm(op, prec, count, *args, _stream_ptr(stream))
    return _check(st, "lr_batched_gemm")


def lr_batched_lrmult(b: Sequence[int], ra: Sequence[int], rb: Sequence[int],
                      AV: Sequence[int], ldav: Sequence[int], BU: Sequence[int], ldbu: Sequence[int],
                      AX: Sequence[int], ldax: Sequence[int], BX: Sequence[int], ldbx: Sequence[int],
                      G: Sequence[int], ldg: Sequence[int], stream=None) -> int:
    count = len(b)
    i32, vp = ctypes.c_int32, ctypes.c_void_p
    args = [_arr(i32, b), _arr(i32, ra), _arr(i32, rb), _arr(vp, AV), _arr(i32, ldav), _arr(vp, BU),
            _arr(i32, ldbu), _arr(vp, AX), _arr(i32, ldax), _arr(vp, BX), _arr(i32, ldbx),
            _arr(vp, G), _arr(i32, ldg)]
    st = load().lr_batched_lrmult(count, *args, _stream_ptr(stream))
    return _check(st, "lr_batched_lrmult")


def _round_arrays(b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv, U, ldu, V, ldv):
    i32, vp = ctypes.c_int32, ctypes.c_void_p
    arrs = [_arr(i32, b), _arr(i32, ra), _arr(i32, rb), _arr(vp, AU), _arr(i32, ldau), _arr(vp, AV),
            _arr(i32, ldav), _arr(vp, AX), _arr(i32, ldax), _arr(vp, BU), _arr(i32, ldbu), _arr(vp, BX),
            _arr(i32, ldbx), _arr(vp, BV), _arr(i32, ldbv)]
    outs = [_arr(vp, U), _arr(i32, ldu), _arr(vp, V), _arr(i32, ldv)]
    return arrs, outs


def lr_batched_lrmult_round(b: Sequence[int], ra: Sequence[int], rb: Sequence[int],
                            AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv,
                            kmax: int, tol: float, U, ldu, V, ldv, sigma: int, kout: int, stream=None) -> int:
    """Pointer-array form of the recompressed low-rank product (see include/lrbg.h);
    sigma and kout are device pointers."""
    ins, outs = _round_arrays(b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv, U, ldu, V, ldv)
    st = load().lr_batched_lrmult_round(len(b), *ins, int(kmax), float(tol), *outs, sigma, kout,
                                        _stream_ptr(stream))
    return _check(st, "lr_batched_lrmult_round")


def lr_batched_lradd_round(b: Sequence[int], ra: Sequence[int], rb: Sequence[int],
                           AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv,
                           kmax: int, tol: float, U, ldu, V, ldv, sigma: int, kout: int, stream=None) -> int:
    """Pointer-array form of the rounded addition of two low-rank blocks (see
    include/lrbg.h); sigma and kout are device pointers."""
    ins, outs = _round_arrays(b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv, U, ldu, V, ldv)
    st = load().lr_batched_lradd_round(len(b), *ins, int(kmax), float(tol), *outs, sigma, kout,
                                       _stream_ptr(stream))
    return _check(st, "lr_batched_lradd_round")


LRBG_NOALLOC_SCRATCH_BYTES = 128 << 20


def lr_batched_lrmult_round_noalloc(b: Sequence[int], ra: Sequence[int], rb: Sequence[int],
                                    AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv,
                                    kmax: int, tol: float, U, ldu, V, ldv, sigma: int, kout: int,
                                    stream=None) -> int:
    """lr_batched_lrmult_round with its scratch in the library's fixed
    per-GPU array (no device allocation; see include/lrbg.h)."""
    ins, outs = _round_arrays(b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv, U, ldu, V, ldv)
    st = load().lr_batched_lrmult_round_noalloc(len(b), *ins, int(kmax), float(tol), *outs, sigma, kout,
                                                _stream_ptr(stream))
    return _check(st, "lr_batched_lrmult_round_noalloc")


class RoundPlan:
    """Owning wrapper of lrbg_round_plan: lr_batched_lrmult_round's arguments
    (without the stream) scheduled once, replayed by execute()."""

    def __init__(self, b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv,
                 kmax: int, tol: float, U, ldu, V, ldv, sigma: int, kout: int, keepalive: Iterable = ()):
        self._keep = list(keepalive)
        ins, outs = _round_arrays(b, ra, rb, AU, ldau, AV, ldav, AX, ldax, BU, ldbu, BX, ldbx, BV, ldbv,
                                  U, ldu, V, ldv)
        h = ctypes.c_void_p()
        _check(load().lrbg_round_plan_create(ctypes.byref(h), len(b), *ins, int(kmax), float(tol), *outs,
                                             sigma, kout), "lrbg_round_plan_create")
        self.handle = h.value

    def execute(self, stream=None):
        _check(load().lrbg_round_plan_execute(self.handle, _stream_ptr(stream)), "lrbg_round_plan_execute")

    def close(self):
        if self.handle:
            load().lrbg_round_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def lrbg_grouped(descs: Sequence[lrbg_desc], stream=None) -> int:
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    return _check(load().lrbg_grouped(arr, len(descs), _stream_ptr(stream)), "lrbg_grouped")


def lrbg_grouped_array(arr, stream=None) -> int:
    """lrbg_grouped over a numpy array of dtype desc_dtype()."""
    if arr.dtype != desc_dtype() or not arr.flags["C_CONTIGUOUS"]:
        raise TypeError("descriptor array must be a contiguous desc_dtype() array")
    ptr = ctypes.cast(arr.ctypes.data, ctypes.POINTER(lrbg_desc))
    return _check(load().lrbg_grouped(ptr, len(arr), _stream_ptr(stream)), "lrbg_grouped")


def lrbg_plan_create(descs: Sequence[lrbg_desc], tune_cache: Optional[str] = None, flags: int = 0) -> int:
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    h = ctypes.c_void_p()
    cache = tune_cache.encode() if tune_cache else None
    _check(load().lrbg_plan_create(ctypes.byref(h), arr, len(descs), cache, flags), "lrbg_plan_create")
    return h.value


def lrbg_plan_execute(plan: int, stream=None) -> int:
    return _check(load().lrbg_plan_execute(plan, _stream_ptr(stream)), "lrbg_plan_execute")


def lrbg_plan_destroy(plan: int) -> int:
    return _check(load().lrbg_plan_destroy(plan), "lrbg_plan_destroy")


def lrbg_plan_get_stats(plan: int) -> dict:
    s = lrbg_plan_stats()
    _check(load().lrbg_plan_get_stats(plan, ctypes.byref(s)), "lrbg_plan_get_stats")
    return {f: getattr(s, f) for f, _ in lrbg_plan_stats._fields_}


def lrbg_schedule_stats(descs: Sequence[lrbg_desc], tune_cache: Optional[str] = None, flags: int = 0) -> dict:
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    s = lrbg_plan_stats()
    cache = tune_cache.encode() if tune_cache else None
    _check(load().lrbg_schedule_stats(arr, len(descs), cache, flags, ctypes.byref(s)), "lrbg_schedule_stats")
    return {f: getattr(s, f) for f, _ in lrbg_plan_stats._fields_}


def lrbg_schedule_variants(descs: Sequence[lrbg_desc], tune_cache: Optional[str] = None, flags: int = 0) -> List[str]:
    """Names of the tile variants a plan over `descs` would run ("nop" for no-op products)."""
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    out = (ctypes.c_int32 * max(len(descs), 1))()
    cache = tune_cache.encode() if tune_cache else None
    lib = load()
    _check(lib.lrbg_schedule_variants(arr, len(descs), cache, flags, out), "lrbg_schedule_variants")
    return [lib.lrbg_variant_name(out[i]).decode() for i in range(len(descs))]


def lrbg_plan_last_ms(plan: int) -> float:
    return float(load().lrbg_plan_last_ms(plan))


def lrbg_autotune(descs: Sequence[lrbg_desc], cache_out: str, reps: int = 3) -> int:
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    return _check(load().lrbg_autotune(arr, len(descs), cache_out.encode(), reps), "lrbg_autotune")


def lrbg_autotune_mix(descs: Sequence[lrbg_desc], cache_in: Optional[str], cache_out: str, reps: int = 5,
                      passes: int = 2, flags: int = 0) -> int:
    arr = (lrbg_desc * max(len(descs), 1))(*descs)
    return _check(load().lrbg_autotune_mix(arr, len(descs), cache_in.encode() if cache_in else None,
                                           cache_out.encode(), reps, passes, flags), "lrbg_autotune_mix")


def lrbg_variant_names() -> List[str]:
    lib = load()
    return [lib.lrbg_variant_name(v).decode() for v in range(lib.lrbg_variant_count())]


def lrbg_last_error() -> str:
    return load().lrbg_last_error().decode(errors="replace")


def lrbg_version() -> int:
    return int(load().lrbg_version())


# ------------------------------------------------------------ conveniences

def _mat(x):
    """(pointer, rows, cols, ld) of a column-major 2-D tensor (or None)."""
    if x is None:
        return 0, 0, 0, 1
    if x.dim() != 2:
        raise ValueError("operands are 2-D")
    rows, cols = x.shape
    if rows > 1 and x.stride(0) != 1:
        raise ValueError("operands must be column-major (stride(0) == 1)")
    ld = x.stride(1) if cols > 1 else max(rows, 1)
    return x.data_ptr(), rows, cols, max(ld, 1)


def desc(op: str, a, b, c, s=None, prec: str = "fp64", e=None) -> lrbg_desc:
    """Descriptor of one product from column-major tensors.

    dense_ts: a = A (m x k), b = U (k x n), c = C (m x n)
    inner:    a = V1 (k x m), b = U2 (k x n), c = T (m x n)
    recomp:   a = U1 (m x k), b = V2 (n x k), s = S (k x k), c = W (m x n)
    lrmult:   a = V_A (k x m), b = U_B (k x n), s = X_A (m x m),
              e = X_B (n x n), c = G (m x n)
    """
    pa, ra, ca, la = _mat(a)
    pb, rb, cb, lb = _mat(b)
    pc, rc, cc, lc = _mat(c)
    ps, rs, cs, ls = _mat(s)
    pe, re, ce, le = _mat(e)
    o = OPS[op]
    if o == LRBG_OP_DENSE_TS:
        m, k, n = ra, ca, cb
    elif o in (LRBG_OP_INNER, LRBG_OP_LRMULT):
        k, m, n = ra, ca, cb
    else:
        m, k, n = ra, ca, rb
    return lrbg_desc(op=o, prec=PRECS[prec], m=m, n=n, k=k, lda=la, ldb=lb, lds=ls if s is not None else 1,
                     ldc=lc, flags=0, lde=le if e is not None else 1, reserved=0,
                     a=pa or None, b=pb or None, s=ps or None, c=pc or None, e=pe or None)


class Plan:
    """Owning wrapper of an lrbg plan (a captured, replayable grouped launch)."""

    def __init__(self, descs: Sequence[lrbg_desc], tune_cache: Optional[str] = None, flags: int = 0,
                 keepalive: Iterable = ()):
        self._keep = list(keepalive)      # tensors whose memory the plan points at
        self.handle = lrbg_plan_create(descs, tune_cache, flags)
        self._execute = load().lrbg_plan_execute   # bound once: replays are short calls

    def execute(self, stream=None):
        st = self._execute(self.handle, stream if stream is None or isinstance(stream, int) else stream.cuda_stream)
        if st != LRBG_OK:
            _check(st, "lrbg_plan_execute")

    def stats(self) -> dict:
        return lrbg_plan_get_stats(self.handle)

    def last_ms(self) -> float:
        return lrbg_plan_last_ms(self.handle)

    def close(self):
        if self.handle:
            lrbg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
