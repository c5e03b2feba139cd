"""The C-ABI library loads, exports every declared entry point and rejects
malformed arguments before launching anything (CPU only: validation runs on
the host before any device call)."""
import ctypes
import os
import re

import pytest

from paper_2311_07602_amd import lrbg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrbg.h")

# Fake, aligned, non-null device addresses: validation never dereferences them.
BASE = 1 << 40


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(l[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("lr_batched_gemm", "lrbg_grouped", "lrbg_plan_create", "lrbg_plan_execute",
                 "lrbg_plan_destroy", "lrbg_autotune", "lrbg_last_error", "lrbg_schedule_stats"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lrbg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings():
    assert lrbg.lrbg_version() >= 100
    lib = lrbg.load()
    assert lib.lrbg_status_string(0) == b"ok"
    assert lib.lrbg_status_string(1) == b"invalid argument"
    names = lrbg.lrbg_variant_names()
    assert names[0] == "nop" and len(names) == lib.lrbg_variant_count()
    assert len(set(names)) == len(names)


def mk(op="dense_ts", prec=0, m=64, n=16, k=64, lda=None, ldb=None, lds=None, ldc=None, a=None, b=None, s=None,
       c=None, base=BASE, e=None, lde=None):
    o = lrbg.OPS[op]
    if lda is None:
        lda = {0: m, 1: k, 2: m, 3: k}[o]
    if ldb is None:
        ldb = {0: k, 1: k, 2: n, 3: k}[o]
    if ldc is None:
        ldc = m
    a = base if a is None else a
    b = base + (1 << 30) if b is None else b
    c = base + (2 << 30) if c is None else c
    if o in (2, 3) and s is None:
        s = base + (3 << 30)
    if o == 3 and e is None:
        e = base + (4 << 30)
    if lds is None:
        lds = {2: k, 3: m}.get(o, 1)
    if lde is None:
        lde = n if o == 3 else 1
    return lrbg.lrbg_desc(op=o, prec=prec, m=m, n=n, k=k, lda=lda, ldb=ldb, lds=lds, ldc=ldc, flags=0,
                          lde=lde, reserved=0, a=a, b=b, s=s, c=c, e=e)


def status(descs):
    try:
        lrbg.lrbg_schedule_stats(descs)
        return 0
    except lrbg.LrbgError as e:
        return e.status


@pytest.mark.parametrize("bad,code", [
    (dict(m=-1), lrbg.LRBG_EINVAL),
    (dict(lda=10), lrbg.LRBG_EINVAL),
    (dict(ldc=3), lrbg.LRBG_EINVAL),
    (dict(a=0), lrbg.LRBG_EINVAL),
    (dict(c=0), lrbg.LRBG_EINVAL),
    (dict(a=BASE + 4), lrbg.LRBG_EINVAL),          # misaligned FP64
    (dict(n=129), lrbg.LRBG_EUNSUPPORTED),         # rank > 128
    (dict(m=70000, lda=70000, ldc=70000), lrbg.LRBG_EUNSUPPORTED),
    (dict(m=65537, lda=65537, ldc=65537), lrbg.LRBG_EUNSUPPORTED),   # one above the block limit
    (dict(m=100, k=65537, lda=100, ldb=65537, ldc=100), lrbg.LRBG_EUNSUPPORTED),
    (dict(m=65536, lda=65536, ldc=65536), 0),                          # the limit itself
    (dict(m=100, k=65536, lda=100, ldb=65536, ldc=100), 0),
    (dict(prec=7), lrbg.LRBG_EINVAL),
    (dict(c=BASE + 8), lrbg.LRBG_EINVAL),          # output overlaps A
])
def test_dense_ts_validation(bad, code):
    assert status([mk(**bad)]) == code


def test_other_ops_validation():
    assert status([mk("inner", m=16, n=16, k=512)]) == 0
    assert status([mk("inner", m=130, n=16, k=512)]) == lrbg.LRBG_EUNSUPPORTED
    assert status([mk("inner", m=16, n=16, k=512, lda=100)]) == lrbg.LRBG_EINVAL
    assert status([mk("recomp", m=512, n=512, k=32)]) == 0
    assert status([mk("recomp", m=512, n=512, k=32, lds=16)]) == lrbg.LRBG_EINVAL
    assert status([mk("recomp", m=512, n=512, k=32, prec=1)]) == lrbg.LRBG_EUNSUPPORTED
    assert status([mk("recomp", m=512, n=512, k=32, s=0)]) == lrbg.LRBG_EINVAL
    d = mk(); d.op = 5
    assert status([d]) == lrbg.LRBG_EINVAL
    d = mk(); d.flags = 1
    assert status([d]) == lrbg.LRBG_EINVAL


def test_lrmult_validation_and_accounting():
    b, r = 1024, 32
    assert status([mk("lrmult", m=r, n=r, k=b)]) == 0
    assert status([mk("lrmult", m=r, n=17, k=b)]) == 0
    assert status([mk("lrmult", m=96, n=128, k=b)]) == 0
    assert status([mk("lrmult", m=129, n=16, k=b)]) == lrbg.LRBG_EUNSUPPORTED    # rank > 128
    assert status([mk("lrmult", m=r, n=r, k=b, prec=1)]) == lrbg.LRBG_EUNSUPPORTED
    assert status([mk("lrmult", m=r, n=r, k=b, e=0)]) == lrbg.LRBG_EINVAL
    assert status([mk("lrmult", m=r, n=r, k=b, s=0)]) == lrbg.LRBG_EINVAL
    assert status([mk("lrmult", m=r, n=r, k=b, lde=r - 1)]) == lrbg.LRBG_EINVAL
    assert status([mk("lrmult", m=r, n=r, k=b, lds=r - 1)]) == lrbg.LRBG_EINVAL
    assert status([mk("lrmult", m=r, n=r, k=b, e=BASE + (4 << 30) + 4)]) == lrbg.LRBG_EINVAL   # misaligned
    assert status([mk("lrmult", m=r, n=r, k=b, c=BASE + (4 << 30) + 8)]) == lrbg.LRBG_EINVAL   # G overlaps X_B
    d = mk("lrmult", m=r, n=r, k=b); d.reserved = 1
    assert status([d]) == lrbg.LRBG_EINVAL
    # e is ignored (may be anything) for the other ops
    d = mk(); d.e = 12345; d.lde = 0
    assert status([d]) == 0
    names = lrbg.lrbg_schedule_variants([mk("lrmult", m=8, n=8, k=b), mk("lrmult", m=32, n=20, k=b, base=BASE * 2),
                                         mk("lrmult", m=64, n=64, k=b, base=BASE * 3),
                                         mk("lrmult", m=100, n=128, k=b, base=BASE * 4),
                                         mk("lrmult", m=0, n=8, k=b, base=BASE * 5, c=0, lds=1, ldc=1)])
    assert names[0].startswith("lrm4_") and names[1].startswith("lrm_") and names[2].startswith("lrm_")
    assert names[3].startswith("lrmb_") and names[4] == "nop"
    st = lrbg.lrbg_schedule_stats([mk("lrmult", m=r, n=r, k=b)])
    assert st["useful_flops"] == pytest.approx(4 * r ** 3 + 2 * r * r * b)   # the paper's Alg. 1 count
    assert st["hbm_bytes"] == pytest.approx(8 * (2 * b * r + 3 * r * r))
    assert st["tiles"] == 8 and st["levels"] == 1                           # one tile, padded to 8 XCD slots
    # X_B written by an INNER of the same call: the product runs one level later
    T = BASE + (10 << 30)
    inner = mk("inner", m=r, n=r, k=512, c=T, ldc=r, base=BASE * 3)
    lm = mk("lrmult", m=r, n=r, k=b, e=T, lde=r)
    assert lrbg.lrbg_schedule_stats([lm, inner])["levels"] == 2
    # lr_batched_gemm does not take LRMULT (it has no X_B operand)
    lib = lrbg.load()
    one = (ctypes.c_int32 * 1)(8)
    ptr = (ctypes.c_void_p * 1)(BASE)
    assert lib.lr_batched_gemm(3, 0, 1, one, one, one, ptr, one, ptr, one, ptr, one, ptr, one, None) == \
        lrbg.LRBG_EINVAL


def test_lrmult_accounting_at_the_papers_tabulated_shapes():
    """The useful-flop count the library reports for a batch of fused
    low-rank products equals the paper's GFLOPS equation (Sec. 7: batch x
    (4 r^3 + 2 r^2 b)) at every (rank, block size) of the paper's printed
    rank-96 and rank-128 tables (tests/golden/paper_tables.json)."""
    import json
    tab = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))
    assert tab["gflops_equation"] == "batch_size * (4*rank^3 + 2*rank^2*block_size) / time"
    shapes = sorted({(t["rank"], b) for t in tab["tables"] for b in t["block_size"]})
    assert shapes == [(96, 512), (96, 1024), (96, 2048), (128, 512), (128, 1024), (128, 2048)]
    batch = 3
    for r, b in shapes:
        descs = [mk("lrmult", m=r, n=r, k=b, base=BASE * (i + 1)) for i in range(batch)]
        st = lrbg.lrbg_schedule_stats(descs)
        assert st["useful_flops"] == batch * (4 * r ** 3 + 2 * r ** 2 * b), (r, b)
        assert st["hbm_bytes"] == batch * 8 * (2 * b * r + 3 * r * r), (r, b)


def test_lrmult_entry_validates_before_launch():
    lib = lrbg.load()
    assert lib.lr_batched_lrmult(1, *([None] * 13), None) == lrbg.LRBG_EINVAL
    assert lib.lr_batched_lrmult(0, *([None] * 13), None) == 0
    i32 = lambda v: (ctypes.c_int32 * 1)(v)
    p = lambda v: (ctypes.c_void_p * 1)(v)
    # rank 129 is rejected by validation (nothing launched, no device touched)
    st = lib.lr_batched_lrmult(1, i32(512), i32(129), i32(8), p(BASE), i32(512), p(BASE + (1 << 30)), i32(512),
                               p(BASE + (2 << 30)), i32(129), p(BASE + (3 << 30)), i32(8), p(BASE + (4 << 30)),
                               i32(129), None)
    assert st == lrbg.LRBG_EUNSUPPORTED


def test_round_entries_validate_before_device_work():
    """lr_batched_lrmult_round and lrbg_round_plan_create reject bad
    arguments before any allocation or launch (so this runs without a GPU)."""
    lib = lrbg.load()
    i32 = lambda v: (ctypes.c_int32 * 1)(v)
    p = lambda v: (ctypes.c_void_p * 1)(v)
    b, r = 256, 16
    def args(kmax=8, tol=1e-8, ra=r, sigma=BASE + (9 << 30), count=1):
        return [count, i32(b), i32(ra), i32(r),
                p(BASE), i32(b), p(BASE + (1 << 30)), i32(b), p(BASE + (2 << 30)), i32(ra),
                p(BASE + (3 << 30)), i32(b), p(BASE + (4 << 30)), i32(r), p(BASE + (5 << 30)), i32(b),
                kmax, tol, p(BASE + (6 << 30)), i32(b), p(BASE + (7 << 30)), i32(b), sigma, BASE + (10 << 30)]
    cases = [(dict(kmax=0), lrbg.LRBG_EUNSUPPORTED), (dict(kmax=65), lrbg.LRBG_EUNSUPPORTED),
             (dict(tol=-1.0), lrbg.LRBG_EINVAL), (dict(tol=float("nan")), lrbg.LRBG_EINVAL),
             (dict(ra=65), lrbg.LRBG_EUNSUPPORTED), (dict(sigma=BASE + 4), lrbg.LRBG_EINVAL),
             (dict(sigma=0), lrbg.LRBG_EINVAL), (dict(count=-1), lrbg.LRBG_EINVAL)]
    for kw, code in cases:
        a = args(**kw)
        assert lib.lr_batched_lrmult_round(*a, None) == code, kw
        assert lib.lr_batched_lrmult_round_noalloc(*a, None) == code, kw
        h = ctypes.c_void_p(12345)
        assert lib.lrbg_round_plan_create(ctypes.byref(h), *a) == code, kw
        assert h.value is None                                 # *out cleared on error
    a = args(); a[1] = None                                    # NULL host array
    assert lib.lr_batched_lrmult_round(*a, None) == lrbg.LRBG_EINVAL
    assert lib.lr_batched_lrmult_round(0, *([None] * 15), 4, 0.0, *([None] * 6), None) == 0
    assert lib.lr_batched_lrmult_round_noalloc(*a, None) == lrbg.LRBG_EINVAL
    assert lib.lr_batched_lrmult_round_noalloc(0, *([None] * 15), 4, 0.0, *([None] * 6), None) == 0
    assert lib.lrbg_round_plan_execute(None, None) == lrbg.LRBG_EINVAL
    assert lib.lrbg_round_plan_destroy(None) == 0


def test_noalloc_round_rejects_batches_beyond_its_scratch():
    """The allocation-free recompressed product sizes its cores and vectors
    on the host and refuses a batch that does not fit the fixed array before
    touching the device: 2000 products of rank 64 with kmax = 64 need
    3 x 32 KiB each, 188 MiB in all, against 128 MiB."""
    lib = lrbg.load()
    n, b, r = 2000, 256, 64
    ia = lambda v: (ctypes.c_int32 * n)(*([v] * n))
    pa = lambda base: (ctypes.c_void_p * n)(*[base + t * (1 << 20) for t in range(n)])
    a = [n, ia(b), ia(r), ia(r)]
    for j in range(6):
        a += [pa(BASE + (j << 32)), ia(b if j in (0, 1, 3, 5) else r)]
    a += [64, 0.0, pa(BASE + (6 << 32)), ia(b), pa(BASE + (7 << 32)), ia(b), BASE + (8 << 32), BASE + (9 << 32)]
    assert lib.lr_batched_lrmult_round_noalloc(*a, None) == lrbg.LRBG_EUNSUPPORTED
    msg = lrbg.lrbg_last_error()
    assert "scratch" in msg and str(lrbg.LRBG_NOALLOC_SCRATCH_BYTES) in msg, msg


def test_lradd_validates_before_device_work():
    """The rounded addition rejects malformed arguments on the host, before
    any device work (so this runs without a GPU)."""
    lib = lrbg.load()
    i32 = lambda *v: (ctypes.c_int32 * len(v))(*v)
    p = lambda *v: (ctypes.c_void_p * len(v))(*v)
    b, ra, rb = 256, 16, 8
    G = 1 << 30

    def args(kmax=8, tol=1e-8, r_a=ra, sigma=BASE + 9 * G, U=BASE + 6 * G, ldu=b, count=1, AX=BASE + 2 * G):
        return [count, i32(b), i32(r_a), i32(rb),
                p(BASE), i32(b), p(BASE + G), i32(b), p(AX), i32(r_a),
                p(BASE + 3 * G), i32(b), p(BASE + 4 * G), i32(rb), p(BASE + 5 * G), i32(b),
                kmax, tol, p(U), i32(ldu), p(BASE + 7 * G), i32(b), sigma, BASE + 10 * G]
    cases = [(dict(kmax=0), lrbg.LRBG_EUNSUPPORTED), (dict(kmax=65), lrbg.LRBG_EUNSUPPORTED),
             (dict(tol=-1.0), lrbg.LRBG_EINVAL), (dict(tol=float("inf")), lrbg.LRBG_EINVAL),
             (dict(r_a=57), lrbg.LRBG_EUNSUPPORTED), (dict(sigma=BASE + 4), lrbg.LRBG_EINVAL),
             (dict(count=-1), lrbg.LRBG_EINVAL), (dict(ldu=b - 1), lrbg.LRBG_EINVAL),
             (dict(U=BASE + 8), lrbg.LRBG_EINVAL),                # U inside A_U
             (dict(U=BASE + 9 * G - 8), lrbg.LRBG_EINVAL),        # U runs into sigma
             (dict(AX=BASE + 7 * G + 64), lrbg.LRBG_EINVAL),      # an input inside V
             (dict(U=0), lrbg.LRBG_EINVAL), (dict(U=BASE + 6 * G + 4), lrbg.LRBG_EINVAL)]
    for kw, code in cases:
        assert lib.lr_batched_lradd_round(*args(**kw), None) == code, kw
    a = args(); a[2] = None
    assert lib.lr_batched_lradd_round(*a, None) == lrbg.LRBG_EINVAL
    assert lib.lr_batched_lradd_round(0, *([None] * 15), 4, 0.0, *([None] * 6), None) == 0


def test_plan_flags_validated():
    d = [mk()]
    for f in (0, lrbg.LRBG_PLAN_NO_GRAPH, lrbg.LRBG_PLAN_UNTIMED, lrbg.LRBG_PLAN_SCHED_MIX | lrbg.LRBG_PLAN_UNTIMED):
        lrbg.lrbg_schedule_stats(d, flags=f)
    with pytest.raises(lrbg.LrbgError) as e:
        lrbg.lrbg_schedule_stats(d, flags=0x20)
    assert e.value.status == lrbg.LRBG_EINVAL


def test_short_contraction_defaults():
    # the new bases of a recompressed product (b x r times r x k) default to
    # the short-contraction tiles; a square contraction keeps the long tiles
    b = 1024
    def pick(m, k, n, i):
        return lrbg.lrbg_schedule_variants([mk(m=m, k=k, n=n, base=BASE * (i + 1))])[0]
    assert pick(b, 8, 4, 0) == "dtss_rm4_rn1_kg2"
    assert pick(b, 16, 8, 1) == "dtss_rm2_rn1_kg4"
    assert pick(b, 32, 16, 2) == "dts64_rm4_rn1_kg8"
    assert pick(b, 32, 32, 3) == "dtss_rm2_rn2_kg2"
    assert pick(b, 64, 64, 4) == "dts64_rm2_rn4_kg4"
    assert pick(b, 24, 64, 5) == "dtss_rm2_rn4_kg1"
    assert not pick(b, b, 8, 6).startswith("dtss")
    assert not pick(64, 64, 16, 7).startswith("dtss")


def test_empty_and_zero_sizes():
    assert lrbg.lrbg_schedule_stats([])["products"] == 0
    st = lrbg.lrbg_schedule_stats([mk(m=0, lda=1, ldc=1, a=0, c=0), mk(n=0, b=0, c=0, base=BASE * 2)])
    assert st["tiles"] == 0 and st["useful_flops"] == 0
    st = lrbg.lrbg_schedule_stats([mk(k=0, lda=64, ldb=1, a=0, b=0)])   # k = 0: output zero-filled
    assert st["tiles"] >= 1


def test_output_overlap_between_products_rejected():
    d1 = mk(); d2 = mk(base=BASE * 2, c=BASE + (2 << 30) + 8 * 64 * 16)
    assert status([d1, d2]) == 0
    d2 = mk(base=BASE * 2, c=BASE + (2 << 30) + 8 * (64 * 16 - 1))
    assert status([d1, d2]) == lrbg.LRBG_EINVAL


def test_chain_levels_and_accounting():
    b, r = 512, 32
    T = BASE + (10 << 30)
    inner = mk("inner", m=r, n=r, k=b, c=T, ldc=r)
    rec = mk("recomp", m=b, n=b, k=r, s=T, lds=r, base=BASE * 3)
    st = lrbg.lrbg_schedule_stats([inner, rec])
    assert st["levels"] == 2
    f_inner = 2 * b * r * r
    f_rec = 2 * b * b * r + 2 * r * r * b
    assert st["useful_flops"] == pytest.approx(f_inner + f_rec)
    by_inner = 8 * (2 * b * r + r * r)
    by_rec = 8 * (2 * b * r + r * r + b * b)
    assert st["hbm_bytes"] == pytest.approx(by_inner + by_rec)
    st1 = lrbg.lrbg_schedule_stats([inner])
    assert st1["levels"] == 1


def test_cycle_rejected():
    X = BASE + (20 << 30); Y = BASE + (21 << 30)
    d1 = mk("inner", m=16, n=16, k=64, a=Y, b=BASE, c=X, ldc=16)
    d2 = mk("inner", m=16, n=16, k=64, a=X, b=BASE + (1 << 32), c=Y, ldc=16, lda=64)
    # d2 reads X (64 x 16 view over a 16 x 16 output: overlapping) and writes Y read by d1
    assert status([d1, d2]) == lrbg.LRBG_EINVAL


def test_tile_counts(tmp_path):
    # DENSE_TS b=1024, r=16 forced to 256-row tiles (RM=4) through a tuning cache
    cache = tmp_path / "t.tune"
    cache.write_text("0 0 1024 16 dts64_rm4_rn1_kg8 0\n")
    st = lrbg.lrbg_schedule_stats([mk(m=1024, n=16, k=1024)], tune_cache=str(cache))
    assert st["tiles"] == 32         # one product: its 4 tiles share one XCD bin, 8 slots per row
    st = lrbg.lrbg_schedule_stats([mk(m=1024, n=16, k=1024)], tune_cache=str(cache),
                                  flags=lrbg.LRBG_PLAN_PERSISTENT)
    assert st["tiles"] == 4
    # RECOMP 512 x 512, rank 32, 64-column tiles -> 8 tiles
    cache.write_text("2 0 512 32 rec64_rb1_bn4_kg8 0\n")
    st = lrbg.lrbg_schedule_stats([mk("recomp", m=512, n=512, k=32)], tune_cache=str(cache),
                                  flags=lrbg.LRBG_PLAN_PERSISTENT)
    assert st["tiles"] == 8
    # an unknown variant name falls back to the built-in choice
    cache.write_text("0 0 1024 16 no_such_variant 0\n")
    assert lrbg.lrbg_schedule_stats([mk(m=1024, n=16, k=1024)], tune_cache=str(cache))["tiles"] > 0


def test_null_host_arrays_rejected():
    lib = lrbg.load()
    st = lib.lr_batched_gemm(0, 0, 1, None, None, None, None, None, None, None, None, None, None, None, None)
    assert st == lrbg.LRBG_EINVAL
    assert lib.lr_batched_gemm(0, 0, 0, None, None, None, None, None, None, None, None, None, None, None, None) == 0
    assert b"NULL" in lib.lrbg_last_error() or lib.lrbg_last_error() != b""


# ------------------------------------------------ element-exact overlaps

def _inner_at(c, ldc, m=8, n=8, k=64, a=BASE, b=BASE + (1 << 30)):
    return mk("inner", m=m, n=n, k=k, a=a, b=b, c=c, ldc=ldc, lda=k, ldb=k)


def test_interleaved_outputs_accepted_and_exact_overlap_rejected():
    X = BASE + (40 << 30)
    # two 8 x 8 outputs in rows [0, 8) and [8, 16) of one 16 x 8 matrix: spans interleave, no element shared
    d1 = _inner_at(X, 16); d2 = _inner_at(X + 8 * 8, 16, a=BASE + (2 << 30))
    assert status([d1, d2]) == 0
    assert lrbg.lrbg_schedule_stats([d1, d2])["levels"] == 1
    # shifted by one row: element (7, j) of the first is element (0, j) of the second
    d3 = _inner_at(X + 7 * 8, 16, a=BASE + (2 << 30))
    assert status([d1, d3]) == lrbg.LRBG_EINVAL


def test_stacked_vector_dependencies_are_exact():
    """Products writing row blocks of a stacked vector and a product reading
    another row block of it: no dependency; reading all of it: one."""
    b, r, nrhs = 64, 8, 8
    L = b + 2 * r
    Xs = BASE + (50 << 30)
    w1 = mk("inner", m=r, n=nrhs, k=b, a=BASE, b=BASE + (1 << 30), c=Xs + 8 * b, ldc=L, lda=b, ldb=b)
    w2 = mk("inner", m=r, n=nrhs, k=b, a=BASE + (2 << 30), b=BASE + (3 << 30), c=Xs + 8 * (b + r), ldc=L,
            lda=b, ldb=b)
    # reads rows [0, b) of Xs only
    rd_top = mk("inner", m=r, n=nrhs, k=b, a=BASE + (4 << 30), b=Xs, c=BASE + (5 << 30), ldc=r, lda=b, ldb=L)
    assert lrbg.lrbg_schedule_stats([w1, w2, rd_top])["levels"] == 1
    # reads all L rows of Xs (the stacked DENSE_TS of a BLR row): after both writers
    rd_all = mk(m=b, n=nrhs, k=L, a=BASE + (6 << 30), b=Xs, c=BASE + (7 << 30), ldc=b, lda=b, ldb=L)
    assert lrbg.lrbg_schedule_stats([w1, w2, rd_all, rd_top])["levels"] == 2
    # a product whose output interleaves with its own input is fine; one sharing an element is not
    own = mk("inner", m=r, n=nrhs, k=b, a=BASE + (8 << 30), b=Xs, c=Xs + 8 * b, ldc=L, lda=b, ldb=L)
    assert status([own]) == 0
    bad = mk("inner", m=r, n=nrhs, k=b, a=BASE + (8 << 30), b=Xs, c=Xs + 8 * (b - 1), ldc=L, lda=b, ldb=L)
    assert status([bad]) == lrbg.LRBG_EINVAL


def test_overlap_decisions_match_brute_force():
    """Random small column-major operands in one buffer: the scheduler's
    overlap (rejection) and dependency (levels) decisions equal those of
    explicit element sets."""
    import random
    rnd = random.Random(7)
    base = BASE + (60 << 30)

    def elems(off, rows, cols, ld):
        return {off + i + j * ld for j in range(cols) for i in range(rows)}

    for trial in range(300):
        ld1, ld2 = rnd.randint(8, 24), rnd.randint(8, 24)
        r1, c1 = rnd.randint(1, 8), rnd.randint(1, 6)       # output of product 1 (inner: m x n)
        r2, c2 = rnd.randint(1, 8), rnd.randint(1, 6)       # output of product 2
        o1, o2 = rnd.randint(0, 200), rnd.randint(0, 200)
        e1, e2 = elems(o1, r1, c1, ld1), elems(o2, r2, c2, ld2)
        p1 = mk("inner", m=r1, n=c1, k=64, a=BASE, b=BASE + (1 << 30), c=base + 8 * o1, ldc=ld1, lda=64, ldb=64)
        p2 = mk("inner", m=r2, n=c2, k=64, a=BASE + (2 << 30), b=BASE + (3 << 30), c=base + 8 * o2, ldc=ld2,
                lda=64, ldb=64)
        st = status([p1, p2])
        assert (st == lrbg.LRBG_EINVAL) == bool(e1 & e2), (trial, st)
        # product 3 reads a k x n operand B at a random place: depends on whichever output it meets
        kr, kc, ldr, orr = rnd.randint(1, 8), rnd.randint(1, 6), rnd.randint(8, 24), rnd.randint(0, 200)
        er = elems(orr, kr, kc, ldr)
        p3 = mk("inner", m=8, n=kc, k=kr, a=BASE + (4 << 30), b=base + 8 * orr, ldb=ldr, lda=kr,
                c=BASE + (5 << 30), ldc=8)
        if e1 & e2:
            continue
        levels = lrbg.lrbg_schedule_stats([p1, p2, p3])["levels"]
        assert levels == (2 if (er & (e1 | e2)) else 1), trial
