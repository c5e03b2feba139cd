// Host side of the lrbg C ABI (include/lrbg.h): argument validation,
// per-bucket tile-variant choice, the XCD-aware tile schedule, dependency
// levels for chained products, plans captured in hipGraphs, and the
// autotuner.  Every step of the products themselves runs in the HIP kernels
// of lrbg_kernels.hip; nothing here computes on matrix data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lrbg.h"
#include "lrbg_internal.h"

namespace lrbg {

// ------------------------------------------------------------- errors

static thread_local std::string g_last_error;

static lrbg_status fail(lrbg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(LRBG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// ------------------------------------------------------------- variants

// Variant table indexed by id (the per-kernel lists are not in id order).
struct VariantTable {
    VariantInfo v[kNumVariants];
    int listed = 0;
    constexpr VariantTable() : v()
    {
#define LRBG_INFO(id, kind, p1, p2, p3, p4) \
    v[id] = VariantInfo{kind, p1, p2, p3, p4};  \
    ++listed;
        LRBG_ALL_VARIANTS(LRBG_INFO)
#undef LRBG_INFO
    }
    constexpr bool dense() const
    {
        for (int i = 1; i < kNumVariants; ++i)
            if (v[i].kind == K_NOP) return false;
        return v[0].kind == K_NOP && listed == kNumVariants - 1;
    }
};
static constexpr VariantTable kVariantTable;
static_assert(kVariantTable.dense(), "variant ids must be 1..kNumVariants-1, each listed once");
static constexpr const VariantInfo *kVariants = kVariantTable.v;

static std::string variant_name(int v)
{
    if (v <= 0 || v >= kNumVariants) return "nop";
    const VariantInfo &vi = kVariants[v];
    char buf[64];
    switch (vi.kind) {
    case K_DTS64: snprintf(buf, sizeof buf, "dts64_rm%d_rn%d_kg%d", vi.p1, vi.p2, vi.p3); break;
    case K_INN64: snprintf(buf, sizeof buf, "inn64_ri%d_rj%d_ks%d_kg%d", vi.p1, vi.p2, vi.p3, vi.p4); break;
    case K_REC64: snprintf(buf, sizeof buf, "rec64_rb%d_bn%d_kg%d", vi.p1, vi.p2, vi.p3); break;
    case K_DTS3: snprintf(buf, sizeof buf, "dts3_rm%d_rn%d_pf%d", vi.p1, vi.p2, vi.p3); break;
    case K_INN3: snprintf(buf, sizeof buf, "inn3_ri%d_rj%d_ks%d_pf%d", vi.p1, vi.p2, vi.p3, vi.p4); break;
    case K_DTSL: snprintf(buf, sizeof buf, "dtsl_rm%d_rn%d_kg%d", vi.p1, vi.p2, vi.p3); break;
    case K_DTSS: snprintf(buf, sizeof buf, "dtss_rm%d_rn%d_kg%d", vi.p1, vi.p2, vi.p3); break;
    case K_INNL: snprintf(buf, sizeof buf, "innl_ri%d_rj%d_wr%d_kg%d", vi.p1, vi.p2, vi.p3, vi.p4); break;
    case K_LRM: snprintf(buf, sizeof buf, "lrm_ri%d_rj%d_ks%d_kg%d", vi.p1, vi.p2, vi.p3, vi.p4); break;
    case K_LRM4: snprintf(buf, sizeof buf, "lrm4_ri%d_rj%d_ks%d_kg%d", vi.p1, vi.p2, vi.p3, vi.p4); break;
    case K_LRMB: snprintf(buf, sizeof buf, "lrmb_ri%d_rj%d_kg%d", vi.p1, vi.p2, vi.p4); break;
    case K_LRM96: snprintf(buf, sizeof buf, "lrm96_ri%d_rj%d_kg%d", vi.p1, vi.p2, vi.p4); break;
    default: snprintf(buf, sizeof buf, "v%d", v);
    }
    return buf;
}

static int kind_of(int op, int prec)
{
    if (prec == LRBG_FP64) {
        if (op == LRBG_OP_DENSE_TS) return K_DTS64;
        if (op == LRBG_OP_INNER) return K_INN64;
        if (op == LRBG_OP_RECOMP) return K_REC64;
        if (op == LRBG_OP_LRMULT) return K_LRM;
    } else if (prec == LRBG_BF16X3) {
        if (op == LRBG_OP_DENSE_TS) return K_DTS3;
        if (op == LRBG_OP_INNER) return K_INN3;
    }
    return K_NOP;
}

// Variant kinds that compute op/prec (several tile designs per product kind).
static bool kind_matches(int kind, int op, int prec)
{
    const int base = kind_of(op, prec);
    if (kind == base) return base != K_NOP;
    if (prec == LRBG_FP64 && op == LRBG_OP_DENSE_TS) return kind == K_DTSL || kind == K_DTSS;
    if (prec == LRBG_FP64 && op == LRBG_OP_INNER) return kind == K_INNL;
    if (prec == LRBG_FP64 && op == LRBG_OP_LRMULT) return kind == K_LRM4 || kind == K_LRMB || kind == K_LRM96;
    return false;
}

// Can variant v compute this product?  (Rank-type limits of the tile.)
static bool variant_fits(int v, const lrbg_desc &d)
{
    if (v <= 0 || v >= kNumVariants) return false;
    const VariantInfo &vi = kVariants[v];
    if (!kind_matches(vi.kind, d.op, d.prec)) return false;
    switch (vi.kind) {
    case K_DTS64: return d.n <= 16 * vi.p2;
    case K_DTSL: return d.n <= 16 * vi.p2;
    case K_DTSS: return d.n <= 16 * vi.p2 && d.k <= 64;
    case K_INNL: return d.n <= 16 * vi.p2 * (4 / vi.p3);
    case K_DTS3: return d.n <= 16 * vi.p2;
    case K_INN64: return d.n <= 16 * vi.p2;
    case K_INN3: return d.n <= 16 * vi.p2;
    case K_LRM: case K_LRM4: return d.m <= 16 * vi.p1 * (4 / vi.p3) && d.n <= 16 * vi.p2;
    case K_LRMB: return d.m <= 128 && d.n <= 128;
    case K_LRM96: return d.m <= 96 && d.n <= 96;
    case K_REC64: {
        const int kp = (d.k + 15) / 16 * 16;
        return (size_t)kp * 16 * vi.p2 * 8 <= (size_t)kLdsBytes;
    }
    }
    return false;
}

// Tile geometry of product d under variant v: tiles start every `step`
// along `extent`; `kc` is the k chunk (a contraction tail needs the guarded
// path) and `rows_full` says whether a tile's block-type rows must be full.
static bool tile_geometry(int v, const lrbg_desc &d, int &step, int &extent, int &kc, bool &rows_full)
{
    const VariantInfo &vi = kVariants[v];
    kc = 1;
    rows_full = false;   // block-type rows must fill the tile
    switch (vi.kind) {
    case K_DTS64: case K_DTSL: case K_DTSS:
        step = 64 * vi.p1; extent = d.m; kc = 4 * vi.p3; rows_full = true; break;
    case K_DTS3:
        step = 64 * vi.p1; extent = d.m; kc = 32; rows_full = true; break;
    case K_INN64:
        step = 16 * vi.p1 * (4 / vi.p3); extent = d.m; kc = 4 * vi.p4; break;
    case K_INN3:
        step = 16 * vi.p1 * (4 / vi.p3); extent = d.m; kc = 32; break;
    case K_LRM: case K_LRM4:   // one tile per product (variant_fits: m <= step)
        step = 16 * vi.p1 * (4 / vi.p3); extent = d.m; kc = 4 * vi.p4; break;
    case K_LRMB:
        step = 128; extent = d.m; kc = 4 * vi.p4; break;
    case K_LRM96:
        step = 96; extent = d.m; kc = 4 * vi.p4; break;
    case K_INNL:
        step = 16 * vi.p1 * vi.p3; extent = d.m; kc = 4 * vi.p4; break;
    case K_REC64:
        step = 16 * vi.p2; extent = d.n; kc = 4 * vi.p3; break;
    default: return false;
    }
    return true;
}

static int64_t tile_count(int v, const lrbg_desc &d)
{
    int step, extent, kc;
    bool rows_full;
    if (!tile_geometry(v, d, step, extent, kc, rows_full) || extent <= 0) return 0;
    return (extent + step - 1) / step;
}

// Tiles of product d under variant v, in order: f(p0, edge) for each, with
// p0 its first row (or column) and edge whether it needs the guarded
// (ragged-edge) code path.
template <class F>
static void for_tiles(int v, const lrbg_desc &d, F &&f)
{
    int step, extent, kc;
    bool rows_full;
    if (!tile_geometry(v, d, step, extent, kc, rows_full)) return;
    const VariantInfo &vi = kVariants[v];
    const bool ktail = d.k % kc != 0 || d.k == 0;
    // RECOMP: every row group of 32 RB rows must be full, and so must the
    // tile's columns (block-type W columns).
    const bool rec_rows_ragged = vi.kind == K_REC64 && d.m % (32 * vi.p1) != 0;
    for (int p = 0; p < extent; p += step) {
        bool e = ktail || rec_rows_ragged;
        if ((rows_full || vi.kind == K_REC64) && p + step > extent) e = true;
        f((int32_t)p, (int32_t)(e ? kTileEdge : 0));
    }
}

// (b, r) of a product: block-type and rank-type dimension.
static void bucket_dims(const lrbg_desc &d, int &b, int &r)
{
    switch (d.op) {
    case LRBG_OP_DENSE_TS: b = std::max(d.m, d.k); r = d.n; break;
    case LRBG_OP_INNER: case LRBG_OP_LRMULT: b = d.k; r = std::max(d.m, d.n); break;
    default: b = std::max(d.m, d.n); r = d.k; break;
    }
}

static int round_bucket(int x, int lo)
{
    int v = lo;
    while (v < x) v *= 2;
    return v;
}

typedef std::tuple<int, int, int, int> BucketKey;   // op, prec, b, r (rounded)

static BucketKey bucket_of(const lrbg_desc &d)
{
    int b, r;
    bucket_dims(d, b, r);
    return BucketKey(d.op, d.prec, round_bucket(b, 64), round_bucket(r, 8));
}

// Built-in choice per bucket (overridden by a tuning cache).
static int default_variant(const lrbg_desc &d)
{
    int b, r;
    bucket_dims(d, b, r);
    const int kind = kind_of(d.op, d.prec);
    auto pick = [&](std::initializer_list<int> cands) {
        for (int v : cands)
            if (variant_fits(v, d)) return v;
        return 0;
    };
    if (kind == K_DTS64) {
        if (4 * d.k <= d.m) {
            // short contraction (a basis update: b x r times r x k): a tile
            // is little work, so take as many rows per tile as the
            // registers allow, and k per lane group to match the contraction
            if (d.n <= 16) return d.k <= 8 ? pick({49, 3}) : d.k <= 16 ? pick({50, 3}) : pick({3, 1});
            if (d.n <= 32) return d.k <= 32 ? pick({51, 5}) : pick({5, 4});
            if (d.n <= 64) return d.k <= 32 ? pick({52, 7}) : pick({7, 6});
        }
        if (d.n <= 16) return pick({1});
        if (d.n <= 32) return pick({4});
        if (d.n <= 64) return pick({d.m >= 512 ? 22 : 6});
        return pick({d.m >= 256 ? 23 : 24});
    }
    if (kind == K_INN64) {
        const int rr = std::max(d.m, d.n);
        if (rr <= 16) return pick({8});
        if (rr <= 32) return pick({9});
        if (rr <= 64) return pick({26, 11});
        return pick({25, 28});
    }
    if (kind == K_DTS3) {
        if (d.n <= 16) return pick({d.m >= 256 ? 29 : 33});
        if (d.n <= 32) return pick({30});
        if (d.n <= 64) return pick({31});
        return pick({32});
    }
    if (kind == K_INN3) {
        const int rr = std::max(d.m, d.n);
        if (rr <= 16) return pick({34});
        if (rr <= 32) return pick({35});
        if (rr <= 64) return pick({36});
        return pick({37});
    }
    if (kind == K_LRM) {
        const int rr = std::max(d.m, d.n);
        if (rr <= 16) return pick({42, 39});   // 4 workgroups per CU: memory-bound, latency-limited
        if (rr <= 32) return pick({40, 44});
        if (rr <= 64) return pick({41});
        if (rr <= 96) return pick({53, 47});
        return pick({47});
    }
    if (kind == K_REC64) {
        if (d.k <= 16) return pick({13});
        if (d.k <= 32) return pick({14});
        if (d.k <= 64) return pick({14, 16});
        return pick({16});
    }
    (void)b;
    (void)r;
    return 0;
}

// ------------------------------------------------------------- validation

static size_t elem_size(int prec) { return prec == LRBG_BF16X3 ? 4 : 8; }

struct Range {
    uintptr_t lo, hi;   // [lo, hi) in bytes
    int64_t idx;
};

static bool overlaps(const Range &a, const Range &b) { return a.lo < b.hi && b.lo < a.hi && a.hi > a.lo && b.hi > b.lo; }

// A column-major operand as the bytes it occupies: `cols` runs of
// `row_bytes` bytes, `ld_bytes` apart (row_bytes <= ld_bytes, validated).
struct Mat {
    uintptr_t p = 0;
    int64_t cols = 0;
    uintptr_t ld_bytes = 0, row_bytes = 0;
    int64_t idx = -1;
    bool empty() const { return !p || cols <= 0 || row_bytes == 0; }
    Range range() const
    {
        if (empty()) return Range{0, 0, idx};
        return Range{p, p + (uintptr_t)(cols - 1) * ld_bytes + row_bytes, idx};
    }
};

static Mat mat_of(const void *p, int rows, int cols, int ld, size_t es, int64_t idx)
{
    Mat m;
    if (!p || rows <= 0 || cols <= 0) return m;
    m.p = (uintptr_t)p;
    m.cols = cols;
    m.ld_bytes = (uintptr_t)ld * es;
    m.row_bytes = (uintptr_t)rows * es;
    m.idx = idx;
    return m;
}

// Element-exact overlap: do some bytes of x and y coincide?  Two operands
// whose byte spans interleave (row blocks of one larger matrix) do not
// overlap unless one of their columns meets one of the other's.
static bool mats_overlap(const Mat &x, const Mat &y)
{
    if (x.empty() || y.empty() || !overlaps(x.range(), y.range())) return false;
    const Mat &a = x.cols <= y.cols ? x : y;
    const Mat &b = x.cols <= y.cols ? y : x;
    for (int64_t j = 0; j < a.cols; ++j) {
        const uintptr_t s = a.p + (uintptr_t)j * a.ld_bytes, e = s + a.row_bytes;   // column j of a
        // first column jb of b that ends after s; columns of b are disjoint and ascending
        int64_t jb = 0;
        if (b.p + b.row_bytes <= s) jb = (int64_t)((s - b.p - b.row_bytes) / b.ld_bytes) + 1;
        if (jb < b.cols && b.p + (uintptr_t)jb * b.ld_bytes < e) return true;
    }
    return false;
}

// Operand shapes (rows, cols) of a product: a, b, s, c, e (0 x 0 when unused).
static void shapes(const lrbg_desc &d, int sh[5][2])
{
    sh[4][0] = sh[4][1] = 0;
    switch (d.op) {
    case LRBG_OP_DENSE_TS:
        sh[0][0] = d.m; sh[0][1] = d.k; sh[1][0] = d.k; sh[1][1] = d.n; sh[2][0] = 0; sh[2][1] = 0;
        break;
    case LRBG_OP_INNER:
        sh[0][0] = d.k; sh[0][1] = d.m; sh[1][0] = d.k; sh[1][1] = d.n; sh[2][0] = 0; sh[2][1] = 0;
        break;
    case LRBG_OP_LRMULT:
        sh[0][0] = d.k; sh[0][1] = d.m; sh[1][0] = d.k; sh[1][1] = d.n; sh[2][0] = d.m; sh[2][1] = d.m;
        sh[4][0] = d.n; sh[4][1] = d.n;
        break;
    default:
        sh[0][0] = d.m; sh[0][1] = d.k; sh[1][0] = d.n; sh[1][1] = d.k; sh[2][0] = d.k; sh[2][1] = d.k;
        break;
    }
    sh[3][0] = d.m;
    sh[3][1] = d.n;
}

static lrbg_status validate_one(const lrbg_desc &d, int64_t i)
{
    if (d.op < 0 || d.op > 3) return fail(LRBG_EINVAL, "product %lld: bad op %d", (long long)i, d.op);
    if (d.prec != LRBG_FP64 && d.prec != LRBG_BF16X3)
        return fail(LRBG_EINVAL, "product %lld: bad precision %d", (long long)i, d.prec);
    if (d.m < 0 || d.n < 0 || d.k < 0)
        return fail(LRBG_EINVAL, "product %lld: negative size (m=%d n=%d k=%d)", (long long)i, d.m, d.n, d.k);
    if (d.flags != 0 || d.reserved != 0)
        return fail(LRBG_EINVAL, "product %lld: flags and reserved must be 0", (long long)i);
    if (kind_of(d.op, d.prec) == K_NOP)
        return fail(LRBG_EUNSUPPORTED, "product %lld: op %d has no bf16x3 form (FP64 only)", (long long)i, d.op);
    int b, r;
    bucket_dims(d, b, r);
    const int rankdims[4][2] = {{d.n, 0}, {d.m, d.n}, {d.k, 0}, {d.m, d.n}};
    const int rankmax = d.op == LRBG_OP_LRMULT ? kMaxLrRank : kMaxRank;
    for (int t = 0; t < 2; ++t)
        if (rankdims[d.op][t] > rankmax)
            return fail(LRBG_EUNSUPPORTED, "product %lld: rank dimension %d exceeds %d", (long long)i,
                        rankdims[d.op][t], rankmax);
    if (b > kMaxBlock)
        return fail(LRBG_EUNSUPPORTED, "product %lld: block dimension %d exceeds %d", (long long)i, b, kMaxBlock);
    int sh[5][2];
    shapes(d, sh);
    const void *ptr[5] = {d.a, d.b, d.s, d.c, d.e};
    const int ld[5] = {d.lda, d.ldb, d.lds, d.ldc, d.lde};
    const char *nm[5] = {"a", "b", "s", "c", "e"};
    const size_t es[5] = {elem_size(d.prec), elem_size(d.prec), 8, 8, 8};
    const bool uses_s = d.op == LRBG_OP_RECOMP || d.op == LRBG_OP_LRMULT, uses_e = d.op == LRBG_OP_LRMULT;
    for (int t = 0; t < 5; ++t) {
        if ((t == 2 && !uses_s) || (t == 4 && !uses_e)) continue;
        const int rows = sh[t][0], cols = sh[t][1];
        if (ld[t] < std::max(1, rows))
            return fail(LRBG_EINVAL, "product %lld: ld%s=%d < rows=%d", (long long)i, nm[t], ld[t], rows);
        if (rows > 0 && cols > 0) {
            if (!ptr[t]) return fail(LRBG_EINVAL, "product %lld: %s is NULL", (long long)i, nm[t]);
            if ((uintptr_t)ptr[t] % es[t])
                return fail(LRBG_EINVAL, "product %lld: %s not %zu-byte aligned", (long long)i, nm[t], es[t]);
        }
    }
    const Mat out = mat_of(d.c, sh[3][0], sh[3][1], d.ldc, 8, i);
    for (int t = 0; t < 5; ++t) {
        if (t == 3 || (t == 2 && !uses_s) || (t == 4 && !uses_e)) continue;
        if (mats_overlap(out, mat_of(ptr[t], sh[t][0], sh[t][1], ld[t], es[t], i)))
            return fail(LRBG_EINVAL, "product %lld: output overlaps input %s", (long long)i, nm[t]);
    }
    return LRBG_OK;
}

// ------------------------------------------------------------- tuning cache

struct TuneTable {
    std::map<BucketKey, int> choice;
};

static int variant_by_name(const std::string &nm)
{
    for (int v = 1; v < kNumVariants; ++v)
        if (variant_name(v) == nm) return v;
    return 0;
}

static void load_tune_cache(const char *path, TuneTable &tt)
{
    if (!path || !*path) return;
    std::ifstream f(path);
    if (!f) return;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        int op, prec, b, r;
        std::string nm;
        if (!(is >> op >> prec >> b >> r >> nm)) continue;
        const int v = variant_by_name(nm);
        if (v) tt.choice[BucketKey(op, prec, b, r)] = v;
    }
}

// ------------------------------------------------------------- cost model

// Useful flops and compulsory bytes of one product (2 flops per multiply-add;
// each operand read once, the output written once).
static void work_of(const lrbg_desc &d, double &flops, double &bytes)
{
    const double m = d.m, n = d.n, k = d.k, es = (double)elem_size(d.prec);
    switch (d.op) {
    case LRBG_OP_DENSE_TS:
        flops = 2.0 * m * n * k;
        bytes = es * (m * k + k * n) + 8.0 * m * n;
        break;
    case LRBG_OP_INNER:
        flops = 2.0 * m * n * k;
        bytes = es * (k * m + k * n) + 8.0 * m * n;
        break;
    case LRBG_OP_LRMULT:   // C = V_A^T U_B, E = X_A C, G = E X_B
        flops = 2.0 * m * n * k + 2.0 * m * m * n + 2.0 * m * n * n;
        bytes = 8.0 * (k * m + k * n + m * m + n * n + m * n);
        break;
    default:
        flops = 2.0 * m * n * k + 2.0 * k * k * n;
        bytes = 8.0 * (m * k + n * k + k * k + m * n);
        break;
    }
    if (d.m == 0 || d.n == 0) flops = bytes = 0.0;
}

// Relative time estimate of a product on the whole chip (seconds).
// Rates of the scheduling cost model (FP64 matrix-core flop/s and HBM
// bytes/s a tile reaches inside a mixed batch); LRBG_COST_MODEL="tf,tbs"
// overrides them (e.g. "70,5.5").
static void cost_rates(double &fr, double &br)
{
    static double f = 0, b = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        f = 70e12;
        b = 5.5e12;
        if (const char *e = getenv("LRBG_COST_MODEL")) {
            double x = 0, y = 0;
            if (sscanf(e, "%lf,%lf", &x, &y) == 2 && x > 0 && y > 0) {
                f = x * 1e12;
                b = y * 1e12;
            }
        }
    });
    fr = f;
    br = b;
}

static double est_time(const lrbg_desc &d)
{
    double f, b, fr, br;
    work_of(d, f, b);
    cost_rates(fr, br);
    return std::max(f / fr, b / br) + 2e-9;
}

static bool compute_bound(const lrbg_desc &d)
{
    double f, b, fr, br;
    work_of(d, f, b);
    cost_rates(fr, br);
    return f / fr > b / br;
}

// ------------------------------------------------------------- plans

constexpr uint32_t kPlanFlags =
    LRBG_PLAN_PERSISTENT | LRBG_PLAN_NO_GRAPH | LRBG_PLAN_SCHED_MIX | LRBG_PLAN_DUAL | LRBG_PLAN_UNTIMED;
constexpr int64_t kDirectLaunchTiles = 4096;   // plans this small (one or two launches) replay directly

struct Level {
    int64_t off[kFamilies] = {};   // per kernel family: first tile in the plan's tile array
    int32_t n[kFamilies] = {};     // and the grid of its one-workgroup-per-tile launch
    int32_t qinfo_off = 0;         // 9 queue offsets (persistent mode, grouped family)
    int32_t grid = 0;
};

}  // namespace lrbg

struct lrbg_plan {
    uint32_t flags = 0;
    int device = 0;
    lrbg::DevDesc *d_descs = nullptr;
    lrbg::Tile *d_tiles = nullptr;
    int32_t *d_qinfo = nullptr;
    int32_t *d_counters = nullptr;
    int32_t *d_cu = nullptr;      // per-CU role flags (LRBG_PLAN_DUAL)
    std::vector<lrbg::Level> levels;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    bool ran_untimed = false;     // LRBG_PLAN_UNTIMED: executed at least once
    lrbg_plan_stats stats{};
};

namespace lrbg {

struct Schedule {
    std::vector<DevDesc> descs;
    std::vector<Tile> tiles;      // all levels, each laid out for its launch
    std::vector<int32_t> qinfo;   // 9 per level
    std::vector<Level> levels;
    std::vector<int> variant;     // per product, 0 = no-op
    lrbg_plan_stats stats{};
};

// Dependency level of every product: a product reading (a, b, s or e)
// memory written by another product runs one level after it.  Overlaps are
// element-exact: outputs may interleave inside one larger matrix (row blocks
// of a stacked vector, for instance) as long as no element is shared.
//
// Outputs are grouped into clusters of intersecting byte spans; within a
// cluster of several outputs the columns of all members are sorted and must
// be disjoint.  An input is then tested against the members of the clusters
// its span meets: one exact test for a single-output cluster, a binary
// search over the sorted columns otherwise.
// `private_b`: every B operand is the library's own scratch, which no output
// can reach, so only the other inputs are tested.
static lrbg_status compute_levels(const lrbg_desc *ds, int64_t n, std::vector<int> &level, bool private_b = false)
{
    level.assign((size_t)n, 0);
    std::vector<Mat> outs;
    outs.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int sh[5][2];
        shapes(ds[i], sh);
        Mat m = mat_of(ds[i].c, sh[3][0], sh[3][1], ds[i].ldc, 8, i);
        if (!m.empty()) outs.push_back(m);
    }
    std::sort(outs.begin(), outs.end(), [](const Mat &x, const Mat &y) { return x.p < y.p; });

    struct Seg {
        uintptr_t lo, hi;
        int64_t idx;
    };
    // clusters as parallel arrays (the input search touches only clo / chi):
    // members outs[cfirst, cfirst + ccount); a multi-member cluster's sorted
    // columns are segs[sbeg, send)
    std::vector<uintptr_t> clo, chi;
    std::vector<size_t> cfirst, ccount, sbeg, send;
    clo.reserve(outs.size());
    chi.reserve(outs.size());
    cfirst.reserve(outs.size());
    ccount.reserve(outs.size());
    for (size_t t = 0; t < outs.size(); ++t) {
        const Range r = outs[t].range();
        if (!clo.empty() && r.lo < chi.back()) {
            chi.back() = std::max(chi.back(), r.hi);
            ++ccount.back();
        } else {
            clo.push_back(r.lo);
            chi.push_back(r.hi);
            cfirst.push_back(t);
            ccount.push_back(1);
        }
    }
    const size_t ncl = clo.size();
    sbeg.assign(ncl, 0);
    send.assign(ncl, 0);
    std::vector<Seg> segs;
    for (size_t c = 0; c < ncl; ++c) {
        if (ccount[c] < 2) continue;
        sbeg[c] = segs.size();
        for (size_t t = cfirst[c]; t < cfirst[c] + ccount[c]; ++t) {
            const Mat &m = outs[t];
            for (int64_t j = 0; j < m.cols; ++j) {
                const uintptr_t lo = m.p + (uintptr_t)j * m.ld_bytes;
                segs.push_back(Seg{lo, lo + m.row_bytes, m.idx});
            }
        }
        send[c] = segs.size();
        std::sort(segs.begin() + (ptrdiff_t)sbeg[c], segs.end(), [](const Seg &x, const Seg &y) { return x.lo < y.lo; });
        for (size_t t = sbeg[c] + 1; t < send[c]; ++t)
            if (segs[t].lo < segs[t - 1].hi)
                return fail(LRBG_EINVAL, "outputs of products %lld and %lld overlap", (long long)segs[t - 1].idx,
                            (long long)segs[t].idx);
    }

    // deps[i]: products whose output product i reads
    std::vector<std::vector<int64_t>> deps((size_t)n);
    bool any = false;
    auto add_dep = [&](int64_t i, int64_t j) {
        if (j == i) return;
        std::vector<int64_t> &v = deps[(size_t)i];
        if (std::find(v.begin(), v.end(), j) == v.end()) v.push_back(j);
        any = true;
    };
    for (int64_t i = 0; i < n; ++i) {
        const lrbg_desc &d = ds[i];
        int sh[5][2];
        shapes(d, sh);
        const void *ptr[4] = {d.a, d.b, d.s, d.e};
        const int ld[4] = {d.lda, d.ldb, d.lds, d.lde};
        const int si[4] = {0, 1, 2, 4};
        const size_t es[4] = {elem_size(d.prec), elem_size(d.prec), 8, 8};
        for (int t = 0; t < 4; ++t) {
            if (t == 1 && private_b) continue;
            if (t == 2 && d.op != LRBG_OP_RECOMP && d.op != LRBG_OP_LRMULT) continue;
            if (t == 3 && d.op != LRBG_OP_LRMULT) continue;
            const Mat in = mat_of(ptr[t], sh[si[t]][0], sh[si[t]][1], ld[t], es[t], i);
            if (in.empty()) continue;
            const Range ir = in.range();
            // clusters starting before ir.hi; walk back while they may meet it (clusters are disjoint)
            size_t c = (size_t)(std::lower_bound(clo.begin(), clo.end(), ir.hi) - clo.begin());
            while (c > 0) {
                --c;
                if (chi[c] <= ir.lo) break;
                if (ccount[c] == 1) {
                    const Mat &m = outs[cfirst[c]];
                    if (mats_overlap(in, m)) add_dep(i, m.idx);
                    continue;
                }
                for (int64_t j = 0; j < in.cols; ++j) {
                    const uintptr_t lo = in.p + (uintptr_t)j * in.ld_bytes, hi = lo + in.row_bytes;
                    auto sg = std::lower_bound(segs.begin() + (ptrdiff_t)sbeg[c], segs.begin() + (ptrdiff_t)send[c], hi,
                                               [](const Seg &x, uintptr_t v) { return x.lo < v; });
                    while (sg != segs.begin() + (ptrdiff_t)sbeg[c]) {
                        --sg;
                        if (sg->hi <= lo) break;   // segments are disjoint and sorted
                        add_dep(i, sg->idx);
                    }
                }
            }
        }
    }
    if (!any) return LRBG_OK;
    // longest-path levels; more passes than products means a cycle
    for (int pass = 0;; ++pass) {
        bool changed = false;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j : deps[(size_t)i])
                if (level[(size_t)i] < level[(size_t)j] + 1) {
                    level[(size_t)i] = level[(size_t)j] + 1;
                    changed = true;
                }
        if (!changed) break;
        if (pass > 64) return fail(LRBG_EINVAL, "product dependencies form a cycle or a chain deeper than 64");
    }
    return LRBG_OK;
}

// Lay out one level's tiles: products are assigned to the 8 XCD bins by
// longest-processing-time on the cost model (a product's tiles stay in one
// bin, so tiles sharing its operands share an L2); within a bin products run
// longest first (or interleaved compute-/memory-bound with SCHED_MIX); the
// bins are interleaved so that tile t is dispatched to XCD t % 8.
static void lay_tiles(const std::vector<int64_t> &prods, const lrbg_desc *ds, const std::vector<int> &variant,
                      uint32_t flags, Schedule &sch, int64_t &tile_off, int32_t &ntiles, bool queues)
{
    struct P {
        int64_t i;
        double t;
    };
    std::vector<P> ps;
    ps.reserve(prods.size());
    bool uniform = true;   // a batch of one shape needs no sorting
    for (int64_t i : prods) {
        ps.push_back(P{i, est_time(ds[i])});
        uniform = uniform && ps.back().t == ps.front().t;
    }
    if (!uniform) std::stable_sort(ps.begin(), ps.end(), [](const P &x, const P &y) { return x.t > y.t; });
    if ((flags & LRBG_PLAN_DUAL) && queues) {
        // 16 queues, role-major: q = role * 8 + xcd; role 0 = matrix-core-bound
        // products, role 1 = memory-bound; each role LPT-balanced over the 8
        // XCD queues, longest first within a queue, a product's tiles adjacent.
        std::vector<std::vector<int64_t>> qs(2 * kXcds);
        std::vector<double> load(2 * kXcds, 0.0);
        for (const P &p : ps) {
            const int role = compute_bound(ds[p.i]) ? 0 : 1;
            int qmin = role * kXcds;
            for (int x = 1; x < kXcds; ++x)
                if (load[role * kXcds + x] < load[qmin]) qmin = role * kXcds + x;
            qs[qmin].push_back(p.i);
            load[qmin] += p.t;
        }
        tile_off = (int64_t)sch.tiles.size();
        int32_t off = 0;
        for (auto &q : qs) {
            sch.qinfo.push_back(off);
            for (int64_t i : q) {
                const int v = variant[(size_t)i];
                for_tiles(v, ds[i], [&](int32_t p0, int32_t e) {
                    sch.tiles.push_back(Tile{(int32_t)i, v, p0, e});
                    ++off;
                });
            }
        }
        sch.qinfo.push_back(off);
        ntiles = off;
        return;
    }
    std::vector<std::vector<int64_t>> bins(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (const P &p : ps) {
        int bmin = 0;
        for (int b = 1; b < kXcds; ++b)
            if (load[b] < load[bmin]) bmin = b;
        bins[bmin].push_back(p.i);
        load[bmin] += p.t;
    }
    if (flags & LRBG_PLAN_SCHED_MIX) {
        for (auto &bin : bins) {
            std::vector<int64_t> cb, mb;
            double tc = 0, tm = 0;
            for (int64_t i : bin) (compute_bound(ds[i]) ? cb : mb).push_back(i);
            for (int64_t i : cb) tc += est_time(ds[i]);
            for (int64_t i : mb) tm += est_time(ds[i]);
            std::vector<int64_t> merged;
            size_t a = 0, b = 0;
            double sc = 0, sm = 0;
            while (a < cb.size() || b < mb.size()) {
                const bool takec = b >= mb.size() || (a < cb.size() && sc / std::max(tc, 1e-30) <= sm / std::max(tm, 1e-30));
                if (takec) {
                    sc += est_time(ds[cb[a]]);
                    merged.push_back(cb[a++]);
                } else {
                    sm += est_time(ds[mb[b]]);
                    merged.push_back(mb[b++]);
                }
            }
            bin.swap(merged);
        }
    }
    // exact tile count of each bin; the tiles are then written straight into
    // their slots
    size_t nbt[kXcds], maxlen = 0, total = 0;
    for (int b = 0; b < kXcds; ++b) {
        nbt[b] = 0;
        for (int64_t i : bins[b]) nbt[b] += (size_t)tile_count(variant[(size_t)i], ds[i]);
        maxlen = std::max(maxlen, nbt[b]);
        total += nbt[b];
    }
    tile_off = (int64_t)sch.tiles.size();
    if (flags & LRBG_PLAN_PERSISTENT) {
        // queue q = bins[q], contiguous
        sch.tiles.resize((size_t)tile_off + total);
        Tile *out = sch.tiles.data() + tile_off;
        int32_t off = 0;
        for (int b = 0; b < kXcds; ++b) {
            sch.qinfo.push_back(off);
            for (int64_t i : bins[b]) {
                const int v = variant[(size_t)i];
                for_tiles(v, ds[i], [&](int32_t p0, int32_t e) { out[off++] = Tile{(int32_t)i, v, p0, e}; });
            }
        }
        sch.qinfo.push_back(off);
        ntiles = off;
    } else {
        // slot-major: bin b's tile j at j kXcds + b, the gaps no-op tiles
        sch.tiles.resize((size_t)tile_off + maxlen * kXcds, Tile{0, 0, 0, 0});
        Tile *out = sch.tiles.data() + tile_off;
        for (int b = 0; b < kXcds; ++b) {
            size_t slot = 0;
            for (int64_t i : bins[b]) {
                const int v = variant[(size_t)i];
                for_tiles(v, ds[i], [&](int32_t p0, int32_t e) {
                    out[slot++ * kXcds + (size_t)b] = Tile{(int32_t)i, v, p0, e};
                });
            }
        }
        ntiles = (int32_t)(maxlen * kXcds);
        if (queues)
            for (int b = 0; b <= kXcds; ++b) sch.qinfo.push_back(0);
    }
}

static int family_of(int v)
{
    const int kind = kVariants[v].kind;
    switch (kind) {
    case K_LRM: return F_LRM;
    case K_LRM4: return F_LRM4;
    case K_LRMB: return F_LRMB;
    case K_LRM96: return F_LRM96;
    case K_DTSS: return F_SHORT;
    default: return F_GROUPED;
    }
}

// A level's products go to one kernel per family: the grouped kernel (or
// its persistent form) and the fused low-rank product kernels.
static void layout_level(const std::vector<int64_t> &prods, const lrbg_desc *ds, const std::vector<int> &variant,
                         uint32_t flags, Schedule &sch, Level &lv)
{
    std::vector<int64_t> fam[kFamilies];
    for (int64_t i : prods) fam[family_of(variant[(size_t)i])].push_back(i);
    lv.qinfo_off = (int32_t)sch.qinfo.size();
    for (int f = 0; f < kFamilies; ++f)
        lay_tiles(fam[f], ds, variant, f == F_GROUPED ? flags : flags & ~(LRBG_PLAN_PERSISTENT | LRBG_PLAN_DUAL),
                  sch, lv.off[f], lv.n[f], f == F_GROUPED);
}

// Scratch the library owns, which no caller buffer can reach:
// kPrivateOut, every output (distinct per product), so there is no
// dependency to find (one level) and no overlap of outputs to reject;
// kPrivateB, every B operand, which then needs no test against outputs.
enum : unsigned { kPrivateOut = 1, kPrivateB = 2 };
static lrbg_status build_schedule(const lrbg_desc *ds, int64_t n, const TuneTable &tt, uint32_t flags,
                                  const int *force_variant, Schedule &sch, unsigned priv = 0)
{
    if (n < 0) return fail(LRBG_EINVAL, "negative count");
    if (n > (int64_t)INT32_MAX / 2) return fail(LRBG_EUNSUPPORTED, "too many products");
    if (n > 0 && !ds) return fail(LRBG_EINVAL, "descriptor array is NULL");
    for (int64_t i = 0; i < n; ++i) {
        lrbg_status st = validate_one(ds[i], i);
        if (st != LRBG_OK) return st;
    }
    std::vector<int> level;
    if (priv & kPrivateOut) {
        level.assign((size_t)n, 0);
    } else {
        lrbg_status st = compute_levels(ds, n, level, (priv & kPrivateB) != 0);
        if (st != LRBG_OK) return st;
    }
    std::vector<int> variant((size_t)n, 0);
    sch.descs.resize((size_t)n);
    double flops = 0, bytes = 0;
    int nlev = 0;
    for (int64_t i = 0; i < n; ++i) {
        const lrbg_desc &d = ds[i];
        int v = 0;
        if (force_variant && variant_fits(*force_variant, d)) v = *force_variant;
        if (!v) {
            auto it = tt.choice.find(bucket_of(d));
            if (it != tt.choice.end() && variant_fits(it->second, d)) v = it->second;
        }
        if (!v) v = default_variant(d);
        if (!v) return fail(LRBG_EUNSUPPORTED, "product %lld: no tile variant fits", (long long)i);
        if (d.m == 0 || d.n == 0) v = 0;   // no-op
        variant[(size_t)i] = v;
        DevDesc &dd = sch.descs[(size_t)i];
        dd.a = d.a;
        dd.b = d.b;
        dd.s = d.s;
        dd.c = d.c;
        dd.e = d.op == LRBG_OP_LRMULT ? d.e : nullptr;
        dd.m = d.m;
        dd.n = d.n;
        dd.k = d.k;
        dd.lda = d.lda;
        dd.ldb = d.ldb;
        dd.lds = d.lds;
        dd.ldc = d.ldc;
        dd.lde = d.op == LRBG_OP_LRMULT ? d.lde : 0;
        double f, b;
        work_of(d, f, b);
        flops += f;
        bytes += b;
        nlev = std::max(nlev, level[(size_t)i] + 1);
    }
    sch.variant = variant;
    std::vector<std::vector<int64_t>> bylevel((size_t)std::max(nlev, 1));
    for (int64_t i = 0; i < n; ++i)
        if (variant[(size_t)i]) bylevel[(size_t)level[(size_t)i]].push_back(i);
    for (auto &prods : bylevel) {
        Level lv;
        layout_level(prods, ds, variant, flags, sch, lv);
        sch.levels.push_back(lv);
    }
    if (sch.tiles.empty()) sch.tiles.push_back(Tile{0, 0, 0, 0});
    if (sch.descs.empty()) sch.descs.push_back(DevDesc{});
    int64_t ntiles = 0;
    int32_t grid = 0;
    for (auto &lv : sch.levels)
        for (int f = 0; f < kFamilies; ++f) {
            ntiles += lv.n[f];
            grid = std::max(grid, lv.n[f]);
        }
    sch.stats.products = n;
    sch.stats.tiles = ntiles;
    sch.stats.levels = (int32_t)sch.levels.size();
    sch.stats.grid = grid;
    sch.stats.useful_flops = flops;
    sch.stats.hbm_bytes = bytes;
    return LRBG_OK;
}

static int g_persist_grid = 0;

static int persistent_grid()
{
    if (!g_persist_grid) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t p;
            if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        }
        g_persist_grid = cus * persistent_blocks_per_cu();
        g_persist_grid = (g_persist_grid + kXcds - 1) / kXcds * kXcds;
    }
    return g_persist_grid;
}

// Enqueue every level of a plan on `stream`.
static lrbg_status enqueue_levels(lrbg_plan *p, hipStream_t stream)
{
    for (auto &lv : p->levels) {
        for (int f = F_GROUPED + 1; f < kFamilies; ++f) {
            const int rc = launch_family(f, p->d_descs, p->d_tiles + lv.off[f], lv.n[f], stream);
            if (rc) return fail(LRBG_EDEVICE, "lrmult launch failed: %s", hipGetErrorString((hipError_t)rc));
        }
        if (lv.n[F_GROUPED] <= 0) continue;
        int rc;
        if (p->flags & LRBG_PLAN_DUAL) {
            rc = launch_reset(p->d_counters + lv.qinfo_off, 2 * kXcds, stream);
            if (!rc) rc = launch_reset(p->d_cu, cu_key_count(), stream);
            if (rc) return fail(LRBG_EDEVICE, "reset launch failed: %s", hipGetErrorString((hipError_t)rc));
            rc = launch_steered(p->d_descs, p->d_tiles + lv.off[F_GROUPED], p->d_qinfo + lv.qinfo_off,
                                p->d_counters + lv.qinfo_off, p->d_cu, lv.n[F_GROUPED], stream);
        } else if (p->flags & LRBG_PLAN_PERSISTENT) {
            rc = launch_reset(p->d_counters + lv.qinfo_off, kXcds, stream);
            if (rc) return fail(LRBG_EDEVICE, "reset launch failed: %s", hipGetErrorString((hipError_t)rc));
            rc = launch_persistent(p->d_descs, p->d_tiles + lv.off[F_GROUPED], p->d_qinfo + lv.qinfo_off,
                                   p->d_counters + lv.qinfo_off, std::min(lv.grid, lv.n[F_GROUPED]), stream);
        } else {
            rc = launch_family(F_GROUPED, p->d_descs, p->d_tiles + lv.off[F_GROUPED], lv.n[F_GROUPED], stream);
        }
        if (rc) return fail(LRBG_EDEVICE, "grouped launch failed: %s", hipGetErrorString((hipError_t)rc));
    }
    return LRBG_OK;
}

static lrbg_status plan_from_schedule(Schedule &sch, uint32_t flags, lrbg_plan **out)
{
    lrbg_plan *p = new (std::nothrow) lrbg_plan();
    if (!p) return fail(LRBG_ENOMEM, "plan allocation failed");
    p->flags = flags;
    p->levels = sch.levels;
    p->stats = sch.stats;
    (void)hipGetDevice(&p->device);
    auto cleanup = [&](lrbg_status st) {
        lrbg_plan_destroy(p);
        return st;
    };
    const size_t nd = sch.descs.size() * sizeof(DevDesc), nt = sch.tiles.size() * sizeof(Tile);
    const size_t nq = std::max<size_t>(sch.qinfo.size(), 1) * sizeof(int32_t);
    if (hipMalloc(&p->d_descs, nd) != hipSuccess || hipMalloc(&p->d_tiles, nt) != hipSuccess ||
        hipMalloc(&p->d_qinfo, nq) != hipSuccess || hipMalloc(&p->d_counters, nq) != hipSuccess)
        return cleanup(fail(LRBG_ENOMEM, "device allocation for the plan failed"));
    if ((flags & LRBG_PLAN_DUAL) && hipMalloc(&p->d_cu, (size_t)cu_key_count() * sizeof(int32_t)) != hipSuccess)
        return cleanup(fail(LRBG_ENOMEM, "device allocation for the plan failed"));
    if (hipMemcpy(p->d_descs, sch.descs.data(), nd, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_tiles, sch.tiles.data(), nt, hipMemcpyHostToDevice) != hipSuccess ||
        (sch.qinfo.size() &&
         hipMemcpy(p->d_qinfo, sch.qinfo.data(), sch.qinfo.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
        return cleanup(fail(LRBG_EDEVICE, "plan upload failed"));
    if (flags & LRBG_PLAN_PERSISTENT) {
        const int grid = persistent_grid();
        for (auto &lv : p->levels) lv.grid = grid;
    }
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
        return cleanup(fail(LRBG_EDEVICE, "event creation failed"));
    // one or two small launches: direct launches are cheaper than a graph
    // launch (measured: 26 -> 19 us for one launch of 256 tiles, 56 -> 49 us
    // for two dependent launches of ~1100 tiles)
    int launches = 0;
    for (const Level &lv : p->levels)
        for (int f = 0; f < kFamilies; ++f) launches += lv.n[f] > 0;
    const bool direct = (flags & LRBG_PLAN_NO_GRAPH) ||
                        (launches <= 2 && !(flags & (LRBG_PLAN_PERSISTENT | LRBG_PLAN_DUAL)) &&
                         sch.stats.tiles <= kDirectLaunchTiles);
    if (!direct) {
        hipStream_t cs;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(LRBG_EDEVICE, "capture stream creation failed"));
        lrbg_status st = LRBG_OK;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            st = fail(LRBG_EDEVICE, "hipStreamBeginCapture failed");
        if (st == LRBG_OK) {
            st = enqueue_levels(p, cs);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &g);
            if (st == LRBG_OK && e != hipSuccess) st = fail(LRBG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            p->graph = g;
        }
        if (st == LRBG_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
            st = fail(LRBG_EDEVICE, "hipGraphInstantiate failed");
        (void)hipStreamDestroy(cs);
        if (st != LRBG_OK) return cleanup(st);
    }
    *out = p;
    return LRBG_OK;
}

// ------------------------------------------------------------- one-shot calls

// One-shot calls stage their schedule (descriptors, tiles) through pooled
// pinned host buffers and pooled device buffers: hipMemcpyAsync on the
// caller's stream, the grouped launch(es), then an event; a buffer pair is
// reused once its event has completed.  After warm-up no call allocates or
// blocks the host on earlier work, so calls on different streams overlap.
struct Staging {
    void *dev = nullptr;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool in_use = false;
    bool recorded = false;   // ev marks the end of the current use (set under g_mu)
    uint64_t seq = 0;        // order in which the uses' events were recorded
};
static std::mutex g_mu;
static std::vector<Staging *> g_staging;
static uint64_t g_seq = 0;
// Scratch this large is not allocated for a third call in flight: the call
// waits for the oldest of two busy buffers instead (allocating tens of GB
// per call is slow, and device memory is finite).  The call it waits for was
// enqueued two calls earlier, so the device stays busy with the one between.
constexpr size_t kBigScratch = size_t(1) << 30;

// with_host: also a pinned host buffer of the same size (for uploads);
// without: device scratch only.
static Staging *acquire_staging(size_t bytes, bool with_host = true)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Staging *best = nullptr;
    for (Staging *st : g_staging) {
        // a buffer in use is free again only once the event recorded after
        // its last enqueued use has completed (an event not yet recorded for
        // this use reads as complete)
        if (st->in_use && st->recorded && hipEventQuery(st->ev) == hipSuccess) st->in_use = false;
        if (!st->in_use && st->cap >= bytes && (st->host != nullptr) == with_host && (!best || st->cap < best->cap))
            best = st;
    }
    if (!best && bytes >= kBigScratch) {
        Staging *oldest = nullptr;
        int busy = 0;
        for (Staging *st : g_staging)
            if (st->in_use && st->recorded && st->cap >= bytes && (st->host != nullptr) == with_host) {
                ++busy;
                if (!oldest || st->seq < oldest->seq) oldest = st;
            }
        if (busy >= 2 && hipEventSynchronize(oldest->ev) == hipSuccess) best = oldest;
    }
    if (best) {
        best->in_use = true;
        best->recorded = false;
        return best;
    }
    // small buffers by powers of two, large ones by 64 MiB steps (a power of
    // two would hold up to twice a large scratch's size)
    size_t cap = 4096;
    while (cap < bytes && cap < (size_t(64) << 20)) cap *= 2;
    if (cap < bytes) cap = (bytes + (size_t(64) << 20) - 1) / (size_t(64) << 20) * (size_t(64) << 20);
    Staging *st = new (std::nothrow) Staging();
    if (!st) return nullptr;
    if (hipMalloc(&st->dev, cap) != hipSuccess) {
        // out of device memory: return the idle buffers of the pool, then retry once
        (void)hipGetLastError();
        for (size_t q = 0; q < g_staging.size();) {
            Staging *o = g_staging[q];
            if (!o->in_use) {
                (void)hipFree(o->dev);
                if (o->host) (void)hipHostFree(o->host);
                if (o->ev) (void)hipEventDestroy(o->ev);
                delete o;
                g_staging.erase(g_staging.begin() + (std::ptrdiff_t)q);
            } else {
                ++q;
            }
        }
        if (hipMalloc(&st->dev, cap) != hipSuccess) {
            (void)hipGetLastError();
            delete st;
            return nullptr;
        }
    }
    if ((with_host && hipHostMalloc(&st->host, cap, hipHostMallocDefault) != hipSuccess) ||
        hipEventCreateWithFlags(&st->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(st->dev);
        if (st->host) (void)hipHostFree(st->host);
        delete st;
        return nullptr;
    }
    st->cap = cap;
    st->in_use = true;
    st->recorded = false;
    g_staging.push_back(st);
    return st;
}

static void release_staging(Staging *sg)
{
    std::lock_guard<std::mutex> lk(g_mu);
    sg->in_use = false;
}

// Record sg's release event on `stream` (after everything that uses sg).
static hipError_t record_release(Staging *sg, hipStream_t stream)
{
    const hipError_t e = hipEventRecord(sg->ev, stream);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_mu);
        sg->recorded = true;
        sg->seq = ++g_seq;
    }
    return e;
}

// Enqueue a built schedule on `stream` through pooled staging buffers.
static lrbg_status enqueue_once(const Schedule &sch, hipStream_t stream)
{
    lrbg_status st = LRBG_OK;
    const size_t nd = sch.descs.size() * sizeof(DevDesc), nt = sch.tiles.size() * sizeof(Tile);
    const size_t toff = (nd + 255) / 256 * 256;
    Staging *sg = acquire_staging(toff + nt);
    if (!sg) return fail(LRBG_ENOMEM, "staging allocation failed");
    memcpy(sg->host, sch.descs.data(), nd);
    memcpy((char *)sg->host + toff, sch.tiles.data(), nt);
    hipError_t e = hipMemcpyAsync(sg->dev, sg->host, toff + nt, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_mu);
        sg->in_use = false;
        return fail(LRBG_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    }
    const DevDesc *dd = (const DevDesc *)sg->dev;
    const Tile *dt = (const Tile *)((char *)sg->dev + toff);
    for (auto &lv : sch.levels) {
        int rc = 0;
        for (int f = 0; f < kFamilies && !rc; ++f) rc = launch_family(f, dd, dt + lv.off[f], lv.n[f], stream);
        if (rc) {
            st = fail(LRBG_EDEVICE, "grouped launch failed: %s", hipGetErrorString((hipError_t)rc));
            break;
        }
    }
    // the buffers are released only after everything enqueued above has run
    e = record_release(sg, stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        release_staging(sg);
        return st != LRBG_OK ? st : fail(LRBG_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    }
    return st;
}

static lrbg_status run_once(const lrbg_desc *ds, int64_t n, hipStream_t stream)
{
    if (n == 0) return LRBG_OK;
    Schedule sch;
    TuneTable tt;
    load_tune_cache(getenv("LRBG_TUNE_CACHE"), tt);
    lrbg_status st = build_schedule(ds, n, tt, 0, nullptr, sch);
    if (st != LRBG_OK) return st;
    return enqueue_once(sch, stream);
}

// ------------------------------------------------- recompressed product

// Product of two low-rank blocks recompressed to rank <= kmax (see
// lr_batched_lrmult_round): G = A_X (A_V^T B_U) B_X by the fused product,
// G = X S Y^T truncated by the batched SVD, U = A_U X_k and V = B_V Y_k by
// DENSE_TS.  Both product schedules are built (and so every argument is
// validated) before anything is launched; G, X, Y live in pooled device
// scratch released by an event after the last launch.
struct RoundArgs {
    int64_t count;
    const int32_t *b, *ra, *rb;
    const double *const *AU, *const *AV, *const *AX, *const *BU, *const *BX, *const *BV;
    const int32_t *ldau, *ldav, *ldax, *ldbu, *ldbx, *ldbv;
    int32_t kmax;
    double tol;
    double *const *U, *const *V;
    const int32_t *ldu, *ldv;
    double *sigma;
    int32_t *kout;
};

// The recompressed product's work, built once for a call or a plan: scratch
// layout (G, X, Y per product), the fused-core and basis-update schedules,
// and the SVD descriptors grouped by size class.
struct RoundBuild {
    size_t total = 0;                       // scratch bytes
    std::vector<size_t> og, ox, oy;         // scratch offsets per product
    Schedule s1, s2;                        // fused core; new bases
    std::vector<SvdDesc> sv;                // by class 16, 32, 64
    int ccount[3] = {0, 0, 0};
};
static const int kSvdClasses[3] = {16, 32, 64};

static lrbg_status round_layout(const RoundArgs &a, RoundBuild &rb)
{
    const int64_t n = a.count;
    if (n < 0) return fail(LRBG_EINVAL, "negative count");
    if (n == 0) return LRBG_OK;
    if (!a.b || !a.ra || !a.rb || !a.AU || !a.AV || !a.AX || !a.BU || !a.BX || !a.BV || !a.ldau || !a.ldav ||
        !a.ldax || !a.ldbu || !a.ldbx || !a.ldbv || !a.U || !a.V || !a.ldu || !a.ldv)
        return fail(LRBG_EINVAL, "a required host array is NULL");
    if (!a.sigma || !a.kout) return fail(LRBG_EINVAL, "sigma and kout must be device arrays");
    if ((uintptr_t)a.sigma % 8 || (uintptr_t)a.kout % 4) return fail(LRBG_EINVAL, "sigma or kout misaligned");
    if (a.kmax < 1 || a.kmax > svd_max_dim())
        return fail(LRBG_EUNSUPPORTED, "kmax must be in [1, %d]", svd_max_dim());
    if (!(a.tol >= 0.0) || !std::isfinite(a.tol)) return fail(LRBG_EINVAL, "tol must be finite and >= 0");
    // scratch: G (ra x rb), X (ra x kmax), Y (rb x kmax) per product, 256-byte aligned
    rb.og.resize((size_t)n);
    rb.ox.resize((size_t)n);
    rb.oy.resize((size_t)n);
    rb.total = 0;
    auto take = [&](size_t elems) {
        const size_t o = rb.total;
        rb.total += (elems * 8 + 255) / 256 * 256;
        return o;
    };
    for (int64_t t = 0; t < n; ++t) {
        if (a.ra[t] < 0 || a.rb[t] < 0 || a.b[t] < 0)
            return fail(LRBG_EINVAL, "product %lld: negative size", (long long)t);
        if (a.ra[t] > svd_max_dim() || a.rb[t] > svd_max_dim())
            return fail(LRBG_EUNSUPPORTED, "product %lld: ranks above %d", (long long)t, svd_max_dim());
        rb.og[(size_t)t] = take((size_t)a.ra[t] * a.rb[t]);
        rb.ox[(size_t)t] = take((size_t)a.ra[t] * a.kmax);
        rb.oy[(size_t)t] = take((size_t)a.rb[t] * a.kmax);
    }
    rb.total = std::max<size_t>(rb.total, 256);
    return LRBG_OK;
}

// Descriptors and schedules with the scratch at `base` (round_layout first).
static lrbg_status round_build(const RoundArgs &a, char *base, RoundBuild &rb)
{
    const int64_t n = a.count;
    std::vector<lrbg_desc> d1((size_t)n), d2((size_t)(2 * n));
    std::vector<SvdDesc> sv((size_t)n);
    for (int64_t t = 0; t < n; ++t) {
        const int ra = a.ra[t], rbk = a.rb[t], bb = a.b[t], km = a.kmax;
        double *G = (double *)(base + rb.og[(size_t)t]), *X = (double *)(base + rb.ox[(size_t)t]),
               *Y = (double *)(base + rb.oy[(size_t)t]);
        lrbg_desc &m = d1[(size_t)t];
        m.op = LRBG_OP_LRMULT;
        m.prec = LRBG_FP64;
        m.m = ra;
        m.n = rbk;
        m.k = bb;
        m.a = a.AV[t];
        m.lda = a.ldav[t];
        m.b = a.BU[t];
        m.ldb = a.ldbu[t];
        m.s = a.AX[t];
        m.lds = a.ldax[t];
        m.e = a.BX[t];
        m.lde = a.ldbx[t];
        m.c = G;
        m.ldc = std::max(ra, 1);
        lrbg_desc &u = d2[(size_t)(2 * t)], &v = d2[(size_t)(2 * t + 1)];
        u.op = v.op = LRBG_OP_DENSE_TS;
        u.prec = v.prec = LRBG_FP64;
        u.m = bb;
        u.k = ra;
        u.n = km;
        u.a = a.AU[t];
        u.lda = a.ldau[t];
        u.b = X;
        u.ldb = std::max(ra, 1);
        u.c = a.U[t];
        u.ldc = a.ldu[t];
        u.lds = 1;
        v.m = bb;
        v.k = rbk;
        v.n = km;
        v.a = a.BV[t];
        v.lda = a.ldbv[t];
        v.b = Y;
        v.ldb = std::max(rbk, 1);
        v.c = a.V[t];
        v.ldc = a.ldv[t];
        v.lds = 1;
        SvdDesc &sd = sv[(size_t)t];
        sd.g = G;
        sd.x = X;
        sd.y = Y;
        sd.sigma = a.sigma + t * km;
        sd.kout = a.kout + t;
        sd.tol = a.tol;
        sd.m = ra;
        sd.n = rbk;
        sd.ldg = std::max(ra, 1);
        sd.ldx = std::max(ra, 1);
        sd.ldy = std::max(rbk, 1);
        sd.kmax = km;
    }
    TuneTable tt;
    load_tune_cache(getenv("LRBG_TUNE_CACHE"), tt);
    // the cores G, and the singular vectors X, Y the basis updates read, are
    // this call's own scratch
    lrbg_status st = build_schedule(d1.data(), n, tt, 0, nullptr, rb.s1, kPrivateOut);
    if (st == LRBG_OK) st = build_schedule(d2.data(), 2 * n, tt, 0, nullptr, rb.s2, kPrivateB);
    if (st != LRBG_OK) return st;
    // group the cores by size class (one SVD launch per class)
    rb.sv.clear();
    rb.sv.reserve(sv.size());
    for (int c = 0; c < 3; ++c) {
        rb.ccount[c] = 0;
        for (const SvdDesc &x : sv) {
            const int dim = std::max(x.m, x.n);
            const int cls = dim <= 16 ? 0 : dim <= 32 ? 1 : 2;
            if (cls == c) {
                rb.sv.push_back(x);
                ++rb.ccount[c];
            }
        }
    }
    return LRBG_OK;
}

static lrbg_status round_svd_launches(const int (&ccount)[3], const SvdDesc *d_sv, hipStream_t stream)
{
    int off = 0;
    for (int c = 0; c < 3; ++c) {
        const int rc = launch_core_svd(kSvdClasses[c], d_sv + off, ccount[c], stream);
        if (rc) return fail(LRBG_EDEVICE, "svd launch failed: %s", hipGetErrorString((hipError_t)rc));
        off += ccount[c];
    }
    return LRBG_OK;
}

static lrbg_status lrmult_round(const RoundArgs &a, hipStream_t stream)
{
    RoundBuild rb;
    lrbg_status st = round_layout(a, rb);
    if (st != LRBG_OK || a.count == 0) return st;
    Staging *scr = acquire_staging(rb.total, false);
    if (!scr) return fail(LRBG_ENOMEM, "scratch allocation failed");
    st = round_build(a, (char *)scr->dev, rb);
    Staging *sd = st == LRBG_OK ? acquire_staging(rb.sv.size() * sizeof(SvdDesc)) : nullptr;
    if (st == LRBG_OK && !sd) st = fail(LRBG_ENOMEM, "staging allocation failed");
    if (st != LRBG_OK) {
        release_staging(scr);
        if (sd) release_staging(sd);
        return st;
    }
    memcpy(sd->host, rb.sv.data(), rb.sv.size() * sizeof(SvdDesc));
    hipError_t e = hipMemcpyAsync(sd->dev, sd->host, rb.sv.size() * sizeof(SvdDesc), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) st = fail(LRBG_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    if (st == LRBG_OK) st = enqueue_once(rb.s1, stream);
    if (st == LRBG_OK) st = round_svd_launches(rb.ccount, (const SvdDesc *)sd->dev, stream);
    if (st == LRBG_OK) st = enqueue_once(rb.s2, stream);
    // scratch and descriptors are released once everything above has run
    if (record_release(scr, stream) != hipSuccess || record_release(sd, stream) != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        release_staging(scr);
        release_staging(sd);
    }
    return st;
}

// ------------------------- recompressed product without allocation
// The same kernels and schedules as lrmult_round, with every device buffer
// the library needs (G, X, Y, the SVD descriptors, both schedules' product
// descriptors and tile lists) placed in the fixed per-device scratch array:
// the cores first, then the tables, each 256-byte aligned.  The tables are
// uploaded with one hipMemcpyAsync from host memory on the caller's stream.

// Launch every level of a schedule whose tables sit at dd / dt.
static lrbg_status launch_levels_at(const Schedule &sch, const DevDesc *dd, const Tile *dt, hipStream_t stream)
{
    for (const Level &lv : sch.levels)
        for (int f = 0; f < kFamilies; ++f) {
            const int rc = launch_family(f, dd, dt + lv.off[f], lv.n[f], stream);
            if (rc) return fail(LRBG_EDEVICE, "grouped launch failed: %s", hipGetErrorString((hipError_t)rc));
        }
    return LRBG_OK;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static lrbg_status lrmult_round_noalloc(const RoundArgs &a, hipStream_t stream)
{
    RoundBuild rb;
    lrbg_status st = round_layout(a, rb);
    if (st != LRBG_OK || a.count == 0) return st;
    const size_t cap = noalloc_scratch_bytes();
    if (rb.total > cap)
        return fail(LRBG_EUNSUPPORTED, "the cores and singular vectors need %zu bytes of scratch; the fixed "
                    "scratch holds %zu (split the batch)", rb.total, cap);
    void *base = nullptr;
    const int e0 = noalloc_scratch(&base);
    if (e0) return fail(LRBG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString((hipError_t)e0));
    char *scr = (char *)base;
    st = round_build(a, scr, rb);
    if (st != LRBG_OK) return st;
    const size_t nsv = rb.sv.size() * sizeof(SvdDesc);
    const size_t nd1 = rb.s1.descs.size() * sizeof(DevDesc), nt1 = rb.s1.tiles.size() * sizeof(Tile);
    const size_t nd2 = rb.s2.descs.size() * sizeof(DevDesc), nt2 = rb.s2.tiles.size() * sizeof(Tile);
    const size_t o_sv = align256(rb.total), o_d1 = o_sv + align256(nsv), o_t1 = o_d1 + align256(nd1);
    const size_t o_d2 = o_t1 + align256(nt1), o_t2 = o_d2 + align256(nd2), end = o_t2 + align256(nt2);
    if (end > cap)
        return fail(LRBG_EUNSUPPORTED, "the call needs %zu bytes of scratch; the fixed scratch holds %zu "
                    "(split the batch)", end, cap);
    std::vector<char> host(end - o_sv);
    memcpy(host.data(), rb.sv.data(), nsv);
    memcpy(host.data() + (o_d1 - o_sv), rb.s1.descs.data(), nd1);
    memcpy(host.data() + (o_t1 - o_sv), rb.s1.tiles.data(), nt1);
    memcpy(host.data() + (o_d2 - o_sv), rb.s2.descs.data(), nd2);
    memcpy(host.data() + (o_t2 - o_sv), rb.s2.tiles.data(), nt2);
    // from pageable host memory: the call returns once the source has been
    // read, so `host` may go out of scope; the copy stays ordered on `stream`
    const hipError_t e = hipMemcpyAsync(scr + o_sv, host.data(), host.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(LRBG_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    st = launch_levels_at(rb.s1, (const DevDesc *)(scr + o_d1), (const Tile *)(scr + o_t1), stream);
    if (st == LRBG_OK) st = round_svd_launches(rb.ccount, (const SvdDesc *)(scr + o_sv), stream);
    if (st == LRBG_OK) st = launch_levels_at(rb.s2, (const DevDesc *)(scr + o_d2), (const Tile *)(scr + o_t2), stream);
    return st;
}

// ------------------------------------------------------ rounded addition
// The sum of two low-rank blocks recompressed (see lr_batched_lradd_round):
// QR of both stacked bases, the core M = R_U diag(A_X, B_X) R_V^T, its
// truncated SVD, and the new bases Q_U X_k and Q_V Y_k; the kernels are in
// lrbg_add.hip, the SVD is the recompressed product's.  Scratch per
// instance: both stacked bases' reflectors and factors, M, X, Y.

static int width_class(int s) { return s <= 16 ? 0 : s <= 32 ? 1 : 2; }
static const int kWidthClasses[3] = {16, 32, 64};

struct AddBuild {
    int kmax = 1;
    size_t total = 0;
    std::vector<size_t> owu, owv, og, ox, oy;
    std::vector<QrDesc> qr[3];
    std::vector<AddCoreDesc> core[3];
    std::vector<SvdDesc> sv[3];
};

// Outputs must be disjoint from each other and from every input: a sweep
// over the operands ordered by first byte, testing element-exact overlap
// only between operands whose byte spans meet.
static lrbg_status check_disjoint(std::vector<std::pair<Mat, bool>> &ops)
{
    std::sort(ops.begin(), ops.end(), [](const std::pair<Mat, bool> &x, const std::pair<Mat, bool> &y) {
        return x.first.range().lo < y.first.range().lo;
    });
    std::vector<const std::pair<Mat, bool> *> active;
    for (const auto &op : ops) {
        if (op.first.empty()) continue;
        const Range r = op.first.range();
        size_t keep = 0;
        for (size_t q = 0; q < active.size(); ++q)
            if (active[q]->first.range().hi > r.lo) active[keep++] = active[q];
        active.resize(keep);
        for (const auto *o : active)
            if ((op.second || o->second) && mats_overlap(op.first, o->first))
                return fail(LRBG_EINVAL, "an output overlaps %s (products %lld and %lld)",
                            op.second && o->second ? "another output" : "an input", (long long)o->first.idx,
                            (long long)op.first.idx);
        active.push_back(&op);
    }
    return LRBG_OK;
}

static lrbg_status add_validate(const RoundArgs &a)
{
    const int64_t n = a.count;
    if (n < 0) return fail(LRBG_EINVAL, "negative count");
    if (n == 0) return LRBG_OK;
    if (!a.b || !a.ra || !a.rb || !a.AU || !a.AV || !a.AX || !a.BU || !a.BX || !a.BV || !a.ldau || !a.ldav ||
        !a.ldax || !a.ldbu || !a.ldbx || !a.ldbv || !a.U || !a.V || !a.ldu || !a.ldv)
        return fail(LRBG_EINVAL, "a required host array is NULL");
    if (!a.sigma || !a.kout) return fail(LRBG_EINVAL, "sigma and kout must be device arrays");
    if ((uintptr_t)a.sigma % 8 || (uintptr_t)a.kout % 4) return fail(LRBG_EINVAL, "sigma or kout misaligned");
    if (a.kmax < 1 || a.kmax > kQrMaxCols) return fail(LRBG_EUNSUPPORTED, "kmax must be in [1, %d]", kQrMaxCols);
    if (!(a.tol >= 0.0) || !std::isfinite(a.tol)) return fail(LRBG_EINVAL, "tol must be finite and >= 0");
    std::vector<std::pair<Mat, bool>> ops;
    ops.reserve((size_t)n * 8 + 2);
    for (int64_t t = 0; t < n; ++t) {
        const int b = a.b[t], ra = a.ra[t], rb = a.rb[t], km = a.kmax;
        if (b < 0 || ra < 0 || rb < 0) return fail(LRBG_EINVAL, "product %lld: negative size", (long long)t);
        if (ra + rb > kQrMaxCols)
            return fail(LRBG_EUNSUPPORTED, "product %lld: ra + rb = %d exceeds %d", (long long)t, ra + rb,
                        kQrMaxCols);
        if (b > kMaxBlock)
            return fail(LRBG_EUNSUPPORTED, "product %lld: block dimension %d exceeds %d", (long long)t, b, kMaxBlock);
        const void *ptr[8] = {a.AU[t], a.AV[t], a.AX[t], a.BU[t], a.BX[t], a.BV[t], a.U[t], a.V[t]};
        const int ld[8] = {a.ldau[t], a.ldav[t], a.ldax[t], a.ldbu[t], a.ldbx[t], a.ldbv[t], a.ldu[t], a.ldv[t]};
        const int rows[8] = {b, b, ra, b, rb, b, b, b}, cols[8] = {ra, ra, ra, rb, rb, rb, km, km};
        const char *nm[8] = {"A_U", "A_V", "A_X", "B_U", "B_X", "B_V", "U", "V"};
        for (int q = 0; q < 8; ++q) {
            if (ld[q] < std::max(1, rows[q]))
                return fail(LRBG_EINVAL, "product %lld: ld of %s = %d < rows = %d", (long long)t, nm[q], ld[q],
                            rows[q]);
            if (rows[q] > 0 && cols[q] > 0) {
                if (!ptr[q]) return fail(LRBG_EINVAL, "product %lld: %s is NULL", (long long)t, nm[q]);
                if ((uintptr_t)ptr[q] % 8)
                    return fail(LRBG_EINVAL, "product %lld: %s not 8-byte aligned", (long long)t, nm[q]);
            }
            ops.emplace_back(mat_of(ptr[q], rows[q], cols[q], ld[q], 8, t), q >= 6);
        }
    }
    Mat sg, ko;
    sg.p = (uintptr_t)a.sigma;
    sg.cols = 1;
    sg.row_bytes = sg.ld_bytes = (uintptr_t)n * (uintptr_t)a.kmax * 8;
    ko.p = (uintptr_t)a.kout;
    ko.cols = 1;
    ko.row_bytes = ko.ld_bytes = (uintptr_t)n * 4;
    ops.emplace_back(sg, true);
    ops.emplace_back(ko, true);
    return check_disjoint(ops);
}

static void add_layout(const RoundArgs &a, AddBuild &ab)
{
    const size_t n = (size_t)a.count;
    ab.kmax = a.kmax;
    ab.total = 0;
    auto take = [&](size_t elems) {
        const size_t o = ab.total;
        ab.total += (elems * 8 + 255) / 256 * 256;
        return o;
    };
    ab.owu.resize(n);
    ab.owv.resize(n);
    ab.og.resize(n);
    ab.ox.resize(n);
    ab.oy.resize(n);
    for (size_t t = 0; t < n; ++t) {
        const int s = a.ra[t] + a.rb[t];
        ab.owu[t] = take(qr_scratch_doubles(a.b[t], s));
        ab.owv[t] = take(qr_scratch_doubles(a.b[t], s));
        ab.og[t] = take((size_t)s * s);
        ab.ox[t] = take((size_t)s * a.kmax);
        ab.oy[t] = take((size_t)s * a.kmax);
    }
    ab.total = std::max<size_t>(ab.total, 256);
}

static void add_build(const RoundArgs &a, char *base, AddBuild &ab)
{
    for (int c = 0; c < 3; ++c) {
        ab.qr[c].clear();
        ab.core[c].clear();
        ab.sv[c].clear();
    }
    for (int64_t t = 0; t < a.count; ++t) {
        const int ra = a.ra[t], rb = a.rb[t], s = ra + rb, c = width_class(s);
        double *wu = (double *)(base + ab.owu[t]), *wv = (double *)(base + ab.owv[t]);
        double *G = (double *)(base + ab.og[t]), *X = (double *)(base + ab.ox[t]), *Y = (double *)(base + ab.oy[t]);
        QrDesc u{}, v{};
        u.w0 = a.AU[t];
        u.ld0 = a.ldau[t];
        u.w1 = a.BU[t];
        u.ld1 = a.ldbu[t];
        u.ws = wu;
        u.xk = X;
        u.out = a.U[t];
        u.ldo = a.ldu[t];
        v.w0 = a.AV[t];
        v.ld0 = a.ldav[t];
        v.w1 = a.BV[t];
        v.ld1 = a.ldbv[t];
        v.ws = wv;
        v.xk = Y;
        v.out = a.V[t];
        v.ldo = a.ldv[t];
        u.b = v.b = a.b[t];
        u.c0 = v.c0 = ra;
        u.c1 = v.c1 = rb;
        u.kmax = v.kmax = a.kmax;
        ab.qr[c].push_back(u);
        ab.qr[c].push_back(v);
        AddCoreDesc cd{};
        cd.ru = wu;
        cd.rv = wv;
        cd.ax = a.AX[t];
        cd.bx = a.BX[t];
        cd.ldax = a.ldax[t];
        cd.ldbx = a.ldbx[t];
        cd.g = G;
        cd.ra = ra;
        cd.rb = rb;
        ab.core[c].push_back(cd);
        SvdDesc sd{};
        sd.g = G;
        sd.x = X;
        sd.y = Y;
        sd.sigma = a.sigma + t * a.kmax;
        sd.kout = a.kout + t;
        sd.tol = a.tol;
        sd.m = sd.n = s;
        sd.ldg = sd.ldx = sd.ldy = std::max(s, 1);
        sd.kmax = a.kmax;
        ab.sv[c].push_back(sd);
    }
    // a wavefront runs 64 / width stacked bases side by side for as many row
    // blocks as the longest of them: keep bases of similar length together
    for (int c = 0; c < 3; ++c)
        std::stable_sort(ab.qr[c].begin(), ab.qr[c].end(), [](const QrDesc &x, const QrDesc &y) { return x.b > y.b; });
}

// Device tables of a built addition, packed in one upload: per width class
// the QR descriptors, the core descriptors, the SVD descriptors.
struct AddTables {
    size_t bytes = 0;
    size_t oq[3], oc[3], os[3];
};

static AddTables add_tables(const AddBuild &ab)
{
    AddTables tb;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    for (int c = 0; c < 3; ++c) {
        tb.oq[c] = take(ab.qr[c].size() * sizeof(QrDesc));
        tb.oc[c] = take(ab.core[c].size() * sizeof(AddCoreDesc));
        tb.os[c] = take(ab.sv[c].size() * sizeof(SvdDesc));
    }
    tb.bytes = std::max<size_t>(off, 256);
    return tb;
}

static void add_pack(const AddBuild &ab, const AddTables &tb, char *host)
{
    for (int c = 0; c < 3; ++c) {
        memcpy(host + tb.oq[c], ab.qr[c].data(), ab.qr[c].size() * sizeof(QrDesc));
        memcpy(host + tb.oc[c], ab.core[c].data(), ab.core[c].size() * sizeof(AddCoreDesc));
        memcpy(host + tb.os[c], ab.sv[c].data(), ab.sv[c].size() * sizeof(SvdDesc));
    }
}

static lrbg_status add_launches(const AddBuild &ab, const AddTables &tb, const char *dev, hipStream_t stream)
{
    int rc = 0;
    for (int c = 0; c < 3 && !rc; ++c)
        rc = launch_qr_factor(kWidthClasses[c], (const QrDesc *)(dev + tb.oq[c]), (int)ab.qr[c].size(), stream);
    for (int c = 0; c < 3 && !rc; ++c)
        rc = launch_add_core(kWidthClasses[c], (const AddCoreDesc *)(dev + tb.oc[c]), (int)ab.core[c].size(),
                             stream);
    for (int c = 0; c < 3 && !rc; ++c)
        rc = launch_core_svd(kWidthClasses[c], (const SvdDesc *)(dev + tb.os[c]), (int)ab.sv[c].size(), stream);
    for (int c = 0; c < 3 && !rc; ++c)
        rc = launch_qr_apply(kWidthClasses[c], ab.kmax, (const QrDesc *)(dev + tb.oq[c]), (int)ab.qr[c].size(),
                             stream);
    if (rc) return fail(LRBG_EDEVICE, "rounded-addition launch failed: %s", hipGetErrorString((hipError_t)rc));
    return LRBG_OK;
}

static lrbg_status lradd_round(const RoundArgs &a, hipStream_t stream)
{
    lrbg_status st = add_validate(a);
    if (st != LRBG_OK || a.count == 0) return st;
    if (a.count > INT32_MAX / 2) return fail(LRBG_EUNSUPPORTED, "count above %d", INT32_MAX / 2);
    AddBuild ab;
    add_layout(a, ab);
    Staging *scr = acquire_staging(ab.total, false);
    if (!scr) return fail(LRBG_ENOMEM, "scratch allocation failed");
    add_build(a, (char *)scr->dev, ab);
    const AddTables tb = add_tables(ab);
    Staging *sd = acquire_staging(tb.bytes);
    if (!sd) {
        release_staging(scr);
        return fail(LRBG_ENOMEM, "staging allocation failed");
    }
    add_pack(ab, tb, (char *)sd->host);
    hipError_t e = hipMemcpyAsync(sd->dev, sd->host, tb.bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) st = fail(LRBG_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
    if (st == LRBG_OK) st = add_launches(ab, tb, (const char *)sd->dev, stream);
    // scratch and tables are released once everything above has run
    if (record_release(scr, stream) != hipSuccess || record_release(sd, stream) != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        release_staging(scr);
        release_staging(sd);
    }
    return st;
}

}  // namespace lrbg

// A recompressed product built once: scratch, the two sub-plans (launched by
// direct enqueue), the SVD descriptors, and one graph over all of it.
struct lrbg_round_plan {
    int64_t count = 0;
    void *d_scratch = nullptr;
    lrbg_plan *core = nullptr, *bases = nullptr;
    lrbg::SvdDesc *d_svd = nullptr;
    int ccount[3] = {0, 0, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
};

// =================================================================== C ABI

using namespace lrbg;

extern "C" {

lrbg_status lr_batched_gemm(int32_t op, int32_t prec, int64_t count, const int32_t *m, const int32_t *n,
                            const int32_t *k, const void *const *A, const int32_t *lda, const void *const *B,
                            const int32_t *ldb, const double *const *S, const int32_t *lds, void *const *C,
                            const int32_t *ldc, void *stream)
{
    if (count < 0) return fail(LRBG_EINVAL, "negative count");
    if (count == 0) return LRBG_OK;
    if (!m || !n || !k || !A || !lda || !B || !ldb || !C || !ldc)
        return fail(LRBG_EINVAL, "a required host array is NULL");
    if (op == LRBG_OP_RECOMP && (!S || !lds)) return fail(LRBG_EINVAL, "RECOMP needs S and lds arrays");
    if (op == LRBG_OP_LRMULT) return fail(LRBG_EINVAL, "LRMULT takes five operands: use lr_batched_lrmult");
    std::vector<lrbg_desc> ds((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        lrbg_desc &d = ds[(size_t)i];
        d.op = op;
        d.prec = prec;
        d.m = m[i];
        d.n = n[i];
        d.k = k[i];
        d.a = A[i];
        d.lda = lda[i];
        d.b = B[i];
        d.ldb = ldb[i];
        d.s = (op == LRBG_OP_RECOMP) ? S[i] : nullptr;
        d.lds = (op == LRBG_OP_RECOMP) ? lds[i] : 1;
        d.c = C[i];
        d.ldc = ldc[i];
        d.flags = 0;
    }
    return run_once(ds.data(), count, (hipStream_t)stream);
}

lrbg_status lr_batched_lrmult(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                              const double *const *AV, const int32_t *ldav, const double *const *BU,
                              const int32_t *ldbu, const double *const *AX, const int32_t *ldax,
                              const double *const *BX, const int32_t *ldbx, double *const *G, const int32_t *ldg,
                              void *stream)
{
    if (count < 0) return fail(LRBG_EINVAL, "negative count");
    if (count == 0) return LRBG_OK;
    if (!b || !ra || !rb || !AV || !ldav || !BU || !ldbu || !AX || !ldax || !BX || !ldbx || !G || !ldg)
        return fail(LRBG_EINVAL, "a required host array is NULL");
    std::vector<lrbg_desc> ds((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        lrbg_desc &d = ds[(size_t)i];
        d.op = LRBG_OP_LRMULT;
        d.prec = LRBG_FP64;
        d.m = ra[i];
        d.n = rb[i];
        d.k = b[i];
        d.a = AV[i];
        d.lda = ldav[i];
        d.b = BU[i];
        d.ldb = ldbu[i];
        d.s = AX[i];
        d.lds = ldax[i];
        d.e = BX[i];
        d.lde = ldbx[i];
        d.c = G[i];
        d.ldc = ldg[i];
    }
    return run_once(ds.data(), count, (hipStream_t)stream);
}

lrbg_status lr_batched_lrmult_round(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                                    const double *const *AU, const int32_t *ldau, const double *const *AV,
                                    const int32_t *ldav, const double *const *AX, const int32_t *ldax,
                                    const double *const *BU, const int32_t *ldbu, const double *const *BX,
                                    const int32_t *ldbx, const double *const *BV, const int32_t *ldbv, int32_t kmax,
                                    double tol, double *const *U, const int32_t *ldu, double *const *V,
                                    const int32_t *ldv, double *sigma, int32_t *kout, void *stream)
{
    RoundArgs a{count, b, ra, rb, AU, AV, AX, BU, BX, BV, ldau, ldav, ldax, ldbu, ldbx, ldbv,
                kmax, tol, U, V, ldu, ldv, sigma, kout};
    return lrmult_round(a, (hipStream_t)stream);
}

lrbg_status lr_batched_lradd_round(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                                   const double *const *AU, const int32_t *ldau, const double *const *AV,
                                   const int32_t *ldav, const double *const *AX, const int32_t *ldax,
                                   const double *const *BU, const int32_t *ldbu, const double *const *BX,
                                   const int32_t *ldbx, const double *const *BV, const int32_t *ldbv, int32_t kmax,
                                   double tol, double *const *U, const int32_t *ldu, double *const *V,
                                   const int32_t *ldv, double *sigma, int32_t *kout, void *stream)
{
    RoundArgs a{count, b, ra, rb, AU, AV, AX, BU, BX, BV, ldau, ldav, ldax, ldbu, ldbx, ldbv,
                kmax, tol, U, V, ldu, ldv, sigma, kout};
    return lradd_round(a, (hipStream_t)stream);
}

lrbg_status lr_batched_lrmult_round_noalloc(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                                            const double *const *AU, const int32_t *ldau, const double *const *AV,
                                            const int32_t *ldav, const double *const *AX, const int32_t *ldax,
                                            const double *const *BU, const int32_t *ldbu, const double *const *BX,
                                            const int32_t *ldbx, const double *const *BV, const int32_t *ldbv,
                                            int32_t kmax, double tol, double *const *U, const int32_t *ldu,
                                            double *const *V, const int32_t *ldv, double *sigma, int32_t *kout,
                                            void *stream)
{
    RoundArgs a{count, b, ra, rb, AU, AV, AX, BU, BX, BV, ldau, ldav, ldax, ldbu, ldbx, ldbv,
                kmax, tol, U, V, ldu, ldv, sigma, kout};
    return lrmult_round_noalloc(a, (hipStream_t)stream);
}

lrbg_status lrbg_round_plan_create(lrbg_round_plan **out, int64_t count, const int32_t *b, const int32_t *ra,
                                   const int32_t *rb, const double *const *AU, const int32_t *ldau,
                                   const double *const *AV, const int32_t *ldav, const double *const *AX,
                                   const int32_t *ldax, const double *const *BU, const int32_t *ldbu,
                                   const double *const *BX, const int32_t *ldbx, const double *const *BV,
                                   const int32_t *ldbv, int32_t kmax, double tol, double *const *U,
                                   const int32_t *ldu, double *const *V, const int32_t *ldv, double *sigma,
                                   int32_t *kout)
{
    if (!out) return fail(LRBG_EINVAL, "out is NULL");
    *out = nullptr;
    RoundArgs a{count, b, ra, rb, AU, AV, AX, BU, BX, BV, ldau, ldav, ldax, ldbu, ldbx, ldbv,
                kmax, tol, U, V, ldu, ldv, sigma, kout};
    RoundBuild bld;
    lrbg_status st = round_layout(a, bld);
    if (st != LRBG_OK) return st;
    lrbg_round_plan *p = new (std::nothrow) lrbg_round_plan();
    if (!p) return fail(LRBG_ENOMEM, "plan allocation failed");
    p->count = count;
    auto cleanup = [&](lrbg_status e) {
        lrbg_round_plan_destroy(p);
        return e;
    };
    if (hipEventCreate(&p->done) != hipSuccess) return cleanup(fail(LRBG_EDEVICE, "event creation failed"));
    if (count == 0) {
        *out = p;
        return LRBG_OK;
    }
    if (hipMalloc(&p->d_scratch, bld.total) != hipSuccess)
        return cleanup(fail(LRBG_ENOMEM, "device allocation for the plan failed"));
    st = round_build(a, (char *)p->d_scratch, bld);
    if (st == LRBG_OK) st = plan_from_schedule(bld.s1, LRBG_PLAN_NO_GRAPH, &p->core);
    if (st == LRBG_OK) st = plan_from_schedule(bld.s2, LRBG_PLAN_NO_GRAPH, &p->bases);
    if (st != LRBG_OK) return cleanup(st);
    const size_t nsv = bld.sv.size() * sizeof(SvdDesc);
    if (hipMalloc(&p->d_svd, std::max<size_t>(nsv, 1)) != hipSuccess)
        return cleanup(fail(LRBG_ENOMEM, "device allocation for the plan failed"));
    if (hipMemcpy(p->d_svd, bld.sv.data(), nsv, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(LRBG_EDEVICE, "plan upload failed"));
    for (int c = 0; c < 3; ++c) p->ccount[c] = bld.ccount[c];
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(LRBG_EDEVICE, "capture stream creation failed"));
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        st = fail(LRBG_EDEVICE, "hipStreamBeginCapture failed");
    if (st == LRBG_OK) {
        st = enqueue_levels(p->core, cs);
        if (st == LRBG_OK) st = round_svd_launches(p->ccount, p->d_svd, cs);
        if (st == LRBG_OK) st = enqueue_levels(p->bases, cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (st == LRBG_OK && e != hipSuccess) st = fail(LRBG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        p->graph = g;
    }
    if (st == LRBG_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        st = fail(LRBG_EDEVICE, "hipGraphInstantiate failed");
    (void)hipStreamDestroy(cs);
    if (st != LRBG_OK) return cleanup(st);
    *out = p;
    return LRBG_OK;
}

lrbg_status lrbg_round_plan_execute(lrbg_round_plan *p, void *stream)
{
    if (!p) return fail(LRBG_EINVAL, "plan is NULL");
    if (p->count == 0) return LRBG_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return fail(LRBG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
    if (hipEventRecord(p->done, s) != hipSuccess) return fail(LRBG_EDEVICE, "event record failed");
    p->launched = true;
    return LRBG_OK;
}

lrbg_status lrbg_round_plan_destroy(lrbg_round_plan *p)
{
    if (!p) return LRBG_OK;
    if (p->launched && p->done) (void)hipEventSynchronize(p->done);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->core) lrbg_plan_destroy(p->core);
    if (p->bases) lrbg_plan_destroy(p->bases);
    if (p->d_svd) (void)hipFree(p->d_svd);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->done) (void)hipEventDestroy(p->done);
    delete p;
    return LRBG_OK;
}

lrbg_status lrbg_grouped(const lrbg_desc *descs, int64_t count, void *stream)
{
    if (count < 0) return fail(LRBG_EINVAL, "negative count");
    return run_once(descs, count, (hipStream_t)stream);
}

lrbg_status lrbg_plan_create(lrbg_plan **out, const lrbg_desc *descs, int64_t count, const char *tune_cache,
                             uint32_t flags)
{
    if (!out) return fail(LRBG_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~kPlanFlags)
        return fail(LRBG_EINVAL, "unknown plan flags 0x%x", flags);
    TuneTable tt;
    load_tune_cache(tune_cache ? tune_cache : getenv("LRBG_TUNE_CACHE"), tt);
    Schedule sch;
    lrbg_status st = build_schedule(descs, count, tt, flags, nullptr, sch);
    if (st != LRBG_OK) return st;
    return plan_from_schedule(sch, flags, out);
}

lrbg_status lrbg_schedule_stats(const lrbg_desc *descs, int64_t count, const char *tune_cache, uint32_t flags,
                                lrbg_plan_stats *out)
{
    if (!out) return fail(LRBG_EINVAL, "out is NULL");
    if (flags & ~kPlanFlags)
        return fail(LRBG_EINVAL, "unknown plan flags 0x%x", flags);
    TuneTable tt;
    load_tune_cache(tune_cache, tt);
    Schedule sch;
    lrbg_status st = build_schedule(descs, count, tt, flags, nullptr, sch);
    if (st != LRBG_OK) return st;
    *out = sch.stats;
    return LRBG_OK;
}

lrbg_status lrbg_schedule_variants(const lrbg_desc *descs, int64_t count, const char *tune_cache, uint32_t flags,
                                   int32_t *variant_out)
{
    if (count > 0 && !variant_out) return fail(LRBG_EINVAL, "variant_out is NULL");
    if (flags & ~kPlanFlags)
        return fail(LRBG_EINVAL, "unknown plan flags 0x%x", flags);
    TuneTable tt;
    load_tune_cache(tune_cache, tt);
    Schedule sch;
    lrbg_status st = build_schedule(descs, count, tt, flags, nullptr, sch);
    if (st != LRBG_OK) return st;
    for (int64_t i = 0; i < count; ++i) variant_out[i] = sch.variant[(size_t)i];
    return LRBG_OK;
}

lrbg_status lrbg_plan_execute(lrbg_plan *p, void *stream)
{
    if (!p) return fail(LRBG_EINVAL, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool timing = !(p->flags & LRBG_PLAN_UNTIMED);
    if (timing && hipEventRecord(p->ev0, s) != hipSuccess) return fail(LRBG_EDEVICE, "event record failed");
    lrbg_status st = LRBG_OK;
    if (p->exec) {
        hipError_t e = hipGraphLaunch(p->exec, s);
        if (e != hipSuccess) st = fail(LRBG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
    } else {
        st = enqueue_levels(p, s);
    }
    if (!timing) {
        p->ran_untimed = true;
        return st;
    }
    if (hipEventRecord(p->ev1, s) != hipSuccess) return fail(LRBG_EDEVICE, "event record failed");
    p->timed = st == LRBG_OK;
    return st;
}

double lrbg_plan_last_ms(lrbg_plan *p)
{
    if (!p || !p->timed) return -1.0;
    if (hipEventSynchronize(p->ev1) != hipSuccess) return -1.0;
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, p->ev0, p->ev1) != hipSuccess) return -1.0;
    return ms;
}

lrbg_status lrbg_plan_destroy(lrbg_plan *p)
{
    if (!p) return LRBG_OK;
    if (p->timed && p->ev1) (void)hipEventSynchronize(p->ev1);
    if (p->ran_untimed) (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->d_descs) (void)hipFree(p->d_descs);
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->d_qinfo) (void)hipFree(p->d_qinfo);
    if (p->d_counters) (void)hipFree(p->d_counters);
    if (p->d_cu) (void)hipFree(p->d_cu);
    delete p;
    return LRBG_OK;
}

lrbg_status lrbg_plan_get_stats(const lrbg_plan *p, lrbg_plan_stats *out)
{
    if (!p || !out) return fail(LRBG_EINVAL, "NULL argument");
    *out = p->stats;
    return LRBG_OK;
}

lrbg_status lrbg_autotune(const lrbg_desc *sample, int64_t count, const char *cache_out, int32_t reps)
{
    if (count <= 0 || !sample) return fail(LRBG_EINVAL, "empty sample");
    if (reps < 1) return fail(LRBG_EINVAL, "reps must be >= 1");
    for (int64_t i = 0; i < count; ++i) {
        lrbg_status st = validate_one(sample[i], i);
        if (st != LRBG_OK) return st;
    }
    std::map<BucketKey, std::vector<lrbg_desc>> buckets;
    for (int64_t i = 0; i < count; ++i) buckets[bucket_of(sample[i])].push_back(sample[i]);
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::ostringstream os;
    os << "# lrbg tuning cache: op prec b r variant ms (#cand lines: every candidate, with the bucket's product count)\n";
    lrbg_status result = LRBG_OK;
    for (auto &kv : buckets) {
        auto &vec = kv.second;
        int best = 0;
        double best_ms = 1e300;
        // candidates from the kernel family of the bucket's default variant:
        // a variant of another family would add a launch to every plan level
        // that holds the bucket, which an isolated timing cannot show
        const int fam = family_of(default_variant(vec[0]));
        for (int v = 1; v < kNumVariants && result == LRBG_OK; ++v) {
            bool ok = family_of(v) == fam;
            for (auto &d : vec) ok = ok && variant_fits(v, d);
            if (!ok) continue;
            Schedule sch;
            TuneTable none;
            if (build_schedule(vec.data(), (int64_t)vec.size(), none, 0, &v, sch) != LRBG_OK) continue;
            lrbg_plan *p = nullptr;
            if (plan_from_schedule(sch, LRBG_PLAN_NO_GRAPH, &p) != LRBG_OK) continue;
            double ms = 1e300;
            for (int r = 0; r <= reps; ++r) {   // first run warms up
                (void)hipEventRecord(e0, s);
                lrbg_status st = enqueue_levels(p, s);
                (void)hipEventRecord(e1, s);
                if (st != LRBG_OK || hipEventSynchronize(e1) != hipSuccess) {
                    result = st != LRBG_OK ? st : fail(LRBG_EDEVICE, "autotune run failed");
                    break;
                }
                float t = 0;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (r > 0) ms = std::min(ms, (double)t);
            }
            lrbg_plan_destroy(p);
            os << "#cand " << std::get<0>(kv.first) << " " << std::get<1>(kv.first) << " " << std::get<2>(kv.first)
               << " " << std::get<3>(kv.first) << " " << variant_name(v) << " " << ms << " " << vec.size() << "\n";
            if (ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        if (best)
            os << std::get<0>(kv.first) << " " << std::get<1>(kv.first) << " " << std::get<2>(kv.first) << " "
               << std::get<3>(kv.first) << " " << variant_name(best) << " " << best_ms << "\n";
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (result != LRBG_OK) return result;
    if (cache_out) {
        std::ofstream f(cache_out);
        if (!f) return fail(LRBG_EINVAL, "cannot write %s", cache_out);
        f << os.str();
    }
    return LRBG_OK;
}

}  // extern "C"

// In-mix coordinate search.  A bucket's fastest variant in isolation is not
// always its fastest inside a mixed batch (neighbouring tiles share the CU's
// LDS, matrix cores and HBM), so starting from the isolation picks of
// `cache_in` each bucket of the sample, largest estimated share first, tries
// every compatible candidate whose isolated time is within kMixIsoSlack of
// the bucket's best: the whole sample is scheduled with that one change and
// its plan is replayed alternately with the current plan; a change that
// makes the median replay faster by more than kMixGain (and again in a
// confirming run with twice the repetitions) is kept.  Passes repeat until
// one keeps nothing.  The output keeps the input's candidate lines (isolated
// times), adds a "#mix" line per trial, and lists every bucket's pick with
// that variant's own isolated time.
namespace lrbg {
constexpr double kMixGain = 0.004;
constexpr double kMixIsoSlack = 1.5;

struct CacheFile {
    TuneTable tt;
    std::vector<std::string> cand_lines;
    std::map<std::pair<BucketKey, int>, double> iso_ms;   // (bucket, variant) -> isolated ms
    std::map<BucketKey, double> best_iso;
};

static void read_cache_file(const char *path, CacheFile &cf)
{
    load_tune_cache(path, cf.tt);
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.rfind("#cand ", 0) != 0) continue;
        cf.cand_lines.push_back(line);
        std::istringstream is(line.substr(6));
        int op, prec, b, r;
        std::string nm;
        double ms;
        if (!(is >> op >> prec >> b >> r >> nm >> ms)) continue;
        const int v = variant_by_name(nm);
        if (!v) continue;
        const BucketKey key(op, prec, b, r);
        cf.iso_ms[{key, v}] = ms;
        auto it = cf.best_iso.find(key);
        if (it == cf.best_iso.end() || ms < it->second) cf.best_iso[key] = ms;
    }
}

// Median of `reps` replays of each plan, replayed alternately (a, b, a, b, ...).
static lrbg_status time_pair(lrbg_plan *a, lrbg_plan *b, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                             double &ma, double &mb)
{
    std::vector<double> ta, tb;
    for (int r = 0; r <= reps; ++r)
        for (int w = 0; w < 2; ++w) {
            lrbg_plan *p = w ? b : a;
            if (hipEventRecord(e0, s) != hipSuccess) return fail(LRBG_EDEVICE, "event record failed");
            lrbg_status st = p->exec ? (hipGraphLaunch(p->exec, s) == hipSuccess ? LRBG_OK : LRBG_EDEVICE)
                                     : enqueue_levels(p, s);
            if (st != LRBG_OK) return fail(LRBG_EDEVICE, "autotune replay failed");
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(LRBG_EDEVICE, "autotune run failed");
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (r > 0) (w ? tb : ta).push_back(t);   // the first replay of each warms up
        }
    auto med = [](std::vector<double> &v) {
        std::sort(v.begin(), v.end());
        const size_t n = v.size();
        return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
    };
    ma = med(ta);
    mb = med(tb);
    return LRBG_OK;
}

static lrbg_status plan_with(const lrbg_desc *ds, int64_t n, const TuneTable &tt, uint32_t flags, lrbg_plan **p)
{
    Schedule sch;
    lrbg_status st = build_schedule(ds, n, tt, flags, nullptr, sch);
    if (st != LRBG_OK) return st;
    return plan_from_schedule(sch, flags, p);
}
}  // namespace lrbg

extern "C" {

lrbg_status lrbg_autotune_mix(const lrbg_desc *sample, int64_t count, const char *cache_in, const char *cache_out,
                              int32_t reps, int32_t passes, uint32_t flags)
{
    if (count <= 0 || !sample) return fail(LRBG_EINVAL, "empty sample");
    if (reps < 1 || passes < 1) return fail(LRBG_EINVAL, "reps and passes must be >= 1");
    if (flags & ~(uint32_t)(LRBG_PLAN_PERSISTENT | LRBG_PLAN_NO_GRAPH | LRBG_PLAN_SCHED_MIX | LRBG_PLAN_DUAL |
                            LRBG_PLAN_UNTIMED))
        return fail(LRBG_EINVAL, "unknown plan flags 0x%x", flags);
    for (int64_t i = 0; i < count; ++i) {
        lrbg_status st = validate_one(sample[i], i);
        if (st != LRBG_OK) return st;
    }
    CacheFile cf;
    read_cache_file(cache_in, cf);
    // buckets of the sample: estimated time, current pick, candidates
    std::map<BucketKey, double> share;
    std::map<BucketKey, std::vector<int64_t>> members;
    for (int64_t i = 0; i < count; ++i) {
        const BucketKey key = bucket_of(sample[i]);
        share[key] += est_time(sample[i]);
        members[key].push_back(i);
    }
    TuneTable cur = cf.tt;
    std::vector<BucketKey> order;
    std::map<BucketKey, std::vector<int>> cands;
    for (auto &kv : members) {
        const BucketKey &key = kv.first;
        auto fits_all = [&](int v) {
            for (int64_t i : kv.second)
                if (!variant_fits(v, sample[i])) return false;
            return true;
        };
        if (!cur.choice.count(key) || !fits_all(cur.choice[key])) cur.choice[key] = default_variant(sample[kv.second[0]]);
        auto bi = cf.best_iso.find(key);
        const int fam = family_of(default_variant(sample[kv.second[0]]));
        for (int v = 1; v < kNumVariants; ++v) {
            if (v == cur.choice[key] || family_of(v) != fam || !fits_all(v)) continue;
            if (bi != cf.best_iso.end()) {
                auto iv = cf.iso_ms.find({key, v});
                if (iv == cf.iso_ms.end() || iv->second > kMixIsoSlack * bi->second) continue;
            }
            cands[key].push_back(v);
        }
        order.push_back(key);
    }
    std::stable_sort(order.begin(), order.end(), [&](const BucketKey &x, const BucketKey &y) { return share[x] > share[y]; });
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::ostringstream mix;
    lrbg_plan *base = nullptr;
    lrbg_status st = LRBG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        st = fail(LRBG_EDEVICE, "event creation failed");
    if (st == LRBG_OK) st = plan_with(sample, count, cur, flags, &base);
    auto key_str = [](const BucketKey &k) {
        std::ostringstream o;
        o << std::get<0>(k) << " " << std::get<1>(k) << " " << std::get<2>(k) << " " << std::get<3>(k);
        return o.str();
    };
    for (int pass = 0; pass < passes && st == LRBG_OK; ++pass) {
        bool changed = false;
        for (const BucketKey &key : order) {
            for (int v : cands[key]) {
                if (st != LRBG_OK || v == cur.choice[key]) continue;
                TuneTable trial = cur;
                trial.choice[key] = v;
                lrbg_plan *p = nullptr;
                if (plan_with(sample, count, trial, flags, &p) != LRBG_OK) continue;
                double mb = 0, mc = 0;
                st = time_pair(base, p, reps, s, e0, e1, mb, mc);
                bool keep = st == LRBG_OK && mc < mb * (1.0 - kMixGain);
                double mb2 = 0, mc2 = 0;
                if (keep) {
                    st = time_pair(base, p, 2 * reps, s, e0, e1, mb2, mc2);
                    keep = st == LRBG_OK && mc2 < mb2 * (1.0 - kMixGain);
                }
                mix << "#mix " << key_str(key) << " " << variant_name(cur.choice[key]) << " -> " << variant_name(v)
                    << " batch_ms " << mb << " " << mc;
                if (mb2 > 0) mix << " confirm " << mb2 << " " << mc2;
                mix << (keep ? " kept" : "") << "\n";
                if (keep) {
                    lrbg_plan_destroy(base);
                    base = p;
                    cur = trial;
                    changed = true;
                } else {
                    lrbg_plan_destroy(p);
                }
            }
        }
        if (!changed) break;
    }
    if (base) lrbg_plan_destroy(base);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (st != LRBG_OK) return st;
    if (cache_out) {
        std::ofstream f(cache_out);
        if (!f) return fail(LRBG_EINVAL, "cannot write %s", cache_out);
        f << "# lrbg tuning cache: op prec b r variant ms (ms: the variant's isolated time in its bucket; #cand: "
             "every candidate in isolation; #mix: whole-sample replays, current -> trial, median ms)\n";
        for (const std::string &l : cf.cand_lines) f << l << "\n";
        f << mix.str();
        for (auto &kv : cur.choice) {
            auto iv = cf.iso_ms.find({kv.first, kv.second});
            f << key_str(kv.first) << " " << variant_name(kv.second) << " ";
            if (iv != cf.iso_ms.end())
                f << iv->second;
            else
                f << "nan";
            f << "\n";
        }
    }
    return LRBG_OK;
}

int32_t lrbg_variant_count(void) { return kNumVariants; }

const char *lrbg_variant_name(int32_t v)
{
    static thread_local std::string s;
    s = variant_name(v);
    return s.c_str();
}

const char *lrbg_status_string(lrbg_status s)
{
    switch (s) {
    case LRBG_OK: return "ok";
    case LRBG_EINVAL: return "invalid argument";
    case LRBG_EUNSUPPORTED: return "unsupported";
    case LRBG_ENOMEM: return "out of memory";
    case LRBG_EDEVICE: return "device error";
    case LRBG_EBUDGET: return "over budget";
    }
    return "unknown status";
}

const char *lrbg_last_error(void) { return g_last_error.c_str(); }

int32_t lrbg_version(void) { return 100; }

}  // extern "C"
