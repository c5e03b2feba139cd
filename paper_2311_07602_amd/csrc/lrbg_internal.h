// Internal definitions shared by the HIP kernels and the host side of the
// library: the device descriptor of one product, the tile record of the
// grouped schedule, and the table of compiled tile variants.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace lrbg {

// One product as the kernels see it (72 bytes).  Element types follow the
// variant: FP64 variants read double a/b, BF16X3 variants read float a/b;
// every output c is double.
struct DevDesc {
    const void *a;
    const void *b;
    const double *s;
    void *c;
    const double *e;
    int32_t m, n, k;
    int32_t lda, ldb, lds, ldc, lde;
};
static_assert(sizeof(DevDesc) == 72, "DevDesc layout");

// One workgroup's unit of work: product `desc`, computed by `variant`,
// starting at row (DENSE_TS, INNER) or column (RECOMP) `p0`.  flags bit 0
// (kTileEdge) marks a tile that touches a ragged block-type edge or a
// contraction tail and must run the guarded code path.
struct Tile {
    int32_t desc;
    int32_t variant;
    int32_t p0;
    int32_t flags;
};
constexpr int32_t kTileEdge = 1;
static_assert(sizeof(Tile) == 16, "Tile layout");

enum Kind : int32_t {
    K_NOP = 0,
    K_DTS64 = 1,   // DENSE_TS, FP64 MFMA          params: RM, RN, KG
    K_INN64 = 2,   // INNER, FP64 MFMA             params: RI, RJ, KS, KG
    K_REC64 = 3,   // RECOMP, FP64 MFMA            params: RB, BNB, KG
    K_DTS3 = 4,    // DENSE_TS, bf16x3 split MFMA  params: RM, RN, PF (prefetch)
    K_INN3 = 5,    // INNER, bf16x3 split MFMA     params: RI, RJ, KS, PF
    K_DTSL = 6,    // DENSE_TS, FP64, U in LDS     params: RM, RN, KG
    K_INNL = 7,    // INNER, FP64, LDS-staged      params: RI, RJ, WR, KG
    K_LRM = 8,     // LRMULT, FP64, fused          params: RI, RJ, KS, KG (INNER phase)
    K_LRM4 = 9,    // as K_LRM in the high-occupancy fused kernel (32 KB LDS, <= 128 VGPRs)
    K_LRMB = 10,   // LRMULT, FP64, fused, ranks <= 128  params: RI, RJ, -, KG (8 waves, 128 KB LDS)
    K_DTSS = 11,   // DENSE_TS, FP64, short contraction (k <= 64)  params: RM, RN, KG (no LDS)
    K_LRM96 = 12,  // LRMULT, FP64, fused, ranks <= 96  params: RI, RJ, -, KG (12 waves, 145 KB LDS)
};

// Kernel families: each family of variants is compiled into its own kernel
// and a plan level issues one launch per non-empty family.
enum Family : int32_t {
    F_GROUPED = 0,   // lrbg_grouped_kernel / lrbg_persistent_kernel
    F_LRM = 1,       // lrbg_lrmult_kernel: 64 KB LDS, 2 workgroups per CU
    F_LRM4 = 2,      // lrbg_lrmult4_kernel: 32 KB LDS, 4 workgroups per CU
    F_LRMB = 3,      // lrbg_lrmultb_kernel: 8 waves, 128 KB LDS, 1 workgroup per CU
    F_SHORT = 4,     // lrbg_short_kernel: no LDS, up to 4 workgroups per CU
    F_LRM96 = 5,     // lrbg_lrmult96_kernel: 12 waves, 145 KB LDS, 1 workgroup per CU
};
constexpr int kFamilies = 6;
constexpr int kThreads96 = 768;
constexpr int kLdsBytes96 = (2 * 24 * 194 + 96 * 97) * 8;   // the KG = 6 staging (24 k x 2 x 97) + the factor region
constexpr int kLdsBytes4 = 32768;
constexpr int kThreadsB = 512;
constexpr int kLdsBytesB = 131072;

constexpr int kThreads = 256;       // 4 wavefronts of 64
constexpr int kWaves = 4;
constexpr int kLdsBytes = 65536;    // static LDS per workgroup (2 workgroups per CU)
constexpr int kMaxRank = 128;
constexpr int kMaxLrRank = 128;    // LRMULT: the rank x rank core staged in LDS
constexpr int kMaxBlock = 65536;
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies

// X(id, kind, p1, p2, p3, p4): the compiled tile variants.  Ids are dense
// and stable within a build; tuning caches refer to variants by name.
// LRBG_VARIANTS run in the grouped kernel; LRBG_LRM_VARIANTS (the fused
// low-rank product) in a kernel of their own, so that their code and
// register pressure stay out of the grouped kernel.
#define LRBG_VARIANTS(X)           \
    X(1, K_DTS64, 1, 1, 8, 0)      \
    X(2, K_DTS64, 2, 1, 8, 0)      \
    X(3, K_DTS64, 4, 1, 8, 0)      \
    X(4, K_DTS64, 1, 2, 8, 0)      \
    X(5, K_DTS64, 2, 2, 8, 0)      \
    X(6, K_DTS64, 1, 4, 4, 0)      \
    X(7, K_DTS64, 2, 4, 4, 0)      \
    X(8, K_INN64, 1, 1, 4, 8)      \
    X(9, K_INN64, 2, 2, 4, 8)      \
    X(10, K_INN64, 2, 2, 2, 8)     \
    X(11, K_INN64, 2, 4, 2, 4)     \
    X(12, K_INN64, 1, 4, 4, 4)     \
    X(13, K_REC64, 1, 4, 2, 0)     \
    X(14, K_REC64, 1, 4, 8, 0)     \
    X(15, K_REC64, 2, 4, 4, 0)     \
    X(16, K_REC64, 1, 2, 8, 0)     \
    X(17, K_REC64, 1, 8, 4, 0)     \
    X(18, K_REC64, 2, 2, 8, 0)     \
    X(19, K_DTSL, 2, 2, 8, 0)      \
    X(20, K_DTSL, 4, 2, 4, 0)      \
    X(21, K_DTSL, 2, 4, 4, 0)      \
    X(22, K_DTSL, 4, 4, 4, 0)      \
    X(23, K_DTSL, 2, 8, 4, 0)      \
    X(24, K_DTSL, 1, 8, 4, 0)      \
    X(25, K_INNL, 4, 4, 2, 2)      \
    X(26, K_INNL, 2, 2, 2, 4)      \
    X(27, K_INNL, 2, 4, 4, 4)      \
    X(28, K_INNL, 4, 4, 2, 3)      \
    X(29, K_DTS3, 4, 1, 0, 0)      \
    X(30, K_DTS3, 2, 2, 1, 0)      \
    X(31, K_DTS3, 2, 4, 0, 0)      \
    X(32, K_DTS3, 1, 8, 0, 0)      \
    X(33, K_DTS3, 1, 2, 1, 0)      \
    X(34, K_INN3, 1, 1, 4, 1)      \
    X(35, K_INN3, 2, 2, 4, 1)      \
    X(36, K_INN3, 1, 4, 4, 1)      \
    X(37, K_INN3, 1, 8, 4, 0)      \
    X(38, K_INN3, 2, 2, 2, 1)

#define LRBG_LRM_VARIANTS(X)          \
    X(39, K_LRM, 1, 1, 4, 8)          \
    X(40, K_LRM, 2, 2, 4, 8)          \
    X(41, K_LRM, 2, 4, 2, 4)

#define LRBG_LRM4_VARIANTS(X)         \
    X(42, K_LRM4, 1, 1, 4, 8)         \
    X(43, K_LRM4, 1, 1, 4, 4)         \
    X(44, K_LRM4, 1, 2, 2, 4)         \
    X(45, K_LRM4, 2, 2, 4, 2)

#define LRBG_LRMB_VARIANTS(X)         \
    X(46, K_LRMB, 4, 2, 0, 4)         \
    X(47, K_LRMB, 2, 4, 0, 4)         \
    X(48, K_LRMB, 4, 2, 0, 2)

// Dense products with a short contraction (the new bases of a recompressed
// product, b x r times r x k): 1-4 k per lane group.
#define LRBG_SHORT_VARIANTS(X)        \
    X(49, K_DTSS, 4, 1, 2, 0)         \
    X(50, K_DTSS, 2, 1, 4, 0)         \
    X(51, K_DTSS, 2, 2, 2, 0)         \
    X(52, K_DTSS, 2, 4, 1, 0)

// Fused low-rank products of ranks 65..96 on a 96-wide tile (12 waves):
// the 128-wide tile would spend 44% of its matrix-core work on padding.
#define LRBG_LRM96_VARIANTS(X)        \
    X(53, K_LRM96, 1, 3, 0, 4)        \
    X(54, K_LRM96, 3, 1, 0, 4)        \
    X(55, K_LRM96, 1, 3, 0, 6)

#define LRBG_ALL_VARIANTS(X) \
    LRBG_VARIANTS(X) LRBG_LRM_VARIANTS(X) LRBG_LRM4_VARIANTS(X) LRBG_LRMB_VARIANTS(X) LRBG_SHORT_VARIANTS(X) \
    LRBG_LRM96_VARIANTS(X)

constexpr int kNumVariants = 56;   // ids 0..55 (0 = no-op tile)

struct VariantInfo {
    int32_t kind, p1, p2, p3, p4;
};

// One small truncated SVD (recompression of a low-rank product's core).
struct SvdDesc {
    const double *g;    // m x n core, column-major, ld ldg
    double *x;          // m x kmax left singular vectors (zero beyond the rank kept)
    double *y;          // n x kmax right singular vectors
    double *sigma;      // kmax singular values, descending (zero beyond the rank kept)
    int32_t *kout;      // the rank kept
    double tol;         // keep sigma_i > tol * sigma_max
    int32_t m, n, ldg, ldx, ldy, kmax;
};

// One stacked basis [W0 | W1] (b x s, s = c0 + c1 <= 64) of a rounded
// addition: the QR factorisation writes its reflectors and triangular factor
// to `ws`; the basis update applies them to the singular vectors `xk`
// (s x kmax, ld s) and writes the new basis `out` (b x kmax, ld ldo).
struct QrDesc {
    const double *w0;   // b x c0, ld ld0 (A_U or A_V)
    const double *w1;   // b x c1, ld ld1 (B_U or B_V)
    double *ws;         // scratch, qr_scratch_doubles(b, s) doubles
    const double *xk;
    double *out;
    int32_t b, c0, c1, ld0, ld1, ldo, kmax, pad;
};

// The core of a rounded addition, M = R_U diag(A_X, B_X) R_V^T (s x s).
struct AddCoreDesc {
    const double *ru, *rv;   // s x s triangular factors, row-major (scratch)
    const double *ax, *bx;   // ra x ra (ld ldax), rb x rb (ld ldbx)
    double *g;               // M, column-major, ld s (scratch)
    int32_t ra, rb, ldax, ldbx;
};

// Rows per block of the QR after the first s0 = min(s, b) rows.
constexpr int kQrRows = 32;
constexpr int kQrMaxCols = 64;

// Scratch of one stacked basis (doubles): the triangular factor R (s x s,
// row-major), the first s0 rows' reflector factors (s taus, then the s0 x s
// reduced rows, row-major: R above the diagonal, reflector tails below),
// then per block of kQrRows rows s taus and the block's reflector tails
// (kQrRows x s, column-major).
inline size_t qr_scratch_doubles(int b, int s)
{
    const int s0 = s < b ? s : b;
    const size_t nblk = b > s0 ? (size_t)(b - s0 + kQrRows - 1) / kQrRows : 0;
    return (size_t)s * s + s + (size_t)s0 * s + nblk * ((size_t)s + (size_t)kQrRows * s);
}

// Kernel launch helpers (defined in the lrbg_*.hip kernel sources).
int launch_persistent(const DevDesc *descs, const Tile *tiles, const int32_t *qinfo,
                      int32_t *counters, int grid, void *stream);
int launch_reset(int32_t *counters, int n, void *stream);
int launch_steered(const DevDesc *descs, const Tile *tiles, const int32_t *qinfo, int32_t *counters,
                   int32_t *cu_busy, int ntiles, void *stream);
int cu_key_count();
int launch_family(int family, const DevDesc *descs, const Tile *tiles, int ntiles, void *stream);
int launch_lrm_family(int family, const DevDesc *descs, const Tile *tiles, int ntiles, void *stream);
int launch_short_family(const DevDesc *descs, const Tile *tiles, int ntiles, void *stream);
int persistent_blocks_per_cu();
int launch_core_svd(int nmax, const SvdDesc *descs, int count, void *stream);
int svd_max_dim();
// Rounded addition: launches for one class of stacked widths (cols in {16, 32, 64}).
int launch_qr_factor(int cols, const QrDesc *descs, int count, void *stream);
int launch_qr_apply(int cols, int kmax, const QrDesc *descs, int count, void *stream);
int launch_add_core(int cols, const AddCoreDesc *descs, int count, void *stream);
// The fixed per-device scratch of the allocation-free entry point.
size_t noalloc_scratch_bytes();
int noalloc_scratch(void **ptr);

}  // namespace lrbg
