// Rounded addition of two low-rank blocks: a batched QR of the stacked
// bases, the small core, its truncated SVD (the kernel of lrbg_round.hip)
// and the new bases.
//
// The sum of A = A_U A_X A_V^T and B = B_U B_X B_V^T (b x b blocks of ranks
// ra and rb, bases of any conditioning) is
//   A + B = [A_U | B_U] diag(A_X, B_X) [A_V | B_V]^T.
// With the thin QR factorisations [A_U | B_U] = Q_U R_U and
// [A_V | B_V] = Q_V R_V this is Q_U M Q_V^T with the s x s core
// M = R_U diag(A_X, B_X) R_V^T (s = ra + rb); the SVD M = X S Y^T truncated
// to k terms gives A + B ~ (Q_U X_k) S_k (Q_V Y_k)^T.  This is the rounded
// addition whose first step Sec. 2 names the low-rank product to be.
//
// QR (s <= 64, lane c of a basis's lane group owns column c): the basis is
// read from HBM once, top to bottom.  Its first s0 = min(s, b) rows are
// reduced in LDS by Householder reflections with pivots on the diagonal (the
// head kernel); every later block of kQrRows rows is then reduced against
// the running triangular factor R (the block kernel).  Reflection j of a
// block acts on row j of R and on the block's rows only, v = [e_j; y_j] (R
// is triangular), so the block's columns stay in the lanes' registers: the
// tail y_j comes from the registers of the lane owning column j (through
// LDS, or for a 64-wide basis by lane reads into scalar registers), and
// every lane to its right applies the reflection to its column.  Reflections follow
// LAPACK's convention: beta = -sign(alpha) sqrt(alpha^2 + |x|^2),
// tau = (beta - alpha) / beta, y = x / (alpha - beta); tau = 0 when x = 0.
// The reflectors and taus go to scratch; Q is never formed.  Every
// transformation is an orthogonal map of the basis's own rows, so Q has
// orthonormal columns to working precision whatever the conditioning of the
// basis (an exactly rank-deficient stack -- two blocks sharing a basis --
// included).
//
// Core (one wavefront per instance): E = R_U diag(A_X, B_X) column by column
// in registers, then M = E R_V^T.
//
// New bases (lane c of a basis's lane group owns output column c < kmax, or
// lanes c and c + S / 2 of an S-lane group (S = 32, 64) when the basis keeps
// at most S / 2 columns): U = Q [X_k; 0], applying the stored reflections in
// reverse order:
// blocks from the last to the first, each producing its kQrRows output rows
// in registers while updating the s x kmax top part Z in LDS, then the
// reflections of the first s0 rows on Z, which gives the top s0 rows.
#include "lrbg_tiles.h"

namespace lrbg {

// Wavefronts per basis in the QR kernels: two for 64-wide bases, whose LDS
// (the first rows' block, the triangle) limits how many wavefronts a CU
// holds -- the head kernel splits the rows of every dot product and update
// between them, the block kernel gives them alternate blocks -- and one for
// narrower bases, which registers limit.
constexpr int qr_waves(int cols) { return cols == 64 ? 2 : 1; }

// G = 64 / S stacked bases per wavefront, one per group of S lanes (group g
// = lanes g S .. g S + S - 1, lane c of a group owns column c).  With several
// groups the per-group LDS arrays are padded so that the groups sharing a
// half-wave of an LDS access fall into different banks (an unpadded stride
// that is a multiple of 32 doubles put every group on the same banks).  Loops run to
// the widest case of the class and to the largest block count of the
// wavefront; a column beyond a basis's width, a row beyond its end and a
// group without a basis are zeros, whose reflections are the identity
// (tau = 0), so every group follows the same control flow.
//
// The factorisation runs as two kernels.  The head kernel reduces the first
// s0 = min(s, b) rows, which needs the whole s0 x s block in LDS, and leaves
// R (zeros below the diagonal) in the scratch; the block kernel, which does
// all later rows, keeps only R's upper triangle in LDS, packed row by row,
// so that a CU holds twice as many of its wavefronts (64-wide bases: 17 KB
// against 33 KB).
template <int S>
__global__ void __launch_bounds__(64 * qr_waves(S)) lrbg_qr_head_kernel(const QrDesc *__restrict__ descs, int count)
{
    constexpr int G = 64 / S, NW = qr_waves(S), RW = S / NW;   // rows per wavefront
    const int wv = NW > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) : 0;
    const int lane = (int)threadIdx.x & 63, g = lane / S, c = lane % S;
    const int t = (int)blockIdx.x * G + g;
    QrDesc d{};
    if (t < count) d = descs[t];
    const int c0 = d.c0, s = d.c0 + d.c1, b = d.b, s0 = s < b ? s : b;
    // rows padded to an odd stride: lane i reading column j (row i) and lane
    // c reading row i (column c) both stay off each other's banks
    constexpr int SP = S + 1, RSTR = S * SP + (G > 1 ? 16 : 0);
    __shared__ double R_[G * RSTR];      // the first rows, row-major, stride SP
    __shared__ double part_[NW > 1 ? NW * 64 : 1];   // the wavefronts' partial dot products
    double *R = R_ + g * RSTR;
    const bool mine = c < s;
    gcp cp = (gcp)(!mine ? d.w0 : c < c0 ? d.w0 + (size_t)c * d.ld0 : d.w1 + (size_t)(c - c0) * d.ld1);
    gp ws = (gp)d.ws;
    gp tau0 = ws + (size_t)s * s;
    gp T = tau0 + s;
    const int rlo = RW * wv, rhi = rlo + RW;   // this wavefront's rows

    // Householder QR in LDS, pivots on the diagonal.  The group forms each
    // reflection together: lane i holds row i of the pivot column, the
    // squared norm is a sum over the group's lanes, and every lane derives
    // beta, tau and the scale itself.  The tails stay unscaled until the end
    // (a column's tail is not read again after its own reflection), so the
    // dot products take the scale once.  For 64-wide bases two wavefronts
    // split the rows of every dot product and update, and join the partial
    // dot products through LDS.
    for (int i = rlo; i < rhi; ++i) R[i * SP + c] = (mine && i < s0) ? cp[i] : 0.0;
    __syncthreads();
    double my_tau = 0.0, my_sc = 0.0;
    for (int j = 0; j < S; ++j) {
        const double xi = (c > j && c < s0) ? R[c * SP + j] : 0.0;
        double nrm2 = xi * xi;
#pragma unroll
        for (int m = 1; m < S; m <<= 1) nrm2 += __shfl_xor(nrm2, m);
        const double alpha = R[j * SP + j];
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (j < s0 && nrm2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + nrm2), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (c == j) {
            my_tau = tau;
            my_sc = scale;
        }
        const bool upd = tau != 0.0 && c > j && mine;
        const int lo = j + 1 > rlo ? j + 1 : rlo, hi = s0 < rhi ? s0 : rhi;
        const double rjc = upd ? R[j * SP + c] : 0.0;   // read before row j is updated
        double p0 = 0.0, p1 = 0.0;
        if (upd) {
            int i = lo;
#pragma unroll 4
            for (; i + 1 < hi; i += 2) {
                p0 += R[i * SP + j] * R[i * SP + c];
                p1 += R[(i + 1) * SP + j] * R[(i + 1) * SP + c];
            }
            if (i < hi) p0 += R[i * SP + j] * R[i * SP + c];
        }
        double p = p0 + p1;
        if constexpr (NW > 1) {
            part_[wv * 64 + lane] = p;
            __syncthreads();
            p = part_[lane] + part_[64 + lane];
        }
        if (c == j && j >= rlo && j < rhi && tau != 0.0) R[j * SP + j] = beta;
        if (upd) {
            const double tw = tau * (rjc + scale * p), f = tw * scale;
            if (j >= rlo && j < rhi) R[j * SP + c] = rjc - tw;
#pragma unroll 4
            for (int i = lo; i < hi; ++i) R[i * SP + c] -= f * R[i * SP + j];
        }
        __syncthreads();
    }
    if (mine) {
        // the tails below the diagonal scaled to the reflectors' y
        for (int i = rlo; i < rhi && i < s0; ++i) {
            const double v = R[i * SP + c];
            T[(size_t)i * s + c] = i > c ? v * my_sc : v;
        }
        if (wv == 0) tau0[c] = my_tau;
        // R so far: the triangle, zeros below it (rows s0 .. s - 1 too)
        for (int i = rlo; i < rhi && i < s; ++i) ws[(size_t)i * s + c] = (i <= c && i < s0) ? R[i * SP + c] : 0.0;
    }
}

// The later blocks: reflections [e_j; y_j] against R, columns in registers.
// The pivot lane publishes its column unscaled with the scale 1 / (alpha -
// beta); every lane scales its own column once, when the block is stored.
// R(j, c), c >= j, sits at j S - j (j - 1) / 2 + c - j of the packed triangle.
//
// For 64-wide bases two wavefronts share one triangle and take alternate
// blocks: wavefront w reduces blocks w, w + 2, w + 4, ..., wavefront 1 one
// reflection behind wavefront 0.  Reflection j of block kb needs row j of R
// as reflection j of block kb - 1 left it, and at any time step the two
// wavefronts work on different rows of R, so one workgroup barrier per step
// orders them.  This doubles the wavefronts a CU holds for the same
// triangles in LDS (which otherwise limit it): a reflection is a dependent
// chain (norm, square root, division, broadcast, dot product), and more
// wavefronts hide its latency.
template <int S>
__global__ void __launch_bounds__(64 * qr_waves(S)) lrbg_qr_blocks_kernel(const QrDesc *__restrict__ descs, int count)
{
    constexpr int G = 64 / S, NW = qr_waves(S);
    // the wavefront index, known to the compiler to be uniform
    const int wv = NW > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) : 0;
    const int lane = (int)threadIdx.x & 63, g = lane / S, c = lane % S;
    const int t = (int)blockIdx.x * G + g;
    QrDesc d{};
    if (t < count) d = descs[t];
    const int c0 = d.c0, s = d.c0 + d.c1, b = d.b, s0 = s < b ? s : b;
    constexpr int TRI = S * (S + 1) / 2;
    constexpr int RSTR = TRI + (G > 1 ? 16 : 0), XSTR = kQrRows + (G > 1 ? 2 : 0);
    __shared__ double R_[G * RSTR];          // R's upper triangle, packed by rows
    __shared__ double xs_[NW * G * XSTR];    // each wavefront's current reflection tail
    __shared__ double tau_[NW * G], sc_[NW * G];
    __shared__ int nb_[G];
    double *R = R_ + g * RSTR, *xs = xs_ + (wv * G + g) * XSTR;
    double *tw_ = tau_ + wv * G, *sw_ = sc_ + wv * G;
    auto rp = [](int j) { return j * S - j * (j - 1) / 2; };   // start of row j
    const bool mine = c < s;
    gcp cp = (gcp)(!mine ? d.w0 : c < c0 ? d.w0 + (size_t)c * d.ld0 : d.w1 + (size_t)(c - c0) * d.ld1);
    gp ws = (gp)d.ws;
    gp tau0 = ws + (size_t)s * s;
    gp T = tau0 + s;
    gp blk = T + (size_t)s0 * s;
    const int nblk = b > s0 ? (b - s0 + kQrRows - 1) / kQrRows : 0;
    if (wv == 0) {
        if (c == 0) nb_[g] = nblk;
        for (int i = 0; i <= c; ++i) R[rp(i) + c - i] = (mine && nblk > 0) ? ws[(size_t)i * s + c] : 0.0;
    }
    __syncthreads();
    int nbmax = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) nbmax = nb_[q] > nbmax ? nb_[q] : nbmax;
    const int steps = (nbmax + NW - 1) / NW * S;   // reflections per wavefront

    double x[kQrRows];
    double my_t = 0.0, my_sc = 0.0;
    int kb = wv - NW, j = S - 1;
    for (int tt = 0; tt < steps + NW - 1; ++tt) {
        const bool on = tt >= wv && tt - wv < steps;   // uniform over the wavefront
        if (on) {
            if (++j == S) {
                j = 0;
                kb += NW;
                const int r0 = s0 + kb * kQrRows;
                const int hb = kb < nblk ? (b - r0 < kQrRows ? b - r0 : kQrRows) : 0;
                if (hb == kQrRows && mine) {
                    // 16-byte loads: a lane's rows are contiguous in its column
                    gcp2 p2 = (gcp2)(cp + r0);
#pragma unroll
                    for (int i = 0; i < kQrRows / 2; ++i) {
                        const d2u v = p2[i];
                        x[2 * i] = v.x;
                        x[2 * i + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < kQrRows; ++i) x[i] = (mine && i < hb) ? cp[r0 + i] : 0.0;
                }
            }
            if constexpr (G == 1) {
                // One basis per wavefront, and every lane forms the
                // reflection itself: three quarters of the pivot column's
                // tail come from lane j's registers (j is uniform) into
                // scalar registers, the last quarter through LDS (the pivot
                // lane stores it, every lane reads it back).  All of it
                // through LDS (32 doubles to every lane, twice per
                // reflection) is more than the CU's LDS keeps up with; all
                // of it by lane reads costs more VALU issue than the split
                // (half or three quarters through LDS measured no faster).
                constexpr int HR = 3 * kQrRows / 4;
                if (c == j) {
#pragma unroll
                    for (int i = HR; i < kQrRows; ++i) xs[i - HR] = x[i];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                double y[kQrRows];
#pragma unroll
                for (int i = 0; i < HR; ++i)
                    y[i] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x[i]), j),
                                            __builtin_amdgcn_readlane(__double2loint(x[i]), j));
#pragma unroll
                for (int i = HR; i < kQrRows; ++i) y[i] = xs[i - HR];
                // every lane's dot product with the tail; the pivot lane's is
                // the tail's squared norm, read out like the tail
                double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
                for (int i = 0; i < kQrRows; i += 4) {
                    w0 += y[i] * x[i];
                    w1 += y[i + 1] * x[i + 1];
                    w2 += y[i + 2] * x[i + 2];
                    w3 += y[i + 3] * x[i + 3];
                }
                const double w = (w0 + w1) + (w2 + w3);
                const double nrm2 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(w), j),
                                                     __builtin_amdgcn_readlane(__double2loint(w), j));
                const double alpha = R[rp(j)];
                double tau = 0.0, scale = 0.0, beta = alpha;
                if (nrm2 > 0.0) {
                    beta = -copysign(sqrt(alpha * alpha + nrm2), alpha);
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                }
                if (c == j) {
                    R[rp(j)] = beta;
                    my_t = tau;
                    my_sc = scale;
                }
                if (tau != 0.0 && c > j) {
                    double *rjc = R + rp(j) + c - j;
                    const double tw = tau * (*rjc + scale * w);
                    *rjc -= tw;
                    const double f = tw * scale;
                    __asm__ volatile("" ::: "memory");   // read the LDS part again
#pragma unroll
                    for (int i = 0; i < HR; ++i) x[i] -= f * y[i];
#pragma unroll
                    for (int i = HR; i < kQrRows; ++i) x[i] -= f * xs[i - HR];
                }
            } else {
            if (c == j) {
                double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
#pragma unroll
                for (int i = 0; i < kQrRows; i += 4) {
                    n0 += x[i] * x[i];
                    n1 += x[i + 1] * x[i + 1];
                    n2 += x[i + 2] * x[i + 2];
                    n3 += x[i + 3] * x[i + 3];
                }
                const double nrm2 = (n0 + n1) + (n2 + n3);
                const double alpha = R[rp(j)];
                double tau = 0.0, scale = 0.0;
                if (nrm2 > 0.0) {
                    const double beta = -copysign(sqrt(alpha * alpha + nrm2), alpha);
                    tau = (beta - alpha) / beta;
                    scale = 1.0 / (alpha - beta);
                    R[rp(j)] = beta;
                }
#pragma unroll
                for (int i = 0; i < kQrRows; ++i) xs[i] = x[i];
                tw_[g] = tau;
                sw_[g] = scale;
                my_t = tau;
                my_sc = scale;
            }
            // the pivot's stores reach the rest of its own wavefront: LDS
            // operations of one wavefront complete in order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double tau = tw_[g];
            if (tau != 0.0 && c > j) {
                const double scale = sw_[g];
                double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
                for (int i = 0; i < kQrRows; i += 4) {
                    w0 += xs[i] * x[i];
                    w1 += xs[i + 1] * x[i + 1];
                    w2 += xs[i + 2] * x[i + 2];
                    w3 += xs[i + 3] * x[i + 3];
                }
                double *rjc = R + rp(j) + c - j;
                const double tw = tau * (*rjc + scale * ((w0 + w1) + (w2 + w3)));
                *rjc -= tw;
                const double f = tw * scale;
                // read the tail again for the update rather than keep 32 more
                // values live: halves the registers, so more waves hide latency
                __asm__ volatile("" ::: "memory");
#pragma unroll
                for (int i = 0; i < kQrRows; ++i) x[i] -= f * xs[i];
            }
            }
            if (j == S - 1 && mine && kb < nblk) {
                gp bp = blk + (size_t)kb * (s + (size_t)kQrRows * s);
                gp2 Y = (gp2)(bp + s + (size_t)c * kQrRows);
#pragma unroll
                for (int i = 0; i < kQrRows / 2; ++i) Y[i] = d2u{x[2 * i] * my_sc, x[2 * i + 1] * my_sc};
                bp[c] = my_t;
            }
        }
        __syncthreads();
    }
    if (wv == 0 && mine && nblk > 0)
        for (int i = 0; i <= c; ++i) ws[(size_t)i * s + c] = R[rp(i) + c - i];
}

// Bases 16 or 32 wide.  As the factorisation, G = 64 / S stacked bases per
// wavefront; lane c of a group computes output column c < min(kmax, S) (a
// basis of width s has rank <= s <= S, so any later columns are zero and are
// filled at the end).  The top part Z is S x KZ with KZ = min(S, kmax
// rounded up to 16): LDS, not registers, decides how many wavefronts a CU
// holds here.  The first s0 rows' reflection tails are staged packed
// (column j's s0 - 1 - j entries at j (2 s0 - j - 1) / 2), so they fit the
// room of one block's tails.  A basis of the 32-wide kernel keeping at most
// 16 columns splits each block's rows between lanes c and c + 16 of its
// group, whose partial dot products meet through one swap of 16-lane rows;
// 16-wide bases keeping at most 16 columns run on that kernel too, which
// stops each block's reflections at the widest basis of the wavefront.
template <int S, int KZ>
__global__ void __launch_bounds__(64) lrbg_qr_apply_kernel(const QrDesc *__restrict__ descs, int count)
{
    static_assert(KZ <= S && KZ % 16 == 0 && S < 64, "top part width, several bases per wavefront");
    constexpr int G = 64 / S;
    constexpr bool SPLIT = S == 32 && 2 * KZ <= S;      // two lanes per output column
    constexpr int RH = SPLIT ? kQrRows / 2 : kQrRows;   // block rows per lane
    const int lane = threadIdx.x, g = lane / S, li = lane % S;   // li: loader index within the group
    const int c = SPLIT ? li & 15 : li, h = SPLIT ? li >> 4 : 0;   // output column, row half
    constexpr int NL = S;                  // loaders per group
    const int t = (int)blockIdx.x * G + g;
    QrDesc d{};
    if (t < count) d = descs[t];
    const int s = d.c0 + d.c1, b = d.b, s0 = s < b ? s : b, km = d.kmax;
    // per-group arrays, padded as in the factorisation
    constexpr int ZSTR = S * KZ + (G > 1 ? 16 : 0);
    // CH reflections' tails of a block at a time (column j at (j - jlo)
    // kQrRows), later the first s0 rows' packed tails (s0 (s0 - 1) / 2 <=
    // S (S - 1) / 2 <= kQrRows CH).  For 32-wide bases a block takes two
    // pieces, the next one loaded into registers while the current one is
    // applied (half the LDS of a whole block: more wavefronts per CU).
    constexpr int CH = 16, NQ = S / CH;
    constexpr bool PREF = NQ > 1;
    constexpr int PF = PREF ? CH * kQrRows / NL : 1;
    constexpr int YL = kQrRows * CH, YSTR = YL + (G > 1 ? 2 : 0), TSTR = S + (G > 1 ? 2 : 0);
    static_assert(S * (S - 1) / 2 <= YL, "packed tails fit");
    static_assert(NL == S, "one tau per loader");
    __shared__ double Z_[G * ZSTR];            // s x kmax top part, Z[j * KZ + c]
    __shared__ double Yl_[G * YSTR];
    __shared__ double tl_[G * TSTR];
    __shared__ int nb_[G], sw_[G];
    double *Z = Z_ + g * ZSTR, *Yl = Yl_ + g * YSTR, *tl = tl_ + g * TSTR;
    const bool mine = c < km && c < KZ;       // km <= S implies km <= KZ
    const bool top = h == 0;                  // the lane that owns Z(., c)
    gcp xk = (gcp)d.xk;
    if (c < KZ && top)
        for (int j = 0; j < S; ++j) Z[j * KZ + c] = (mine && j < s) ? xk[j + (size_t)c * s] : 0.0;
    gcp ws = (gcp)d.ws;
    gcp tau0 = ws + (size_t)s * s;
    gcp T = tau0 + s;
    gcp blk = T + (size_t)s0 * s;
    const int nblk = b > s0 ? (b - s0 + kQrRows - 1) / kQrRows : 0;
    if (li == 0) {
        nb_[g] = nblk;
        sw_[g] = s;
    }
    __syncthreads();
    int nbmax = 0, smax = 1;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        nbmax = nb_[q] > nbmax ? nb_[q] : nbmax;
        smax = sw_[q] > smax ? sw_[q] : smax;
    }
    // reflections past the widest basis of the wavefront are the identity
    // for every group: the pieces of a block stop there
    const int jmax = smax - 1, qtop = jmax / CH;
    // this group's piece q of block kb's tails, and the block's taus
    double pf[PF], pt = 0.0;
    auto fetch = [&](int kb, int q) {
        const bool lv = kb < nblk;
        gcp bp = blk + (size_t)kb * (s + (size_t)kQrRows * s);
        const int base = q * YL;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int e = li + NL * p;
            pf[p] = (lv && base + e < s * kQrRows) ? bp[s + base + e] : 0.0;
        }
        pt = (lv && li < s) ? bp[li] : 0.0;
    };
    if constexpr (PREF) {
        if (nbmax > 0) fetch(nbmax - 1, qtop);
    }
    for (int kb = nbmax - 1; kb >= 0; --kb) {
        const bool live = kb < nblk;
        gcp bp = blk + (size_t)kb * (s + (size_t)kQrRows * s);
        const int r0 = s0 + kb * kQrRows, hb = live ? (b - r0 < kQrRows ? b - r0 : kQrRows) : 0;
        double u[RH];
#pragma unroll
        for (int i = 0; i < RH; ++i) u[i] = 0.0;
        for (int q = qtop; q >= 0; --q) {
            __syncthreads();                       // the previous piece's reads of Yl are done
            if constexpr (PREF) {
#pragma unroll
                for (int p = 0; p < PF; ++p) Yl[li + NL * p] = pf[p];
                if (q == qtop) tl[li] = pt;
            } else {
                for (int e = li; e < YL; e += NL) Yl[e] = (live && e < s * kQrRows) ? bp[s + e] : 0.0;
                tl[li] = (live && li < s) ? bp[li] : 0.0;
            }
            __syncthreads();
            if constexpr (PREF) {
                if (q > 0)
                    fetch(kb, q - 1);
                else if (kb > 0)
                    fetch(kb - 1, qtop);
            }
            const int jlo = q * CH;
            // Reflections past the basis's width are the identity (tau = 0), and
            // so is any other with tau = 0: it is applied as such rather than
            // skipped, so that no branch waits on the LDS read of tau.  The tail
            // stays in registers for the update and the next reflection's tail is
            // read a step ahead (LDS, not registers, limits the wavefronts here).
            const int jtop = jlo + CH - 1 < jmax ? jlo + CH - 1 : jmax;
            // reflection j with its tail in yc, loading the next one into yn;
            // two at a time with the buffers' roles swapped, so no copies
            auto reflect = [&](int j, const double (&yc)[RH], double (&yn)[RH]) {
                const double tau = tl[j];
                const double zj = (mine && top) ? Z[j * KZ + c] : 0.0;
                {
                    const double *y = Yl + (j > jlo ? j - 1 - jlo : 0) * kQrRows + RH * h;
#pragma unroll
                    for (int i = 0; i < RH; ++i) yn[i] = y[i];
                }
                double w0 = zj, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
                for (int i = 0; i < RH; i += 4) {
                    w0 += yc[i] * u[i];
                    w1 += yc[i + 1] * u[i + 1];
                    w2 += yc[i + 2] * u[i + 2];
                    w3 += yc[i + 3] * u[i + 3];
                }
                double w = (w0 + w1) + (w2 + w3);
                if constexpr (SPLIT) {
                    // after the swap one result holds this lane's partial and the
                    // other its partner's (lane ^ 16), in either order
                    const unsigned lo = __double2loint(w), hi = __double2hiint(w);
                    const auto sl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
                    const auto sh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
                    w = __hiloint2double((int)sh[0], (int)sl[0]) + __hiloint2double((int)sh[1], (int)sl[1]);
                }
                const double tw = tau * w;
                if (mine && top) Z[j * KZ + c] = zj - tw;
#pragma unroll
                for (int i = 0; i < RH; ++i) u[i] -= tw * yc[i];
            };
            double ya[RH], yb[RH];
            {
                const double *y = Yl + (jtop - jlo) * kQrRows + RH * h;
#pragma unroll
                for (int i = 0; i < RH; ++i) ya[i] = y[i];
            }
            int j = jtop;
            for (; j > jlo; j -= 2) {
                reflect(j, ya, yb);
                reflect(j - 1, yb, ya);
            }
            if (j == jlo) reflect(jlo, ya, yb);
        }
        if (mine && live) {
            gp o = (gp)d.out + (size_t)c * d.ldo + r0 + RH * h;
            const int hv = hb - RH * h;        // valid rows of this lane's part
            if (hv >= RH) {
                gp2 o2 = (gp2)o;
#pragma unroll
                for (int i = 0; i < RH / 2; ++i) o2[i] = d2u{u[2 * i], u[2 * i + 1]};
            } else {
#pragma unroll
                for (int i = 0; i < RH; ++i)
                    if (i < hv) o[i] = u[i];
            }
        }
    }
    // the first s0 rows: reflections with pivots on the diagonal
    __syncthreads();
    auto pk = [s0](int j) { return j * (2 * s0 - j - 1) / 2; };
    for (int j = 0; j < s0; ++j)
        for (int i = j + 1 + li; i < s0; i += NL) Yl[pk(j) + i - j - 1] = T[(size_t)i * s + j];
    for (int e = li; e < S; e += NL) tl[e] = e < s ? tau0[e] : 0.0;
    __syncthreads();
    if (mine && top) {
        for (int j = S - 1; j >= 0; --j) {
            const double tau = j < s0 ? tl[j] : 0.0;
            if (tau == 0.0) continue;
            const double *y = Yl + pk(j) - j - 1;   // y[i] for i > j
            double w = Z[j * KZ + c];
#pragma unroll 4
            for (int i = j + 1; i < s0; ++i) w += y[i] * Z[i * KZ + c];
            const double tw = tau * w;
            Z[j * KZ + c] -= tw;
#pragma unroll 4
            for (int i = j + 1; i < s0; ++i) Z[i * KZ + c] -= tw * y[i];
        }
        gp o = (gp)d.out + (size_t)c * d.ldo;
        for (int i = 0; i < s0; ++i) o[i] = Z[i * KZ + c];
    }
    // output columns S .. kmax - 1 (kmax above the class width): zero
    for (int col = S + li; col < km; col += S) {
        gp o = (gp)d.out + (size_t)col * d.ldo;
        for (int i = 0; i < b; ++i) o[i] = 0.0;
    }
}

// The same application for 64-wide bases (one basis per wavefront), with the
// tails staged CH = 16 reflections at a time instead of a whole block and
// the taus in registers (lane j holds tau_j, read out by the uniform j): LDS
// then holds Z and 4 KB of tails (20 KB against 33 KB at kmax <= 32, eight
// wavefronts per CU instead of four), to hide each reflection's dependent
// chain.  The next piece of tails is loaded into registers while the
// current one is applied and written to LDS at the piece boundary, so no
// wavefront waits on HBM there.  The first s0 rows' tails are staged in
// pieces of at most the same size, packed by columns as above.
template <int KZ>
__global__ void __launch_bounds__(64) lrbg_qr_apply64_kernel(const QrDesc *__restrict__ descs, int count)
{
    constexpr int S = 64;
    static_assert(KZ <= S && KZ % 16 == 0, "top part width");
    constexpr bool SPLIT = 2 * KZ <= S;                 // two lanes per output column
    constexpr int RH = SPLIT ? kQrRows / 2 : kQrRows;   // block rows per lane
    constexpr int CH = 16, YC = CH * kQrRows, PF = YC / 64;
    const int lane = threadIdx.x, c = SPLIT ? lane & 31 : lane;
    const int h = SPLIT ? lane >> 5 : 0;   // row half of a block
    if ((int)blockIdx.x >= count) return;
    const QrDesc d = descs[blockIdx.x];
    const int s = d.c0 + d.c1, b = d.b, s0 = s < b ? s : b, km = d.kmax;
    __shared__ double Z[S * KZ];    // s x kmax top part, Z[j * KZ + c]
    __shared__ double Yl[YC];       // tails of reflections jlo .. jlo + CH - 1 (column j at (j - jlo) kQrRows)
    auto bcast = [](double v, int l) {    // lane l's v, l uniform
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                                __builtin_amdgcn_readlane(__double2loint(v), l));
    };
    const bool mine = c < km && c < KZ;
    const bool top = h == 0;        // the lane that owns Z(., c)
    gcp xk = (gcp)d.xk;
    if (c < KZ && top)
        for (int j = 0; j < S; ++j) Z[j * KZ + c] = (mine && j < s) ? xk[j + (size_t)c * s] : 0.0;
    gcp ws = (gcp)d.ws;
    gcp tau0 = ws + (size_t)s * s;
    gcp T = tau0 + s;
    gcp blk = T + (size_t)s0 * s;
    const int nblk = b > s0 ? (b - s0 + kQrRows - 1) / kQrRows : 0;
    const int jtop = s - 1, qtop = jtop > 0 ? jtop / CH : 0;

    // piece q of block kb's tails (reflections q CH .. q CH + CH - 1) and the
    // block's taus, into registers
    double pf[PF], pt = 0.0;
    auto fetch = [&](int kb, int q) {
        gcp bp = blk + (size_t)kb * (s + (size_t)kQrRows * s);
        const int base = q * YC;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int e = lane + 64 * p;
            pf[p] = base + e < s * kQrRows ? bp[s + base + e] : 0.0;
        }
        pt = lane < s ? bp[lane] : 0.0;
    };
    if (nblk > 0) fetch(nblk - 1, qtop);
    double tc = 0.0;                           // this block's tau of the lane's index
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int r0 = s0 + kb * kQrRows, hb = b - r0 < kQrRows ? b - r0 : kQrRows;
        double u[RH];
#pragma unroll
        for (int i = 0; i < RH; ++i) u[i] = 0.0;
        for (int q = qtop; q >= 0; --q) {
            __syncthreads();                   // the previous piece's reads are done
#pragma unroll
            for (int p = 0; p < PF; ++p) Yl[lane + 64 * p] = pf[p];
            if (q == qtop) tc = pt;
            __syncthreads();
            if (q > 0)
                fetch(kb, q - 1);
            else if (kb > 0)
                fetch(kb - 1, qtop);
            // as in the general kernel: every reflection applied (tau = 0 is
            // the identity), the tail kept in registers and the next one
            // read a step ahead
            const int jlo = q * CH, jhi = jtop < jlo + CH - 1 ? jtop : jlo + CH - 1;
            // reflection j with its tail in yc, loading the next one into yn;
            // two at a time with the buffers' roles swapped, so no copies
            auto reflect = [&](int j, const double (&yc)[RH], double (&yn)[RH]) {
                const double tau = bcast(tc, j);
                const double zj = (mine && top) ? Z[j * KZ + c] : 0.0;
                {
                    const double *y = Yl + (j > jlo ? j - 1 - jlo : 0) * kQrRows + RH * h;
#pragma unroll
                    for (int i = 0; i < RH; ++i) yn[i] = y[i];
                }
                double w0 = zj, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
                for (int i = 0; i < RH; i += 4) {
                    w0 += yc[i] * u[i];
                    w1 += yc[i + 1] * u[i + 1];
                    w2 += yc[i + 2] * u[i + 2];
                    w3 += yc[i + 3] * u[i + 3];
                }
                double w = (w0 + w1) + (w2 + w3);
                if constexpr (SPLIT) {
                    const unsigned lo = __double2loint(w), hi = __double2hiint(w);
                    const auto sl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
                    const auto sh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
                    w = __hiloint2double((int)sh[0], (int)sl[0]) + __hiloint2double((int)sh[1], (int)sl[1]);
                }
                const double tw = tau * w;
                if (mine && top) Z[j * KZ + c] = zj - tw;
#pragma unroll
                for (int i = 0; i < RH; ++i) u[i] -= tw * yc[i];
            };
            double ya[RH], yb[RH];
            {
                const double *y = Yl + (jhi > jlo ? jhi - jlo : 0) * kQrRows + RH * h;
#pragma unroll
                for (int i = 0; i < RH; ++i) ya[i] = y[i];
            }
            int j = jhi;
            for (; j > jlo; j -= 2) {
                reflect(j, ya, yb);
                reflect(j - 1, yb, ya);
            }
            if (j == jlo) reflect(j, ya, yb);
        }
        if (mine) {
            gp o = (gp)d.out + (size_t)c * d.ldo + r0 + RH * h;
            const int hv = hb - RH * h;        // valid rows of this lane's half
            if (hv >= RH) {
                gp2 o2 = (gp2)o;
#pragma unroll
                for (int i = 0; i < RH / 2; ++i) o2[i] = d2u{u[2 * i], u[2 * i + 1]};
            } else {
#pragma unroll
                for (int i = 0; i < RH; ++i)
                    if (i < hv) o[i] = u[i];
            }
        }
    }

    // the first s0 rows: reflections with pivots on the diagonal, j = s0 - 1
    // down to 0; column j's tail (rows j + 1 .. s0 - 1) at pk(j) of the
    // packed order, staged in pieces of consecutive columns of at most YC
    // entries
    auto pk = [s0](int j) { return j * (2 * s0 - j - 1) / 2; };
    tc = lane < s ? tau0[lane] : 0.0;
    for (int jhi = s0 - 1; jhi >= 0;) {
        int jlo = jhi;
        while (jlo > 0 && pk(jhi + 1) - pk(jlo - 1) <= YC) --jlo;
        const int e0 = pk(jlo), ne = pk(jhi + 1) - e0;
        double g[PF];
        int jj = jlo;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int e = lane + 64 * p;
            g[p] = 0.0;
            if (e < ne) {
                while (pk(jj + 1) <= e0 + e) ++jj;
                g[p] = T[(size_t)(e0 + e - pk(jj) + jj + 1) * s + jj];
            }
        }
        __syncthreads();                       // the previous piece's reads are done
#pragma unroll
        for (int p = 0; p < PF; ++p) Yl[lane + 64 * p] = g[p];
        __syncthreads();
        for (int j = jhi; j >= jlo; --j) {
            const double tau = bcast(tc, j);
            if (mine && top) {
                const double *y = Yl + pk(j) - e0 - j - 1;   // y[i] for i > j
                double w = Z[j * KZ + c];
#pragma unroll 4
                for (int i = j + 1; i < s0; ++i) w += y[i] * Z[i * KZ + c];
                const double tw = tau * w;
                Z[j * KZ + c] -= tw;
#pragma unroll 4
                for (int i = j + 1; i < s0; ++i) Z[i * KZ + c] -= tw * y[i];
            }
        }
        jhi = jlo - 1;
    }
    if (mine && top) {
        gp o = (gp)d.out + (size_t)c * d.ldo;
        for (int i = 0; i < s0; ++i) o[i] = Z[i * KZ + c];
    }
}

template <int S>
__global__ void __launch_bounds__(64) lrbg_add_core_kernel(const AddCoreDesc *__restrict__ descs, int count)
{
    if ((int)blockIdx.x >= count) return;
    const AddCoreDesc d = descs[blockIdx.x];
    const int lane = threadIdx.x, ra = d.ra, rb = d.rb, s = d.ra + d.rb;
    __shared__ double RU[S * S];    // R_U, then E = R_U diag(A_X, B_X); row-major, stride S
    // R_V transposed, rows padded to an odd stride so that the transposing
    // stores (consecutive lanes, consecutive rows) fall into different banks:
    // RVt[l * (S + 1) + c] = R_V(c, l)
    __shared__ double RVt[S * (S + 1)];
    gcp ru = (gcp)d.ru, rv = (gcp)d.rv;
    // row by row, lane = column (row-major factors: coalesced), several rows'
    // loads in flight at once
#pragma unroll 8
    for (int i = 0; i < s; ++i)
        if (lane < s) {
            RU[i * S + lane] = ru[(size_t)i * s + lane];
            RVt[lane * (S + 1) + i] = rv[(size_t)i * s + lane];
        }
    __syncthreads();
    // E(:, l) = R_U(:, block of l) * D(block of l, l), lane l
    double e_[S];
#pragma unroll
    for (int i = 0; i < S; ++i) e_[i] = 0.0;
    if (lane < ra) {
        gcp ax = (gcp)d.ax + (size_t)lane * d.ldax;
        for (int m = 0; m < ra; ++m) {
            const double dx = ax[m];
#pragma unroll
            for (int i = 0; i < S; ++i) e_[i] += RU[i * S + m] * dx;
        }
    } else if (lane < s) {
        gcp bx = (gcp)d.bx + (size_t)(lane - ra) * d.ldbx;
        for (int m = 0; m < rb; ++m) {
            const double dx = bx[m];
#pragma unroll
            for (int i = 0; i < S; ++i) e_[i] += RU[i * S + ra + m] * dx;
        }
    }
    __syncthreads();
    if (lane < S) {
#pragma unroll
        for (int i = 0; i < S; ++i) RU[i * S + lane] = e_[i];
    }
    __syncthreads();
    // M(:, c) = sum_l E(:, l) R_V(c, l), lane c
    if (lane < s) {
        double mc[S];
#pragma unroll
        for (int i = 0; i < S; ++i) mc[i] = 0.0;
        for (int l = 0; l < s; ++l) {
            const double v = RVt[l * (S + 1) + lane];
#pragma unroll
            for (int i = 0; i < S; ++i) mc[i] += RU[i * S + l] * v;
        }
        gp g = (gp)d.g + (size_t)lane * s;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (i < s) g[i] = mc[i];
    }
}

// per: descriptors per workgroup of each class (16, 32, 64 wide)
template <typename D, typename K16, typename K32, typename K64>
static int launch_by_class(int cols, const D *descs, int count, void *stream, K16 k16, K32 k32, K64 k64,
                           const int (&per)[3], int threads = 64)
{
    if (count <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    auto grid = [&](int q) { return dim3((unsigned)((count + per[q] - 1) / per[q])); };
    if (cols == 16)
        hipLaunchKernelGGL(k16, grid(0), dim3(threads), 0, st, descs, count);
    else if (cols == 32)
        hipLaunchKernelGGL(k32, grid(1), dim3(threads), 0, st, descs, count);
    else if (cols == 64)
        hipLaunchKernelGGL(k64, grid(2), dim3(threads), 0, st, descs, count);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int launch_qr_factor(int cols, const QrDesc *descs, int count, void *stream)
{
    const int rc = launch_by_class(cols, descs, count, stream, lrbg_qr_head_kernel<16>, lrbg_qr_head_kernel<32>,
                                   lrbg_qr_head_kernel<64>, {4, 2, 1}, 64 * qr_waves(cols));
    if (rc != 0) return rc;
    return launch_by_class(cols, descs, count, stream, lrbg_qr_blocks_kernel<16>, lrbg_qr_blocks_kernel<32>,
                           lrbg_qr_blocks_kernel<64>, {4, 2, 1}, 64 * qr_waves(cols));
}

int launch_qr_apply(int cols, int kmax, const QrDesc *descs, int count, void *stream)
{
    if (count <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const int kz = kmax <= 16 ? 16 : kmax <= 32 ? 32 : 64;
    if (cols == 16 && kz == 16)   // two lanes per column: as a 32-wide class with the later reflections skipped
        hipLaunchKernelGGL((lrbg_qr_apply_kernel<32, 16>), dim3((count + 1) / 2), dim3(64), 0, st, descs, count);
    else if (cols == 16)
        hipLaunchKernelGGL((lrbg_qr_apply_kernel<16, 16>), dim3((count + 3) / 4), dim3(64), 0, st, descs, count);
    else if (cols == 32 && kz == 16)
        hipLaunchKernelGGL((lrbg_qr_apply_kernel<32, 16>), dim3((count + 1) / 2), dim3(64), 0, st, descs, count);
    else if (cols == 32)
        hipLaunchKernelGGL((lrbg_qr_apply_kernel<32, 32>), dim3((count + 1) / 2), dim3(64), 0, st, descs, count);
    else if (cols == 64 && kz == 16)
        hipLaunchKernelGGL(lrbg_qr_apply64_kernel<16>, dim3(count), dim3(64), 0, st, descs, count);
    else if (cols == 64 && kz == 32)
        hipLaunchKernelGGL(lrbg_qr_apply64_kernel<32>, dim3(count), dim3(64), 0, st, descs, count);
    else if (cols == 64)
        hipLaunchKernelGGL(lrbg_qr_apply64_kernel<64>, dim3(count), dim3(64), 0, st, descs, count);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int launch_add_core(int cols, const AddCoreDesc *descs, int count, void *stream)
{
    return launch_by_class(cols, descs, count, stream, lrbg_add_core_kernel<16>, lrbg_add_core_kernel<32>,
                           lrbg_add_core_kernel<64>, {1, 1, 1});
}

}  // namespace lrbg
