// Kernels of the fused low-rank product G = X_A (V_A^T U_B) X_B (Alg. 1).
// They share the INNER accumulation of lrbg_tiles.h with the grouped kernel
// but are compiled into kernels of their own, each with the LDS size and
// register budget its tiles need.
#include "lrbg_tiles.h"

namespace lrbg {

// ---------------------------------------------------------------------------
// LRMULT, FP64, fused.  G = X_A (V_A^T U_B) X_B for one product per
// workgroup (ranks m, n <= R = 16 RI NG = 16 RJ), in the order of Alg. 1:
//   C = V_A^T U_B   the INNER accumulation above (the long k = b contraction)
//   E = X_A C       from LDS, on the matrix cores
//   G = E X_B       from LDS, on the matrix cores; only G is written to HBM.
// Alg. 2 fuses the same chain so that the rank-sized intermediates never
// leave the cache; here they never leave LDS.  LDS (LDSD doubles), R x R
// doubles each:
//   R0 (bottom): C row-major (the E phase reads C(kk, J0 + c): consecutive
//       lanes, consecutive banks), then E column-major (the G phase reads
//       E(I0 + rho(c), kk), again consecutive)
//   R1 (top, clear of the reduction slots of the C phase): X_A column-major,
//       then X_B row-major.
// X_A is fetched before the long contraction and parked in R1 once the first
// chunk's loads are in flight; X_B is fetched with it when it fits in a few
// registers, else at the start of the E phase.  The small contractions run
// over k in steps of 4 with k >= rank read as 0; rows and columns beyond the
// ranks hold finite filler and are never stored.
template <int RI, int RJ, int KS, int KG, bool GUARD, int LDSD>
__device__ __forceinline__ void lrm_tile(const DevDesc &d, int i0, double *lds)
{
    constexpr int NG = 4 / KS;
    constexpr int R = 16 * RJ;
    static_assert(16 * RI * NG == R, "LRMULT tile covers a square R x R core");
    constexpr int SLOTS = (KS - 1) * NG * RI * RJ * 4 * 64;   // reduction doubles of the C phase
    static_assert(SLOTS + R * R <= LDSD && 2 * R * R <= LDSD, "LRMULT staging exceeds LDS");
    constexpr int XE = (R * R + kThreads - 1) / kThreads;   // X elements per thread
    constexpr bool XB_EARLY = XE <= 4;
    constexpr int NB = R / 16;                             // 16 x 16 blocks per side
    constexpr int QB = (NB * NB + kWaves - 1) / kWaves;    // blocks per wave
    const int tid = threadIdx.x, lane = tid & 63, c = lane & 15, g = lane >> 4, w = tid >> 6;
    const int ra = d.m, rb = d.n;
    double *R0 = lds, *R1 = lds + LDSD - R * R;

    // Thread tid takes linear elements idx = tid + 256 e of the R x R square
    // (row = idx % R, col = idx / R): coalesced down the columns.
    auto fetch = [&](double (&x)[XE], const double *p, int ld, int r) {
#pragma unroll
        for (int e = 0; e < XE; ++e) {
            const int idx = tid + kThreads * e, row = idx % R, col = idx / R;
            x[e] = (idx < R * R && row < r && col < r) ? gin(p)[row + (size_t)col * ld] : 0.0;
        }
    };
    double xa[XE], xb[XE];
    fetch(xa, d.s, d.lds, ra);
    if constexpr (XB_EARLY) fetch(xb, d.e, d.lde, rb);

    d4 acc[RI][RJ];
    inn64_accumulate<RI, RJ, KS, KG, GUARD>(d, i0, lds, acc, [&] {
#pragma unroll
        for (int e = 0; e < XE; ++e) {
            const int idx = tid + kThreads * e;
            if (idx < R * R) R1[idx] = xa[e];   // column-major
        }
    });

    // C -> R0, row-major
    const int og = w / KS, ks = w % KS;
    if (ks == 0) {
        const int rowbase = i0 + og * 16 * RI;
#pragma unroll
        for (int bi = 0; bi < RI; ++bi)
#pragma unroll
            for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) R0[(rowbase + bi * 16 + 4 * g + v) * R + bj * 16 + c] = acc[bi][bj][v];
    }
    __syncthreads();
    if constexpr (!XB_EARLY) fetch(xb, d.e, d.lde, rb);

    // Wave w owns output blocks q = w + 4 qq (I-blocks fastest).
    const int nbi = (ra + 15) / 16, nbj = (rb + 15) / 16, nb = nbi * nbj;
    int I0[QB], J0[QB];
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
        const int q = w + kWaves * qq;
        I0[qq] = q < nb ? (q % nbi) * 16 : 0;
        J0[qq] = q < nb ? (q / nbi) * 16 : 0;
    }
    d4 o[QB];

    // E = X_A C, contraction over ra
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) o[qq] = d4{0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < ra; l0 += 4) {
        const bool ok = l0 + g < ra;
        const int kk = ok ? l0 + g : 0;   // masked lanes read a valid LDS address
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) {
            if (w + kWaves * qq >= nb) continue;
            const double a = ok ? R1[I0[qq] + rho(c) + kk * R] : 0.0;
            const double b = ok ? R0[kk * R + J0[qq] + c] : 0.0;
            o[qq] = mfma64(a, b, o[qq]);
        }
    }
    __syncthreads();   // C and X_A are dead

    // E -> R0 (column-major), X_B -> R1 (row-major)
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
        if (w + kWaves * qq >= nb) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) R0[I0[qq] + 4 * g + v + (J0[qq] + c) * R] = o[qq][v];
    }
#pragma unroll
    for (int e = 0; e < XE; ++e) {
        const int idx = tid + kThreads * e, row = idx % R, col = idx / R;
        if (idx < R * R) R1[row * R + col] = xb[e];
    }
    __syncthreads();

    // G = E X_B, contraction over rb
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) o[qq] = d4{0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < rb; l0 += 4) {
        const bool ok = l0 + g < rb;
        const int kk = ok ? l0 + g : 0;
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) {
            if (w + kWaves * qq >= nb) continue;
            const double a = ok ? R0[I0[qq] + rho(c) + kk * R] : 0.0;
            const double b = ok ? R1[kk * R + J0[qq] + c] : 0.0;
            o[qq] = mfma64(a, b, o[qq]);
        }
    }
    const size_t ldg = (size_t)d.ldc;
#pragma unroll
    for (int qq = 0; qq < QB; ++qq) {
        if (w + kWaves * qq >= nb) continue;
        const int orow = I0[qq] + 4 * g, col = J0[qq] + c;
        if (orow >= ra || col >= rb) continue;
        double out[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v] = o[qq][v];
        store_run<4, true>(gout(d.c) + orow + (size_t)col * ldg, out, ra - orow, false);
    }
    __syncthreads();   // LDS is reused by the next tile of a persistent workgroup
}

// ---------------------------------------------------------------------------
// LRMULT for ranks up to R = 128 (8 waves, 128 KB of LDS, one workgroup per
// CU), fused: the R x R intermediates in LDS (C, then E over it); one wave
// per 16 rows of E and G.
//   C phase: wave (wr, wc) of a WR x WC grid accumulates C rows
//            [16 RI wr, +16 RI) x columns [16 RJ wc, +16 RJ) over all of k,
//            each k chunk of V_A and U_B staged once in LDS for all 8 waves
//            (inner_staged); C -> LDS row-major.
//   E phase: wave w forms E rows [16 w, 16 w + 16) x all columns: its strip
//            X_A(16 w + rho(c), Q g + s), s < Q = R / 4, sits in registers
//            (lane group g takes Q consecutive k), C(Q g + s, 16 J + c) comes
//            from LDS (consecutive lanes, consecutive banks); E -> LDS
//            column-major over C.
//   G phase: wave w forms G rows [16 w, 16 w + 16): its E strip comes from
//            LDS into registers, the X_B column strips X_B(Q g + s, 16 J + c)
//            stream from L2 (Q contiguous doubles per lane), one column
//            block ahead, and G is stored block by block.
// Rows and columns beyond the ranks hold finite filler or zeros: X_A columns
// >= ra and X_B rows >= rb read as 0, so they never reach an output, and
// output rows/columns beyond the ranks are not stored.
template <int RI, int RJ, int KG, bool GUARD>
__device__ __forceinline__ void lrmb_tile(const DevDesc &d, double *lds)
{
    constexpr int R = 128, NTHR = kThreadsB, LDSB = kLdsBytesB;
    constexpr int WR = R / (16 * RI), WC = R / (16 * RJ);
    static_assert(WR * WC == NTHR / 64 && 16 * (NTHR / 64) == R, "one C block group and one E row block per wave");
    static_assert(R * R * 8 <= LDSB, "LRMULT core exceeds LDS");
    constexpr int NBJ = R / 16, Q = R / 4;
    const int tid = threadIdx.x, lane = tid & 63, c = lane & 15, g = lane >> 4, w = tid >> 6;
    const int ra = d.m, rb = d.n;
    const int wr = w / WC, wc = w % WC;
    const int row0 = 16 * RI * wr, col0 = 16 * RJ * wc;

    d4 acc[RI][RJ];
    inner_staged<RI, RJ, WR, WC, KG, GUARD, NTHR, LDSB>(d, 0, lds, acc);

    // X_A strip of the E phase, issued before the C store
    const int erow = 16 * w + rho(c);
    double xa[Q];
    {
        gcp p = gin(d.s) + (erow < ra ? erow : 0);
        const size_t ldx = (size_t)d.lds;
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int kk = Q * g + s;
            xa[s] = kk < ra ? p[kk * ldx] : 0.0;
        }
    }

#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[(row0 + 16 * bi + 4 * g + v) * R + col0 + 16 * bj + c] = acc[bi][bj][v];
    __syncthreads();

    // E = X_A C
    const int nbj = (rb + 15) / 16;
    const bool rows_live = 16 * w < ra;
    d4 e[NBJ];
#pragma unroll
    for (int J = 0; J < NBJ; ++J) e[J] = d4{0.0, 0.0, 0.0, 0.0};
    if (rows_live) {
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const double *crow = lds + (Q * g + s) * R + c;
#pragma unroll
            for (int J = 0; J < NBJ; ++J)
                if (J < nbj) e[J] = mfma64(xa[s], crow[16 * J], e[J]);
        }
    }

    auto fetch_xb = [&](int J, double (&xb)[Q]) {
        const int col = 16 * J + c;
        gcp p = gin(d.e) + (size_t)(col < rb ? col : 0) * d.lde + Q * g;
        load_run<Q, true>(xb, p, rb - Q * g);   // rows >= rb read 0
    };
    double xb0[Q], xb1[Q];
    fetch_xb(0, xb0);
    __syncthreads();   // C is dead

#pragma unroll
    for (int J = 0; J < NBJ; ++J)
        if (J < nbj)
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[(16 * w + 4 * g + v) + (16 * J + c) * R] = e[J][v];
    __syncthreads();

    // G = E X_B
    if (!rows_live) return;
    double ea[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) ea[s] = lds[erow + (Q * g + s) * R];
    const size_t ldg = (size_t)d.ldc;
    const int orow = 16 * w + 4 * g;
    auto block = [&](int J, const double (&xb)[Q]) {
        d4 o = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < Q; ++s) o = mfma64(ea[s], xb[s], o);
        const int col = 16 * J + c;
        if (orow < ra && col < rb) {
            double out[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = o[v];
            store_run<4, true>(gout(d.c) + orow + (size_t)col * ldg, out, ra - orow, false);
        }
    };
    // X_B strips one column block ahead (two register buffers)
#pragma unroll
    for (int J = 0; J < NBJ; J += 2) {
        if (J >= nbj) break;
        if (J + 1 < nbj) fetch_xb(J + 1, xb1);
        block(J, xb0);
        if (J + 1 >= nbj) break;
        if (J + 2 < nbj) fetch_xb(J + 2, xb0);
        block(J + 1, xb1);
    }
}

// ---------------------------------------------------------------------------
// LRMULT for ranks up to R = 96, fused, on a 96-wide tile: 12 waves (three
// per SIMD; a workgroup of 6 waves spreads 2-2-1-1 over the four SIMDs and
// left the matrix cores of half of them waiting at every barrier) and 145 KB
// of LDS, one workgroup per CU.  The small factors are staged in LDS, so
// the E and G phases read no operand from L2 and hold no register strips.
// LDS: region 0 holds the INNER staging, then C row-major, then E
// column-major over it; region 1 (R x (R + 1), padded against bank
// conflicts) holds X_A with column k at k (R + 1), then X_B with row k at
// k (R + 1).
//   C phase: wave (wr, wc) of a WR x WC grid accumulates C rows
//            [16 RI wr, +16 RI) x columns [16 RJ wc, +16 RJ) (inner_staged);
//            X_A is fetched into registers before it and parked in region 1
//            with C.
//   E phase: the two waves w and w + 6 share E rows [16 (w % 6), +16), each
//            forming three of the six column blocks; X_B is in flight
//            meanwhile and is parked in region 1 once X_A is dead.
//   G phase: the same split; E rows from region 0, X_B rows from region 1,
//            G stored block by block.
// X_A columns >= ra and X_B rows >= rb are staged as zeros, so they never
// reach an output; rows and columns of G beyond the ranks are not stored.
template <int RI, int RJ, int KG, bool GUARD>
__device__ __forceinline__ void lrm96_tile(const DevDesc &d, double *lds)
{
    constexpr int R = 96, NW = kThreads96 / 64, NTHR = kThreads96, P1 = R + 1;
    constexpr int WR = R / (16 * RI), WC = R / (16 * RJ);
    constexpr int NRB = R / 16, NBJ = R / 16, NBJW = NBJ / (NW / NRB), Q = R / 4;
    static_assert(WR * WC == NW && NRB * (NW / NRB) == NW, "one C block group per wave, two waves per E row block");
    constexpr int KC = 4 * KG, STG = 2 * KC * (2 * R + 2), REG0 = STG > R * R ? STG : R * R;
    static_assert((REG0 + R * P1) * 8 <= kLdsBytes96, "96-wide fused tile exceeds LDS");
    constexpr int NST = R * R / 2 / NTHR;   // 16-byte pairs per thread of an R x R factor
    static_assert(NST * NTHR * 2 == R * R, "factor staging split");
    const int tid = threadIdx.x, lane = tid & 63, c = lane & 15, g = lane >> 4, w = tid >> 6;
    const int ra = d.m, rb = d.n;
    const int wr = w / WC, wc = w % WC;
    const int row0 = 16 * RI * wr, col0 = 16 * RJ * wc;
    const int rbk = w % NRB, jb0 = (w / NRB) * NBJW;
    double *reg1 = lds + REG0;

    // an n x n factor (column-major, ld) into registers: pair p of a thread is
    // rows i, i + 1 of column k; rows and columns >= n read as zeros
    double xst[NST][2];
    auto fetch_factor = [&](gcp base, size_t ld, int n) {
#pragma unroll
        for (int p = 0; p < NST; ++p) {
            const int idx = tid + NTHR * p;
            const int k = idx / (R / 2), i = 2 * (idx % (R / 2));
            load_run<2, true>(xst[p], base + i + (size_t)(k < n ? k : 0) * ld, k < n ? n - i : 0);
        }
    };
    fetch_factor(gin(d.s), (size_t)d.lds, ra);

    d4 acc[RI][RJ];
    inner_staged<RI, RJ, WR, WC, KG, GUARD, NTHR, REG0 * 8>(d, 0, lds, acc);

#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[(row0 + 16 * bi + 4 * g + v) * R + col0 + 16 * bj + c] = acc[bi][bj][v];
#pragma unroll
    for (int p = 0; p < NST; ++p) {   // X_A(i, k) at k P1 + i
        const int idx = tid + NTHR * p;
        const int k = idx / (R / 2), i = 2 * (idx % (R / 2));
        reg1[k * P1 + i] = xst[p][0];
        reg1[k * P1 + i + 1] = xst[p][1];
    }
    fetch_factor(gin(d.e), (size_t)d.lde, rb);   // X_B, in flight during the E phase
    __syncthreads();

    // E = X_A C
    const int nbj = (rb + 15) / 16;
    const bool rows_live = 16 * rbk < ra;
    const int erow = 16 * rbk + rho(c);
    d4 e[NBJW];
#pragma unroll
    for (int J = 0; J < NBJW; ++J) e[J] = d4{0.0, 0.0, 0.0, 0.0};
    if (rows_live) {
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const double a = reg1[(Q * g + s) * P1 + erow];
            const double *crow = lds + (Q * g + s) * R + c;
#pragma unroll
            for (int J = 0; J < NBJW; ++J)
                if (jb0 + J < nbj) e[J] = mfma64(a, crow[16 * (jb0 + J)], e[J]);
        }
    }
    __syncthreads();   // C and X_A are dead

#pragma unroll
    for (int J = 0; J < NBJW; ++J)
        if (jb0 + J < nbj)
#pragma unroll
            for (int v = 0; v < 4; ++v) lds[(16 * rbk + 4 * g + v) + (16 * (jb0 + J) + c) * R] = e[J][v];
#pragma unroll
    for (int p = 0; p < NST; ++p) {   // X_B(k, col) at k P1 + col
        const int idx = tid + NTHR * p;
        const int col = idx / (R / 2), k = 2 * (idx % (R / 2));
        reg1[k * P1 + col] = xst[p][0];
        reg1[(k + 1) * P1 + col] = xst[p][1];
    }
    __syncthreads();

    // G = E X_B
    if (!rows_live) return;
    double ea[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) ea[s] = lds[erow + (Q * g + s) * R];
    const size_t ldg = (size_t)d.ldc;
    const int orow = 16 * rbk + 4 * g;
#pragma unroll
    for (int J = 0; J < NBJW; ++J) {
        const int col = 16 * (jb0 + J) + c;
        if (jb0 + J >= nbj) break;
        d4 o = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < Q; ++s) o = mfma64(ea[s], reg1[(Q * g + s) * P1 + col], o);
        if (orow < ra && col < rb) {
            double out[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = o[v];
            store_run<4, true>(gout(d.c) + orow + (size_t)col * ldg, out, ra - orow, false);
        }
    }
}

template <int KIND, int P1, int P2, int P3, int P4>
__device__ __forceinline__ void run_lrm_variant(const DevDesc &d, int p0, bool edge, double *lds)
{
    if constexpr (KIND == K_LRMB) {
        if (edge)
            lrmb_tile<P1, P2, P4, true>(d, lds);
        else
            lrmb_tile<P1, P2, P4, false>(d, lds);
    } else if constexpr (KIND == K_LRM96) {
        if (edge)
            lrm96_tile<P1, P2, P4, true>(d, lds);
        else
            lrm96_tile<P1, P2, P4, false>(d, lds);
    } else {
        constexpr int LDSD = (KIND == K_LRM ? kLdsBytes : kLdsBytes4) / 8;
        if (edge)
            lrm_tile<P1, P2, P3, P4, true, LDSD>(d, p0, lds);
        else
            lrm_tile<P1, P2, P3, P4, false, LDSD>(d, p0, lds);
    }
}

template <int FAMILY>
__device__ __forceinline__ void run_lrm_tile(const DevDesc *__restrict__ descs, const Tile &t, double *lds)
{
    if (t.variant <= 0) return;
    const DevDesc d = descs[t.desc];
    const bool edge = (t.flags & kTileEdge) != 0;
#define LRBG_LRM_CASE(id, kind, p1, p2, p3, p4) \
    case id:                                \
        run_lrm_variant<kind, p1, p2, p3, p4>(d, t.p0, edge, lds); break;
    if constexpr (FAMILY == F_LRM) {
        switch (t.variant) {
            LRBG_LRM_VARIANTS(LRBG_LRM_CASE)
        default:
            break;
        }
    } else if constexpr (FAMILY == F_LRMB) {
        switch (t.variant) {
            LRBG_LRMB_VARIANTS(LRBG_LRM_CASE)
        default:
            break;
        }
    } else if constexpr (FAMILY == F_LRM96) {
        switch (t.variant) {
            LRBG_LRM96_VARIANTS(LRBG_LRM_CASE)
        default:
            break;
        }
    } else {
        switch (t.variant) {
            LRBG_LRM4_VARIANTS(LRBG_LRM_CASE)
        default:
            break;
        }
    }
#undef LRBG_LRM_CASE
}

// The fused low-rank products, one workgroup per tile (same tile layout and
// XCD interleave as the grouped kernel): ranks up to 64 with 64 KB of LDS
// (2 workgroups per CU), and ranks up to 32 with 32 KB and at most 128
// VGPRs (4 workgroups per CU, twice the loads in flight per CU for the
// memory-bound small ranks).
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
lrbg_lrmult_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[kLdsBytes / 8];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_lrm_tile<F_LRM>(descs, tl, lds);
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
lrbg_lrmult4_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[kLdsBytes4 / 8];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_lrm_tile<F_LRM4>(descs, tl, lds);
}

// Ranks up to 128: 8 waves and 128 KB of LDS, one workgroup per CU.
__global__ void __launch_bounds__(kThreadsB) __attribute__((amdgpu_waves_per_eu(2, 2)))
lrbg_lrmultb_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[kLdsBytesB / 8];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_lrm_tile<F_LRMB>(descs, tl, lds);
}

// Ranks up to 96: 12 waves and 145 KB of LDS, one workgroup per CU.
__global__ void __launch_bounds__(kThreads96) __attribute__((amdgpu_waves_per_eu(3, 3)))
lrbg_lrmult96_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[kLdsBytes96 / 8];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_lrm_tile<F_LRM96>(descs, tl, lds);
}

int launch_lrm_family(int family, const DevDesc *descs, const Tile *tiles, int ntiles, void *stream)
{
    if (ntiles <= 0) return 0;
    const dim3 grid(ntiles), block(kThreads);
    hipStream_t s = (hipStream_t)stream;
    if (family == F_LRM)
        hipLaunchKernelGGL(lrbg_lrmult_kernel, grid, block, 0, s, descs, tiles, ntiles);
    else if (family == F_LRM4)
        hipLaunchKernelGGL(lrbg_lrmult4_kernel, grid, block, 0, s, descs, tiles, ntiles);
    else if (family == F_LRMB)
        hipLaunchKernelGGL(lrbg_lrmultb_kernel, grid, dim3(kThreadsB), 0, s, descs, tiles, ntiles);
    else if (family == F_LRM96)
        hipLaunchKernelGGL(lrbg_lrmult96_kernel, grid, dim3(kThreads96), 0, s, descs, tiles, ntiles);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

}  // namespace lrbg
