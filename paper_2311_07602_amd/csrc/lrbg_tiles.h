// Device tiles for batched low-rank products on gfx950 (MI355X), shared by
// the kernels of lrbg_kernels.hip and lrbg_lrmult.hip.
//
// Every product is cut into workgroup tiles (4 wavefronts); one grouped
// kernel runs a heterogeneous list of tiles, dispatching on the tile's
// variant.  All contractions run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): per instruction a wavefront multiplies a 16x4 by
// a 4x16 block; lane l = c + 16 g supplies A(row c, k g) and B(k g, col c),
// and receives D(i, c) for the four rows i with i % 4 == g (item i / 4).
// Accumulators stay in VGPRs: on gfx950 the FP64 MFMA reaches its full rate
// from VGPR accumulators even at one wave per SIMD, not from AGPRs.
//
// Two index remappings keep HBM traffic coalesced without any transposition:
//  * k permutation: the contraction order inside a chunk is free, so lane
//    group g consumes KG consecutive k (k0 + KG g + s at step s).  A lane then
//    reads KG contiguous doubles of a column of a k-contiguous operand (U, V1,
//    U2), i.e. whole 16-byte vectors.
//  * row permutation: with rho(c) = 4 (c % 4) + c / 4, MFMA row c of row
//    block mm reads actual row rho(c) (RM = 1) or 32 h + 2 rho(c) + e with
//    mm = 2 h + e (RM even).  A lane then loads whole 16-byte row pairs of a
//    row-contiguous operand (A, U1), one load instruction covers 256
//    contiguous bytes of a column per lane group, and a lane's outputs are
//    runs of contiguous rows: 4g .. 4g+3 (RM = 1) or 32 h + 8g .. +7.
//
// Ragged edges: a lane's A-operand value only reaches output row c and its
// B-operand value only output column c, so lanes beyond a rank-type edge
// load from a clamped, valid address and their outputs are never stored.
// Only contraction tails must read zeros; they, and block-type edges, are
// handled by a GUARD instantiation of each tile that the host selects per
// tile (Tile::flags bit 0); interior tiles run straight-line vector loads.
// Loads of chunk i+1 are issued before the matrix-core work of chunk i into
// a second register buffer (explicit ping-pong, no copies), and no loaded
// value is touched before it is consumed, so each wait covers one chunk.
//
// The products (column-major, see include/lrbg.h):
//   DENSE_TS C = A U          (dense block x skinny basis)
//   INNER    T = V1^T U2      (Alg. 1 step 1 / Alg. 2 loop 4 of the paper)
//   RECOMP   W = U1 (S V2^T)  (S V2^T formed in LDS, then streamed against U1)
//   LRMULT   G = X_A (V_A^T U_B) X_B  (Alg. 1, rank-sized intermediates in LDS)
#ifndef LRBG_TILES_H
#define LRBG_TILES_H

#include <hip/hip_runtime.h>
#include "lrbg_internal.h"

namespace lrbg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// Operand pointers come out of the descriptor table, so the compiler cannot
// infer their address space; flat accesses would also count against the LDS
// wait counter and serialise HBM prefetches with LDS traffic.  All operand
// accesses therefore go through explicit global-space pointers.
#define GLB __attribute__((address_space(1)))
typedef const GLB double *gcp;
typedef GLB double *gp;
typedef const GLB d2u *gcp2;
typedef GLB d2u *gp2;

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int rho(int c) { return 4 * (c & 3) + (c >> 2); }

__device__ __forceinline__ gcp gin(const void *p) { return (gcp)(p); }
__device__ __forceinline__ gp gout(void *p) { return (gp)(p); }

// NV contiguous doubles from p.  With GUARD, elements at or beyond `valid`
// read 0 (ragged edges); otherwise all NV are in range and the load is
// straight-line 16-byte vector loads.  NT: non-temporal loads, for an
// operand that no other tile reads (it then does not push the shared
// operands of the tiles around it out of L2).
template <int NV, bool GUARD, bool NT = false>
__device__ __forceinline__ void load_run(double (&dst)[NV], gcp p, int valid)
{
    if (!GUARD || valid >= NV) {
        if constexpr (NV % 2 == 0) {
#pragma unroll
            for (int t = 0; t < NV; t += 2) {
                d2u v;
                if constexpr (NT)
                    v = __builtin_nontemporal_load(reinterpret_cast<gcp2>(p + t));
                else
                    v = *reinterpret_cast<gcp2>(p + t);
                dst[t] = v.x;
                dst[t + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int t = 0; t < NV; ++t) dst[t] = NT ? __builtin_nontemporal_load(p + t) : p[t];
        }
    } else {
#pragma unroll
        for (int t = 0; t < NV; ++t) dst[t] = (t < valid) ? (NT ? __builtin_nontemporal_load(p + t) : p[t]) : 0.0;
    }
}

template <int NV, bool GUARD>
__device__ __forceinline__ void store_run(gp p, const double (&src)[NV], int valid, bool nt)
{
    if (!GUARD || valid >= NV) {
        if constexpr (NV % 2 == 0) {
#pragma unroll
            for (int t = 0; t < NV; t += 2) {
                d2u v;
                v.x = src[t];
                v.y = src[t + 1];
                if (nt)
                    __builtin_nontemporal_store(v, reinterpret_cast<gp2>(p + t));
                else
                    *reinterpret_cast<gp2>(p + t) = v;
            }
        } else {
#pragma unroll
            for (int t = 0; t < NV; ++t) p[t] = src[t];
        }
    } else {
#pragma unroll
        for (int t = 0; t < NV; ++t)
            if (t < valid) p[t] = src[t];
    }
}

// The lane's RM rows of one column (col = row 0 of the wave's span); with
// GUARD, rows at or beyond `valid` (relative to the span) read 0.
template <int RM, bool GUARD, bool NT = false>
__device__ __forceinline__ void load_rows(double (&dst)[RM], gcp col, int c, int valid)
{
    if constexpr (RM == 1) {
        double t[1];
        load_run<1, GUARD, NT>(t, col + rho(c), valid - rho(c));
        dst[0] = t[0];
    } else {
#pragma unroll
        for (int h = 0; h < RM / 2; ++h) {
            const int r0 = 32 * h + 2 * rho(c);
            double t[2];
            load_run<2, GUARD, NT>(t, col + r0, valid - r0);
            dst[2 * h] = t[0];
            dst[2 * h + 1] = t[1];
        }
    }
}

// Store the lane's outputs of one column: acc[mm] is row block mm, item v
// holding MFMA row 4v + g.  col = row 0 of the wave's span.
template <int RM, bool GUARD>
__device__ __forceinline__ void store_rows(gp col, const d4 (&acc)[RM], int g, int valid, bool nt)
{
    if constexpr (RM == 1) {
        double o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = acc[0][v];
        store_run<4, GUARD>(col + 4 * g, o, valid - 4 * g, nt);
    } else {
#pragma unroll
        for (int h = 0; h < RM / 2; ++h) {
            const int r0 = 32 * h + 8 * g;
            double o[8];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                o[2 * v] = acc[2 * h][v];
                o[2 * v + 1] = acc[2 * h + 1][v];
            }
            store_run<8, GUARD>(col + r0, o, valid - r0, nt);
        }
    }
}

// ---------------------------------------------------------------------------
// Staging of a k-contiguous operand chunk (KC rows of NCOL columns of a
// column-major matrix) into LDS as buf[kk * P + j] (the thread-count test is
// resolved at compile time when NPAIR is a multiple of NTHR: a per-thread
// branch around the store lets the compiler sink a load into it, right
// before its use, which exposes that load's whole latency): threads read 16-byte row
// pairs, consecutive threads walking down a column, and write them
// transposed so that the matrix-core operand reads (16 consecutive j per
// lane group) are conflict-free.  Columns at or beyond `nvalid` hold
// clamped (valid) data, used only for outputs that are never stored; with
// GUARD, rows at or beyond `kvalid` are stored as 0.
template <int NCOL, int KC, bool GUARD, int NTHR = kThreads>
struct StageK {
    static_assert(KC % 2 == 0, "row pairs");
    static constexpr int NPAIR = NCOL * (KC / 2);
    static constexpr int PPT = (NPAIR + NTHR - 1) / NTHR;
    double r[PPT][2];

    __device__ __forceinline__ void fetch(gcp base, size_t ld, int kvalid, int nvalid)
    {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = threadIdx.x + NTHR * p;
            const int j = idx / (KC / 2), kk = 2 * (idx % (KC / 2));
            const int jc = ((NPAIR % NTHR == 0 || idx < NPAIR) && j < nvalid) ? j : 0;
            load_run<2, GUARD>(r[p], base + kk + (size_t)jc * ld, kvalid - kk);
        }
    }
    __device__ __forceinline__ void store(double *buf, int P) const
    {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = threadIdx.x + NTHR * p;
            if (NPAIR % NTHR == 0 || idx < NPAIR) {   // decided at compile time when NPAIR divides
                const int j = idx / (KC / 2), kk = 2 * (idx % (KC / 2));
                buf[kk * P + j] = r[p][0];
                buf[(kk + 1) * P + j] = r[p][1];
            }
        }
    }
};

// ---------------------------------------------------------------------------
// DENSE_TS, FP64.  Workgroup tile: rows [i0, i0 + 64 RM) x all n (<= 16 RN)
// columns, full contraction.  Wave w owns rows i0 + 16 RM w + [0, 16 RM).
// A streams from HBM exactly once (each element feeds RN MFMAs in registers)
// through non-temporal loads; U chunks are re-read from L2 by every wave and
// by the product's other row tiles.  No barriers.  (With A loaded normally,
// a mixed batch's streaming A evicted U between the row tiles of a product:
// 8% more HBM reads than the compulsory bytes, against 0.5% when each
// bucket runs alone; with non-temporal A loads, 0.9%.)
template <int RM, int RN, int KG, bool GUARD>
__device__ __forceinline__ void dts64_tile(const DevDesc &d, int i0)
{
    constexpr int KSTEP = 4 * KG;
    static_assert(RM == 1 || RM % 2 == 0, "RM is 1 or even");
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t lda = (size_t)d.lda, ldu = (size_t)d.ldb, ldc = (size_t)d.ldc;

    const int wrow = i0 + 16 * RM * w;
    if (GUARD && wrow >= M) return;
    const int rvalid = M - wrow;
    const gcp Ap = gin(d.a) + wrow;

    gcp Up[RN];
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        const int col = jb * 16 + c;
        Up[jb] = gin(d.b) + (size_t)(col < N ? col : 0) * ldu;
    }

    d4 acc[RM][RN];
#pragma unroll
    for (int mm = 0; mm < RM; ++mm)
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) acc[mm][jb] = d4{0.0, 0.0, 0.0, 0.0};

    auto load = [&](int k0, double (&aa)[KG][RM], double (&uu)[RN][KG]) {
        const int kb = k0 + KG * g;
        const int kvalid = K - kb;
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            if (!GUARD || s < kvalid)
                load_rows<RM, GUARD, true>(aa[s], Ap + (size_t)(kb + s) * lda, c, rvalid);
            else
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) aa[s][mm] = 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) load_run<KG, GUARD>(uu[jb], Up[jb] + kb, kvalid);
    };
    auto compute = [&](const double (&aa)[KG][RM], const double (&uu)[RN][KG]) {
#pragma unroll
        for (int s = 0; s < KG; ++s)
#pragma unroll
            for (int jb = 0; jb < RN; ++jb)
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) acc[mm][jb] = mfma64(aa[s][mm], uu[jb][s], acc[mm][jb]);
    };

    // One chunk in flight while the previous one is multiplied.  Inside the
    // loop the prefetch is unconditional and handed over by copy at the end
    // of the step; the last chunk is peeled off.  A conditional prefetch, or
    // a two-buffer loop with an exit between the halves, lets the compiler
    // drain or sink the loads in front of the matrix-core work that should
    // hide them.
    double a[KG][RM], u[RN][KG];
    if (K > 0) load(0, a, u);
    for (int k0 = 0; k0 + KSTEP < K; k0 += KSTEP) {
        double an[KG][RM], un[RN][KG];
        load(k0 + KSTEP, an, un);
        compute(a, u);
        __builtin_amdgcn_sched_barrier(0);   // keep the hand-off behind the products
#pragma unroll
        for (int s = 0; s < KG; ++s) {
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) a[s][mm] = an[s][mm];
#pragma unroll
            for (int nn = 0; nn < RN; ++nn) u[nn][s] = un[nn][s];
        }
    }
    if (K > 0) compute(a, u);

#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        if (jb * 16 + c >= N) continue;
        d4 o[RM];
#pragma unroll
        for (int mm = 0; mm < RM; ++mm) o[mm] = acc[mm][jb];
        store_rows<RM, GUARD>(gout(d.c) + wrow + (size_t)(jb * 16 + c) * ldc, o, g, rvalid, false);
    }
}

// ---------------------------------------------------------------------------
// DENSE_TS, FP64, U staged in LDS (for the matrix-core-bound buckets): the 4
// waves share each U chunk from LDS instead of each re-reading it from L2;
// A streams from HBM straight into registers (non-temporal, as in dts64_tile).  Tile: rows [i0, i0 + 64 RM) x
// all n (<= 16 RN) columns.  Two LDS buffers, one barrier per chunk.
template <int RM, int RN, int KG, bool GUARD>
__device__ __forceinline__ void dtsl_tile(const DevDesc &d, int i0, double *lds)
{
    constexpr int KC = 4 * KG;
    constexpr int NC = 16 * RN;
    constexpr int P = NC + 1;
    constexpr int BUF = KC * P;
    static_assert(2 * BUF * 8 <= kLdsBytes, "DENSE_TS U staging exceeds LDS");
    static_assert(RM == 1 || RM % 2 == 0, "RM is 1 or even");
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t lda = (size_t)d.lda, ldu = (size_t)d.ldb, ldc = (size_t)d.ldc;

    const int wrow = i0 + 16 * RM * w;
    const bool active = !GUARD || wrow < M;     // inactive waves still stage and sync
    const int rvalid = M - wrow;
    const gcp Ap = gin(d.a) + (active ? wrow : 0);
    const gcp U = gin(d.b);

    d4 acc[RM][RN];
#pragma unroll
    for (int mm = 0; mm < RM; ++mm)
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) acc[mm][jb] = d4{0.0, 0.0, 0.0, 0.0};

    auto load_a = [&](int k0, double (&aa)[KG][RM]) {
        const int kb = k0 + KG * g;
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            if (!GUARD || (active && kb + s < K))
                load_rows<RM, GUARD, true>(aa[s], Ap + (size_t)(kb + s) * lda, c, rvalid);
            else
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) aa[s][mm] = 0.0;
        }
    };
    auto compute = [&](const double *cur, const double (&aa)[KG][RM]) {
        if (!active) return;
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            double b[RN];
#pragma unroll
            for (int jb = 0; jb < RN; ++jb) b[jb] = cur[(KG * g + s) * P + jb * 16 + c];
#pragma unroll
            for (int jb = 0; jb < RN; ++jb)
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) acc[mm][jb] = mfma64(aa[s][mm], b[jb], acc[mm][jb]);
        }
    };

    // Chunk i lives in LDS buffer i % 2.  The next chunk's U and A are
    // fetched before this chunk's matrix-core work and first touched after
    // it (LDS store, register copy), so their latency is covered by one chunk.
    StageK<NC, KC, GUARD> st;
    double a[KG][RM];
    if (K > 0) {
        st.fetch(U, ldu, K, N);
        load_a(0, a);
        st.store(lds, P);
    }
    __syncthreads();
    // The loop body is straight-line and the last chunk is peeled off: with
    // the loads and stores inside `if (more)` the compiler's wait placement
    // stalled each k step of a chunk on that chunk's own prefetch.
    int it = 0;
    for (int k0 = 0; k0 + KC < K; k0 += KC, ++it) {
        const int kn = k0 + KC;
        double an[KG][RM];
        st.fetch(U + kn, ldu, K - kn, N);
        load_a(kn, an);
        compute(lds + (it & 1) * BUF, a);
        st.store(lds + ((it + 1) & 1) * BUF, P);
#pragma unroll
        for (int s = 0; s < KG; ++s)
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) a[s][mm] = an[s][mm];
        __syncthreads();
    }
    if (K > 0) {
        compute(lds + (it & 1) * BUF, a);
        __syncthreads();
    }

    if (!active) return;
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        const int col = jb * 16 + c;
        if (col >= N) continue;
        d4 o[RM];
#pragma unroll
        for (int mm = 0; mm < RM; ++mm) o[mm] = acc[mm][jb];
        store_rows<RM, GUARD>(gout(d.c) + wrow + (size_t)col * ldc, o, g, rvalid, false);
    }
}

// ---------------------------------------------------------------------------
// INNER, FP64.  T = V1^T U2 with a long contraction (k = b) into a small
// output (m, n = ranks).  Waves form NG = 4 / KS output groups of RI row
// blocks x RJ column blocks, and KS waves split the k chunks of one group
// (interleaved, so the group streams neighbouring rows together).  Partial
// sums meet in LDS and are added in a fixed order: deterministic, no atomics.
// Workgroup tile: T rows [i0, i0 + 16 RI NG) x all n columns.
//
// One wave's share of an INNER contraction: T(row0 + [0, 16 RI), col0 +
// [0, 16 RJ)) summed over the k chunks kb, kb + kstride, ... (chunks of
// 4 KG), into acc (zeroed here).  Lane (c, g) ends with
// T(row0 + 16 bi + 4 g + v, col0 + 16 bj + c) in acc[bi][bj][v]; rows >= m
// and columns >= n hold finite filler (clamped operand columns), never an
// output.  `after_first` runs once the first chunk's loads are in flight.
template <int RI, int RJ, int KG, bool GUARD, typename Hook>
__device__ __forceinline__ void inner_stream(const DevDesc &d, int row0, int col0, int kb0, int kstride,
                                             d4 (&acc)[RI][RJ], Hook after_first)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldv = (size_t)d.lda, ldu = (size_t)d.ldb;

    gcp Vp[RI], Up[RJ];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int col = row0 + bi * 16 + rho(c);   // V1 column = T row
        Vp[bi] = gin(d.a) + (size_t)(col < M ? col : 0) * ldv;
    }
#pragma unroll
    for (int bj = 0; bj < RJ; ++bj) {
        const int col = col0 + bj * 16 + c;
        Up[bj] = gin(d.b) + (size_t)(col < N ? col : 0) * ldu;
    }

#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

    auto load = [&](int k0, double (&aa)[RI][KG], double (&uu)[RJ][KG]) {
        const int kb = k0 + KG * g;
        const int kvalid = K - kb;
#pragma unroll
        for (int bi = 0; bi < RI; ++bi) load_run<KG, GUARD>(aa[bi], Vp[bi] + kb, kvalid);
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) load_run<KG, GUARD>(uu[bj], Up[bj] + kb, kvalid);
    };
    auto compute = [&](const double (&aa)[RI][KG], const double (&uu)[RJ][KG]) {
#pragma unroll
        for (int s = 0; s < KG; ++s)
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj) acc[bi][bj] = mfma64(aa[bi][s], uu[bj][s], acc[bi][bj]);
    };

    // Two register buffers, chunks taken in pairs: every load in the loop is
    // unconditional and no exit sits between a load and its use, so the
    // compiler neither drains nor sinks the prefetch; the last one or two
    // chunks are peeled off.  (With split k a wave sees only a few chunks,
    // so a per-step register hand-off or a redundant last load shows.)
    double a0[RI][KG], u0[RJ][KG], a1[RI][KG], u1[RJ][KG];
    if (kb0 < K) load(kb0, a0, u0);
    after_first();
    int k0 = kb0;
    // The scheduling barriers keep each prefetch ahead of the products (and
    // of the waits for their operands) that it is meant to overlap.
    for (; k0 + 2 * kstride < K; k0 += 2 * kstride) {
        load(k0 + kstride, a1, u1);
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, u0);
        load(k0 + 2 * kstride, a0, u0);
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, u1);
    }
    if (k0 + kstride < K) {
        load(k0 + kstride, a1, u1);
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, u0);
        compute(a1, u1);
    } else if (k0 < K) {
        compute(a0, u0);
    }
}

// inn64_accumulate leaves the finished sums in the ks == 0 waves: lane
// (c, g) of output group og holds T(rowbase + 16 bi + 4 g + v, 16 bj + c) in
// acc[bi][bj][v], rowbase = i0 + 16 RI og.  Rows >= m and columns >= n hold
// finite filler, never an output.  LDS is free again when it returns.
// `after_first` runs once the first chunk's loads are in flight (before any
// LDS use of the reduction).
template <int RI, int RJ, int KS, int KG, bool GUARD, typename Hook>
__device__ __forceinline__ void inn64_accumulate(const DevDesc &d, int i0, double *lds, d4 (&acc)[RI][RJ],
                                                 Hook after_first)
{
    constexpr int NG = 4 / KS;
    constexpr int KSTEP = 4 * KG;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int og = w / KS, ks = w % KS;
    inner_stream<RI, RJ, KG, GUARD>(d, i0 + og * 16 * RI, 0, ks * KSTEP, KS * KSTEP, acc, after_first);

    if constexpr (KS > 1) {
        // slot (og, ks-1): RI*RJ*4 doubles per lane, lane-fastest
        constexpr int PER = RI * RJ * 4;
        static_assert((KS - 1) * NG * PER * 64 * 8 <= kLdsBytes, "INNER reduction exceeds LDS");
        if (ks > 0) {
            double *slot = lds + (size_t)((og * (KS - 1) + ks - 1) * PER) * 64;
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) slot[((bi * RJ + bj) * 4 + v) * 64 + lane] = acc[bi][bj][v];
        }
        __syncthreads();
        if (ks == 0) {
#pragma unroll 1
            for (int p = 1; p < KS; ++p) {
                const double *slot = lds + (size_t)((og * (KS - 1) + p - 1) * PER) * 64;
#pragma unroll
                for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[bi][bj][v] += slot[((bi * RJ + bj) * 4 + v) * 64 + lane];
            }
        }
        __syncthreads();   // LDS is reused after this
    }
}

template <int RI, int RJ, int KS, int KG, bool GUARD>
__device__ __forceinline__ void inn64_tile(const DevDesc &d, int i0, double *lds)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int og = w / KS, ks = w % KS;
    const int M = d.m, N = d.n;
    const size_t ldt = (size_t)d.ldc;
    const int rowbase = i0 + og * 16 * RI;
    d4 acc[RI][RJ];
    inn64_accumulate<RI, RJ, KS, KG, GUARD>(d, i0, lds, acc, [] {});
    if (ks != 0) return;
#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int orow = rowbase + bi * 16 + 4 * g;
        const int ovalid = M - orow;
        if (ovalid <= 0) continue;
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) {
            if (bj * 16 + c >= N) continue;
            double o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = acc[bi][bj][v];
            store_run<4, true>(gout(d.c) + orow + (size_t)(bj * 16 + c) * ldt, o, ovalid, false);
        }
    }
}

// ---------------------------------------------------------------------------
// INNER, FP64, both operands staged in LDS (ranks >= 64, matrix-core-bound):
// each k chunk of V1 (tile rows) and U2 (all columns) crosses HBM -> LDS
// once, and the waves, arranged WR x WC over the output, each own a
// 16 RI x 16 RJ block group for the whole contraction (no reduction).
// inner_staged accumulates T rows [i0, i0 + 16 RI WR) x columns
// [0, 16 RJ WC) with NTHR threads and LDSB bytes of LDS: wave (wr, wc) ends
// with T(i0 + 16 RI wr + 16 bi + 4 g + v, 16 RJ wc + 16 bj + c) in
// acc[bi][bj][v].  It ends with a barrier, so LDS is free on return.
template <int RI, int RJ, int WR, int WC, int KG, bool GUARD, int NTHR, int LDSB>
__device__ __forceinline__ void inner_staged(const DevDesc &d, int i0, double *lds, d4 (&acc)[RI][RJ])
{
    static_assert(WR * WC * 64 == NTHR, "one block group per wave");
    constexpr int KC = 4 * KG;
    constexpr int MT = 16 * RI * WR, NT = 16 * RJ * WC;
    constexpr int PV = MT + 1, PU = NT + 1;
    constexpr int BUF = KC * (PV + PU);
    static_assert(2 * BUF * 8 <= LDSB, "INNER staging exceeds LDS");
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int wr = w / WC, wc = w % WC;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldv = (size_t)d.lda, ldu = (size_t)d.ldb;
    const gcp V1t = gin(d.a) + (size_t)i0 * ldv;   // column i0 of V1 = T row i0
    const gcp U2 = gin(d.b);
    const int mvalid = M - i0;

#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

    const int arow = wr * 16 * RI, bcol = wc * 16 * RJ;
    auto compute = [&](const double *cv) {
        const double *cu = cv + KC * PV;
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            const int kk = KG * g + s;
            double a[RI], b[RJ];
#pragma unroll
            for (int bi = 0; bi < RI; ++bi) a[bi] = cv[kk * PV + arow + bi * 16 + rho(c)];
#pragma unroll
            for (int bj = 0; bj < RJ; ++bj) b[bj] = cu[kk * PU + bcol + bj * 16 + c];
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj) acc[bi][bj] = mfma64(a[bi], b[bj], acc[bi][bj]);
        }
    };
    StageK<MT, KC, GUARD, NTHR> sv;
    StageK<NT, KC, GUARD, NTHR> su;
    if (K > 0) {
        sv.fetch(V1t, ldv, K, mvalid);
        su.fetch(U2, ldu, K, N);
        sv.store(lds, PV);
        su.store(lds + KC * PV, PU);
    }
    __syncthreads();
    int it = 0;
    for (int k0 = 0; k0 + KC < K; k0 += KC, ++it) {   // loop shape as in dtsl_tile
        const int kn = k0 + KC;
        sv.fetch(V1t + kn, ldv, K - kn, mvalid);
        su.fetch(U2 + kn, ldu, K - kn, N);
        compute(lds + (it & 1) * BUF);
        double *nv = lds + ((it + 1) & 1) * BUF;
        sv.store(nv, PV);
        su.store(nv + KC * PV, PU);
        __syncthreads();
    }
    if (K > 0) {
        compute(lds + (it & 1) * BUF);
        __syncthreads();
    }
}

// Tile: T rows [i0, i0 + 16 RI WR) x columns [0, 16 RJ WC), 4 waves.
template <int RI, int RJ, int WR, int KG, bool GUARD>
__device__ __forceinline__ void innl_tile(const DevDesc &d, int i0, double *lds)
{
    constexpr int WC = 4 / WR;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int wr = w / WC, wc = w % WC;
    const int M = d.m, N = d.n;
    const size_t ldt = (size_t)d.ldc;
    const int arow = wr * 16 * RI, bcol = wc * 16 * RJ;
    d4 acc[RI][RJ];
    inner_staged<RI, RJ, WR, WC, KG, GUARD, kThreads, kLdsBytes>(d, i0, lds, acc);

#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int orow = i0 + arow + bi * 16 + 4 * g;
        const int ovalid = M - orow;
        if (ovalid <= 0) continue;
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) {
            const int col = bcol + bj * 16 + c;
            if (col >= N) continue;
            double o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = acc[bi][bj][v];
            store_run<4, true>(gout(d.c) + orow + (size_t)col * ldt, o, ovalid, false);
        }
    }
}

// ---------------------------------------------------------------------------
// RECOMP, FP64.  W = U1 (S V2^T).  Workgroup tile: columns [j0, j0 + 16 BNB)
// x all rows.  First P = S V2^T restricted to the tile's columns (k x 16 BNB)
// is formed once on the matrix cores into LDS.  The waves then sweep row
// groups of 32 RB rows computing the transposed product W^T = P^T U1^T:
// in that orientation the matrix-core output puts 16 consecutive W rows on
// 16 consecutive lanes, and with two row-interleaved blocks (rows 2c, 2c+1)
// each lane stores 16 contiguous bytes, so one store instruction writes four
// contiguous 256-byte column segments of W (non-temporal: the b x b output
// is the dominant HBM traffic).  U1 row pairs (L2-resident, shared by the
// product's column tiles) are prefetched one step ahead across row groups.
template <int RB, int BNB, int KG, bool GUARD>
__device__ __forceinline__ void rec64_tile(const DevDesc &d, int j0, double *lds)
{
    constexpr int PW = 16 * BNB;
    constexpr int KSTEP = 4 * KG;
    constexpr int RG = 32 * RB;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldu = (size_t)d.lda, ldv = (size_t)d.ldb, lds_ = (size_t)d.lds, ldw = (size_t)d.ldc;
    const gcp U1 = gin(d.a), V2 = gin(d.b), S = gin(d.s);
    const gp W = gout(d.c);
    double *P = lds;   // P[l * PW + jj], l < 16 * ceil(K / 16)

    // ---- P = S V2^T on the tile's columns (rank-sized, masked branch-free)
    const int KB = (K + 15) >> 4;
    for (int blk = w; blk < KB * BNB; blk += kWaves) {
        const int lb = blk / BNB, jb = blk % BNB;
        const int l = lb * 16 + c;              // A operand row (P row)
        const int jj = j0 + jb * 16 + c;        // B operand column (W column)
        const bool lok = l < K, jok = jj < N;
        const gcp Sp = S + (lok ? l : 0);
        const gcp Vp = V2 + (jok ? jj : 0);
        d4 p = d4{0.0, 0.0, 0.0, 0.0};
        // all loads of a batch of QB steps are issued before its MFMAs, so a
        // block waits for one memory round trip per batch, not per step
        constexpr int QB = 8;
        for (int q0 = 0; q0 < K; q0 += 4 * QB) {
            double sv[QB], vv[QB];
#pragma unroll
            for (int t = 0; t < QB; ++t) {
                const int q = q0 + 4 * t + g;
                const bool qok = q < K;
                const size_t qc = (size_t)(qok ? q : 0);
                sv[t] = Sp[qc * lds_];
                vv[t] = Vp[qc * ldv];
                sv[t] = (lok && qok) ? sv[t] : 0.0;
                vv[t] = (jok && qok) ? vv[t] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < QB; ++t) p = mfma64(sv[t], vv[t], p);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(lb * 16 + 4 * v + g) * PW + jb * 16 + c] = p[v];
    }
    __syncthreads();

    // ---- W^T = P^T U1^T, flattened over (row group, k chunk) with prefetch
    auto load_u = [&](int wrow, int l0, double (&u)[RB][KG][2]) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int row0 = wrow + 32 * rb + 2 * c;
#pragma unroll
            for (int s = 0; s < KG; ++s) {
                const int l = l0 + KG * g + s;
                if (!GUARD || l < K)
                    load_run<2, GUARD>(u[rb][s], U1 + row0 + (size_t)l * ldu, M - row0);
                else
                    u[rb][s][0] = u[rb][s][1] = 0.0;
            }
        }
    };
    d4 acc[RB][2][BNB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int bi = 0; bi < BNB; ++bi) acc[rb][e][bi] = d4{0.0, 0.0, 0.0, 0.0};

    int rg = w, l0 = 0;
    double u[RB][KG][2];
    if (rg * RG < M) load_u(rg * RG, 0, u);
    while (rg * RG < M) {
        int nl0 = l0 + KSTEP, nrg = rg;
        if (nl0 >= K) {
            nl0 = 0;
            nrg = rg + kWaves;
        }
        const bool has_next = nrg * RG < M;
        double un[RB][KG][2];
        // unconditional prefetch (the last step re-reads its own chunk)
        load_u(has_next ? nrg * RG : rg * RG, has_next ? nl0 : l0, un);
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            const int l = l0 + KG * g + s;
            double pa[BNB];
#pragma unroll
            for (int bi = 0; bi < BNB; ++bi) pa[bi] = (!GUARD || l < K) ? P[l * PW + bi * 16 + c] : 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int bi = 0; bi < BNB; ++bi) acc[rb][e][bi] = mfma64(pa[bi], u[rb][s][e], acc[rb][e][bi]);
        }
        if (nl0 == 0) {   // row group complete: store and reset
            const int wrow = rg * RG;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int row0 = wrow + 32 * rb + 2 * c;
#pragma unroll
                for (int bi = 0; bi < BNB; ++bi)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int col = j0 + bi * 16 + 4 * v + g;
                        if (GUARD && col >= N) continue;
                        const double o[2] = {acc[rb][0][bi][v], acc[rb][1][bi][v]};
                        store_run<2, GUARD>(W + row0 + (size_t)col * ldw, o, M - row0, true);
                    }
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int bi = 0; bi < BNB; ++bi) acc[rb][e][bi] = d4{0.0, 0.0, 0.0, 0.0};
            }
        }
        rg = nrg;
        l0 = nl0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int s = 0; s < KG; ++s) {
                u[rb][s][0] = un[rb][s][0];
                u[rb][s][1] = un[rb][s][1];
            }
    }
    __syncthreads();   // P is reused by the next tile of a persistent workgroup
}


// ---------------------------------------------------------------------------
// BF16x3 split precision (FP32 operands, FP64 output).  Each FP32 value x is
// split as x = x0 + x1 + x2 with x0 = RNE_bf16(x), x1 = RNE_bf16(x - x0),
// x2 = RNE_bf16(x - x0 - x1); the differences are exact in FP32, and three
// 8-bit-significand terms hold the 24-bit significand.  A product keeps the
// six term pairs of order i + j <= 2 (Henry, Tang, Heinecke, ARITH 2019),
// accumulated on v_mfma_f32_16x16x32_bf16 into three FP32 accumulators by
// order (hi: x0 y0; mid: x0 y1 + x1 y0; lo: x0 y2 + x1 y1 + x2 y0), which are
// added in FP64 smallest first.  The dropped terms are below 2^-24 relative.
// The bf16 matrix core takes 8 consecutive k per lane: lane l = c + 16 g
// holds A(row c, k 8g..8g+7) and B(k 8g..8g+7, col c) and receives D(4g + v,
// c) as item v.

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef const GLB float *gcf;
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ gcf ginf(const void *p) { return (gcf)(p); }

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

struct Split3 {
    bf8 t0, t1, t2;
};

// The three terms of 8 values, two at a time: round to nearest even to
// bfloat16 on the hardware conversion (v_cvt_pk_bf16_f32 on gfx950, one
// instruction per pair), widen back exactly (a shift of the bit pattern) and
// take the exact FP32 remainder.  Infinities and NaN keep their class (their
// remainders are NaN).  About 5 instructions per value instead of the ~25 of
// a rounding written out on the encoding, which had left the split tiles
// bound by the vector ALU rather than by HBM.
__device__ __forceinline__ Split3 split3(const float (&x)[8])
{
    Split3 s;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f2v v = f2v{x[2 * t], x[2 * t + 1]};
        const bf2 h0 = __builtin_convertvector(v, bf2);
        const f2v r1 = v - __builtin_convertvector(h0, f2v);
        const bf2 h1 = __builtin_convertvector(r1, bf2);
        const f2v r2 = r1 - __builtin_convertvector(h1, f2v);
        const bf2 h2 = __builtin_convertvector(r2, bf2);
        s.t0[2 * t] = h0.x;
        s.t0[2 * t + 1] = h0.y;
        s.t1[2 * t] = h1.x;
        s.t1[2 * t + 1] = h1.y;
        s.t2[2 * t] = h2.x;
        s.t2[2 * t + 1] = h2.y;
    }
    return s;
}

__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// acc[0] hi, acc[1] mid, acc[2] lo
__device__ __forceinline__ void mfma_x6(const Split3 &a, const Split3 &b, f4 (&acc)[3])
{
    acc[0] = mfma_bf16(a.t0, b.t0, acc[0]);
    acc[1] = mfma_bf16(a.t0, b.t1, acc[1]);
    acc[1] = mfma_bf16(a.t1, b.t0, acc[1]);
    acc[2] = mfma_bf16(a.t0, b.t2, acc[2]);
    acc[2] = mfma_bf16(a.t1, b.t1, acc[2]);
    acc[2] = mfma_bf16(a.t2, b.t0, acc[2]);
}

__device__ __forceinline__ double combine3(const f4 (&acc)[3], int v)
{
    return ((double)acc[2][v] + (double)acc[1][v]) + (double)acc[0][v];
}

// 8 contiguous floats; with GUARD, elements at or beyond `valid` read 0.
template <bool GUARD>
__device__ __forceinline__ void load8f(float (&dst)[8], gcf p, int valid)
{
    if (!GUARD || valid >= 8) {
        const f4u v0 = *reinterpret_cast<const GLB f4u *>(p);
        const f4u v1 = *reinterpret_cast<const GLB f4u *>(p + 4);
        dst[0] = v0.x; dst[1] = v0.y; dst[2] = v0.z; dst[3] = v0.w;
        dst[4] = v1.x; dst[5] = v1.y; dst[6] = v1.z; dst[7] = v1.w;
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) dst[t] = (t < valid) ? p[t] : 0.0f;
    }
}

// INNER, bf16x3.  Same work split as the FP64 INNER tile: NG = 4 / KS output
// groups of RI x RJ blocks, KS waves splitting 32-wide k chunks, FP64
// partials reduced through LDS in a fixed order.
template <int RI, int RJ, int KS, int PF, bool GUARD>
__device__ __forceinline__ void inn3_tile(const DevDesc &d, int i0, double *lds)
{
    constexpr int NG = 4 / KS;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int og = w / KS, ks = w % KS;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldv = (size_t)d.lda, ldu = (size_t)d.ldb, ldt = (size_t)d.ldc;

    const int rowbase = i0 + og * 16 * RI;
    gcf Vp[RI], Up[RJ];
    bool cok[RJ];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int col = rowbase + bi * 16 + c;
        Vp[bi] = ginf(d.a) + (size_t)(col < M ? col : 0) * ldv;
    }
#pragma unroll
    for (int bj = 0; bj < RJ; ++bj) {
        const int col = bj * 16 + c;
        cok[bj] = col < N;
        Up[bj] = ginf(d.b) + (size_t)(cok[bj] ? col : 0) * ldu;
    }
    f4 acc[RI][RJ][3];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
            for (int o = 0; o < 3; ++o) acc[bi][bj][o] = f4{0.f, 0.f, 0.f, 0.f};

    float a[RI][8], u[RJ][8];
    auto load = [&](int k0, float (&aa)[RI][8], float (&uu)[RJ][8]) {
        const int kb = k0 + 8 * g, kv = K - kb;
#pragma unroll
        for (int bi = 0; bi < RI; ++bi) load8f<GUARD>(aa[bi], Vp[bi] + kb, kv);
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) load8f<GUARD>(uu[bj], Up[bj] + kb, kv);
    };
    auto compute = [&]() {
        Split3 sa[RI];
#pragma unroll
        for (int bi = 0; bi < RI; ++bi) sa[bi] = split3(a[bi]);
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) {
            const Split3 sb = split3(u[bj]);
#pragma unroll
            for (int bi = 0; bi < RI; ++bi) mfma_x6(sa[bi], sb, acc[bi][bj]);
        }
    };
    constexpr int KSTEP = KS * 32;
    const int kb0 = ks * 32;
    if constexpr (PF) {   // loop shape as in dts64_tile: prefetch, last chunk peeled
        if (kb0 < K) load(kb0, a, u);
        for (int k0 = kb0; k0 + KSTEP < K; k0 += KSTEP) {
            float an[RI][8], un[RJ][8];
            load(k0 + KSTEP, an, un);
            compute();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
#pragma unroll
                for (int bi = 0; bi < RI; ++bi) a[bi][t] = an[bi][t];
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj) u[bj][t] = un[bj][t];
            }
        }
        if (kb0 < K) compute();
    } else {
        for (int k0 = kb0; k0 < K; k0 += KSTEP) {
            load(k0, a, u);
            compute();
        }
    }

    double res[RI][RJ][4];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) res[bi][bj][v] = combine3(acc[bi][bj], v);

    if constexpr (KS > 1) {
        constexpr int PER = RI * RJ * 4;
        static_assert((KS - 1) * NG * PER * 64 * 8 <= kLdsBytes, "INNER reduction exceeds LDS");
        if (ks > 0) {
            double *slot = lds + (size_t)((og * (KS - 1) + ks - 1) * PER) * 64;
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) slot[((bi * RJ + bj) * 4 + v) * 64 + lane] = res[bi][bj][v];
        }
        __syncthreads();
        if (ks == 0) {
#pragma unroll 1
            for (int p = 1; p < KS; ++p) {
                const double *slot = lds + (size_t)((og * (KS - 1) + p - 1) * PER) * 64;
#pragma unroll
                for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                        for (int v = 0; v < 4; ++v) res[bi][bj][v] += slot[((bi * RJ + bj) * 4 + v) * 64 + lane];
            }
        }
        __syncthreads();
    }
    if (ks != 0) return;
#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int orow = rowbase + bi * 16 + 4 * g;
        const int ovalid = M - orow;
        if (ovalid <= 0) continue;
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) {
            if (!cok[bj]) continue;
            double o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = res[bi][bj][v];
            store_run<4, true>(gout(d.c) + orow + (size_t)(bj * 16 + c) * ldt, o, ovalid, false);
        }
    }
}

// DENSE_TS, bf16x3.  Wave w owns rows i0 + 16 RM w + [0, 16 RM); lane c loads
// the RM consecutive rows RM c .. RM c + RM - 1 of each of its 8 columns, so
// row block mm uses row RM c + mm and the lane's outputs are the 4 RM
// contiguous rows 4 RM g .. 4 RM g + 4 RM - 1.  U columns are 8 contiguous
// floats per lane.  No barriers.
template <int RM, int RN, int PF, bool GUARD>
__device__ __forceinline__ void dts3_tile(const DevDesc &d, int i0)
{
    static_assert(RM == 1 || RM == 2 || RM == 4, "RM in {1,2,4}");
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t lda = (size_t)d.lda, ldu = (size_t)d.ldb, ldc = (size_t)d.ldc;
    const int wrow = i0 + 16 * RM * w;
    if (GUARD && wrow >= M) return;
    const int lrow = wrow + RM * c;
    const int rvalid = M - lrow;
    const gcf Ap = ginf(d.a) + lrow;
    gcf Up[RN];
    bool colok[RN];
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        const int col = jb * 16 + c;
        colok[jb] = col < N;
        Up[jb] = ginf(d.b) + (size_t)(colok[jb] ? col : 0) * ldu;
    }
    f4 acc[RM][RN][3];
#pragma unroll
    for (int mm = 0; mm < RM; ++mm)
#pragma unroll
        for (int jb = 0; jb < RN; ++jb)
#pragma unroll
            for (int o = 0; o < 3; ++o) acc[mm][jb][o] = f4{0.f, 0.f, 0.f, 0.f};

    float a[RM][8], u[RN][8];
    auto load = [&](int k0, float (&aa)[RM][8], float (&uu)[RN][8]) {
        const int kb = k0 + 8 * g, kv = K - kb;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            float r[RM];
            if (!GUARD || (t < kv && rvalid >= RM)) {
                const gcf p = Ap + (size_t)(kb + t) * lda;
                if constexpr (RM == 4) {
                    const f4u v = *reinterpret_cast<const GLB f4u *>(p);
                    r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
                } else if constexpr (RM == 2) {
                    const f2u v = *reinterpret_cast<const GLB f2u *>(p);
                    r[0] = v.x; r[1] = v.y;
                } else {
                    r[0] = p[0];
                }
            } else {
#pragma unroll
                for (int mm = 0; mm < RM; ++mm)
                    r[mm] = (t < kv && mm < rvalid) ? Ap[(size_t)(kb + t) * lda + mm] : 0.0f;
            }
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) aa[mm][t] = r[mm];
        }
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) load8f<GUARD>(uu[jb], Up[jb] + kb, kv);
    };
    auto compute = [&]() {
        Split3 sa[RM];
#pragma unroll
        for (int mm = 0; mm < RM; ++mm) sa[mm] = split3(a[mm]);
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) {
            const Split3 sb = split3(u[jb]);
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) mfma_x6(sa[mm], sb, acc[mm][jb]);
        }
    };
    if constexpr (PF) {   // loop shape as in dts64_tile
        if (K > 0) load(0, a, u);
        for (int k0 = 0; k0 + 32 < K; k0 += 32) {
            float an[RM][8], un[RN][8];
            load(k0 + 32, an, un);
            compute();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) a[mm][t] = an[mm][t];
#pragma unroll
                for (int jb = 0; jb < RN; ++jb) u[jb][t] = un[jb][t];
            }
        }
        if (K > 0) compute();
    } else {
        for (int k0 = 0; k0 < K; k0 += 32) {
            load(k0, a, u);
            compute();
        }
    }
    // lane (c, g): MFMA row 4g + v of block mm is row wrow + RM (4g + v) + mm
    const int orow = wrow + 4 * RM * g;
    const int ovalid = M - orow;
    if (GUARD && ovalid <= 0) return;
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        if (!colok[jb]) continue;
        double o[4 * RM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) o[RM * v + mm] = combine3(acc[mm][jb], v);
        store_run<4 * RM, GUARD>(gout(d.c) + orow + (size_t)(jb * 16 + c) * ldc, o, ovalid, false);
    }
}

// ---------------------------------------------------------------------------
// Dispatch over the compiled variants.

template <int KIND, int P1, int P2, int P3, int P4, bool GUARD>
__device__ __forceinline__ void run_variant_g(const DevDesc &d, int p0, double *lds)
{
    if constexpr (KIND == K_DTS64)
        dts64_tile<P1, P2, P3, GUARD>(d, p0);
    else if constexpr (KIND == K_INN64)
        inn64_tile<P1, P2, P3, P4, GUARD>(d, p0, lds);
    else if constexpr (KIND == K_REC64)
        rec64_tile<P1, P2, P3, GUARD>(d, p0, lds);
    else if constexpr (KIND == K_DTSL)
        dtsl_tile<P1, P2, P3, GUARD>(d, p0, lds);
    else if constexpr (KIND == K_INNL)
        innl_tile<P1, P2, P3, P4, GUARD>(d, p0, lds);
    else if constexpr (KIND == K_DTS3)
        dts3_tile<P1, P2, P3, GUARD>(d, p0);
    else if constexpr (KIND == K_INN3)
        inn3_tile<P1, P2, P3, P4, GUARD>(d, p0, lds);
}

template <int KIND, int P1, int P2, int P3, int P4>
__device__ __forceinline__ void run_variant(const DevDesc &d, int p0, bool edge, double *lds)
{
    if (edge)
        run_variant_g<KIND, P1, P2, P3, P4, true>(d, p0, lds);
    else
        run_variant_g<KIND, P1, P2, P3, P4, false>(d, p0, lds);
}

// Run tile t with the variants of one kernel (LIST: an X-macro variant list).
#define LRBG_CASE(id, kind, p1, p2, p3, p4) \
    case id:                                \
        run_variant<kind, p1, p2, p3, p4>(lrbg_d_, lrbg_t_.p0, lrbg_edge_, lrbg_lds_); break;
#define LRBG_RUN_TILE(LIST, descs, t, lds)                        \
    do {                                                          \
        const Tile &lrbg_t_ = (t);                                \
        double *lrbg_lds_ = (lds);                                \
        if (lrbg_t_.variant <= 0) break;                          \
        const DevDesc lrbg_d_ = (descs)[lrbg_t_.desc];            \
        const bool lrbg_edge_ = (lrbg_t_.flags & kTileEdge) != 0; \
        switch (lrbg_t_.variant) {                                \
            LIST(LRBG_CASE)                                       \
        default:                                                  \
            break;                                                \
        }                                                         \
    } while (0)

}  // namespace lrbg

#endif  // LRBG_TILES_H
