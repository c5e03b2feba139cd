// HIP kernels for batched low-rank products on gfx950 (MI355X).
//
// Every product is cut into workgroup tiles (4 wavefronts); one grouped
// kernel runs a heterogeneous list of tiles, dispatching on the tile's
// variant.  All contractions run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): per instruction a wavefront multiplies a 16x4 by
// a 4x16 block; lane l = c + 16 g supplies A(row c, k g) and B(k g, col c),
// and receives D(i, c) for the four rows i with i % 4 == g (item i / 4).
//
// Two index remappings keep HBM traffic coalesced without any LDS
// transposition:
//  * k permutation: the contraction order inside a chunk is free, so lane
//    group g consumes KG consecutive k (k0 + KG g + s at step s).  A lane then
//    reads KG contiguous doubles of a column of a k-contiguous operand (U, V1,
//    U2), i.e. whole 16-byte vectors.
//  * row permutation: MFMA row c of row-block mm reads actual row
//    RM * rho(c) + mm with rho(c) = 4 (c % 4) + c / 4.  A lane then loads RM
//    contiguous rows of a row-contiguous operand (A, U1) per column, and its
//    outputs are the 4 RM contiguous rows RM*4g .. RM*4g + 4RM - 1.
//
// The products (column-major, see include/lrbg.h):
//   DENSE_TS C = A U          (dense block x skinny basis)
//   INNER    T = V1^T U2      (Alg. 1 step 1 / Alg. 2 loop 4 of the paper)
//   RECOMP   W = U1 (S V2^T)  (S V2^T formed in LDS, then streamed against U1)
#include <hip/hip_runtime.h>
#include "lrbg_internal.h"

namespace lrbg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int rho(int c) { return 4 * (c & 3) + (c >> 2); }

// n contiguous doubles from p into dst; elements at or beyond `valid` read 0.
template <int NV>
__device__ __forceinline__ void load_run(double (&dst)[NV], const double *p, int valid)
{
    if (valid >= NV) {
        if constexpr (NV % 2 == 0) {
#pragma unroll
            for (int t = 0; t < NV; t += 2) {
                d2u v = *reinterpret_cast<const d2u *>(p + t);
                dst[t] = v.x;
                dst[t + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int t = 0; t < NV; ++t) dst[t] = p[t];
        }
    } else {
#pragma unroll
        for (int t = 0; t < NV; ++t) dst[t] = (t < valid) ? p[t] : 0.0;
    }
}

template <int NV>
__device__ __forceinline__ void store_run(double *p, const double (&src)[NV], int valid, bool nt)
{
    if (valid >= NV) {
        if constexpr (NV % 2 == 0) {
#pragma unroll
            for (int t = 0; t < NV; t += 2) {
                d2u v;
                v.x = src[t];
                v.y = src[t + 1];
                if (nt)
                    __builtin_nontemporal_store(v, reinterpret_cast<d2u *>(p + t));
                else
                    *reinterpret_cast<d2u *>(p + t) = v;
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

// ---------------------------------------------------------------------------
// DENSE_TS, FP64.  Workgroup tile: rows [i0, i0 + 64 RM) x all n (<= 16 RN)
// columns, full contraction.  Wave w owns rows i0 + 16 RM w + [0, 16 RM).
// A streams from HBM exactly once (each element feeds RN MFMAs in registers);
// U chunks are re-read from L2 by every wave.
template <int RM, int RN, int KG>
__device__ __forceinline__ void dts64_tile(const DevDesc &d, int i0)
{
    constexpr int KSTEP = 4 * KG;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t lda = (size_t)d.lda, ldu = (size_t)d.ldb, ldc = (size_t)d.ldc;
    const double *__restrict__ A = static_cast<const double *>(d.a);
    const double *__restrict__ U = static_cast<const double *>(d.b);
    double *__restrict__ C = static_cast<double *>(d.c);

    const int wrow = i0 + 16 * RM * w;
    if (wrow >= M) return;                       // no barriers in this tile
    const int lrow = wrow + RM * rho(c);         // first of the lane's RM load rows
    const int rvalid = M - lrow;                 // rows left from lrow (may be <= 0)

    const double *Ap = A + lrow;                 // + col * lda
    const double *Up[RN];
    bool colok[RN];
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        const int col = jb * 16 + c;
        colok[jb] = col < N;
        Up[jb] = U + (size_t)(colok[jb] ? col : 0) * ldu;
    }

    d4 acc[RM][RN];
#pragma unroll
    for (int mm = 0; mm < RM; ++mm)
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) acc[mm][jb] = d4{0.0, 0.0, 0.0, 0.0};

    double a[KG][RM], u[RN][KG];

    auto load = [&](int k0, double (&aa)[KG][RM], double (&uu)[RN][KG]) {
        const int kb = k0 + KG * g;              // this lane group's first k
        const int kvalid = K - kb;
#pragma unroll
        for (int s = 0; s < KG; ++s) {
            if (s < kvalid)
                load_run<RM>(aa[s], Ap + (size_t)(kb + s) * lda, rvalid);
            else
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) aa[s][mm] = 0.0;
        }
#pragma unroll
        for (int jb = 0; jb < RN; ++jb) {
            if (colok[jb])
                load_run<KG>(uu[jb], Up[jb] + kb, kvalid);
            else
#pragma unroll
                for (int s = 0; s < KG; ++s) uu[jb][s] = 0.0;
        }
    };

    load(0, a, u);
    for (int k0 = 0; k0 < K; k0 += KSTEP) {
        double an[KG][RM], un[RN][KG];
        const bool more = k0 + KSTEP < K;
        if (more) load(k0 + KSTEP, an, un);
#pragma unroll
        for (int s = 0; s < KG; ++s)
#pragma unroll
            for (int jb = 0; jb < RN; ++jb)
#pragma unroll
                for (int mm = 0; mm < RM; ++mm)
                    acc[mm][jb] = mfma64(a[s][mm], u[jb][s], acc[mm][jb]);
        if (more) {
#pragma unroll
            for (int s = 0; s < KG; ++s)
#pragma unroll
                for (int mm = 0; mm < RM; ++mm) a[s][mm] = an[s][mm];
#pragma unroll
            for (int jb = 0; jb < RN; ++jb)
#pragma unroll
                for (int s = 0; s < KG; ++s) u[jb][s] = un[jb][s];
        }
    }

    // lane (c, g) holds rows wrow + 4 RM g + (RM v + mm) of column jb*16 + c
    const int orow = wrow + 4 * RM * g;
    const int ovalid = M - orow;
    if (ovalid <= 0) return;
#pragma unroll
    for (int jb = 0; jb < RN; ++jb) {
        if (!colok[jb]) continue;
        double o[4 * RM];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int mm = 0; mm < RM; ++mm) o[RM * v + mm] = acc[mm][jb][v];
        store_run<4 * RM>(C + orow + (size_t)(jb * 16 + c) * ldc, o, ovalid, false);
    }
}

// ---------------------------------------------------------------------------
// INNER, FP64.  T = V1^T U2 with a long contraction (k = b) into a small
// output (m, n = ranks).  Waves form NG = 4 / KS output groups of RI row
// blocks x RJ column blocks, and KS waves split the k chunks of one group
// (interleaved, so the group streams neighbouring rows together).  Partial
// sums meet in LDS and are added in a fixed order: deterministic, no atomics.
// Workgroup tile: T rows [i0, i0 + 16 RI NG) x all n columns.
template <int RI, int RJ, int KS, int KG>
__device__ __forceinline__ void inn64_tile(const DevDesc &d, int i0, double *lds)
{
    constexpr int NG = 4 / KS;
    constexpr int KSTEP = 4 * KG;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int og = w / KS, ks = w % KS;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldv = (size_t)d.lda, ldu = (size_t)d.ldb, ldt = (size_t)d.ldc;
    const double *__restrict__ V1 = static_cast<const double *>(d.a);
    const double *__restrict__ U2 = static_cast<const double *>(d.b);
    double *__restrict__ T = static_cast<double *>(d.c);

    const int rowbase = i0 + og * 16 * RI;
    const double *Vp[RI];
    bool rok[RI];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi) {
        const int col = rowbase + bi * 16 + rho(c);   // V1 column = T row
        rok[bi] = col < M;
        Vp[bi] = V1 + (size_t)(rok[bi] ? col : 0) * ldv;
    }
    const double *Up[RJ];
    bool cok[RJ];
#pragma unroll
    for (int bj = 0; bj < RJ; ++bj) {
        const int col = bj * 16 + c;
        cok[bj] = col < N;
        Up[bj] = U2 + (size_t)(cok[bj] ? col : 0) * ldu;
    }

    d4 acc[RI][RJ];
#pragma unroll
    for (int bi = 0; bi < RI; ++bi)
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

    double a[RI][KG], u[RJ][KG];
    auto load = [&](int k0, double (&aa)[RI][KG], double (&uu)[RJ][KG]) {
        const int kb = k0 + KG * g;
        const int kvalid = K - kb;
#pragma unroll
        for (int bi = 0; bi < RI; ++bi) {
            if (rok[bi])
                load_run<KG>(aa[bi], Vp[bi] + kb, kvalid);
            else
#pragma unroll
                for (int s = 0; s < KG; ++s) aa[bi][s] = 0.0;
        }
#pragma unroll
        for (int bj = 0; bj < RJ; ++bj) {
            if (cok[bj])
                load_run<KG>(uu[bj], Up[bj] + kb, kvalid);
            else
#pragma unroll
                for (int s = 0; s < KG; ++s) uu[bj][s] = 0.0;
        }
    };

    int k0 = ks * KSTEP;
    if (k0 < K) load(k0, a, u);
    for (; k0 < K; k0 += KS * KSTEP) {
        double an[RI][KG], un[RJ][KG];
        const bool more = k0 + KS * KSTEP < K;
        if (more) load(k0 + KS * KSTEP, an, un);
#pragma unroll
        for (int s = 0; s < KG; ++s)
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int bj = 0; bj < RJ; ++bj)
                    acc[bi][bj] = mfma64(a[bi][s], u[bj][s], acc[bi][bj]);
        if (more) {
#pragma unroll
            for (int bi = 0; bi < RI; ++bi)
#pragma unroll
                for (int s = 0; s < KG; ++s) a[bi][s] = an[bi][s];
#pragma unroll
            for (int bj = 0; bj < RJ; ++bj)
#pragma unroll
                for (int s = 0; s < KG; ++s) u[bj][s] = un[bj][s];
        }
    }

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
        __syncthreads();   // LDS is reused by the next tile of a persistent workgroup
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
            for (int v = 0; v < 4; ++v) o[v] = acc[bi][bj][v];
            store_run<4>(T + orow + (size_t)(bj * 16 + c) * ldt, o, ovalid, false);
        }
    }
}

// ---------------------------------------------------------------------------
// RECOMP, FP64.  W = U1 (S V2^T).  Workgroup tile: columns [j0, j0 + 16 BNB)
// x all rows.  First P = S V2^T restricted to the tile's columns (k x 16 BNB)
// is formed once on the matrix cores into LDS; then the waves sweep row
// groups of 16 RM rows, streaming U1 (L2-resident, shared by the product's
// column tiles) against P and writing W with non-temporal stores: the b x b
// output is the dominant HBM traffic.
template <int RM, int BNB, int KG>
__device__ __forceinline__ void rec64_tile(const DevDesc &d, int j0, double *lds)
{
    constexpr int PW = 16 * BNB;
    constexpr int KSTEP = 4 * KG;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    const int M = d.m, N = d.n, K = d.k;
    const size_t ldu = (size_t)d.lda, ldv = (size_t)d.ldb, lds_ = (size_t)d.lds, ldw = (size_t)d.ldc;
    const double *__restrict__ U1 = static_cast<const double *>(d.a);
    const double *__restrict__ V2 = static_cast<const double *>(d.b);
    const double *__restrict__ S = d.s;
    double *__restrict__ W = static_cast<double *>(d.c);
    double *P = lds;   // P[l * PW + jj], l < 16 * ceil(K / 16)

    // ---- P = S V2^T on the tile's columns
    const int KB = (K + 15) >> 4;
    for (int blk = w; blk < KB * BNB; blk += kWaves) {
        const int lb = blk / BNB, jb = blk % BNB;
        const int l = lb * 16 + c;              // A operand row (P row)
        const int jj = j0 + jb * 16 + c;        // B operand column (W column)
        const bool lok = l < K, jok = jj < N;
        d4 p = d4{0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < K; q0 += 4) {
            const int q = q0 + g;
            const double sa = (lok && q < K) ? S[l + (size_t)q * lds_] : 0.0;
            const double vb = (jok && q < K) ? V2[jj + (size_t)q * ldv] : 0.0;
            p = mfma64(sa, vb, p);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(lb * 16 + 4 * v + g) * PW + jb * 16 + c] = p[v];
    }
    __syncthreads();

    bool colok[BNB];
    size_t coff[BNB];
#pragma unroll
    for (int jb = 0; jb < BNB; ++jb) {
        const int col = j0 + jb * 16 + c;
        colok[jb] = col < N;
        coff[jb] = (size_t)col * ldw;
    }

    for (int rg = w; rg * 16 * RM < M; rg += kWaves) {
        const int wrow = rg * 16 * RM;
        const int lrow = wrow + RM * rho(c);
        const int rvalid = M - lrow;
        d4 acc[RM][BNB];
#pragma unroll
        for (int mm = 0; mm < RM; ++mm)
#pragma unroll
            for (int jb = 0; jb < BNB; ++jb) acc[mm][jb] = d4{0.0, 0.0, 0.0, 0.0};

        for (int l0 = 0; l0 < K; l0 += KSTEP) {
            const int lb0 = l0 + KG * g;
            double a[KG][RM];
#pragma unroll
            for (int s = 0; s < KG; ++s) {
                if (lb0 + s < K)
                    load_run<RM>(a[s], U1 + lrow + (size_t)(lb0 + s) * ldu, rvalid);
                else
#pragma unroll
                    for (int mm = 0; mm < RM; ++mm) a[s][mm] = 0.0;
            }
#pragma unroll
            for (int s = 0; s < KG; ++s) {
                const int l = lb0 + s;
#pragma unroll
                for (int jb = 0; jb < BNB; ++jb) {
                    const double b = (l < K) ? P[l * PW + jb * 16 + c] : 0.0;
#pragma unroll
                    for (int mm = 0; mm < RM; ++mm) acc[mm][jb] = mfma64(a[s][mm], b, acc[mm][jb]);
                }
            }
        }

        const int orow = wrow + 4 * RM * g;
        const int ovalid = M - orow;
        if (ovalid > 0) {
#pragma unroll
            for (int jb = 0; jb < BNB; ++jb) {
                if (!colok[jb]) continue;
                double o[4 * RM];
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int mm = 0; mm < RM; ++mm) o[RM * v + mm] = acc[mm][jb][v];
                store_run<4 * RM>(W + orow + coff[jb], o, ovalid, true);
            }
        }
    }
    __syncthreads();   // P is reused by the next tile of a persistent workgroup
}

// ---------------------------------------------------------------------------
// Dispatch over the compiled variants.

template <int KIND, int P1, int P2, int P3, int P4>
__device__ __forceinline__ void run_variant(const DevDesc &d, int p0, double *lds)
{
    if constexpr (KIND == K_DTS64)
        dts64_tile<P1, P2, P3>(d, p0);
    else if constexpr (KIND == K_INN64)
        inn64_tile<P1, P2, P3, P4>(d, p0, lds);
    else if constexpr (KIND == K_REC64)
        rec64_tile<P1, P2, P3>(d, p0, lds);
}

__device__ __forceinline__ void run_tile(const DevDesc *__restrict__ descs, const Tile &t, double *lds)
{
    if (t.variant <= 0) return;
    const DevDesc d = descs[t.desc];
    switch (t.variant) {
#define LRBG_CASE(id, kind, p1, p2, p3, p4) \
    case id:                                \
        run_variant<kind, p1, p2, p3, p4>(d, t.p0, lds); break;
        LRBG_VARIANTS(LRBG_CASE)
#undef LRBG_CASE
    default:
        break;
    }
}

// One workgroup per tile.  The host lays the tile list out so that tile t
// lands on XCD t % 8 under the hardware's round-robin dispatch.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) lrbg_grouped_kernel(const DevDesc *__restrict__ descs,
                                                                const Tile *__restrict__ tiles, int ntiles)
{
    __shared__ double lds[kLdsBytes / 8];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_tile(descs, tl, lds);
}

// Persistent workgroups: workgroup b serves queue b % 8 first (its XCD under
// round-robin dispatch), then steals from the other queues.  qinfo holds the
// 9 queue offsets into `tiles`.  Every workgroup leaves once all 8 counters
// have passed their queue lengths, so the grid always drains.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) lrbg_persistent_kernel(const DevDesc *__restrict__ descs,
                                                                   const Tile *__restrict__ tiles,
                                                                   const int32_t *__restrict__ qinfo,
                                                                   int32_t *counters)
{
    __shared__ double lds[kLdsBytes / 8];
    __shared__ int32_t next;
    const int home = blockIdx.x % kXcds;
    for (int qi = 0; qi < kXcds; ++qi) {
        const int q = (home + qi) % kXcds;
        const int32_t qbeg = qinfo[q], qlen = qinfo[q + 1] - qinfo[q];
        for (;;) {
            if (threadIdx.x == 0) next = atomicAdd(&counters[q], 1);
            __syncthreads();
            const int32_t idx = next;
            __syncthreads();
            if (idx >= qlen) break;
            const Tile tl = tiles[qbeg + idx];
            run_tile(descs, tl, lds);
        }
    }
}

__global__ void lrbg_reset_kernel(int32_t *counters, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0;
}

int launch_grouped(const DevDesc *descs, const Tile *tiles, int ntiles, void *stream)
{
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL(lrbg_grouped_kernel, dim3(ntiles), dim3(kThreads), 0, (hipStream_t)stream, descs, tiles,
                       ntiles);
    return (int)hipGetLastError();
}

int launch_persistent(const DevDesc *descs, const Tile *tiles, const int32_t *qinfo, int32_t *counters, int grid,
                      void *stream)
{
    if (grid <= 0) return 0;
    hipLaunchKernelGGL(lrbg_persistent_kernel, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, descs, tiles,
                       qinfo, counters);
    return (int)hipGetLastError();
}

int launch_reset(int32_t *counters, int n, void *stream)
{
    hipLaunchKernelGGL(lrbg_reset_kernel, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, counters, n);
    return (int)hipGetLastError();
}

int persistent_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lrbg_persistent_kernel, kThreads, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace lrbg
