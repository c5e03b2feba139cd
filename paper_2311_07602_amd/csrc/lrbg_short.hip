// Dense products with a short contraction: C = A U with A b x k, U k x n,
// k and n at most 64 -- the new bases A_U X_k and B_V Y_k of a recompressed
// low-rank product.  The DENSE_TS register tile streams A once and keeps U
// in registers, but with KG = 8 k per lane group a contraction of 8 or 16
// leaves three or two of the four lane groups of the matrix-core operand
// idle (they load nothing, so a wave has a quarter of its loads in flight).
// These variants take 1-4 k per lane group and run in their own kernel,
// which needs no LDS, so several workgroups share a CU: the products are
// pure streams (read A, write C) and need loads in flight, not reuse.
#include "lrbg_tiles.h"

namespace lrbg {

__device__ __forceinline__ void run_short_tile(const DevDesc *__restrict__ descs, const Tile &t)
{
    if (t.variant <= 0) return;
    const DevDesc d = descs[t.desc];
    const bool edge = (t.flags & kTileEdge) != 0;
#define LRBG_SHORT_CASE(id, kind, p1, p2, p3, p4)      \
    case id:                                           \
        if (edge)                                      \
            dts64_tile<p1, p2, p3, true>(d, t.p0);     \
        else                                           \
            dts64_tile<p1, p2, p3, false>(d, t.p0);    \
        break;
    switch (t.variant) {
        LRBG_SHORT_VARIANTS(LRBG_SHORT_CASE)
    default:
        break;
    }
#undef LRBG_SHORT_CASE
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
lrbg_short_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
{
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    run_short_tile(descs, tl);
}

int launch_short_family(const DevDesc *descs, const Tile *tiles, int ntiles, void *stream)
{
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL(lrbg_short_kernel, dim3(ntiles), dim3(kThreads), 0, (hipStream_t)stream, descs, tiles,
                       ntiles);
    return (int)hipGetLastError();
}

}  // namespace lrbg
