// The grouped kernel (one workgroup per tile over a heterogeneous tile list)
// and its persistent form, for the DENSE_TS, INNER and RECOMP tiles of
// lrbg_tiles.h (FP64 and BF16x3); the fused low-rank product kernels live
// in lrbg_lrmult.hip.
#include "lrbg_tiles.h"

namespace lrbg {

__device__ __forceinline__ void run_tile(const DevDesc *__restrict__ descs, const Tile &t, double *lds)
{
    LRBG_RUN_TILE(LRBG_VARIANTS, descs, t, lds);
}

// Out-of-line tile call for the persistent kernel: keeps each variant's
// register state out of the persistent loop.
__device__ __noinline__ void run_tile_call(const DevDesc *__restrict__ descs, const Tile *tp, double *lds)
{
    const Tile t = *tp;
    run_tile(descs, t, lds);
}

// One workgroup per tile.  The host lays the tile list out so that tile t
// lands on XCD t % 8 under the hardware's round-robin dispatch.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
lrbg_grouped_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles, int ntiles)
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
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
lrbg_persistent_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles,
                       const int32_t *__restrict__ qinfo, int32_t *counters)
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
            run_tile_call(descs, tiles + qbeg + idx, lds);
        }
    }
}

__global__ void lrbg_reset_kernel(int32_t *counters, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0;
}

int launch_persistent(const DevDesc *descs, const Tile *tiles, const int32_t *qinfo, int32_t *counters, int grid,
                      void *stream)
{
    if (grid <= 0) return 0;
    hipLaunchKernelGGL(lrbg_persistent_kernel, dim3(grid), dim3(kThreads), 0, (hipStream_t)stream, descs, tiles,
                       qinfo, counters);
    return (int)hipGetLastError();
}

int launch_family(int family, const DevDesc *descs, const Tile *tiles, int ntiles, void *stream)
{
    if (ntiles <= 0) return 0;
    const dim3 grid(ntiles), block(kThreads);
    hipStream_t s = (hipStream_t)stream;
    if (family != F_GROUPED) return launch_lrm_family(family, descs, tiles, ntiles, stream);
    hipLaunchKernelGGL(lrbg_grouped_kernel, grid, block, 0, s, descs, tiles, ntiles);
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
