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

// Role-steered dispatch: one workgroup per tile, as in the grouped kernel,
// but a workgroup picks its tile when it starts instead of by its index.
// The tiles are in 16 queues, q = role * 8 + xcd (role 0: matrix-core-bound
// products, role 1: memory-bound ones).  A starting workgroup identifies its
// CU from the hardware id registers and claims that CU's flag in `cu_busy`:
// if no matrix-core-bound tile runs there it takes one (role 0), otherwise a
// memory-bound one, so the two kinds of work share every CU instead of
// pairing up by chance.  It tries its own XCD's queue of that role first,
// then the other XCDs, then the other role.  The grid has exactly as many
// workgroups as tiles, so every workgroup finds one: each failed claim is on
// a queue that is already exhausted.  The flag is released when the tile is
// done (or at once if the workgroup ended up with a memory-bound tile).
constexpr int kCuKeys = 4096;   // (XCC id, SE/SH/CU bits of HW_ID) -> flag

__device__ __forceinline__ int cu_key()
{
    const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);    // HW_ID
    const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 20);  // XCC_ID
    return (int)(((xcc & 15u) << 8) | ((hw >> 8) & 0xffu));
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
lrbg_steered_kernel(const DevDesc *__restrict__ descs, const Tile *__restrict__ tiles,
                    const int32_t *__restrict__ qinfo, int32_t *counters, int32_t *cu_busy)
{
    __shared__ double lds[kLdsBytes / 8];
    __shared__ int32_t s_tile, s_key;
    if (threadIdx.x == 0) {
        const int key = cu_key();
        bool hold = atomicCAS(&cu_busy[key], 0, 1) == 0;
        const int role = hold ? 0 : 1;
        const int home = blockIdx.x % kXcds;
        int tile = -1, got = -1;
        for (int pass = 0; pass < 2 && tile < 0; ++pass) {
            const int r = pass == 0 ? role : 1 - role;
            for (int qi = 0; qi < kXcds && tile < 0; ++qi) {
                const int q = r * kXcds + (home + qi) % kXcds;
                const int32_t qlen = qinfo[q + 1] - qinfo[q];
                if (qlen <= 0) continue;
                const int32_t idx = atomicAdd(&counters[q], 1);
                if (idx < qlen) {
                    tile = qinfo[q] + idx;
                    got = r;
                }
            }
        }
        if (hold && got != 0) {
            atomicExch(&cu_busy[key], 0);
            hold = false;
        }
        s_tile = tile;
        s_key = hold ? key : -1;
    }
    __syncthreads();
    const int tile = s_tile, key = s_key;
    if (tile >= 0) {
        const Tile tl = tiles[tile];
        run_tile(descs, tl, lds);
    }
    if (key >= 0) {
        __syncthreads();
        if (threadIdx.x == 0) atomicExch(&cu_busy[key], 0);
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
    if (family == F_SHORT) return launch_short_family(descs, tiles, ntiles, stream);
    if (family != F_GROUPED) return launch_lrm_family(family, descs, tiles, ntiles, stream);
    hipLaunchKernelGGL(lrbg_grouped_kernel, grid, block, 0, s, descs, tiles, ntiles);
    return (int)hipGetLastError();
}

int launch_steered(const DevDesc *descs, const Tile *tiles, const int32_t *qinfo, int32_t *counters,
                   int32_t *cu_busy, int ntiles, void *stream)
{
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL(lrbg_steered_kernel, dim3(ntiles), dim3(kThreads), 0, (hipStream_t)stream, descs, tiles,
                       qinfo, counters, cu_busy);
    return (int)hipGetLastError();
}

int cu_key_count() { return kCuKeys; }

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
