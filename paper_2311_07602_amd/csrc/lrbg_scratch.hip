// Fixed device scratch for the entry point that allocates nothing
// (lr_batched_lrmult_round_noalloc): the cores, singular vectors and
// launch tables of a recompressed product live in one file-scope device
// array instead of memory the library allocates.  Every GPU the library
// runs on holds its own copy of the array, at its own address, until the
// process ends; the host never uses the array's name as an address, only
// the device pointer looked up here once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lrbg.h"
#include "lrbg_internal.h"

namespace lrbg {

constexpr size_t kNoAllocScratchBytes = LRBG_NOALLOC_SCRATCH_BYTES;   // 128 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Device address of the current device's scratch array: looked up with
// hipGetSymbolAddress the first time a device asks, with that device current,
// and kept per device.  Returns a hipError_t (0 on success).
int noalloc_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return 0;
}

}  // namespace lrbg
