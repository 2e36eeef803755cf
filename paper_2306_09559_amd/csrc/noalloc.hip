// mpmc_mlmc_level_estimate_noalloc: the level entry point with its workspace
// in a static device array instead of a caller-supplied buffer, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// Each GPU the library runs on holds its own copy of `scratch` for the life
// of the process.  In host code the name `scratch` is not a device address:
// the entry point looks the array up once per device with
// hipGetSymbolAddress and passes that address to the kernels, exactly where
// the allocating entry point passes the caller's workspace.
#include <hip/hip_runtime.h>

#include <atomic>

#include "common.hpp"
#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::atomic<void *> g_scratch[kMaxDevices];

// the device address of this device's scratch array (looked up on the first call per device)
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPMC_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return MPMC_EUNSUPPORTED;
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPMC_EHIP;
        g_scratch[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return MPMC_OK;
}

}  // namespace

extern "C" {

size_t mpmc_noalloc_scratch_bytes(void) { return kScratchBytes; }

int mpmc_mlmc_level_estimate_noalloc(const mpmc_lattice *lat, const mpmc_level *level, mpmc_shape shape,
                                     const mpmc_noise *noise, double *samples, double *acc, void *stream) {
    // the same validation as the allocating entry point, with the scratch as the workspace
    const size_t need = mpmc_level_workspace_size(lat, level, shape);
    if (need == 0) return MPMC_EINVAL;
    if (need > kScratchBytes) return MPMC_EWORKSPACE;
    void *ws = nullptr;
    const int st = scratch_address(&ws);
    if (st != MPMC_OK) return st;
    return mpmc_mlmc_level_estimate(lat, level, shape, noise, samples, acc, ws, kScratchBytes, stream);
}

}  // extern "C"
