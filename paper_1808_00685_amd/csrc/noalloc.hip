// noalloc.hip -- homocorrelation entry point that allocates nothing, for
// callers that cannot allocate device or pinned memory (code under graph
// capture, serving loops, harnesses that forbid hipMalloc).  It runs the same
// launch sequence as corr2d_homo with a fixed device array of this library,
// `scratch`, as the workspace.
//
// The array is a file-scope device variable: each GPU the library runs on
// holds its own copy, for as long as the process lives.  Host code never
// passes the array's name to a kernel (on the host that name is a host-side
// stand-in, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "corr2d.h"
#include "corr2d_internal.h"

namespace {

// Largest workspace the fixed scratch serves (64 MiB: the m = 256,
// n = 16384 homocorrelation in split-BF16, FP32 or BF16 needs 33 MiB).
constexpr size_t kScratchBytes = CORR2D_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace corr2d {
// api.cpp: validation of a plan for this entry point (no interpolation, a
// homocorrelation plan, its workspace within max_bytes).
corr2d_status noalloc_check(corr2d_plan_t p, size_t max_bytes);
corr2d_status noalloc_fail(corr2d_status s, const char* what);
}  // namespace corr2d

extern "C" corr2d_status corr2d_homo_noalloc(corr2d_plan_t plan, const void* y, const double* ref,
                                             void* phi, void* psi, void* stream) {
    corr2d_status st = corr2d::noalloc_check(plan, kScratchBytes);
    if (st != CORR2D_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return corr2d::noalloc_fail(CORR2D_EDEVICE, "no current device for the fixed scratch");
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_ptr[dev]) {
            // the device copy of `scratch` on the current device
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return corr2d::noalloc_fail(CORR2D_EDEVICE, "hipGetSymbolAddress of the fixed scratch failed");
            g_ptr[dev] = ptr;
        }
        ws = g_ptr[dev];
    }
    return corr2d_homo(plan, y, ref, phi, psi, ws, kScratchBytes, stream);
}
