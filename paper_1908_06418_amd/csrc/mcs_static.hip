// The library's static device scratch: the workspace of
// mcs_solve_batch_static, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array.  In host code its name stands for
// a host-side shadow, not a device address, so the device address is looked
// up here once per device (with that device current) and only that address
// is handed to the plan, the kernels and the copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mcs.h"

namespace {

constexpr size_t kScratchBytes = (size_t)MCS_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];  // device address of scratch per device (null: not looked up)

}  // namespace

// The device address of the current device's scratch and its size, or null
// (with *err naming the HIP error) if the device or the lookup fails.
extern "C" void *mcs_internal_static_scratch(size_t *bytes, int *err) {
    *bytes = kScratchBytes;
    *err = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? (int)e : -1;
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            *err = e != hipSuccess ? (int)e : -1;
            (void)hipGetLastError();
            return nullptr;
        }
        g_addr[dev] = p;
    }
    return g_addr[dev];
}
