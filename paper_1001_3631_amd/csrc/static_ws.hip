// The library's own device workspace for callers that cannot allocate
// (teuk_init_grid_static): one file-scope array per device, found through
// its symbol address once per device and used only through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace {

// Each GPU the library runs on holds its own copy until the process ends.
__device__ __align__(256) unsigned char scratch[teuk::kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace teuk {

// Device address of the current device's array (the host-side name of the
// array is not a device address and is never passed to a kernel or a copy).
hipError_t static_workspace(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace teuk
