// Static device scratch area of the allocation-free autotune entry point
// (tk_autotune_static): a fixed-size array in the library's code object, so
// that a caller that cannot allocate device memory can still have the
// autotuner save and restore its state.  Each GPU the library runs on holds
// its own copy from the first use until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tk_scratch.h"

static __device__ __align__(256) unsigned char scratch[tk::kScratchBytes];

namespace tk {

namespace {

std::mutex g_lock;                       // guards g_addr and serialises users
void *g_addr[kScratchMaxDevices] = {};  // device address of `scratch` per device

}  // namespace

hipError_t scratch_area(int device, void **ptr)
{
    if (device < 0 || device >= kScratchMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_addr[device]) {
        // The array's name is a host-side stand-in; its address on this
        // device comes from the runtime, with the device current.
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    return hipSuccess;
}

std::mutex &scratch_user_lock()
{
    static std::mutex m;
    return m;
}

}  // namespace tk
