// Fixed device scratch for the entry point that allocates nothing
// (llg_step_adjoint_noalloc): a file-scope device array of
// MM_NOALLOC_SCRATCH_BYTES that the code object brings with it, so each GPU
// the library runs on holds one copy from the first use until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol): the device address comes from
// hipGetSymbolAddress, once per device with that device current, and every
// later use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mmx.h"

static __device__ __align__(256) unsigned char scratch[MM_NOALLOC_SCRATCH_BYTES];

namespace mmx {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's copy of the array, looked up on the first
// call for `device` (made current for the lookup, then restored).
hipError_t noalloc_scratch(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace mmx
