// Device scratch of the allocation-free entry point (mgwr_toeplitz_apply_static).
//
// One file-scope array in device memory: every GPU the library runs on holds
// its own copy, at its own address, from module load until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory, so
// its device address is looked up with hipGetSymbolAddress once per device
// (with that device current) and only that address is ever handed to
// kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mgwr.h"
#include "mgwr_internal.h"

namespace mgwr {

static __device__ __align__(256) unsigned char scratch[MGWR_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return set_error(MGWR_EDEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device)
            return set_error(MGWR_EDEVICE, "static scratch looked up with another device current");
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return set_error(MGWR_EDEVICE, "hipGetSymbolAddress of the static scratch failed");
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return MGWR_OK;
}

}  // namespace mgwr
