// Fixed device scratch of the entry points that allocate nothing.
//
// One file-scope device array per GPU the library runs on (each device
// holds its own copy, at its own address, until the process ends).  Host
// code never uses the array's name as an address: the device address of
// each GPU's copy is looked up once per device, with that device current,
// and kept here; kernels receive that address as an argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sdc_internal.h"

namespace sdc {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

int static_scratch(int device, void** ptr) {
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return (int)e;
        if (cur != device) {
            e = hipSetDevice(device);
            if (e != hipSuccess) return (int)e;
        }
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return (int)e;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return 0;
}

}  // namespace sdc
