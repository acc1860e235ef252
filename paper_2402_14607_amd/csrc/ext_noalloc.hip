// ext_noalloc.hip -- the static device scratch of the allocation-free entry
// point (ext_growing_extract_noalloc).
//
// The array lives in the library's code object: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  In
// host code the name `scratch` is only a host-side stand-in, so the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; host code uses
// that address, never the name, for kernel arguments and copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "ext_internal.h"

namespace {

static __device__ __align__(256) uint8_t scratch[qext::kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_looked_up[kMaxDevices] = {};
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace qext {

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_looked_up[device]) return g_ptr[device] ? hipSuccess : hipErrorInvalidSymbol;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_ptr[device] = p;
    g_looked_up[device] = true;
    return hipSuccess;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_looked_up[device] ? g_ptr[device] : nullptr;
}

}  // namespace qext
