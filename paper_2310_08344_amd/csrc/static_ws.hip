// The library's static device scratch: the workspace of lx_phi_leja_static,
// for callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation).  Every GPU the library
// runs on holds its own copy of the array until the process ends; its
// address on a device is looked up once, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lx_device.h"

namespace lx {
namespace {

__device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device] == nullptr) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<double*>(p);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace lx
