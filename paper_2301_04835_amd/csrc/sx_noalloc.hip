// Fixed device scratch for the entry point that allocates nothing
// (sx_bias_eval_noalloc): the partial sums of its kernels live in this
// file-scope array, one copy per GPU, held until the process ends.  Its
// device address is looked up once per device at set-up (sx_create, with
// that device current); host code uses only that address, never the
// array's name, which on the host is a stand-in, not device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sx_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per GPU
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // per device: the array's device address (null: not looked up)

}  // namespace

namespace sx {

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) g_ptr[device] = static_cast<double *>(p);
    return e;
}

double *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace sx
