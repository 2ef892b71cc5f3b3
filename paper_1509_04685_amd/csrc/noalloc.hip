// cola_pm_force without a caller workspace, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace of cola_pm_force -- the three padded spectra, the interleaved force mesh, the
// deposit's sort buffers and the twiddle tables -- lives in a fixed device array of kNoAllocBytes per GPU, defined here.  Host
// code never passes the array's name to a kernel (on the host it is only a stand-in symbol): the
// first call on a device looks up that device's address of the array with hipGetSymbolAddress,
// with the device current, and every later call on that device passes the looked-up pointer as
// the workspace of the ordinary entry point.  Nothing here calls hipMalloc or hipFree.

#include <mutex>

#include "cola_internal.h"

namespace {

constexpr size_t kNoAllocBytes = size_t(96) << 20;  // 96 MiB per GPU, held until the process ends
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per device.
int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cola::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return COLA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return cola::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return COLA_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return COLA_OK;
}

}  // namespace

extern "C" {

int cola_pm_force_noalloc(const cola_problem* prob, const cola_particles* in, float* acc[3], void* stream) {
    const size_t need = cola_workspace_bytes(prob, 0);
    if (need == 0) return COLA_ERR_INVALID_ARG;
    if (need > kNoAllocBytes) return COLA_ERR_WORKSPACE_TOO_SMALL;  // beyond the fixed array
    void* ws = nullptr;
    const int s = scratch_ptr(&ws);
    if (s != COLA_OK) return s;
    return cola_pm_force(prob, in, acc, ws, kNoAllocBytes, stream);
}

}  // extern "C"
