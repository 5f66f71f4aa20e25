// psd_noalloc.hip -- psd_deposit_uniform for callers that cannot allocate.
//
// The deposit's workspace (the queue's work counter; with cost ordering the
// chunk buckets and order; with the surrogate the per-chunk mask; with
// PSD_CHECK_FINITE the count of bad coordinates) lives here in one fixed
// device array instead of a caller buffer.  Each GPU the library runs on holds
// its own copy of the array until the process ends; its device address is
// looked up once per device and every launch gets that address, never the
// array's name (in host code the name is only a host-side stand-in).
#include <stdio.h>

#include <mutex>

#include "psd.h"
#include "psd_internal.h"

namespace psd {
psd_status set_error(psd_status s, const char* detail);
}  // namespace psd

namespace {

constexpr size_t kScratchBytes = (size_t)PSD_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up with the device
// current on the first call that runs on it.
hipError_t scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

psd_status psd_deposit_uniform_noalloc(const float* pos, const psd_particles* p, const int32_t nc[3],
                                       void* out, double* mass_sum, const psd_options* opt,
                                       void* stream)
{
    size_t need = 0;
    psd_status s = psd_uniform_workspace_size(p, nc, opt, &need);
    if (s != PSD_OK) return s;
    if (need > kScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof(msg),
                 "deposit_uniform_noalloc: this problem needs %zu workspace bytes, more than the "
                 "%zu of the fixed device scratch; use psd_deposit_uniform with a workspace",
                 need, kScratchBytes);
        return psd::set_error(PSD_ERR_WORKSPACE, msg);
    }
    void* ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) {
        char msg[200];
        snprintf(msg, sizeof(msg), "deposit_uniform_noalloc: scratch address: %s",
                 hipGetErrorString(e));
        return psd::set_error(PSD_ERR_HIP, msg);
    }
    return psd_deposit_uniform(pos, p, nc, out, mass_sum, opt, ws, kScratchBytes, stream);
}

}  // extern "C"
