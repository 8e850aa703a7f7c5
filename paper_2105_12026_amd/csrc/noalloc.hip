// Multi-set evaluation for callers that cannot allocate device memory.
//
// ebc_eval_sets needs a few per-set tables (unit prefix sums, validation
// flags, per-(set, ground-set split) float64 partial sums). Here they live in
// one file-scope device array, so the call needs no workspace argument and no
// allocation. Each device that the library runs on holds its own copy of the
// array at its own address; host code never uses the array's name as a device
// pointer (on the host it is only a stand-in) but the address returned by
// hipGetSymbolAddress, looked up once per device with that device current.
#include <mutex>

#include "ebc_internal.h"

namespace ebc {
namespace {

constexpr size_t kFixedScratchBytes = EBC_FIXED_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`; nullptr if the device id is out
// of range or the lookup fails.
void* device_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return nullptr;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace ebc

using namespace ebc;

extern "C" {

ebc_status ebc_eval_sets_noalloc(ebc_dataset* ds, const int64_t* offsets, const int32_t* idx, int64_t l,
                                 double* f_out, int32_t in_dtype, void* stream) {
    if (!ds || l < 0 || l > (int64_t(1) << 31) - 1) return EBC_E_INVALID_ARG;
    if (l == 0) return EBC_OK;
    if (!offsets || !idx || !f_out) return EBC_E_INVALID_ARG;
    if (in_dtype != 0 && in_dtype != 1) return EBC_E_INVALID_ARG;
    if (eval_sets_scratch_bytes(ds->n, l) > kFixedScratchBytes) return EBC_E_NOMEM;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return EBC_E_DEVICE;
    void* p = device_scratch(dev);
    if (!p) return EBC_E_DEVICE;
    const hipError_t e =
        launch_eval_sets(ds, offsets, idx, l, f_out, in_dtype != 0, p, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? EBC_OK : EBC_E_DEVICE;
}

}  // extern "C"
