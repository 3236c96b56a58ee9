// sp2_noalloc.hip -- sp2_density_noalloc: the SP2 solve of sp2_density with its
// workspace in a fixed device array of this library instead of a caller or
// library allocation, for callers that cannot allocate device memory.
//
// `scratch` below is a file-scope __device__ array.  Its name in host code is
// a host-side stand-in, not a device address: the device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and only
// that pointer is handed to the kernels.  Each GPU holds its own copy of the
// array for the life of the process.  Every call on one GPU shares that GPU's
// copy: calls that overlap on one GPU (two host threads, or two streams) race
// and must be serialised by the caller.  Everything the solve needs zeroed
// (loop state, arrival counters) is reset by its first kernel.
#include <mutex>

#include "sp2_internal.h"

namespace sp2 {

constexpr size_t kScratchBytes = size_t(64) << 20;  // SP2_NOALLOC_MAX_BYTES in sp2.h
static_assert(kScratchBytes == SP2_NOALLOC_MAX_BYTES, "header and library agree on the cap");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 16;
void* g_scratch_ptr[kMaxDevices] = {};
int g_scratch_err[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];

// Device address of this device's `scratch` (looked up once per device).
hipError_t scratch_for_current(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[dev], [dev]() {
        void* p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = (int)r;
        g_scratch_ptr[dev] = (r == hipSuccess) ? p : nullptr;
    });
    if (g_scratch_err[dev] != (int)hipSuccess || !g_scratch_ptr[dev]) return hipErrorInvalidSymbol;
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace sp2

extern "C" {

int sp2_density_noalloc(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                        sp2_dtype dtype, sp2_compute compute, int fp64_prefix_iters,
                        void* hip_stream, sp2_info* info) {
    const size_t need = sp2_workspace_size(n, dtype, compute);
    if (need == 0)  // invalid arguments: reported by the checks, before any HIP call
        return sp2::density_impl(H, D, n, ld, n_occ, tol, max_iter, dtype, compute,
                                 fp64_prefix_iters, nullptr, 0, hip_stream, info, true);
    if (need > sp2::kScratchBytes) {
        if (info) {
            *info = sp2_info{};
            info->status = SP2_E_WORKSPACE;
        }
        return SP2_E_WORKSPACE;
    }
    void* ws = nullptr;
    if (sp2::scratch_for_current(&ws) != hipSuccess) {
        if (info) {
            *info = sp2_info{};
            info->status = SP2_E_HIP;
        }
        return SP2_E_HIP;
    }
    return sp2::density_impl(H, D, n, ld, n_occ, tol, max_iter, dtype, compute, fp64_prefix_iters,
                             ws, sp2::kScratchBytes, hip_stream, info, true);
}

}  // extern "C"
