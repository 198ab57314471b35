// The sweep nest as a call of its own: one 19-point weighted-Jacobi sweep
// with its FP64 residual on caller buffers, the offloaded form of the sweep
// that generated code can call directly (as a function block replaces a
// library call, Sec. 3.2).  The per-wave residual partials live in device
// memory the library allocates once per device (ofl_sweep19), or in a fixed
// device array of the library (ofl_sweep19_noalloc, for callers that cannot
// allocate).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/ofl.h"
#include "kernels.hpp"
#include "status.hpp"

using namespace ofl;

// Scratch of the no-allocation form: room for the residual partials of one
// sweep (one double per wave; 8224 on a 256-CU device), 128 KiB held on every
// device the library runs on until the process ends.  In host code the name
// stands for no device address: kernels get the address looked up per device.
static __device__ __align__(256) double scratch[16384];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_partials[kMaxDevices] = {};
int64_t g_capacity[kMaxDevices] = {};

constexpr int64_t kNoAllocPartials = sizeof(scratch) / sizeof(double);
double *g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// The device address of `scratch` on device `dev` (current), looked up once.
int scratch_address(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(OFL_E_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return OFL_OK;
}

}  // namespace

namespace ofl {

// Arguments of a sweep call: OFL_OK or the error.
int check_sweep_args(const float *p, const float *q, int64_t I, int64_t J, int64_t K, const double *res_slot) {
    if (!p || !q || !res_slot) return fail(OFL_E_ARG, "null pointer");
    if (p == q) return fail(OFL_E_ARG, "p and q must be distinct grids");
    if ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(q)) % 16)
        return fail(OFL_E_ARG, "grids must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(res_slot) % 8) return fail(OFL_E_ARG, "residual slot must be 8-byte aligned");
    if (I < 1 || J < 1 || K < 1) return fail(OFL_E_RANGE, "extents must be >= 1");
    if ((I + 6) * J * K * 4 >= (1ll << 31))
        return fail(OFL_E_RANGE, "grid too large: the grid plus six planes must hold under 2 GiB");
    return OFL_OK;
}

}  // namespace ofl

extern "C" int ofl_sweep19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                           void *stream) {
    int rc = check_sweep_args(p, q, I, J, K, res_slot);
    if (rc != OFL_OK) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(OFL_E_RANGE, "device index out of range");
    const int64_t need = k::stencil_partials(I, J, K);
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_capacity[dev] < need) {
            if (g_partials[dev]) (void)hipFree(g_partials[dev]);
            g_partials[dev] = nullptr;
            g_capacity[dev] = 0;
            e = hipMalloc(&g_partials[dev], (size_t)need * sizeof(double));
            if (e != hipSuccess)
                return e == hipErrorOutOfMemory ? fail(OFL_E_NOMEM, "sweep scratch") : hip_fail(e, "hipMalloc");
            g_capacity[dev] = need;
        }
        part = g_partials[dev];
    }
    k::ReduceScratch rs{part, need};
    e = k::stencil19(p, q, I, J, K, res_slot, rs, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? OFL_OK : hip_fail(e, "sweep launch");
}

extern "C" int ofl_sweep19_noalloc(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                                   void *stream) {
    int rc = check_sweep_args(p, q, I, J, K, res_slot);
    if (rc != OFL_OK) return rc;
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(OFL_E_RANGE, "device index out of range");
    if (k::stencil_partials(I, J, K) > kNoAllocPartials)
        return fail(OFL_E_RANGE, "the sweep needs more residual partials than the fixed scratch holds");
    double *part = nullptr;
    rc = scratch_address(dev, &part);
    if (rc != OFL_OK) return rc;
    // every wave of the sweep stores its partial before the finish reads it:
    // nothing in the scratch needs clearing
    const k::ReduceScratch rs{part, kNoAllocPartials};
    const hipError_t le = k::stencil19(p, q, I, J, K, res_slot, rs, static_cast<hipStream_t>(stream));
    return le == hipSuccess ? OFL_OK : hip_fail(le, "sweep launch");
}
