// pa_apply_unfused_noalloc: the unfused apply with its quadrature-point tensor staged in a
// fixed device array instead of handle memory that the library allocates on first use.
//
// `scratch` below is a file-scope device array: one copy per GPU, resident from module
// load to process end.  Host code never passes its name to a kernel (on the host the name
// is only a stand-in symbol, not a device address): the device address of each GPU's copy
// is fetched once per device with hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "capi_util.h"
#include "internal.h"

namespace hexpa {

namespace {

constexpr size_t kScratchDoubles = size_t(16) << 20;  // 128 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {nullptr};

// device address of this device's copy of `scratch` (looked up once per device)
int scratch_ptr(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return arg_error("pa_apply_unfused_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("pa_apply_unfused_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                      hipGetErrorString(e));
            return PA_ERR_HIP;
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PA_OK;
}

}  // namespace

}  // namespace hexpa

using namespace hexpa;

extern "C" int pa_apply_unfused_noalloc(pa_op *op, int variant, const double *x, double *y, void *stream)
{
    PA_TRY
    if (!op || !x || !y) return arg_error("pa_apply_unfused_noalloc: NULL argument");
    if (x == y) return arg_error("pa_apply_unfused_noalloc: x and y must not alias");
    if (variant != PA_VARIANT_MFMA_UNFUSED && variant != PA_VARIANT_VALU_UNFUSED)
        return arg_error("pa_apply_unfused_noalloc: variant must be PA_VARIANT_MFMA_UNFUSED or PA_VARIANT_VALU_UNFUSED");
    const size_t channels = (op->ops & PA_DIFFUSION) ? ((op->ops & PA_MASS) ? 4 : 3) : 1;
    const size_t need = (size_t)op->nelem * channels * op->q * op->q * op->q;
    if (need > kScratchDoubles)
        return arg_error("pa_apply_unfused_noalloc: the quadrature-point tensor (nelem x channels x q1d^3 doubles) "
                         "exceeds the 16 Mi doubles of the fixed scratch array");
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != op->device) return arg_error("pa_apply_unfused_noalloc: the operator's device must be current");
    double *buf = nullptr;
    int rc = scratch_ptr(dev, &buf);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    HIP_OK(vec_fill(y, 0.0, op->ndof, s));
    bool ok = true;
    HIP_OK(launch_apply(op, variant, x, y, nullptr, op->nelem, s, &ok, buf));
    if (!ok) {
        set_error("pa_apply_unfused_noalloc: apply kernel not instantiated for this (p, q1d, ops)");
        return PA_ERR_UNSUPPORTED;
    }
    return PA_OK;
    PA_CATCH
}
