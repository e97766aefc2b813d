// pit_coarse_sweep_noalloc: the coarse preconditioner solve with its staging
// in a fixed device array of the library, for callers that may not allocate
// (code under stream capture, serving loops that forbid allocation).
//
// `scratch` is one array per GPU, created when the code object loads and held
// until the process ends.  Its name in host code is not a device address: the
// address comes from hipGetSymbolAddress, taken once per device with that
// device current and kept in g_scratch[device].  Every call on a device shares
// that device's array, so calls that overlap on one GPU race.
#include "ctx.hpp"

#include <mutex>

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[PIT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch`.
int scratch_of_current_device(double **out)
{
    int dev = -1;
    PIT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return PIT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        PIT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return PIT_EHIP;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return PIT_OK;
}

}  // namespace

extern "C" int pit_coarse_sweep_noalloc(pit_ctx *ctx, const double *v, double *z, void *stream)
{
    if (!ctx || !ctx->ws || !v || !z) return PIT_EINVAL;
    if (sweep_staging_bytes(ctx) > PIT_NOALLOC_SCRATCH_BYTES) return PIT_ENOMEM;
    double *stage = nullptr;
    if (int rc = scratch_of_current_device(&stage)) return rc;
    PIT_HIP(sweep_staged(ctx, v, z, stage, static_cast<hipStream_t>(stream)));
    return PIT_OK;
}
