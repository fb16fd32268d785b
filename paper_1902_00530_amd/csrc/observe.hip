// lbm_observe (include/lbm.h): fields and observables of a population buffer
// with no context and no workspace, for callers that cannot allocate device
// memory (code under graph capture, serving loops).  It runs the kernels of
// lbm_moments with their reduction partials in the library's static scratch.
#include <mutex>
#include <string>

#include "internal.h"

namespace lbm {

// The scratch array is one per device (each GPU that runs this library holds
// its copy until the process ends); host code reaches it only through the
// address hipGetSymbolAddress returns for the current device, never through
// the array's name.  Every call on a device shares that device's array; the
// kernels write every partial they later read before reading it, so nothing
// has to start at zero, and calls that overlap on one device race.
constexpr size_t kObserveScratchBytes = 12ull << 20;
constexpr size_t kObserveDoubles = kObserveScratchBytes / sizeof(double);
static __device__ __align__(256) double scratch[kObserveDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Address of this device's scratch array (looked up once per device, with
// that device current).
static hipError_t observe_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace lbm

using namespace lbm;

extern "C" int32_t lbm_observe(const lbm_params *p, const void *f, int64_t pitch, int64_t step, float *rho,
                               float *ux, float *uy, void *stream, lbm_obs *obs)
{
    int32_t rc = validate_params(p, pitch);
    if (rc)
        return rc;
    if (!f)
        return fail(LBM_EINVAL, "null population buffer");
    if (step < 0)
        return fail(LBM_EINVAL, "negative step index");
    const size_t need = moments_scratch_doubles(*p) + 8;
    if (need > kObserveDoubles)
        return fail(LBM_EINVAL, "lattice too large for lbm_observe's static scratch (" + std::to_string(need * 8) +
                                    " bytes needed, " + std::to_string(kObserveScratchBytes) +
                                    " available): use lbm_moments");
    double *sc = nullptr;
    LBM_HIP_TRY(observe_scratch(&sc));
    hipStream_t s = (hipStream_t)stream;
    const StepArgs a = make_step_args(*p, pitch);
    double *result = sc + (need - 8);
    LBM_HIP_TRY(launch_moments(*p, a, f, rho, ux, uy, sc, result, s));
    if (!obs)
        return LBM_OK;
    double r[8];
    LBM_HIP_TRY(hipMemcpyAsync(r, result, sizeof r, hipMemcpyDeviceToHost, s));
    LBM_HIP_TRY(hipStreamSynchronize(s));
    finish_obs(*p, r, step, obs);
    if (obs->nonfinite)
        return fail(LBM_ENONFINITE, "non-finite populations in the state");
    return LBM_OK;
}
