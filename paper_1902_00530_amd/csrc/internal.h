// Host-side internals of the library: the context object and the kernel
// launchers that the C ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/lbm.h"
#include "device.h"

namespace lbm {

void set_error(const std::string &msg);
int32_t fail(int32_t code, const std::string &msg);
int32_t hip_fail(hipError_t e, const char *what);

#define LBM_HIP_TRY(expr)                                      \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return ::lbm::hip_fail(e_, #expr); \
    } while (0)

// Fill the kernel argument block from validated parameters.
StepArgs make_step_args(const lbm_params &p, int64_t pitch);
// Parameter validation shared by lbm_create and lbm_sweep_batch.
int32_t validate_params(const lbm_params *p, int64_t pitch);

// Compile-time variant of the site body for these arguments (kUnitTau, kNoisy).
int step_flags(const StepArgs &a);
// One fused step src -> dst; the step index comes from clock slot `slot`
// and the next index goes to the other slot.
hipError_t launch_step(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                       hipStream_t s);
// Initial state into dst.
hipError_t launch_init(const lbm_params &p, const lbm_init &in, const StepArgs &a, void *dst, hipStream_t s);
// f_i += drho / 7 in place.
hipError_t launch_add_density(const lbm_params &p, const StepArgs &a, void *buf, double drho, hipStream_t s);
// The same three on the square (D2Q9) lattice (f_i += drho / 9).
hipError_t launch_step_q9(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk,
                          int slot, hipStream_t s);
// Set clock slot `slot` to step index t (enqueued; a kernel, so it may be
// captured into a graph).
hipError_t launch_set_clock(StepClock *clk, int slot, int64_t t, hipStream_t s);
hipError_t launch_init_q9(const lbm_params &p, const lbm_init &in, const StepArgs &a, void *dst, hipStream_t s);
hipError_t launch_add_density_q9(const lbm_params &p, const StepArgs &a, void *buf, double drho, hipStream_t s);

// Moments and FP64 reductions.  scratch: device doubles of
// moments_scratch_doubles(p); result: 8 device doubles
// {M, Jx, Jy, sum |j|, nonfinite, mean_x rho_y, var_x rho_y, unused}.
size_t moments_scratch_doubles(const lbm_params &p);
hipError_t launch_moments(const lbm_params &p, const StepArgs &a, const void *src, float *rho, float *ux,
                          float *uy, double *scratch, double *result, hipStream_t s);
// The surrogate form of lbm_sweep_batch (opts->surrogate set; arguments
// validated as for a plain sweep).
// Adam (as lbm_cnn_adam) on up to kAdamMax tensors in one launch.
constexpr int kAdamMax = 6;
struct AdamJobs {
    float *theta[kAdamMax], *m[kAdamMax], *v[kAdamMax];
    const float *g[kAdamMax];
    int64_t count[kAdamMax];
    uint16_t *bf16[kAdamMax];  // bf16 copies of theta, or null
};
hipError_t launch_adam_many(const AdamJobs &j, int n, float lr, float beta1, float beta2, float eps, int64_t t,
                            hipStream_t s);

int32_t surrogate_sweep(const lbm_params *ps, int n, const lbm_sweep_opts *o, void *const *bufs, void *ws,
                        size_t ws_bytes, hipStream_t st, lbm_obs *out);
// Turn the 8 reduced doubles into an lbm_obs (host).
void finish_obs(const lbm_params &p, const double *r, int64_t step, lbm_obs *o);

}  // namespace lbm

struct lbm_ctx {
    lbm_params p;
    lbm::StepArgs args;
    int device;
    hipStream_t stream;
    void *buf[2];
    int cur;
    int64_t pitch;
    int64_t step;
    // in the caller's workspace
    lbm::StepClock *clk;  // device step index (two slots)
    double *d_result;     // 8 doubles
    double *d_scratch;    // reductions
    // graphs of kGraphSteps steps starting from buffer 0 and from buffer 1,
    // captured on first use
    hipGraphExec_t graph[2];
};
