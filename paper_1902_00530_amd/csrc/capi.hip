// C ABI of the library (include/lbm.h): validation, context management and
// the single-lattice entry points.
#include <math.h>
#include <string.h>

#include <new>
#include <string>

#include "internal.h"

namespace lbm {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

int32_t fail(int32_t code, const std::string &msg)
{
    g_error = msg;
    return code;
}

int32_t hip_fail(hipError_t e, const char *what)
{
    g_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return LBM_EHIP;
}

static bool finite_nonneg(double v) { return isfinite(v) && v >= 0.0; }

int32_t validate_params(const lbm_params *p, int64_t pitch)
{
    if (!p)
        return fail(LBM_EINVAL, "null parameters");
    if (p->lattice != LBM_D2Q7 && p->lattice != LBM_D2Q9)
        return fail(LBM_EINVAL, "unknown lattice");
    if (p->nx < 2 || p->ny < 2)
        return fail(LBM_EINVAL, "nx and ny must be >= 2");
    if (p->lattice == LBM_D2Q7 && (p->ny & 1))
        return fail(LBM_EINVAL, "ny must be even (offset-row triangular lattice)");
    if (p->ny > 65535)
        return fail(LBM_EINVAL, "ny must be <= 65535 (one grid row of blocks per lattice row)");
    if ((uint64_t)p->nx * (uint64_t)p->ny >= (1ull << 32))
        return fail(LBM_EINVAL, "nx*ny must be < 2^32 (32-bit site counter of the noise)");
    if (pitch < p->nx)
        return fail(LBM_EINVAL, "pitch must be >= nx");
    if (p->model < LBM_PASSIVE || p->model > LBM_CIL)
        return fail(LBM_EINVAL, "unknown model");
    if (p->storage < LBM_F32 || p->storage > LBM_BF16_DEV_R32)
        return fail(LBM_EINVAL, "unknown storage");
    if (p->storage == LBM_BF16_DEV_R32 && p->lattice == LBM_D2Q9)
        return fail(LBM_EUNSUPPORTED, "the float32 rest plane storage takes D2Q7 lattices");
    if (!(p->tau >= 1.0))
        return fail(LBM_EINVAL, "tau must be >= 1 (or +inf for streaming only)");
    if (!finite_nonneg(p->sigma))
        return fail(LBM_EINVAL, "sigma must be finite and >= 0");
    if (!finite_nonneg(p->A) || !finite_nonneg(p->B) || !finite_nonneg(p->C) || !finite_nonneg(p->u_max))
        return fail(LBM_EINVAL, "A, B, C and u_max must be finite and >= 0");
    if (p->model == LBM_MIPS && !(isfinite(p->rho_star) && p->rho_star > 0.0))
        return fail(LBM_EINVAL, "rho_star must be finite and > 0 for MIPS");
    if (p->storage != LBM_F32 && !finite_nonneg(p->rho_ref))
        return fail(LBM_EINVAL, "rho_ref must be finite and >= 0 for deviation storage");
    if (p->lattice == LBM_D2Q9 && (uint64_t)p->ny * (uint64_t)pitch * (p->storage == LBM_F32 ? 4u : 2u) >= (1ull << 32))
        return fail(LBM_EUNSUPPORTED, "D2Q9 population planes must be below 2^32 bytes");
    return LBM_OK;
}

// w rho_ref rounded to the storage format, so that a population of exactly 0
// (what the negative correction leaves) is stored and read back exactly:
// with an unrepresentable reference every corrected zero came back a little
// negative, a mass leak that ran away in disordered states
static float storage_reference(double v, int storage)
{
    float f = (float)v;
    if (storage == LBM_BF16_DEV) {
        uint32_t b;
        memcpy(&b, &f, 4);
        b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest even (finite values)
        b &= 0xffff0000u;
        memcpy(&f, &b, 4);
    } else if (storage == LBM_F16_DEV) {
        f = (float)(_Float16)f;
    }
    return f;
}

StepArgs make_step_args(const lbm_params &p, int64_t pitch)
{
    StepArgs a;
    a.nx = p.nx;
    a.ny = p.ny;
    a.pitch = pitch;
    a.plane = (int64_t)p.ny * pitch;
    a.omega = (float)(1.0 / p.tau);
    const bool q9 = p.lattice == LBM_D2Q9;
    a.noise_scale = (float)(q9 ? p.sigma / 73728.0 : p.sigma / 229376.0);
    a.noise_h = (float)(q9 ? p.sigma / 8192.0 : p.sigma / 32768.0);
    a.A16 = (float)p.A * 65536.0f;
    a.B16 = (float)p.B * 65536.0f;
    a.C = (float)p.C;
    a.rho_star = p.model == LBM_MIPS ? (float)p.rho_star : 1.0f;
    a.inv_rho_star = p.model == LBM_MIPS ? (float)(1.0 / p.rho_star) : 1.0f;
    a.u_max = (float)p.u_max;
    const double rr = p.storage == LBM_F32 ? 0.0 : p.rho_ref;
    // the float32 rest plane of LBM_BF16_DEV_R32 holds f_0 itself
    const int moving = p.storage == LBM_BF16_DEV_R32 ? LBM_BF16_DEV : p.storage;
    a.wr0 = p.storage == LBM_BF16_DEV_R32 ? 0.0f : storage_reference(q9 ? 4.0 * rr / 9.0 : 0.5 * rr, p.storage);
    a.wr1 = storage_reference(q9 ? rr / 9.0 : rr / 12.0, moving);
    a.wr2 = storage_reference(q9 ? rr / 36.0 : rr / 12.0, moving);
    a.key0 = (uint32_t)(p.seed & 0xffffffffu);
    a.key1 = (uint32_t)(p.seed >> 32);
    a.noisy = p.sigma != 0.0;
    return a;
}

__global__ void k_set_clock(StepClock *clk, int slot, int64_t t)
{
    if ((blockIdx.x | threadIdx.x) == 0)
        clk->t[slot] = t;
}

hipError_t launch_set_clock(StepClock *clk, int slot, int64_t t, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, s, clk, slot, t);
    return hipGetLastError();
}

// A context's workspace: the step clock, the 8 reduced doubles of a sample,
// then the reduction scratch.
constexpr size_t kWsClock = 0, kWsResult = 256, kWsScratch = 512;

static size_t ctx_workspace_bytes(const lbm_params &p)
{
    return kWsScratch + ((moments_scratch_doubles(p) * sizeof(double) + 255) & ~(size_t)255);
}

// Steps per captured graph of lbm_step (even, so a replay leaves the state in
// the buffer it started from).
constexpr int64_t kGraphSteps = 64;

static hipError_t enqueue_steps(lbm_ctx *c, int from, int64_t n, hipStream_t s)
{
    for (int64_t k = 0; k < n; ++k) {
        const int slot = (from + (int)(k & 1)) & 1;
        hipError_t e = c->p.lattice == LBM_D2Q9
                           ? launch_step_q9(c->p, c->args, c->buf[slot], c->buf[slot ^ 1], c->clk, slot, s)
                           : launch_step(c->p, c->args, c->buf[slot], c->buf[slot ^ 1], c->clk, slot, s);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// kGraphSteps steps from buffer `from`, captured on a private stream (the
// caller's may be the legacy null stream, which cannot be captured).
static hipError_t capture_steps(lbm_ctx *c, int from)
{
    hipStream_t cap;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess)
        return e;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t ce = e == hipSuccess ? enqueue_steps(c, from, kGraphSteps, cap) : e;
    hipError_t ee = e == hipSuccess ? hipStreamEndCapture(cap, &g) : e;
    (void)hipStreamDestroy(cap);
    e = ce != hipSuccess ? ce : ee;
    if (e == hipSuccess)
        e = hipGraphInstantiate(&c->graph[from], g, nullptr, nullptr, 0);
    if (g)
        (void)hipGraphDestroy(g);
    return e;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

const char *lbm_last_error(void) { return g_error.c_str(); }

int32_t lbm_deviation_reference(const lbm_params *p, float *wr)
{
    int32_t rc = validate_params(p, p ? p->nx : 0);
    if (rc)
        return rc;
    if (!wr)
        return fail(LBM_EINVAL, "null output");
    const StepArgs a = make_step_args(*p, p->nx);
    const int q = p->lattice == LBM_D2Q9 ? 9 : 7;
    for (int i = 0; i < q; ++i)
        wr[i] = i == 0 ? a.wr0 : (q == 7 || i <= 4 ? a.wr1 : a.wr2);
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params *p, int64_t pitch)
{
    if (validate_params(p, pitch) != LBM_OK)
        return 0;
    return ctx_workspace_bytes(*p);
}

int32_t lbm_create(const lbm_params *p, void *f_a, void *f_b, int64_t pitch, const lbm_init *init, void *ws,
                   size_t ws_bytes, void *stream, lbm_ctx **out)
{
    if (!out)
        return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    int32_t rc = validate_params(p, pitch);
    if (rc)
        return rc;
    if (!f_a || !f_b)
        return fail(LBM_EINVAL, "null population buffer");
    if (f_a == f_b)
        return fail(LBM_EINVAL, "f_a and f_b must be distinct buffers");
    if (!ws)
        return fail(LBM_EINVAL, "null workspace");
    if ((uintptr_t)ws % 256 != 0)
        return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < ctx_workspace_bytes(*p))
        return fail(LBM_EINVAL, "workspace smaller than lbm_workspace_bytes()");
    if (init && (init->mode < LBM_INIT_NONE || init->mode > LBM_INIT_GAUSS_DIR))
        return fail(LBM_EINVAL, "unknown init mode");
    if (init && init->mode != LBM_INIT_NONE &&
        !(isfinite(init->rho_mean) && init->rho_mean >= 0.0 && finite_nonneg(init->rho_spread) &&
          init->rho_spread <= 1.0 && isfinite(init->angle_std) && isfinite(init->u_mag) &&
          isfinite(init->pop_noise)))
        return fail(LBM_EINVAL, "invalid init parameters");
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c)
        return fail(LBM_EINVAL, "out of host memory");
    c->p = *p;
    c->pitch = pitch;
    c->args = make_step_args(*p, pitch);
    c->stream = (hipStream_t)stream;
    c->buf[0] = f_a;
    c->buf[1] = f_b;
    c->cur = 0;
    c->step = 0;
    char *w = (char *)ws;
    c->clk = (StepClock *)(w + kWsClock);
    c->d_result = (double *)(w + kWsResult);
    c->d_scratch = (double *)(w + kWsScratch);
    c->graph[0] = c->graph[1] = nullptr;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = launch_set_clock(c->clk, 0, 0, c->stream);
    if (e == hipSuccess && init && init->mode != LBM_INIT_NONE)
        e = p->lattice == LBM_D2Q9 ? launch_init_q9(*p, *init, c->args, f_a, c->stream)
                                   : launch_init(*p, *init, c->args, f_a, c->stream);
    if (e != hipSuccess) {
        rc = hip_fail(e, "lbm_create");
        delete c;
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int32_t lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    if (n < 0)
        return fail(LBM_EINVAL, "negative step count");
    // whole graphs of kGraphSteps steps, then single launches; a stream that
    // the caller is capturing gets single launches only
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusNone;
    }
    int64_t left = n;
    if (cs == hipStreamCaptureStatusNone && n >= kGraphSteps) {
        if (!c->graph[c->cur])
            LBM_HIP_TRY(capture_steps(c, c->cur));
        for (; left >= kGraphSteps; left -= kGraphSteps)
            LBM_HIP_TRY(hipGraphLaunch(c->graph[c->cur], c->stream));
    }
    LBM_HIP_TRY(enqueue_steps(c, c->cur, left, c->stream));
    c->cur ^= (int)(n & 1);
    c->step += n;
    return LBM_OK;
}

int32_t lbm_moments(lbm_ctx *c, float *rho, float *ux, float *uy, lbm_obs *obs)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    LBM_HIP_TRY(launch_moments(c->p, c->args, c->buf[c->cur], rho, ux, uy, c->d_scratch, c->d_result, c->stream));
    if (!obs)
        return LBM_OK;
    double r[8];
    LBM_HIP_TRY(hipMemcpyAsync(r, c->d_result, sizeof r, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
    finish_obs(c->p, r, c->step, obs);
    if (obs->nonfinite)
        return fail(LBM_ENONFINITE, "non-finite populations in the state");
    return LBM_OK;
}

int32_t lbm_current_buffer(const lbm_ctx *c)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    return c->cur;
}

int64_t lbm_get_step(const lbm_ctx *c)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    return c->step;
}

int32_t lbm_set_step(lbm_ctx *c, int64_t step)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    if (step < 0)
        return fail(LBM_EINVAL, "negative step index");
    LBM_HIP_TRY(launch_set_clock(c->clk, c->cur, step, c->stream));
    c->step = step;
    return LBM_OK;
}

int32_t lbm_add_density(lbm_ctx *c, double drho)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    if (!isfinite(drho))
        return fail(LBM_EINVAL, "drho must be finite");
    if (c->p.lattice == LBM_D2Q9)
        LBM_HIP_TRY(launch_add_density_q9(c->p, c->args, c->buf[c->cur], drho, c->stream));
    else
        LBM_HIP_TRY(launch_add_density(c->p, c->args, c->buf[c->cur], drho, c->stream));
    return LBM_OK;
}

int32_t lbm_destroy(lbm_ctx *c)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    hipError_t e = hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k)
        if (c->graph[k])
            (void)hipGraphExecDestroy(c->graph[k]);
    delete c;
    if (e != hipSuccess)
        return hip_fail(e, "lbm_destroy");
    return LBM_OK;
}

}  // extern "C"
