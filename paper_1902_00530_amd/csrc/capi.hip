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
    if (p->storage < LBM_F32 || p->storage > LBM_F16_DEV)
        return fail(LBM_EINVAL, "unknown storage");
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
    a.A16 = (float)p.A * 65536.0f;
    a.B16 = (float)p.B * 65536.0f;
    a.C = (float)p.C;
    a.rho_star = p.model == LBM_MIPS ? (float)p.rho_star : 1.0f;
    a.inv_rho_star = p.model == LBM_MIPS ? (float)(1.0 / p.rho_star) : 1.0f;
    a.u_max = (float)p.u_max;
    const double rr = p.storage == LBM_F32 ? 0.0 : p.rho_ref;
    a.wr0 = (float)(q9 ? 4.0 * rr / 9.0 : 0.5 * rr);
    a.wr1 = (float)(q9 ? rr / 9.0 : rr / 12.0);
    a.wr2 = (float)(q9 ? rr / 36.0 : rr / 12.0);
    a.key0 = (uint32_t)(p.seed & 0xffffffffu);
    a.key1 = (uint32_t)(p.seed >> 32);
    a.noisy = p.sigma != 0.0;
    return a;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

const char *lbm_last_error(void) { return g_error.c_str(); }

int32_t lbm_create(const lbm_params *p, void *f_a, void *f_b, int64_t pitch, const lbm_init *init, void *stream,
                   lbm_ctx **out)
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
    hipError_t e = hipGetDevice(&c->device);
    const size_t nd = moments_scratch_doubles(*p);
    if (e == hipSuccess)
        e = hipMalloc((void **)&c->d_scratch, nd * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&c->d_result, 8 * sizeof(double));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->h_result, 8 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess && init && init->mode != LBM_INIT_NONE)
        e = p->lattice == LBM_D2Q9 ? launch_init_q9(*p, *init, c->args, f_a, c->stream)
                                   : launch_init(*p, *init, c->args, f_a, c->stream);
    if (e != hipSuccess) {
        rc = hip_fail(e, "lbm_create");
        if (c->d_scratch) hipFree(c->d_scratch);
        if (c->d_result) hipFree(c->d_result);
        if (c->h_result) hipHostFree(c->h_result);
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
    for (int64_t k = 0; k < n; ++k) {
        hipError_t e = c->p.lattice == LBM_D2Q9
                           ? launch_step_q9(c->p, c->args, c->buf[c->cur], c->buf[c->cur ^ 1], c->step, c->stream)
                           : launch_step(c->p, c->args, c->buf[c->cur], c->buf[c->cur ^ 1], c->step, c->stream);
        if (e != hipSuccess)
            return hip_fail(e, "lbm_step");
        c->cur ^= 1;
        c->step += 1;
    }
    return LBM_OK;
}

int32_t lbm_moments(lbm_ctx *c, float *rho, float *ux, float *uy, lbm_obs *obs)
{
    if (!c)
        return fail(LBM_ESTATE, "null context");
    LBM_HIP_TRY(launch_moments(c->p, c->args, c->buf[c->cur], rho, ux, uy, c->d_scratch, c->d_result, c->stream));
    if (!obs)
        return LBM_OK;
    LBM_HIP_TRY(hipMemcpyAsync(c->h_result, c->d_result, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LBM_HIP_TRY(hipStreamSynchronize(c->stream));
    finish_obs(c->p, c->h_result, c->step, obs);
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
    hipFree(c->d_scratch);
    hipFree(c->d_result);
    hipHostFree(c->h_result);
    delete c;
    if (e != hipSuccess)
        return hip_fail(e, "lbm_destroy");
    return LBM_OK;
}

}  // extern "C"
