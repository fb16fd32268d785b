// The learned surrogate as a library object (include/lbm_cnn.h): a handle
// that owns nothing on the device, whose weights, Adam moments and field
// normalisation live in one caller-owned parameter block, and whose
// activations live in a caller-owned workspace; training and prediction
// calls; and the surrogate form of a batched sweep, in which the network
// advances the coarse fields of every lattice by k steps per evaluation,
// the lattice Boltzmann method judges them every check_every evaluations and
// a lattice whose error exceeds the bound continues with the method.  The
// surrogate is not part of the paper's method; the method is its data source
// and its judge.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/lbm_cnn.h"
#include "internal.h"

namespace lbm {

constexpr int kHidden = 32, kOut = 3;

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Parameter block: six float32 tensors (w1, b1, w2, b2, w3, b3), their Adam
// moments m and v, the bfloat16 copies of w1..w3, and the normalisation
// (scale, shift of the inputs; inv_scale, inv_shift of the outputs: cin
// floats each).
struct ParamLayout {
    int64_t count[6];
    size_t theta[6], m[6], v[6], wb[3], norm, total;
};

static ParamLayout param_layout(int cin)
{
    ParamLayout P{};
    const int64_t c[6] = {(int64_t)kHidden * cin * 9, kHidden, (int64_t)kHidden * kHidden * 9, kHidden,
                          (int64_t)kOut * kHidden * 9, kOut};
    size_t off = 0;
    for (int k = 0; k < 6; ++k) {
        P.count[k] = c[k];
        P.theta[k] = off;
        off = al256(off + c[k] * sizeof(float));
    }
    for (int k = 0; k < 6; ++k) {
        P.m[k] = off;
        off = al256(off + c[k] * sizeof(float));
    }
    for (int k = 0; k < 6; ++k) {
        P.v[k] = off;
        off = al256(off + c[k] * sizeof(float));
    }
    for (int k = 0; k < 3; ++k) {
        P.wb[k] = off;
        off = al256(off + c[2 * k] * sizeof(uint16_t));
    }
    P.norm = off;
    off = al256(off + 4 * (size_t)cin * sizeof(float));
    P.total = off;
    return P;
}

// Workspace: normalised inputs and targets, activations, the network's own
// workspace, gradients, statistics, and the sweep's coarse fields.
struct WorkLayout {
    size_t xn, tn, a1, a2, y, cnn, grad[6], mean, stdev, stats, loss, X, Y, F, err, mask, ptrs, act, total;
    size_t cnn_bytes;
};

static WorkLayout work_layout(const lbm_surrogate_desc &d)
{
    WorkLayout W{};
    const int64_t hw = (int64_t)d.h * d.w, mb = d.max_batch;
    lbm_cnn_shape sh{(int32_t)mb, d.cin, kHidden, kOut, d.h, d.w};
    W.cnn_bytes = lbm_cnn_workspace_bytes(&sh);
    const ParamLayout P = param_layout(d.cin);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al256(off + bytes);
        return o;
    };
    W.xn = take(mb * d.cin * hw * sizeof(float));
    W.tn = take(mb * kOut * hw * sizeof(float));
    W.a1 = take(mb * kHidden * hw * sizeof(float));
    W.a2 = take(mb * kHidden * hw * sizeof(float));
    W.y = take(mb * kOut * hw * sizeof(float));
    W.cnn = take(W.cnn_bytes);
    for (int k = 0; k < 6; ++k)
        W.grad[k] = take(P.count[k] * sizeof(float));
    W.mean = take(d.cin * sizeof(double));
    W.stdev = take(d.cin * sizeof(double));
    W.stats = take(lbm_channel_stats_workspace_bytes(d.cin));
    W.loss = take(sizeof(float));
    W.X = take(mb * d.cin * hw * sizeof(float));
    W.Y = take(mb * d.cin * hw * sizeof(float));
    W.F = take(mb * d.cin * hw * sizeof(float));
    W.err = take(mb * sizeof(double));
    W.mask = take(mb * sizeof(int32_t));
    W.ptrs = take(2 * mb * sizeof(void *));
    W.act = take(mb * sizeof(float));
    W.total = off;
    return W;
}

static bool desc_ok(const lbm_surrogate_desc *d)
{
    return d && d->cin >= 3 && d->cin <= 4 && d->h > 0 && d->w > 0 && (int64_t)d->h * d->w <= (1 << 20) &&
           d->coarse >= 1 && (d->coarse == 1 || d->coarse % 2 == 0) && d->k >= 1 && d->max_batch >= 1 &&
           d->max_batch <= 65535;
}

// out[i][c][p] = src[idx ? idx[i] : i][c][p] * scale[c] + shift[c] for
// c < nc; src holds sc channels per sample, out nc.
__global__ __launch_bounds__(256) void k_gather_affine(const float *__restrict__ src, int sc, const int32_t *__restrict__ idx,
                                                       int n, int nc, int64_t hw, const float *__restrict__ scale,
                                                       const float *__restrict__ shift, float *__restrict__ out)
{
    const int64_t total = (int64_t)n * nc * hw;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t p = e % hw;
        const int c = (int)((e / hw) % nc);
        const int i = (int)(e / (hw * nc));
        const int64_t s = idx ? idx[i] : i;
        out[e] = src[(s * sc + c) * hw + p] * scale[c] + shift[c];
    }
}

// y[i][c] = yn[i][c] * inv_scale[c] + inv_shift[c] for the three fields, and
// the constant channels copied from x.
__global__ __launch_bounds__(256) void k_denorm_merge(const float *__restrict__ yn, const float *__restrict__ x, int n,
                                                      int cin, int64_t hw, const float *__restrict__ inv_scale,
                                                      const float *__restrict__ inv_shift, float *__restrict__ y)
{
    const int64_t total = (int64_t)n * cin * hw;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t p = e % hw;
        const int c = (int)((e / hw) % cin);
        const int64_t i = e / (hw * cin);
        y[e] = c < kOut ? yn[(i * kOut + c) * hw + p] * inv_scale[c] + inv_shift[c] : x[e];
    }
}

// Normalisation from the channel statistics: inputs to (x - mean) / std,
// outputs back by std and mean (a channel with no spread keeps scale 1).
__global__ void k_set_norm(const double *__restrict__ mean, const double *__restrict__ stdev, int cin,
                           float *__restrict__ norm)
{
    const int c = threadIdx.x;
    if (c >= cin)
        return;
    const double sd = stdev[c] > 0.0 ? stdev[c] : 1.0;
    norm[c] = (float)(1.0 / sd);
    norm[cin + c] = (float)(-mean[c] / sd);
    norm[2 * cin + c] = (float)sd;
    norm[3 * cin + c] = (float)mean[c];
}

// dst[l] = src[l] (rows of len floats) where mask[l] != 0.
__global__ __launch_bounds__(256) void k_select_rows(float *__restrict__ dst, const float *__restrict__ src,
                                                     const int32_t *__restrict__ mask, int64_t len)
{
    const int l = blockIdx.y;
    if (!mask[l])
        return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < len; e += (int64_t)gridDim.x * 256)
        dst[(int64_t)l * len + e] = src[(int64_t)l * len + e];
}

static unsigned grid_for(int64_t total) { return (unsigned)std::min<int64_t>((total + 255) / 256, 16384); }

}  // namespace lbm

struct lbm_surrogate {
    lbm_surrogate_desc d;
    lbm::ParamLayout P;
    lbm::WorkLayout W;
    char *params;
    char *ws;
    hipStream_t stream;
    int64_t t;  // Adam steps taken
    float *norm() const { return (float *)(params + P.norm); }
    lbm_cnn_params cnn_params() const
    {
        lbm_cnn_params p;
        for (int k = 0; k < 3; ++k) {
            p.w[k] = (const uint16_t *)(params + P.wb[k]);
            p.b[k] = (const float *)(params + P.theta[2 * k + 1]);
        }
        return p;
    }
    lbm_cnn_shape shape(int n) const { return lbm_cnn_shape{n, d.cin, lbm::kHidden, lbm::kOut, d.h, d.w}; }
};

namespace lbm {

// Network output for the samples already normalised in W.xn.
static int32_t forward_n(lbm_surrogate *s, int n)
{
    const lbm_cnn_shape sh = s->shape(n);
    const lbm_cnn_params p = s->cnn_params();
    return lbm_cnn_forward(&sh, &p, (const float *)(s->ws + s->W.xn), (float *)(s->ws + s->W.a1),
                           (float *)(s->ws + s->W.a2), (float *)(s->ws + s->W.y), s->ws + s->W.cnn, s->W.cnn_bytes,
                           s->stream);
}

static int32_t predict_into(lbm_surrogate *s, const float *x, int n, float *y)
{
    const int64_t hw = (int64_t)s->d.h * s->d.w;
    const float *nm = s->norm();
    hipLaunchKernelGGL(k_gather_affine, dim3(grid_for((int64_t)n * s->d.cin * hw)), dim3(256), 0, s->stream, x,
                       s->d.cin, (const int32_t *)nullptr, n, s->d.cin, hw, nm, nm + s->d.cin,
                       (float *)(s->ws + s->W.xn));
    LBM_HIP_TRY(hipGetLastError());
    int32_t rc = forward_n(s, n);
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_denorm_merge, dim3(grid_for((int64_t)n * s->d.cin * hw)), dim3(256), 0, s->stream,
                       (const float *)(s->ws + s->W.y), x, n, s->d.cin, hw, nm + 2 * s->d.cin, nm + 3 * s->d.cin, y);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Surrogate form of lbm_sweep_batch (called by it when opts->surrogate is
// set; arguments already validated as for a plain sweep).
// ---------------------------------------------------------------------------
int32_t surrogate_sweep(const lbm_params *ps, int n, const lbm_sweep_opts *o, void *const *bufs, void *ws,
                        size_t ws_bytes, hipStream_t st, lbm_obs *out)
{
    lbm_surrogate *s = o->surrogate;
    const lbm_surrogate_desc &d = s->d;
    if (s->stream != st)
        return fail(LBM_EINVAL, "the sweep's stream must be the surrogate's");
    if (o->k != d.k)
        return fail(LBM_EINVAL, "opts.k must equal the k the surrogate was created for");
    if (o->check_every < 1 || !(o->tol >= 0.0))
        return fail(LBM_EINVAL, "check_every must be >= 1 and tol >= 0");
    if (n > d.max_batch)
        return fail(LBM_EINVAL, "more lattices than the surrogate's max_batch");
    if (o->n_steps % d.k != 0)
        return fail(LBM_EINVAL, "n_steps must be a multiple of k");
    if (o->sample_every != 0 && o->sample_every != o->n_steps)
        return fail(LBM_EINVAL, "a surrogate sweep samples once, at the end (sample_every 0 or n_steps)");
    if (o->drho)
        return fail(LBM_EINVAL, "a surrogate sweep takes no density ramp");
    for (int l = 0; l < n; ++l) {
        const lbm_params &p = ps[l];
        if (p.lattice != LBM_D2Q7 || p.model == LBM_MIPS || p.storage != LBM_F32)
            return fail(LBM_EUNSUPPORTED, "surrogate sweeps take D2Q7 CIL or passive lattices in F32 storage");
        if (p.nx != d.w * d.coarse || p.ny != d.h * d.coarse)
            return fail(LBM_EINVAL, "every lattice must be (w * coarse) x (h * coarse) sites");
    }
    const int64_t hw = (int64_t)d.h * d.w, row = (int64_t)d.cin * hw;
    const int64_t jumps = o->n_steps / d.k;
    const int k = d.k;
    const WorkLayout &W = s->W;
    float *X = (float *)(s->ws + W.X), *Y = (float *)(s->ws + W.Y), *F = (float *)(s->ws + W.F);
    double *d_err = (double *)(s->ws + W.err);
    int32_t *d_mask = (int32_t *)(s->ws + W.mask);
    void **d_ptrs = (void **)(s->ws + W.ptrs);
    float *d_act = (float *)(s->ws + W.act);

    // which buffer of each pair holds the lattice's state
    std::vector<int> cur(n, 0);
    std::vector<int32_t> fallen(n, 0);
    std::vector<float> act(n);
    for (int l = 0; l < n; ++l)
        act[l] = (float)ps[l].B;
    std::vector<void *> ptrs(2 * (size_t)n);
    auto upload_ptrs = [&]() -> hipError_t {  // the state buffer of every lattice
        for (int l = 0; l < n; ++l)
            ptrs[l] = bufs[2 * l + cur[l]];
        return hipMemcpyAsync(d_ptrs, ptrs.data(), sizeof(void *) * n, hipMemcpyHostToDevice, st);
    };
    auto coarse_all = [&](float *dst) -> int32_t {
        LBM_HIP_TRY(upload_ptrs());
        int32_t rc = lbm_coarsen_many(&ps[0], n, (const float *const *)d_ptrs, d.coarse, dst, row, st);
        if (rc)
            return rc;
        if (d.cin > 3)
            return lbm_fill_channel(dst, n, d.cin, 3, hw, d_act, st);
        return LBM_OK;
    };
    // lift the coarse fields src of the lattices where pick[l] into their
    // state buffers
    std::vector<int32_t> pick(n);
    auto lift_some = [&](const float *src) -> int32_t {
        for (int l = 0; l < n; ++l)
            ptrs[n + l] = pick[l] ? bufs[2 * l + cur[l]] : nullptr;
        std::vector<int> idx;
        for (int l = 0; l < n; ++l)
            if (pick[l])
                idx.push_back(l);
        // one launch per run of consecutive picked lattices (lift_many reads
        // rows in_stride apart)
        for (size_t a = 0; a < idx.size();) {
            size_t b = a + 1;
            while (b < idx.size() && idx[b] == idx[b - 1] + 1)
                ++b;
            LBM_HIP_TRY(hipMemcpyAsync(d_ptrs + n, &ptrs[n + idx[a]], sizeof(void *) * (b - a), hipMemcpyHostToDevice,
                                       st));
            int32_t rc = lbm_lift_many(&ps[0], (int32_t)(b - a), src + (int64_t)idx[a] * row, row, d.coarse,
                                       (float *const *)(d_ptrs + n), st);
            if (rc)
                return rc;
            a = b;  // the next run's pointer upload is ordered after this lift on the stream
        }
        return LBM_OK;
    };
    // k lattice Boltzmann steps of the lattices where pick[l], one batched
    // call (a fixed two-step tile, so a new subset is not tuned)
    auto advance_some = [&](int64_t step0) -> int32_t {
        std::vector<lbm_params> sp;
        std::vector<void *> sb;
        std::vector<int> idx;
        for (int l = 0; l < n; ++l)
            if (pick[l]) {
                sp.push_back(ps[l]);
                sb.push_back(bufs[2 * l + cur[l]]);
                sb.push_back(bufs[2 * l + (cur[l] ^ 1)]);
                idx.push_back(l);
            }
        if (sp.empty())
            return LBM_OK;
        lbm_sweep_opts io{};
        io.n_steps = k;
        io.sample_every = 0;
        io.step0 = step0;
        io.tile_rows = o->tile_rows ? o->tile_rows : 16;
        io.use_graph = 1;
        int32_t rc = lbm_sweep_batch(sp.data(), (int32_t)sp.size(), &io, sb.data(), ws, ws_bytes, st, nullptr);
        if (rc)
            return rc;
        for (int l : idx)
            cur[l] ^= k & 1;
        return LBM_OK;
    };

    LBM_HIP_TRY(hipMemcpyAsync(d_act, act.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
    int32_t rc = coarse_all(X);
    if (rc)
        return rc;
    std::vector<double> err(n);
    std::vector<double> errors;  // per check, per lattice (NaN where fallen before the check)
    int64_t n_checks = 0;
    for (int64_t j = 0; j < jumps; ++j) {
        rc = predict_into(s, X, n, Y);
        if (rc)
            return rc;
        bool any_live = false;
        for (int l = 0; l < n; ++l)
            any_live = any_live || !fallen[l];
        const bool check = (j + 1) % o->check_every == 0 && any_live;
        const int64_t step0 = o->step0 + j * k;
        if (check) {
            for (int l = 0; l < n; ++l)
                pick[l] = !fallen[l];
            rc = lift_some(X);  // the judge starts from the surrogate's coarse state
            if (rc)
                return rc;
        }
        for (int l = 0; l < n; ++l)
            pick[l] = fallen[l] || check;
        rc = advance_some(step0);
        if (rc)
            return rc;
        rc = coarse_all(F);
        if (rc)
            return rc;
        // fallen lattices take the method's fields
        LBM_HIP_TRY(hipMemcpyAsync(d_mask, fallen.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_select_rows, dim3(grid_for(row), n), dim3(256), 0, st, Y, F, d_mask, row);
        LBM_HIP_TRY(hipGetLastError());
        if (check) {
            rc = lbm_field_error(Y, F, n, d.cin, kOut, hw, d_err, st);
            if (rc)
                return rc;
            LBM_HIP_TRY(hipMemcpyAsync(err.data(), d_err, sizeof(double) * n, hipMemcpyDeviceToHost, st));
            LBM_HIP_TRY(hipStreamSynchronize(st));
            std::vector<int32_t> newly(n, 0);
            for (int l = 0; l < n; ++l) {
                errors.push_back(fallen[l] ? NAN : err[l]);
                if (!fallen[l] && !(err[l] <= o->tol))
                    newly[l] = 1;
            }
            ++n_checks;
            for (int l = 0; l < n; ++l)
                fallen[l] |= newly[l];
            LBM_HIP_TRY(hipMemcpyAsync(d_mask, newly.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_select_rows, dim3(grid_for(row), n), dim3(256), 0, st, Y, F, d_mask, row);
            LBM_HIP_TRY(hipGetLastError());
            LBM_HIP_TRY(hipStreamSynchronize(st));  // host vectors of this check are released
        }
        std::swap(X, Y);
    }
    // lattices still on the surrogate: their state becomes the lift of their
    // coarse fields; every state goes to the buffer the step count names
    for (int l = 0; l < n; ++l)
        pick[l] = !fallen[l];
    rc = lift_some(X);
    if (rc)
        return rc;
    const int last = (int)(o->n_steps & 1);
    for (int l = 0; l < n; ++l)
        if (cur[l] != last) {
            const size_t bytes = (size_t)7 * ps[l].nx * ps[l].ny * sizeof(float);
            LBM_HIP_TRY(hipMemcpyAsync(bufs[2 * l + last], bufs[2 * l + cur[l]], bytes, hipMemcpyDeviceToDevice, st));
            cur[l] = last;
        }
    if (o->coarse_out)
        LBM_HIP_TRY(hipMemcpyAsync(o->coarse_out, X, sizeof(float) * n * row, hipMemcpyDeviceToDevice, st));
    if (o->fallen_out)
        memcpy(o->fallen_out, fallen.data(), sizeof(int32_t) * n);
    if (o->check_errors_out)
        for (size_t e = 0; e < errors.size() && (int64_t)e < (int64_t)n * o->max_checks; ++e)
            o->check_errors_out[e] = errors[e];
    if (o->n_checks_out)
        *o->n_checks_out = n_checks;
    // the sample: a plain sweep of zero steps samples the final states
    std::vector<void *> fb(2 * (size_t)n);
    for (int l = 0; l < n; ++l) {
        fb[2 * l] = bufs[2 * l + last];
        fb[2 * l + 1] = bufs[2 * l + (last ^ 1)];
    }
    lbm_sweep_opts so{};
    so.n_steps = 0;
    so.step0 = o->step0 + o->n_steps;
    so.tile_rows = o->tile_rows ? o->tile_rows : 16;
    so.use_graph = 0;
    if (!out) {
        LBM_HIP_TRY(hipStreamSynchronize(st));  // host arrays of the uploads are released
        return LBM_OK;
    }
    return lbm_sweep_batch(ps, n, &so, fb.data(), ws, ws_bytes, st, out);
}

}  // namespace lbm

using namespace lbm;

extern "C" {

size_t lbm_surrogate_param_bytes(const lbm_surrogate_desc *d)
{
    return desc_ok(d) ? param_layout(d->cin).total : 0;
}

size_t lbm_surrogate_workspace_bytes(const lbm_surrogate_desc *d)
{
    return desc_ok(d) ? work_layout(*d).total : 0;
}

int32_t lbm_surrogate_create(const lbm_surrogate_desc *d, void *params, int32_t init, uint64_t seed, void *ws,
                             size_t ws_bytes, void *stream, lbm_surrogate **out)
{
    if (!out)
        return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!desc_ok(d))
        return fail(LBM_EINVAL, "invalid surrogate description (cin 3 or 4, h, w > 0, coarse 1 or even, k >= 1, "
                                "1 <= max_batch <= 65535)");
    if (!params || !ws || (uintptr_t)params % 256 || (uintptr_t)ws % 256)
        return fail(LBM_EINVAL, "null or misaligned (256 B) parameter block or workspace");
    const WorkLayout W = work_layout(*d);
    if (ws_bytes < W.total)
        return fail(LBM_EINVAL, "workspace smaller than lbm_surrogate_workspace_bytes()");
    lbm_surrogate *s = new (std::nothrow) lbm_surrogate();
    if (!s)
        return fail(LBM_EINVAL, "out of host memory");
    s->d = *d;
    s->P = param_layout(d->cin);
    s->W = W;
    s->params = (char *)params;
    s->ws = (char *)ws;
    s->stream = (hipStream_t)stream;
    s->t = 0;
    if (init) {
        // He-uniform weights (bound sqrt(6 / fan_in), a tenth of it on the
        // output layer, so the untrained network starts near the identity of
        // the residual connection), zero biases and moments, identity
        // normalisation
        std::vector<char> host(s->P.total, 0);
        std::mt19937_64 rng(seed);
        const int fan[3] = {9 * d->cin, 9 * kHidden, 9 * kHidden};
        for (int k = 0; k < 3; ++k) {
            const double lim = sqrt(6.0 / fan[k]) * (k == 2 ? 0.1 : 1.0);
            std::uniform_real_distribution<double> u(-lim, lim);
            float *w = (float *)(host.data() + s->P.theta[2 * k]);
            uint16_t *wb = (uint16_t *)(host.data() + s->P.wb[k]);
            for (int64_t e = 0; e < s->P.count[2 * k]; ++e) {
                w[e] = (float)u(rng);
                // bfloat16 round to nearest even of a finite float
                uint32_t b;
                memcpy(&b, &w[e], 4);
                b += 0x7fffu + ((b >> 16) & 1u);
                wb[e] = (uint16_t)(b >> 16);
            }
        }
        float *nm = (float *)(host.data() + s->P.norm);
        for (int c = 0; c < d->cin; ++c) {
            nm[c] = 1.0f;
            nm[2 * d->cin + c] = 1.0f;
        }
        hipError_t e = hipMemcpyAsync(params, host.data(), host.size(), hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "lbm_surrogate_create");
        }
    }
    *out = s;
    return LBM_OK;
}

int32_t lbm_surrogate_fit_normalisation(lbm_surrogate *s, const float *x, int32_t n)
{
    if (!s)
        return fail(LBM_ESTATE, "null surrogate");
    if (!x || n < 1)
        return fail(LBM_EINVAL, "null samples or n < 1");
    const int64_t hw = (int64_t)s->d.h * s->d.w;
    double *mean = (double *)(s->ws + s->W.mean), *sd = (double *)(s->ws + s->W.stdev);
    int32_t rc = lbm_channel_stats(x, n, s->d.cin, hw, mean, sd, s->ws + s->W.stats,
                                   lbm_channel_stats_workspace_bytes(s->d.cin), s->stream);
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_set_norm, dim3(1), dim3(64), 0, s->stream, mean, sd, s->d.cin, s->norm());
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_surrogate_train_step(lbm_surrogate *s, const float *x, const float *target, const int32_t *idx,
                                 int32_t n, float lr, float *loss)
{
    if (!s)
        return fail(LBM_ESTATE, "null surrogate");
    if (!x || !target || n < 1 || n > s->d.max_batch)
        return fail(LBM_EINVAL, "null samples, or n outside 1..max_batch");
    if (!(lr >= 0.0f))
        return fail(LBM_EINVAL, "lr must be >= 0");
    const int64_t hw = (int64_t)s->d.h * s->d.w;
    const int cin = s->d.cin;
    const float *nm = s->norm();
    float *xn = (float *)(s->ws + s->W.xn), *tn = (float *)(s->ws + s->W.tn);
    hipLaunchKernelGGL(k_gather_affine, dim3(grid_for((int64_t)n * cin * hw)), dim3(256), 0, s->stream, x, cin, idx, n,
                       cin, hw, nm, nm + cin, xn);
    hipLaunchKernelGGL(k_gather_affine, dim3(grid_for((int64_t)n * kOut * hw)), dim3(256), 0, s->stream, target, cin,
                       idx, n, kOut, hw, nm, nm + cin, tn);
    LBM_HIP_TRY(hipGetLastError());
    int32_t rc = forward_n(s, n);
    if (rc)
        return rc;
    const lbm_cnn_shape sh = s->shape(n);
    const lbm_cnn_params p = s->cnn_params();
    lbm_cnn_grads g;
    for (int k = 0; k < 3; ++k) {
        g.w[k] = (float *)(s->ws + s->W.grad[2 * k]);
        g.b[k] = (float *)(s->ws + s->W.grad[2 * k + 1]);
    }
    float *d_loss = (float *)(s->ws + s->W.loss);
    rc = lbm_cnn_backward(&sh, &p, xn, (const float *)(s->ws + s->W.a1), (const float *)(s->ws + s->W.a2),
                          (const float *)(s->ws + s->W.y), tn, &g, d_loss, s->ws + s->W.cnn, s->W.cnn_bytes,
                          s->stream);
    if (rc)
        return rc;
    s->t += 1;
    AdamJobs aj{};
    for (int k = 0; k < 6; ++k) {
        aj.theta[k] = (float *)(s->params + s->P.theta[k]);
        aj.m[k] = (float *)(s->params + s->P.m[k]);
        aj.v[k] = (float *)(s->params + s->P.v[k]);
        aj.g[k] = (const float *)(s->ws + s->W.grad[k]);
        aj.count[k] = s->P.count[k];
        aj.bf16[k] = k % 2 == 0 ? (uint16_t *)(s->params + s->P.wb[k / 2]) : nullptr;
    }
    LBM_HIP_TRY(launch_adam_many(aj, 6, lr, 0.9f, 0.999f, 1e-8f, s->t, s->stream));
    if (loss)
        LBM_HIP_TRY(hipMemcpyAsync(loss, d_loss, sizeof(float), hipMemcpyDeviceToDevice, s->stream));
    return LBM_OK;
}

int32_t lbm_surrogate_predict(lbm_surrogate *s, const float *x, int32_t n, float *y)
{
    if (!s)
        return fail(LBM_ESTATE, "null surrogate");
    if (!x || !y || n < 1 || n > s->d.max_batch)
        return fail(LBM_EINVAL, "null fields, or n outside 1..max_batch");
    if (x == y)
        return fail(LBM_EINVAL, "x and y must be distinct arrays");
    return predict_into(s, x, n, y);
}

int32_t lbm_surrogate_view_of(const lbm_surrogate *s, lbm_surrogate_view *v)
{
    if (!s)
        return fail(LBM_ESTATE, "null surrogate");
    if (!v)
        return fail(LBM_EINVAL, "null view");
    for (int k = 0; k < 6; ++k) {
        v->theta[k] = (float *)(s->params + s->P.theta[k]);
        v->m[k] = (float *)(s->params + s->P.m[k]);
        v->v[k] = (float *)(s->params + s->P.v[k]);
        v->count[k] = s->P.count[k];
    }
    for (int k = 0; k < 3; ++k)
        v->w_bf16[k] = (uint16_t *)(s->params + s->P.wb[k]);
    v->norm = s->norm();
    v->adam_steps = s->t;
    return LBM_OK;
}

int32_t lbm_surrogate_destroy(lbm_surrogate *s)
{
    if (!s)
        return fail(LBM_ESTATE, "null surrogate");
    hipError_t e = hipStreamSynchronize(s->stream);
    delete s;
    if (e != hipSuccess)
        return hip_fail(e, "lbm_surrogate_destroy");
    return LBM_OK;
}

}  // extern "C"
