// Surrogate network kernels: a three-layer convolutional net (3x3 kernels,
// circular padding, ReLU, residual on the predicted fields) that advances the
// coarse density and momentum fields of a lattice by k steps, its training
// (mean-squared error, backward pass, Adam) and the maps between populations
// and coarse fields.  Not part of the paper; it is judged by the lattice
// Boltzmann step itself.
//
// Layout: activations NCHW float32; weights stored as bfloat16 (the Adam
// step keeps float32 master copies) and widened once per pass to float32, so
// every product is a bf16 x f32 -> f32 product with float32 accumulation.
// Convolutions: one block = one sample x a 16 x 16 pixel tile x all output
// channels; the input tile with its one-pixel halo sits in LDS, weights are
// read with wave-uniform addresses (scalar loads), each thread keeps one
// pixel's output channels in registers.  Reductions (weight gradients, loss)
// use fixed partitions and orders, so results are deterministic.
#include <math.h>

#include <algorithm>

#include "../../include/lbm_cnn.h"
#include "internal.h"

namespace lbm {

constexpr int kTile = 16;

// ---------------------------------------------------------------------------
// 3x3 convolution.  TR = 0: y[n,o,i,j] = b[o] + sum_c sum_k w[o,c,k]
// x[n,c,i+ky-1,j+kx-1].  TR = 1 (input gradient of a convolution with
// weights w[Cin_orig=co][Cout_orig=ci]): y[n,c,..] = sum_o sum_k
// w[o,c,8-k] x[n,o,..], i.e. the same sum with transposed, flipped weights.
// Epilogue in order: bias, ReLU, + resid[n, o] (first co channels of a
// tensor with resid_c channels), * (mask[n, o] > 0).
//
// One block = one sample x a 16 x 16 pixel tile x OG of the co_n output
// channels (blockIdx.z = sample * groups + group), so small batches of small
// fields still give several blocks per CU; the input tile with its halo is
// staged in LDS kChunk channels at a time.  Every output sums over c and k in
// increasing order, as the definition reads.
// ---------------------------------------------------------------------------
constexpr int kChunk = 8;

template <int OG, int TR>
__global__ __launch_bounds__(256) void k_conv3x3(const float *__restrict__ x, int ci_n, const float *__restrict__ w,
                                                 int co_n, const float *__restrict__ bias,
                                                 const float *__restrict__ resid, int resid_c,
                                                 const float *__restrict__ mask, int relu, float *__restrict__ y,
                                                 int H, int W)
{
    constexpr int L = kTile + 2;
    __shared__ float s_in[kChunk * L * L];
    const int groups = co_n / OG;
    const int n = blockIdx.z / groups, o0 = (blockIdx.z - n * groups) * OG;
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
    const int tid = threadIdx.x;
    const size_t HW = (size_t)H * W;
    const float *xn = x + (size_t)n * ci_n * HW;
    const int pi = tid >> 4, pj = tid & 15;
    const int i = i0 + pi, j = j0 + pj;
    float acc[OG];
#pragma unroll
    for (int o = 0; o < OG; ++o)
        acc[o] = bias ? bias[o0 + o] : 0.0f;
    for (int c0 = 0; c0 < ci_n; c0 += kChunk) {
        const int cc = min(kChunk, ci_n - c0);
        __syncthreads();  // the previous chunk is no longer read
        for (int e = tid; e < cc * L * L; e += 256) {
            const int c = e / (L * L), r = e - c * (L * L), li = r / L, lj = r - li * L;
            int gi = i0 + li - 1, gj = j0 + lj - 1;
            gi = gi < 0 ? gi + H : (gi >= H ? gi - H : gi);
            gj = gj < 0 ? gj + W : (gj >= W ? gj - W : gj);
            s_in[e] = xn[(size_t)(c0 + c) * HW + (size_t)gi * W + gj];
        }
        __syncthreads();
        for (int c = 0; c < cc; ++c) {
            const float *t = s_in + c * L * L + pi * L + pj;
            float v[9];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    v[ky * 3 + kx] = t[ky * L + kx];
            const int cg = c0 + c;
#pragma unroll
            for (int o = 0; o < OG; ++o) {
                float sum = acc[o];
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const float wk = TR ? w[((size_t)cg * co_n + o0 + o) * 9 + (8 - k)]
                                        : w[((size_t)(o0 + o) * ci_n + cg) * 9 + k];
                    sum = fmaf(wk, v[k], sum);
                }
                acc[o] = sum;
            }
        }
    }
    if (i >= H || j >= W)
        return;
    const size_t pix = (size_t)i * W + j;
#pragma unroll
    for (int o = 0; o < OG; ++o) {
        const int og = o0 + o;
        float r = acc[o];
        if (relu)
            r = fmaxf(r, 0.0f);
        if (resid)
            r += resid[((size_t)n * resid_c + og) * HW + pix];
        if (mask)
            r = mask[((size_t)n * co_n + og) * HW + pix] > 0.0f ? r : 0.0f;
        y[((size_t)n * co_n + og) * HW + pix] = r;
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dw[o,c,k] = sum_{n,i,j} dy[n,o,i,j]
// x[n,c,i+ky-1,j+kx-1], db[o] = sum dy[n,o,i,j].  One block per (sample,
// 16 x 16 tile) writes its partial sums (float, in pixel order) to
// part[block][co_n ci_n 9 + co_n]; k_grad_reduce adds the blocks in order in
// float64.  Per chunk of kChunk input channels, thread t takes the pair
// (OG output channels, one input channel) t mod pairs and the pixel group
// t / pairs; the pixel groups of a pair are then added in order through LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cwave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

template <int OG>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const float *__restrict__ dy, int co_n,
                                                       const float *__restrict__ x, int ci_n, int H, int W,
                                                       float *__restrict__ part)
{
    constexpr int L = kTile + 2;
    __shared__ float s_x[kChunk * L * L];      // x tile, kChunk input channels
    __shared__ float s_d[32 * kTile * kTile];  // dy tile, all (<= 32) output channels
    __shared__ float s_red[256 * 9];           // pixel-group partials
    const int tiles_j = (W + kTile - 1) / kTile, tiles_i = (H + kTile - 1) / kTile;
    const int n = blockIdx.x / (tiles_i * tiles_j), tt = blockIdx.x - n * (tiles_i * tiles_j);
    const int ti = tt / tiles_j;
    const int i0 = ti * kTile, j0 = (tt - ti * tiles_j) * kTile;
    const int tid = threadIdx.x;
    const size_t HW = (size_t)H * W;
    const int pairs = (co_n / OG) * kChunk;  // divides 256 (checked on the host)
    const int pg = 256 / pairs;              // pixel groups
    const int pair = tid % pairs, grp = tid / pairs;
    const int og = pair / kChunk, cl = pair - og * kChunk;
    const int nw = co_n * ci_n * 9;
    float *out = part + (size_t)blockIdx.x * (nw + co_n);
    // dy tile (zero outside the field)
    for (int e = tid; e < co_n * kTile * kTile; e += 256) {
        const int o = e / (kTile * kTile), r = e - o * (kTile * kTile), li = r / kTile, lj = r - li * kTile;
        const int gi = i0 + li, gj = j0 + lj;
        s_d[e] = (gi < H && gj < W) ? dy[((size_t)n * co_n + o) * HW + (size_t)gi * W + gj] : 0.0f;
    }
    for (int c0 = 0; c0 < ci_n; c0 += kChunk) {
        __syncthreads();
        for (int e = tid; e < kChunk * L * L; e += 256) {
            const int c = e / (L * L), r = e - c * (L * L), li = r / L, lj = r - li * L;
            int gi = i0 + li - 1, gj = j0 + lj - 1;
            gi = gi < 0 ? gi + H : (gi >= H ? gi - H : gi);
            gj = gj < 0 ? gj + W : (gj >= W ? gj - W : gj);
            s_x[e] = c0 + c < ci_n ? x[((size_t)n * ci_n + c0 + c) * HW + (size_t)gi * W + gj] : 0.0f;
        }
        __syncthreads();
        float acc[OG][9];
#pragma unroll
        for (int o = 0; o < OG; ++o)
#pragma unroll
            for (int k = 0; k < 9; ++k)
                acc[o][k] = 0.0f;
        for (int p = grp; p < kTile * kTile; p += pg) {
            const int pi = p >> 4, pj = p & 15;
            const float *t = s_x + cl * L * L + pi * L + pj;
            float v[9];
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    v[ky * 3 + kx] = t[ky * L + kx];
#pragma unroll
            for (int o = 0; o < OG; ++o) {
                const float d = s_d[(og * OG + o) * kTile * kTile + p];
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    acc[o][k] = fmaf(d, v[k], acc[o][k]);
            }
        }
        // the pixel groups of one (pair, tap), added in group order, one
        // (pair, tap) per thread
#pragma unroll
        for (int o = 0; o < OG; ++o) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 9; ++k)
                s_red[tid * 9 + k] = acc[o][k];
            __syncthreads();
            for (int q = tid; q < pairs * 9; q += 256) {
                const int qp = q / 9, k = q - qp * 9;
                const int qog = qp / kChunk, qcl = qp - qog * kChunk;
                if (c0 + qcl < ci_n) {
                    float sum = 0.0f;
                    for (int g = 0; g < pg; ++g)
                        sum += s_red[(g * pairs + qp) * 9 + k];
                    out[((size_t)(qog * OG + o) * ci_n + c0 + qcl) * 9 + k] = sum;
                }
            }
        }
    }
    // bias: thread o adds its dy tile in pixel order
    if (tid < co_n) {
        float sum = 0.0f;
        for (int p = 0; p < kTile * kTile; ++p)
            sum += s_d[tid * kTile * kTile + p];
        out[nw + tid] = sum;
    }
}

// g[e] = the sum over blocks b of part[b][e] (float64); e < nw goes to the
// weight gradient, e >= nw to the bias gradient.  A block takes 64 entries
// with 4 threads each: thread slice s adds blocks s, s + 4, ... in order, then
// the four slices are added in order.
__global__ __launch_bounds__(256) void k_grad_reduce(const float *__restrict__ part, int nblocks, int nw, int nb,
                                                     float *__restrict__ gw, float *__restrict__ gb)
{
    __shared__ double s_sum[4][64];
    const int col = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + col;
    double sum = 0.0;
    if (e < nw + nb)
        for (int b = slice; b < nblocks; b += 4)
            sum += (double)part[(size_t)b * (nw + nb) + e];
    s_sum[slice][col] = sum;
    __syncthreads();
    if (slice == 0 && e < nw + nb) {
        const double t = ((s_sum[0][col] + s_sum[1][col]) + s_sum[2][col]) + s_sum[3][col];
        if (e < nw)
            gw[e] = (float)t;
        else
            gb[e - nw] = (float)t;
    }
}

// Mean squared error: dy = 2 (y - t) / count, per-block float64 partials of
// sum (y - t)^2; k_mse_final adds them in order.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, int64_t count,
                                             float *__restrict__ dy, double *__restrict__ part)
{
    __shared__ double s_red[4];
    double acc = 0.0;
    const float scale = (float)(2.0 / (double)count);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        const float d = y[e] - t[e];
        dy[e] = d * scale;
        acc += (double)d * (double)d;
    }
    acc = cwave_sum(acc);
    if ((threadIdx.x & 63) == 0)
        s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

// One block of 256: thread t adds partials t, t + 256, ... in order, then a
// fixed tree over the threads.
__global__ __launch_bounds__(256) void k_mse_final(const double *__restrict__ part, int nparts, int64_t count,
                                                   float *__restrict__ loss)
{
    __shared__ double s_red[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256)
        s += part[b];
    s = cwave_sum(s);
    if ((threadIdx.x & 63) == 0)
        s_red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        *loss = (float)((((s_red[0] + s_red[1]) + s_red[2]) + s_red[3]) / (double)count);
}

// bf16 weights -> float32 working copy.
__global__ void k_widen_bf16(const uint16_t *__restrict__ w, int64_t count, float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count)
        out[e] = bf16_bits_to_float(w[e]);
}

// Adam (Kingma & Ba, algorithm 1) on a float32 master tensor; writes the
// bf16 copy when bf16_out is given.
__global__ void k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t count, float lr, float beta1, float beta2, float eps,
                       float bc1, float bc2, uint16_t *__restrict__ bf16_out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count)
        return;
    const float gi = g[e];
    const float mi = beta1 * m[e] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[e] + (1.0f - beta2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float th = theta[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    theta[e] = th;
    if (bf16_out)
        bf16_out[e] = float_to_bf16_rne(th);
}

// x[n, c, p] = x[n, c, p] * scale[c] + shift[c] for c < nc (in place).
__global__ void k_channel_affine(float *__restrict__ x, int N, int C, int nc, int64_t HW,
                                 const float *__restrict__ scale, const float *__restrict__ shift)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nc * HW;
    if (e >= (int64_t)N * per)
        return;
    const int64_t n = e / per, r = e - n * per;
    const int c = (int)(r / HW);
    float *p = x + (n * C + c) * HW + (r - (int64_t)c * HW);
    *p = *p * scale[c] + shift[c];
}

// Per-sample relative L2 error of the first nc channels: out[s] =
// |a_s - b_s| / |b_s| (float64 sums, one block per sample, fixed order).
__global__ __launch_bounds__(256) void k_field_error(const float *__restrict__ a, const float *__restrict__ b, int C,
                                                     int nc, int64_t hw, double *__restrict__ out)
{
    __shared__ double s_red[2][4];
    const int smp = blockIdx.x;
    double num = 0.0, den = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)nc * hw; e += 256) {
        const int64_t o = (int64_t)smp * C * hw + e;
        const double d = (double)a[o] - (double)b[o];
        num += d * d;
        den += (double)b[o] * (double)b[o];
    }
    num = cwave_sum(num);
    den = cwave_sum(den);
    if ((threadIdx.x & 63) == 0) {
        s_red[0][threadIdx.x >> 6] = num;
        s_red[1][threadIdx.x >> 6] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nn = ((s_red[0][0] + s_red[0][1]) + s_red[0][2]) + s_red[0][3];
        const double dd = ((s_red[1][0] + s_red[1][1]) + s_red[1][2]) + s_red[1][3];
        out[smp] = dd > 0.0 ? sqrt(nn / dd) : (nn > 0.0 ? INFINITY : 0.0);
    }
}

// Per-channel mean and standard deviation over n samples and hw pixels, in
// float64 and in a fixed order: each of kStatBlocks blocks of a channel sums
// its contiguous share of the channel's n * hw values (pass 1: values, pass
// 3: squared deviations from the mean), and one block per channel adds the
// shares in block order (passes 2 and 4).
constexpr int kStatBlocks = 256;

__device__ __forceinline__ double stat_block_sum(double acc)
{
    __shared__ double s_red[4];
    acc = cwave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    return ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];  // valid in every thread
}

// pass 1 (mean == nullptr) or 3: partial sums of x, or of (x - mean)^2
__global__ __launch_bounds__(256) void k_stat_partial(const float *__restrict__ x, int n, int C, int64_t hw,
                                                      const double *__restrict__ mean, double *__restrict__ part)
{
    const int c = blockIdx.y, b = blockIdx.x;
    const int64_t cnt = (int64_t)n * hw;
    const int64_t lo = cnt * b / kStatBlocks, hi = cnt * (b + 1) / kStatBlocks;
    const double m = mean ? mean[c] : 0.0;
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const int64_t smp = e / hw, px = e - smp * hw;
        const double v = (double)x[(smp * C + c) * hw + px];
        acc += mean ? (v - m) * (v - m) : v;
    }
    acc = stat_block_sum(acc);
    if (threadIdx.x == 0)
        part[(int64_t)c * kStatBlocks + b] = acc;
}

// pass 2 (mean of the partial sums) or 4 (standard deviation)
__global__ __launch_bounds__(256) void k_stat_final(const double *__restrict__ part, int64_t cnt,
                                                    double *__restrict__ out, int root)
{
    const int c = blockIdx.x;
    double acc = threadIdx.x < kStatBlocks ? part[(int64_t)c * kStatBlocks + threadIdx.x] : 0.0;
    acc = stat_block_sum(acc);
    if (threadIdx.x == 0)
        out[c] = root ? sqrt(acc / (double)cnt) : acc / (double)cnt;
}

// x[s, ch, :] = values[s]
__global__ void k_fill_channel(float *__restrict__ x, int n, int C, int ch, int64_t hw,
                               const float *__restrict__ values)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * hw)
        return;
    const int64_t s = e / hw;
    x[(s * C + ch) * hw + (e - s * hw)] = values[s];
}

// ---------------------------------------------------------------------------
// Coarse fields of a lattice: the mean over c x c blocks of sites of rho, jx,
// jy of the streamed populations (the fields step (ii) of the algorithm
// sees), out[3][ny/c][nx/c].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_coarsen(const float *__restrict__ f, StepArgs a, int cs, int cw, int chh,
                                                 float *__restrict__ out)
{
    const int cx = blockIdx.x * blockDim.x + threadIdx.x, cy = blockIdx.y;
    if (cx >= cw)
        return;
    float r = 0.0f, jxs = 0.0f, jys = 0.0f;
    for (int dy = 0; dy < cs; ++dy)
        for (int dx = 0; dx < cs; ++dx) {
            const int x = cx * cs + dx, y = cy * cs + dy;
            const PullSources32 g = pull_sources32(a, x, y);
            float v[7];
#pragma unroll
            for (int i = 0; i < 7; ++i)
                v[i] = ld32(f + (size_t)i * (uint32_t)a.plane, g.idx[i]);
            float rho, jx, jy;
            site_moments(v, rho, jx, jy);
            r += rho;
            jxs += jx;
            jys += jy;
        }
    const float inv = 1.0f / (float)(cs * cs);
    const size_t cp = (size_t)chh * cw;
    out[(size_t)cy * cw + cx] = r * inv;
    out[cp + (size_t)cy * cw + cx] = jxs * inv;
    out[2 * cp + (size_t)cy * cw + cx] = jys * inv;
}

// Many lattices of one shape: blockIdx.z selects the lattice, whose stored
// state is bufs[z]; output rows of lattice z start at out + z * out_stride.
__global__ __launch_bounds__(256) void k_coarsen_many(const float *const *__restrict__ bufs, StepArgs a, int cs,
                                                      int cw, int chh, float *__restrict__ out, int64_t out_stride)
{
    const int cx = blockIdx.x * blockDim.x + threadIdx.x, cy = blockIdx.y;
    if (cx >= cw)
        return;
    const float *f = bufs[blockIdx.z];
    float r = 0.0f, jxs = 0.0f, jys = 0.0f;
    for (int dy = 0; dy < cs; ++dy)
        for (int dx = 0; dx < cs; ++dx) {
            const PullSources32 g = pull_sources32(a, cx * cs + dx, cy * cs + dy);
            float v[7];
#pragma unroll
            for (int i = 0; i < 7; ++i)
                v[i] = ld32(f + (size_t)i * (uint32_t)a.plane, g.idx[i]);
            float rho, jx, jy;
            site_moments(v, rho, jx, jy);
            r += rho;
            jxs += jx;
            jys += jy;
        }
    const float inv = 1.0f / (float)(cs * cs);
    const size_t cp = (size_t)chh * cw;
    float *o = out + (int64_t)blockIdx.z * out_stride;
    o[(size_t)cy * cw + cx] = r * inv;
    o[cp + (size_t)cy * cw + cx] = jxs * inv;
    o[2 * cp + (size_t)cy * cw + cx] = jys * inv;
}

__global__ __launch_bounds__(256) void k_lift_many(const float *__restrict__ coarse, int64_t in_stride, StepArgs a,
                                                   int cs, int cw, int chh, float *const *__restrict__ bufs)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= a.nx)
        return;
    const float *cf = coarse + (int64_t)blockIdx.z * in_stride;
    float *f = bufs[blockIdx.z];
    const int cx = x / cs, cy = y / cs;
    const size_t cp = (size_t)chh * cw;
    const float rho = fmaxf(cf[(size_t)cy * cw + cx], 0.0f);
    const float jx = cf[cp + (size_t)cy * cw + cx], jy = cf[2 * cp + (size_t)cy * cw + cx];
    const float r = rho > 0.0f ? 1.0f / rho : 0.0f;
    float eq[7];
    site_equilibrium(rho, jx * r, jy * r, eq);
    const uint32_t own = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
#pragma unroll
    for (int i = 0; i < 7; ++i)
        st32(f + (size_t)i * (uint32_t)a.plane, own, eq[i]);
}

// Populations from coarse fields: every site of a c x c block gets the
// steady state xi(rho, j/rho) of its block (eq. fssD2Q7 with u* = u), as a
// stored state.  rho <= 0 gives empty sites.
__global__ __launch_bounds__(256) void k_lift(const float *__restrict__ coarse, StepArgs a, int cs, int cw, int chh,
                                              float *__restrict__ f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= a.nx)
        return;
    const int cx = x / cs, cy = y / cs;
    const size_t cp = (size_t)chh * cw;
    const float rho = fmaxf(coarse[(size_t)cy * cw + cx], 0.0f);
    const float jx = coarse[cp + (size_t)cy * cw + cx], jy = coarse[2 * cp + (size_t)cy * cw + cx];
    const float r = rho > 0.0f ? 1.0f / rho : 0.0f;
    float eq[7];
    site_equilibrium(rho, jx * r, jy * r, eq);
    const uint32_t own = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
#pragma unroll
    for (int i = 0; i < 7; ++i)
        st32(f + (size_t)i * (uint32_t)a.plane, own, eq[i]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int64_t n_w(int a, int b) { return (int64_t)a * b * 9; }

static bool shape_ok(const lbm_cnn_shape *s)
{
    return s && s->n > 0 && s->h > 0 && s->w > 0 && s->hidden == 32 && s->cout == 3 && s->cin >= 3 &&
           s->cin <= 32 && (int64_t)s->h * s->w <= (1 << 26) && s->n <= 65535;
}

// co output channels in groups of OG (co % OG == 0)
template <int OG, int TR>
static hipError_t conv(const float *x, int ci, const float *w, int co, const float *b, const float *resid,
                       int resid_c, const float *mask, int relu, float *y, int N, int H, int W, hipStream_t s)
{
    dim3 grd((W + kTile - 1) / kTile, (H + kTile - 1) / kTile, N * (co / OG));
    hipLaunchKernelGGL((k_conv3x3<OG, TR>), grd, dim3(256), 0, s, x, ci, w, co, b, resid, resid_c, mask, relu, y, H,
                       W);
    return hipGetLastError();
}

static int conv_tiles(int H, int W) { return ((H + kTile - 1) / kTile) * ((W + kTile - 1) / kTile); }

// Weight and bias gradients of one layer (co output, ci input channels):
// per-tile partials, then their ordered sum.
template <int OG>
static hipError_t wgrad(const float *dy, int co, const float *x, int ci, int N, int H, int W, float *part, float *gw,
                        float *gb, hipStream_t s)
{
    const int blocks = N * conv_tiles(H, W);
    hipLaunchKernelGGL((k_conv3x3_wgrad<OG>), dim3(blocks), dim3(256), 0, s, dy, co, x, ci, H, W, part);
    const int total = co * ci * 9 + co;
    hipLaunchKernelGGL(k_grad_reduce, dim3((total + 63) / 64), dim3(256), 0, s, part, blocks, co * ci * 9, co, gw,
                       gb);
    return hipGetLastError();
}

struct CnnWs {
    float *w[3];     // widened weights
    double *part;    // loss partials
    float *gpart;    // per-tile gradient partials
    float *dy;       // dL/dy [n][cout][hw]
    float *dz2;      // [n][hidden][hw]
    float *dz1;      // [n][hidden][hw]
    size_t total;
};

static const int kMseBlocks = 1024;

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace: widened weights, loss partials and the backward pass's
// intermediate gradients.  base == nullptr only measures the size.
static CnnWs cnn_layout(const lbm_cnn_shape *s, char *base)
{
    CnnWs L{};
    size_t off = 0, o[7];
    const int64_t hw = (int64_t)s->h * s->w;
    const int64_t sizes[3] = {n_w(s->hidden, s->cin), n_w(s->hidden, s->hidden), n_w(s->cout, s->hidden)};
    for (int k = 0; k < 3; ++k) {
        o[k] = off;
        off = align256(off + sizes[k] * sizeof(float));
    }
    o[3] = off;
    off = align256(off + kMseBlocks * sizeof(double));
    const size_t gpart = off;  // the largest layer: hidden x hidden weights
    off = align256(off + (size_t)s->n * conv_tiles(s->h, s->w) *
                             (size_t)(s->hidden * std::max(s->hidden, s->cin) * 9 + s->hidden) * sizeof(float));
    o[4] = off;
    off = align256(off + (size_t)s->n * s->cout * hw * sizeof(float));
    o[5] = off;
    off = align256(off + (size_t)s->n * s->hidden * hw * sizeof(float));
    o[6] = off;
    off = align256(off + (size_t)s->n * s->hidden * hw * sizeof(float));
    L.total = off;
    if (base) {
        for (int k = 0; k < 3; ++k)
            L.w[k] = (float *)(base + o[k]);
        L.part = (double *)(base + o[3]);
        L.gpart = (float *)(base + gpart);
        L.dy = (float *)(base + o[4]);
        L.dz2 = (float *)(base + o[5]);
        L.dz1 = (float *)(base + o[6]);
    }
    return L;
}

static hipError_t widen(const lbm_cnn_shape *s, const lbm_cnn_params *p, const CnnWs &L, hipStream_t st)
{
    const int64_t sizes[3] = {n_w(s->hidden, s->cin), n_w(s->hidden, s->hidden), n_w(s->cout, s->hidden)};
    for (int k = 0; k < 3; ++k)
        hipLaunchKernelGGL(k_widen_bf16, dim3((unsigned)((sizes[k] + 255) / 256)), dim3(256), 0, st, p->w[k], sizes[k],
                           L.w[k]);
    return hipGetLastError();
}

}  // namespace lbm

using namespace lbm;

extern "C" {

size_t lbm_cnn_workspace_bytes(const lbm_cnn_shape *s)
{
    if (!shape_ok(s))
        return 0;
    return cnn_layout(s, nullptr).total;
}

int32_t lbm_cnn_forward(const lbm_cnn_shape *s, const lbm_cnn_params *p, const float *x, float *a1, float *a2,
                        float *y, void *ws, size_t ws_bytes, void *stream)
{
    if (!shape_ok(s))
        return fail(LBM_EINVAL, "invalid network shape (hidden must be 32, cout 3, 3 <= cin <= 32)");
    if (!p || !x || !a1 || !a2 || !y || !ws)
        return fail(LBM_EINVAL, "null pointer");
    for (int k = 0; k < 3; ++k)
        if (!p->w[k] || !p->b[k])
            return fail(LBM_EINVAL, "null weight or bias");
    const CnnWs L = cnn_layout(s, (char *)ws);
    if (ws_bytes < L.total)
        return fail(LBM_EINVAL, "workspace smaller than lbm_cnn_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    LBM_HIP_TRY(widen(s, p, L, st));
    LBM_HIP_TRY((conv<8, 0>(x, s->cin, L.w[0], 32, p->b[0], nullptr, 0, nullptr, 1, a1, s->n, s->h, s->w, st)));
    LBM_HIP_TRY((conv<8, 0>(a1, 32, L.w[1], 32, p->b[1], nullptr, 0, nullptr, 1, a2, s->n, s->h, s->w, st)));
    LBM_HIP_TRY((conv<3, 0>(a2, 32, L.w[2], 3, p->b[2], x, s->cin, nullptr, 0, y, s->n, s->h, s->w, st)));
    return LBM_OK;
}

int32_t lbm_cnn_backward(const lbm_cnn_shape *s, const lbm_cnn_params *p, const float *x, const float *a1,
                         const float *a2, const float *y, const float *target, const lbm_cnn_grads *g,
                         float *loss, void *ws, size_t ws_bytes, void *stream)
{
    if (!shape_ok(s))
        return fail(LBM_EINVAL, "invalid network shape (hidden must be 32, cout 3, 3 <= cin <= 32)");
    if (!p || !x || !a1 || !a2 || !y || !target || !g || !loss || !ws)
        return fail(LBM_EINVAL, "null pointer");
    for (int k = 0; k < 3; ++k)
        if (!g->w[k] || !g->b[k])
            return fail(LBM_EINVAL, "null gradient buffer");
    const CnnWs L = cnn_layout(s, (char *)ws);
    if (ws_bytes < L.total)
        return fail(LBM_EINVAL, "workspace smaller than lbm_cnn_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    const int N = s->n, H = s->h, W = s->w;
    const int64_t hw = (int64_t)H * W, count = (int64_t)N * s->cout * hw;
    LBM_HIP_TRY(widen(s, p, L, st));
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, st, y, target, count, L.dy, L.part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, L.part, kMseBlocks, count, loss);
    // layer 3: y = x[:cout] + conv(a2, w2) + b2
    LBM_HIP_TRY(wgrad<3>(L.dy, s->cout, a2, 32, N, H, W, L.gpart, g->w[2], g->b[2], st));
    LBM_HIP_TRY((conv<8, 1>(L.dy, s->cout, L.w[2], 32, nullptr, nullptr, 0, a2, 0, L.dz2, N, H, W, st)));
    // layer 2: a2 = relu(conv(a1, w1) + b1)
    LBM_HIP_TRY(wgrad<4>(L.dz2, 32, a1, 32, N, H, W, L.gpart, g->w[1], g->b[1], st));
    LBM_HIP_TRY((conv<8, 1>(L.dz2, 32, L.w[1], 32, nullptr, nullptr, 0, a1, 0, L.dz1, N, H, W, st)));
    // layer 1: a1 = relu(conv(x, w0) + b0)
    LBM_HIP_TRY(wgrad<4>(L.dz1, 32, x, s->cin, N, H, W, L.gpart, g->w[0], g->b[0], st));
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_cnn_adam(float *theta, float *m, float *v, const float *grad, int64_t count, float lr, float beta1,
                     float beta2, float eps, int64_t t, uint16_t *bf16_out, void *stream)
{
    if (!theta || !m || !v || !grad || count < 0 || t < 1)
        return fail(LBM_EINVAL, "invalid Adam arguments");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(LBM_EINVAL, "invalid Adam hyper-parameters");
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
    if (count > 0)
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, theta, m,
                           v, grad, count, lr, beta1, beta2, eps, bc1, bc2, bf16_out);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_channel_affine(float *x, int32_t n, int32_t c, int32_t nc, int64_t hw, const float *scale,
                           const float *shift, void *stream)
{
    if (!x || !scale || !shift || n < 0 || c < 1 || nc < 0 || nc > c || hw < 0)
        return fail(LBM_EINVAL, "invalid channel_affine arguments");
    const int64_t total = (int64_t)n * nc * hw;
    if (total > 0)
        hipLaunchKernelGGL(k_channel_affine, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           x, n, c, nc, hw, scale, shift);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_field_error(const float *a, const float *b, int32_t n, int32_t c, int32_t nc, int64_t hw, double *out,
                        void *stream)
{
    if (!a || !b || !out || n < 0 || c < 1 || nc < 1 || nc > c || hw < 1)
        return fail(LBM_EINVAL, "invalid field_error arguments");
    if (n > 0)
        hipLaunchKernelGGL(k_field_error, dim3(n), dim3(256), 0, (hipStream_t)stream, a, b, c, nc, hw, out);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

size_t lbm_channel_stats_workspace_bytes(int32_t c) { return c < 1 ? 0 : (size_t)c * kStatBlocks * sizeof(double); }

int32_t lbm_channel_stats(const float *x, int32_t n, int32_t c, int64_t hw, double *mean, double *stdev, void *ws,
                          size_t ws_bytes, void *stream)
{
    if (!x || !mean || !stdev || !ws || n < 1 || c < 1 || hw < 1)
        return fail(LBM_EINVAL, "invalid channel_stats arguments");
    if (ws_bytes < lbm_channel_stats_workspace_bytes(c))
        return fail(LBM_EINVAL, "workspace smaller than lbm_channel_stats_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    double *part = (double *)ws;
    const int64_t cnt = (int64_t)n * hw;
    hipLaunchKernelGGL(k_stat_partial, dim3(kStatBlocks, c), dim3(256), 0, st, x, n, c, hw, (const double *)nullptr,
                       part);
    hipLaunchKernelGGL(k_stat_final, dim3(c), dim3(256), 0, st, part, cnt, mean, 0);
    hipLaunchKernelGGL(k_stat_partial, dim3(kStatBlocks, c), dim3(256), 0, st, x, n, c, hw, (const double *)mean,
                       part);
    hipLaunchKernelGGL(k_stat_final, dim3(c), dim3(256), 0, st, part, cnt, stdev, 1);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_fill_channel(float *x, int32_t n, int32_t c, int32_t ch, int64_t hw, const float *values, void *stream)
{
    if (!x || !values || n < 0 || c < 1 || ch < 0 || ch >= c || hw < 1)
        return fail(LBM_EINVAL, "invalid fill_channel arguments");
    const int64_t total = (int64_t)n * hw;
    if (total > 0)
        hipLaunchKernelGGL(k_fill_channel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           x, n, c, ch, hw, values);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_coarsen(const lbm_params *p, const float *f, int32_t c, float *out, void *stream)
{
    int32_t rc = validate_params(p, p ? p->nx : 0);
    if (rc)
        return rc;
    if (!f || !out)
        return fail(LBM_EINVAL, "null pointer");
    if (p->lattice != LBM_D2Q7)
        return fail(LBM_EUNSUPPORTED, "coarse fields take the D2Q7 lattice");
    if (p->storage != LBM_F32)
        return fail(LBM_EUNSUPPORTED, "coarse fields take F32 storage");
    if (c < 1 || p->nx % c || p->ny % c || ((c & 1) && c != 1))
        return fail(LBM_EINVAL, "c must divide nx and ny and be 1 or even");
    if ((uint64_t)p->nx * p->ny * 7ull >= (1ull << 30))
        return fail(LBM_EINVAL, "lattice too large");
    const StepArgs a = make_step_args(*p, p->nx);
    const int cw = p->nx / c, chh = p->ny / c;
    hipLaunchKernelGGL(k_coarsen, dim3((cw + 255) / 256, chh), dim3(256), 0, (hipStream_t)stream, f, a,
                       c, cw, chh, out);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

static int32_t check_fields(const lbm_params *p, int32_t c)
{
    int32_t rc = validate_params(p, p ? p->nx : 0);
    if (rc)
        return rc;
    if (p->lattice != LBM_D2Q7)
        return fail(LBM_EUNSUPPORTED, "coarse fields take the D2Q7 lattice");
    if (p->storage != LBM_F32)
        return fail(LBM_EUNSUPPORTED, "coarse fields take F32 storage");
    if (c < 1 || p->nx % c || p->ny % c || ((c & 1) && c != 1))
        return fail(LBM_EINVAL, "c must divide nx and ny and be 1 or even");
    if ((uint64_t)p->nx * p->ny * 7ull >= (1ull << 30))
        return fail(LBM_EINVAL, "lattice too large");
    return LBM_OK;
}

int32_t lbm_coarsen_many(const lbm_params *p, int32_t n, const float *const *bufs, int32_t c, float *out,
                         int64_t out_stride, void *stream)
{
    int32_t rc = check_fields(p, c);
    if (rc)
        return rc;
    const int cw = p->nx / c, chh = p->ny / c;
    if (!bufs || !out || n < 0 || n > 65535 || out_stride < 3ll * cw * chh)
        return fail(LBM_EINVAL, "invalid coarsen_many arguments");
    const StepArgs a = make_step_args(*p, p->nx);
    if (n > 0)
        hipLaunchKernelGGL(k_coarsen_many, dim3((cw + 255) / 256, chh, n), dim3(256), 0, (hipStream_t)stream, bufs,
                           a, c, cw, chh, out, out_stride);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_lift_many(const lbm_params *p, int32_t n, const float *coarse, int64_t in_stride, int32_t c,
                      float *const *bufs, void *stream)
{
    int32_t rc = check_fields(p, c);
    if (rc)
        return rc;
    const int cw = p->nx / c, chh = p->ny / c;
    if (!bufs || !coarse || n < 0 || n > 65535 || in_stride < 3ll * cw * chh)
        return fail(LBM_EINVAL, "invalid lift_many arguments");
    const StepArgs a = make_step_args(*p, p->nx);
    if (n > 0)
        hipLaunchKernelGGL(k_lift_many, dim3((p->nx + 255) / 256, p->ny, n), dim3(256), 0, (hipStream_t)stream,
                           coarse, in_stride, a, c, cw, chh, bufs);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int32_t lbm_lift(const lbm_params *p, const float *coarse, int32_t c, float *f, void *stream)
{
    int32_t rc = validate_params(p, p ? p->nx : 0);
    if (rc)
        return rc;
    if (!f || !coarse)
        return fail(LBM_EINVAL, "null pointer");
    if (p->lattice != LBM_D2Q7)
        return fail(LBM_EUNSUPPORTED, "lifting takes the D2Q7 lattice");
    if (p->storage != LBM_F32)
        return fail(LBM_EUNSUPPORTED, "lifting writes F32 storage");
    if (c < 1 || p->nx % c || p->ny % c || ((c & 1) && c != 1))
        return fail(LBM_EINVAL, "c must divide nx and ny and be 1 or even");
    if ((uint64_t)p->nx * p->ny * 7ull >= (1ull << 30))
        return fail(LBM_EINVAL, "lattice too large");
    const StepArgs a = make_step_args(*p, p->nx);
    hipLaunchKernelGGL(k_lift, dim3((p->nx + 255) / 256, p->ny), dim3(256), 0, (hipStream_t)stream, coarse, a, c,
                       p->nx / c, p->ny / c, f);
    LBM_HIP_TRY(hipGetLastError());
    return LBM_OK;
}

}  // extern "C"
