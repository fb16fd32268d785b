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
// Convolutions (bf16 operands: the weights, and each activation split into
// three bf16 parts) and weight gradients (FP32 operands) are matrix products
// on the matrix cores over 16 x 8 pixel tiles staged in LDS with their halo.
// Reductions (weight gradients, loss) use fixed partitions and orders, so
// results are deterministic.
#include <math.h>

#include <algorithm>

#include "../../include/lbm_cnn.h"
#include "internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// 3x3 convolutions on the matrix cores, bf16 operands with float32
// accumulation (v_mfma_f32_32x32x16_bf16).  The weights are bf16 values
// already; each float32 activation x is split into three bf16 parts, x = h +
// m + l + r with |r| < 2^-24 |x| (h: x with its low 16 bits cleared, m and l
// the same of the exact remainders), and the product of each part with the
// weight is exact, so the three products together give the float32 product
// and only the order of the float32 sums differs from the definition.  A
// 16 x 8 pixel tile of one sample per block (four waves, one 32-pixel slab
// each: two image rows of 16), its input split and stored channel-last in
// LDS with the one-pixel circular halo, every channel at once (ci, co <= 32).
//
// Convolution as a matrix product per slab: D[pixel][o] = sum_k A[pixel][k]
// B[k][o], k = tap * CP + c (tap = 3 ky + kx, c < CP = ci rounded up to 16
// with zero channels), A the input at the pixel shifted by the tap, B[k][o]
// = wb[o][tap][c] (bf16).  TR = 0 weights: wb[o][tap][c] = w[o][c][tap]: y =
// b[o] + sum_c sum_tap w[o,c,tap] x[n,c,i+ky-1,j+kx-1].  The input gradient
// of a convolution whose weights are w[c][o][tap] takes wb[o][tap][c] =
// w[c][o][8 - tap], the transposed, flipped weights (both written by
// k_widen).  Epilogue in order: bias, ReLU, + resid[n, o] (first co channels
// of a tensor with resid_c channels), * (mask[n, o] > 0).
//
// MFMA 32x32x16 operand layout (per lane l of the wave): A row l mod 32 with
// k = 8 (l / 32) + j, j < 8; B column l mod 32, the same k; result register r
// holds row 8 (r / 4) + 4 (l / 32) + r mod 4 of column l mod 32.  Each step
// takes one tap and 16 channels, so a lane's eight A values (channels c0 +
// 8 (l / 32) ..) and eight B values are 16 contiguous bytes of LDS.
// ---------------------------------------------------------------------------
constexpr int kTW = 16, kTH = 8;                   // pixel tile
constexpr int kHW_ = kTW + 2, kHH = kTH + 2;       // with the halo
constexpr int kHalo = kHW_ * kHH;                  // 180 pixels
constexpr int kMaxC = 32;                          // channels

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// v in [-1, n + kHW_ - 2] wrapped into [0, n); SMALL: n may be smaller than
// the halo tile, so v may wrap more than once
template <bool SMALL>
__device__ __forceinline__ int wrap_index(int v, int n)
{
    if (SMALL)
        return (v + n) % n;
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// LDS staging with every global load of a thread in flight before the first
// LDS write: element e < count (count > 0) of the block's copy is get(e) (a
// load from an address that is valid for every e < count) stored by put(e).
template <int NT, int MAXE, class Get, class Put>
__device__ __forceinline__ void stage(int count, Get get, Put put)
{
    constexpr int U = (MAXE + NT - 1) / NT;
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        v[u] = get(min((int)threadIdx.x + u * NT, count - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = threadIdx.x + u * NT;
        if (e < count)
            put(e, v[u]);
    }
}

// element e = c * kHalo + hy * kHW_ + hx of the input tile of sample n with
// its circular halo (0 for c >= ci_n); offsets within a sample fit 32 bits
// (ci h w < 2^31)
template <bool SMALL>
__device__ __forceinline__ float halo_value(const float *__restrict__ xn, int ci_n, int H, int W, int i0, int j0, int e)
{
    const int c = e / kHalo, r = e - c * kHalo, hy = r / kHW_, hx = r - hy * kHW_;
    const int gi = wrap_index<SMALL>(i0 + hy - 1, H), gj = wrap_index<SMALL>(j0 + hx - 1, W);
    const float v = xn[(unsigned)min(c, ci_n - 1) * (unsigned)H * (unsigned)W + (unsigned)gi * (unsigned)W + (unsigned)gj];
    return c < ci_n ? v : 0.0f;
}

// the input tile as float32, s[c][hy][hx], c < cpad <= MAXC (halo values of
// pixels outside the field feed no output)
template <int NT, int MAXC>
__device__ __forceinline__ void stage_halo(const float *__restrict__ x, int n, int ci_n, int cpad, int H, int W, int i0,
                                           int j0, float *s)
{
    const float *xn = x + (size_t)n * ci_n * H * W;
    auto put = [&](int e, float v) { s[e] = v; };
    if (H >= kHH && W >= kHW_)
        stage<NT, MAXC * kHalo>(cpad * kHalo, [&](int e) { return halo_value<false>(xn, ci_n, H, W, i0, j0, e); }, put);
    else
        stage<NT, MAXC * kHalo>(cpad * kHalo, [&](int e) { return halo_value<true>(xn, ci_n, H, W, i0, j0, e); }, put);
}

// the three bf16 parts of x (bit patterns): x = h + m + l + r, |r| < 2^-24 |x|
__device__ __forceinline__ void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l)
{
    const uint32_t hb = __float_as_uint(x) & 0xffff0000u;
    const float r1 = x - __uint_as_float(hb);  // exact: the low 16 bits of x
    const uint32_t mb = __float_as_uint(r1) & 0xffff0000u;
    const float r2 = r1 - __uint_as_float(mb);  // exact
    h = (uint16_t)(hb >> 16);
    m = (uint16_t)(mb >> 16);
    l = (uint16_t)(__float_as_uint(r2) >> 16);
}

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// CP: input channels rounded up to 16 (16 or 32).
template <int CP>
__global__ __launch_bounds__(256) void k_conv3x3(const float *__restrict__ x, int ci_n, const uint16_t *__restrict__ wb,
                                                 int co_n, const float *__restrict__ bias,
                                                 const float *__restrict__ resid, int resid_c,
                                                 const float *__restrict__ mask, int relu, float *__restrict__ y,
                                                 int H, int W)
{
    // strides (bf16 elements) padded so that eight consecutive lanes' 16-byte
    // reads fall in distinct banks
    constexpr int CPS = CP + 8, WS = 9 * CP + 8;
    __shared__ __attribute__((aligned(16))) uint16_t s_x[3 * kHalo * CPS];  // [part][pixel][channel]
    __shared__ __attribute__((aligned(16))) uint16_t s_w[kMaxC * WS];      // [out][tap][channel]
    const int n = blockIdx.z, i0 = blockIdx.y * kTH, j0 = blockIdx.x * kTW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    {
        const float *xn = x + (size_t)n * ci_n * H * W;
        auto put = [&](int e, float v) {
            const int c = e / kHalo, pix = e - c * kHalo;
            uint16_t h, m, l;
            split3(v, h, m, l);
            s_x[pix * CPS + c] = h;
            s_x[(kHalo + pix) * CPS + c] = m;
            s_x[(2 * kHalo + pix) * CPS + c] = l;
        };
        if (H >= kHH && W >= kHW_)
            stage<256, CP * kHalo>(CP * kHalo, [&](int e) { return halo_value<false>(xn, ci_n, H, W, i0, j0, e); },
                                   put);
        else
            stage<256, CP * kHalo>(CP * kHalo, [&](int e) { return halo_value<true>(xn, ci_n, H, W, i0, j0, e); },
                                   put);
    }
    // B: rows o < co_n of wb (9 CP bf16 each, 16-byte pieces), zero rows after
    {
        constexpr int RQ = 9 * CP / 8;  // 16-byte pieces per row
        const uint4 *src = (const uint4 *)wb;
        for (int e = threadIdx.x; e < kMaxC * RQ; e += 256) {
            const int o = e / RQ, q = e - o * RQ;
            const uint4 v = o < co_n ? src[(size_t)o * RQ + q] : make_uint4(0u, 0u, 0u, 0u);
            *(uint4 *)(s_w + o * WS + q * 8) = v;
        }
    }
    __syncthreads();
    const int m = lane & 31, hk = lane >> 5;        // A row (pixel of the slab) / B column, k half
    const int pr = 2 * wv + (m >> 4), pc = m & 15;  // tile row and column of the A row's pixel
    const uint16_t *pa = s_x + (pr * kHW_ + pc) * CPS + 8 * hk;
    const uint16_t *pb = s_w + m * WS + 8 * hk;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r)
        acc[r] = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
        for (int c0 = 0; c0 < CP; c0 += 16) {
            const bf16x8 b = *(const bf16x8 *)(pb + t * CP + c0);
            const int off = ((t / 3) * kHW_ + t % 3) * CPS + c0;
#pragma unroll
            for (int part = 0; part < 3; ++part)
                acc = mfma_bf16(*(const bf16x8 *)(pa + part * kHalo * CPS + off), b, acc);
        }
    }
    // lane: output channel o = m; register group g holds the four pixels
    // 8 g + 4 hk .. + 3 of the slab, one image row, consecutive columns
    const int o = m;
    if (o >= co_n)
        return;
    const size_t HW = (size_t)H * W;
    const float bo = bias ? bias[o] : 0.0f;
    float *yo = y + ((size_t)n * co_n + o) * HW;
    const float *ro = resid ? resid + ((size_t)n * resid_c + o) * HW : nullptr;
    const float *mo = mask ? mask + ((size_t)n * co_n + o) * HW : nullptr;
    if ((W & 3) == 0) {
        // four 16-byte groups (j + 3 < W whenever j < W); the residual and
        // mask loads of all groups are issued before the first use
        size_t pix[4];
        bool ok[4];
        float4 rq[4], mq[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int i = i0 + 2 * wv + (g >> 1), j = j0 + 8 * (g & 1) + 4 * hk;
            ok[g] = i < H && j < W;
            pix[g] = ok[g] ? (size_t)i * W + j : 0;
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            rq[g] = ro ? *(const float4 *)(ro + pix[g]) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            mq[g] = mo ? *(const float4 *)(mo + pix[g]) : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = acc[4 * g + u] + bo;
                if (relu)
                    v[u] = fmaxf(v[u], 0.0f);
            }
            if (ro)
                v[0] += rq[g].x, v[1] += rq[g].y, v[2] += rq[g].z, v[3] += rq[g].w;
            if (mo) {
                v[0] = mq[g].x > 0.0f ? v[0] : 0.0f, v[1] = mq[g].y > 0.0f ? v[1] : 0.0f;
                v[2] = mq[g].z > 0.0f ? v[2] : 0.0f, v[3] = mq[g].w > 0.0f ? v[3] : 0.0f;
            }
            if (ok[g])
                *(float4 *)(yo + pix[g]) = make_float4(v[0], v[1], v[2], v[3]);
        }
        return;
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int i = i0 + 2 * wv + (g >> 1), j = j0 + 8 * (g & 1) + 4 * hk;
        if (i >= H || j >= W)
            continue;
        const size_t pix = (size_t)i * W + j;
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = acc[4 * g + u] + bo;
            if (relu)
                v[u] = fmaxf(v[u], 0.0f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j + u >= W)
                break;
            float w = v[u];
            if (ro)
                w += ro[pix + u];
            if (mo)
                w = mo[pix + u] > 0.0f ? w : 0.0f;
            yo[pix + u] = w;
        }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dw[o,c,tap] = sum_{n,i,j} dy[n,o,i,j]
// x[n,c,i+ky-1,j+kx-1], db[o] = sum dy[n,o,i,j].  One block per (sample,
// 16 x 8 tile) writes its partial sums to part[block][co_n ci_n 9 + co_n];
// k_grad_reduce adds the blocks in order in float64.  Per block a matrix
// product on the matrix cores (v_mfma_f32_16x16x4_f32): D[o][k] = sum_p
// A[o][p] B[p][k], p the tile's 128 pixels in groups of four neighbours
// (lane group q = l / 16 takes pixel 4 s + q of step s), k = c * 9 + tap.
// The output is cut into 16 x 16 blocks (rows o, columns k), dealt to the
// four waves in turn; the bias sums are per-row wave reductions of the dy
// tile in a fixed order.
//
// 16x16x4 operand layout (lane l): A row l mod 16, k = l / 16; B column
// l mod 16, k = l / 16; result register r holds row 4 (l / 16) + r of
// column l mod 16.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cwave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWgWaves = 4;

__global__ __launch_bounds__(64 * kWgWaves) void k_conv3x3_wgrad(const float *__restrict__ dy, int co_n,
                                                                 const float *__restrict__ x, int ci_n, int H, int W,
                                                                 float *__restrict__ part)
{
    constexpr int NT = 64 * kWgWaves, NP = kTW * kTH, DS = NP + 1;  // threads, pixels, dy row stride
    __shared__ float s_x[kMaxC * kHalo];
    __shared__ float s_d[kMaxC * DS];  // dy tile [o][p] (rows o >= co_n zero; pixels outside the field zero)
    const int tiles_j = (W + kTW - 1) / kTW, tiles_i = (H + kTH - 1) / kTH;
    const int n = blockIdx.x / (tiles_i * tiles_j), tt = blockIdx.x - n * (tiles_i * tiles_j);
    const int ti = tt / tiles_j;
    const int i0 = ti * kTH, j0 = (tt - ti * tiles_j) * kTW;
    const size_t HW = (size_t)H * W;
    stage_halo<NT, kMaxC>(x, n, ci_n, ci_n, H, W, i0, j0, s_x);
    const float *dyn = dy + (size_t)n * co_n * HW;
    stage<NT, kMaxC * NP>(
        kMaxC * NP,
        [&](int e) {
            const int o = e / NP, pq = e - o * NP, gi = i0 + pq / kTW, gj = j0 + pq % kTW;
            const bool ok = o < co_n && gi < H && gj < W;
            const float v = dyn[ok ? (size_t)o * HW + (size_t)gi * W + gj : 0];
            return ok ? v : 0.0f;
        },
        [&](int e, float v) { s_d[(e / NP) * DS + e % NP] = v; });
    __syncthreads();
    const int K = ci_n * 9, nw = co_n * K;
    float *out = part + (size_t)blockIdx.x * (nw + co_n);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, q = lane >> 4;
    const int nrb = (co_n + 15) >> 4, ncb = (K + 15) >> 4;
    for (int tb = wv; tb < nrb * ncb; tb += kWgWaves) {
        const int rb = tb / ncb, cb = tb - rb * ncb;
        const int col = cb * 16 + l16;  // this lane's B column k
        const int cc = col < K ? col / 9 : 0, t = col < K ? col - cc * 9 : 0, ty = t / 3, tx = t - ty * 3;
        const float *pa = s_d + (rb * 16 + l16) * DS + q;
        const float *pb = s_x + cc * kHalo + ty * kHW_ + tx + q;
        // all of the block's operands first, then the products
        float av[NP / 4], bv[NP / 4];
#pragma unroll
        for (int s4 = 0; s4 < NP / 4; ++s4) {  // pixel 4 s4 + q: row s4 / 4, column 4 s4 mod 16 + q
            av[s4] = pa[4 * s4];
            bv[s4] = pb[(s4 >> 2) * kHW_ + ((4 * s4) & 15)];
        }
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s4 = 0; s4 < NP / 4; ++s4)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s4], bv[s4], acc, 0, 0, 0);
        if (col < K) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = rb * 16 + 4 * q + r;
                if (o < co_n)
                    out[(size_t)o * K + col] = acc[r];
            }
        }
    }
    // bias: wave w takes rows w, w + 4, ...; lane l adds pixels l and l + 64,
    // then a fixed butterfly over the wave
    for (int o = wv; o < co_n; o += kWgWaves) {
        float v = s_d[o * DS + lane] + s_d[o * DS + lane + 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            v += __shfl_xor(v, off, 64);
        if (lane == 0)
            out[nw + o] = v;
    }
}

// g[e] = the sum over blocks b of part[b][e] (float64); e < nw goes to the
// weight gradient, e >= nw to the bias gradient.  A block takes kReduceCols
// entries with 256 / kReduceCols threads each: thread slice s adds blocks s,
// s + slices, ... in order, then the slices are added in order.
constexpr int kReduceCols = 16, kReduceSlices = 256 / kReduceCols;

__global__ __launch_bounds__(256) void k_grad_reduce(const float *__restrict__ part, int nblocks, int nw, int nb,
                                                     float *__restrict__ gw, float *__restrict__ gb)
{
    __shared__ double s_sum[kReduceSlices][kReduceCols];
    const int col = threadIdx.x % kReduceCols, slice = threadIdx.x / kReduceCols;
    const int e = blockIdx.x * kReduceCols + col;
    const size_t stride = (size_t)(nw + nb);
    double sum = 0.0;
    if (e < nw + nb) {
        const float *p = part + e;
        int b = slice;
        constexpr int U = 8;  // loads in flight per thread; the additions stay in block order
        for (; b + (U - 1) * kReduceSlices < nblocks; b += U * kReduceSlices) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = p[(size_t)(b + u * kReduceSlices) * stride];
#pragma unroll
            for (int u = 0; u < U; ++u)
                sum += (double)v[u];
        }
        for (; b < nblocks; b += kReduceSlices)
            sum += (double)p[(size_t)b * stride];
    }
    s_sum[slice][col] = sum;
    __syncthreads();
    if (slice == 0 && e < nw + nb) {
        double t = s_sum[0][col];
        for (int k = 1; k < kReduceSlices; ++k)
            t += s_sum[k][col];
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

// bf16 weights -> the B layout of a convolution, out[o][tap][c] (c < cp, zero
// for c >= ci), up to three tensors per launch (blockIdx.y).  tr = 0: the
// convolution's own weights w[o][c][tap]; tr = 1: the input gradient of a
// convolution whose weights are w[c][o][tap], out[o][tap][c] = w[c][o][8 -
// tap].
struct WidenJobs {
    const uint16_t *w[3];
    uint16_t *out[3];
    int co[3], ci[3], cp[3], tr[3];
};

__global__ void k_widen(WidenJobs j)
{
    const int q = blockIdx.y, co = j.co[q], ci = j.ci[q], cp = j.cp[q];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= co * 9 * cp)
        return;
    const int o = e / (9 * cp), r = e - o * (9 * cp), t = r / cp, c = r - t * cp;
    uint16_t v = 0;
    if (c < ci)
        v = j.tr[q] ? j.w[q][(c * co + o) * 9 + (8 - t)] : j.w[q][(o * ci + c) * 9 + t];
    j.out[q][e] = v;
}

// Adam (Kingma & Ba, algorithm 1) on float32 master tensors, up to kAdamMax
// of them in one launch (blockIdx.y selects the tensor; every tensor has its
// own moments and gradient); writes the bf16 copy where one is given.
__global__ void k_adam_many(AdamJobs j, float lr, float beta1, float beta2, float eps, float bc1, float bc2)
{
    const int q = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= j.count[q])
        return;
    float *theta = j.theta[q], *m = j.m[q], *v = j.v[q];
    const float gi = j.g[q][e];
    const float mi = beta1 * m[e] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[e] + (1.0f - beta2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float th = theta[e] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    theta[e] = th;
    if (j.bf16[q])
        j.bf16[q][e] = float_to_bf16_rne(th);
}

hipError_t launch_adam_many(const AdamJobs &j, int n, float lr, float beta1, float beta2, float eps, int64_t t,
                            hipStream_t s)
{
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
    int64_t most = 0;
    for (int q = 0; q < n; ++q)
        most = std::max(most, j.count[q]);
    if (n > 0 && most > 0)
        hipLaunchKernelGGL(k_adam_many, dim3((unsigned)((most + 255) / 256), n), dim3(256), 0, s, j, lr, beta1, beta2,
                           eps, bc1, bc2);
    return hipGetLastError();
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
static bool shape_ok(const lbm_cnn_shape *s)
{
    return s && s->n > 0 && s->h > 0 && s->w > 0 && s->hidden == 32 && s->cout == 3 && s->cin >= 3 &&
           s->cin <= 32 && (int64_t)s->h * s->w <= (1 << 26) && s->n <= 65535;
}

static int pad16(int c) { return c <= 16 ? 16 : 32; }

// wb: bf16 weights in the B layout [co][9][pad16(ci)] (k_widen)
static hipError_t conv(const float *x, int ci, const uint16_t *wb, int co, const float *b, const float *resid,
                       int resid_c, const float *mask, int relu, float *y, int N, int H, int W, hipStream_t s)
{
    dim3 grd((W + kTW - 1) / kTW, (H + kTH - 1) / kTH, N);
    if (pad16(ci) == 16)
        hipLaunchKernelGGL(k_conv3x3<16>, grd, dim3(256), 0, s, x, ci, wb, co, b, resid, resid_c, mask, relu, y, H, W);
    else
        hipLaunchKernelGGL(k_conv3x3<32>, grd, dim3(256), 0, s, x, ci, wb, co, b, resid, resid_c, mask, relu, y, H, W);
    return hipGetLastError();
}

static int conv_tiles(int H, int W) { return ((H + kTH - 1) / kTH) * ((W + kTW - 1) / kTW); }

// Weight and bias gradients of one layer (co output, ci input channels):
// per-tile partials, then their ordered sum.
static hipError_t wgrad(const float *dy, int co, const float *x, int ci, int N, int H, int W, float *part, float *gw,
                        float *gb, hipStream_t s)
{
    const int blocks = N * conv_tiles(H, W);
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(blocks), dim3(64 * kWgWaves), 0, s, dy, co, x, ci, H, W, part);
    const int total = co * ci * 9 + co;
    hipLaunchKernelGGL(k_grad_reduce, dim3((total + kReduceCols - 1) / kReduceCols), dim3(256), 0, s, part, blocks,
                       co * ci * 9, co, gw, gb);
    return hipGetLastError();
}

struct CnnWs {
    uint16_t *wb[3];   // the layers' weights in the convolutions' B layout [co][9][pad16(ci)]
    uint16_t *wbt[3];  // the input-gradient convolutions' weights (layers 2 and 3)
    double *part;      // loss partials
    float *gpart;      // per-tile gradient partials
    float *dy;         // dL/dy [n][cout][hw]
    float *dz2;        // [n][hidden][hw]
    float *dz1;        // [n][hidden][hw]
    size_t total;
};

static const int kMseBlocks = 1024;

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace: the weights in the B layout, loss partials and the backward
// pass's intermediate gradients.  base == nullptr only measures the size.
static CnnWs cnn_layout(const lbm_cnn_shape *s, char *base)
{
    CnnWs L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return base ? base + o : nullptr;
    };
    const int64_t hw = (int64_t)s->h * s->w;
    const int co[3] = {s->hidden, s->hidden, s->cout}, ci[3] = {s->cin, s->hidden, s->hidden};
    for (int k = 0; k < 3; ++k)
        L.wb[k] = (uint16_t *)take((size_t)co[k] * 9 * pad16(ci[k]) * sizeof(uint16_t));
    for (int k = 1; k < 3; ++k)
        L.wbt[k] = (uint16_t *)take((size_t)ci[k] * 9 * pad16(co[k]) * sizeof(uint16_t));
    L.part = (double *)take(kMseBlocks * sizeof(double));
    // per-tile partials of the largest layer (hidden x max(hidden, cin) weights)
    L.gpart = (float *)take((size_t)s->n * conv_tiles(s->h, s->w) *
                            (size_t)(s->hidden * std::max(s->hidden, s->cin) * 9 + s->hidden) * sizeof(float));
    L.dy = (float *)take((size_t)s->n * s->cout * hw * sizeof(float));
    L.dz2 = (float *)take((size_t)s->n * s->hidden * hw * sizeof(float));
    L.dz1 = (float *)take((size_t)s->n * s->hidden * hw * sizeof(float));
    L.total = off;
    return L;
}

// forward: the three layers' convolutions; backward: the input-gradient
// convolutions of layers 2 and 3 (their output channels are the layer's
// inputs)
static hipError_t widen(const lbm_cnn_shape *s, const lbm_cnn_params *p, const CnnWs &L, bool backward,
                        hipStream_t st)
{
    const int co[3] = {s->hidden, s->hidden, s->cout}, ci[3] = {s->cin, s->hidden, s->hidden};
    WidenJobs j{};
    int nj = 0, most = 0;
    for (int k = backward ? 1 : 0; k < 3; ++k, ++nj) {
        j.w[nj] = p->w[k];
        j.out[nj] = backward ? L.wbt[k] : L.wb[k];
        j.co[nj] = backward ? ci[k] : co[k];
        j.ci[nj] = backward ? co[k] : ci[k];
        j.cp[nj] = pad16(j.ci[nj]);
        j.tr[nj] = backward;
        most = std::max(most, j.co[nj] * 9 * j.cp[nj]);
    }
    hipLaunchKernelGGL(k_widen, dim3((most + 255) / 256, nj), dim3(256), 0, st, j);
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
    LBM_HIP_TRY(widen(s, p, L, false, st));
    LBM_HIP_TRY(conv(x, s->cin, L.wb[0], 32, p->b[0], nullptr, 0, nullptr, 1, a1, s->n, s->h, s->w, st));
    LBM_HIP_TRY(conv(a1, 32, L.wb[1], 32, p->b[1], nullptr, 0, nullptr, 1, a2, s->n, s->h, s->w, st));
    LBM_HIP_TRY(conv(a2, 32, L.wb[2], 3, p->b[2], x, s->cin, nullptr, 0, y, s->n, s->h, s->w, st));
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
    LBM_HIP_TRY(widen(s, p, L, true, st));
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, st, y, target, count, L.dy, L.part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, L.part, kMseBlocks, count, loss);
    // layer 3: y = x[:cout] + conv(a2, w2) + b2
    LBM_HIP_TRY(wgrad(L.dy, s->cout, a2, 32, N, H, W, L.gpart, g->w[2], g->b[2], st));
    LBM_HIP_TRY(conv(L.dy, s->cout, L.wbt[2], 32, nullptr, nullptr, 0, a2, 0, L.dz2, N, H, W, st));
    // layer 2: a2 = relu(conv(a1, w1) + b1)
    LBM_HIP_TRY(wgrad(L.dz2, 32, a1, 32, N, H, W, L.gpart, g->w[1], g->b[1], st));
    LBM_HIP_TRY(conv(L.dz2, 32, L.wbt[1], 32, nullptr, nullptr, 0, a1, 0, L.dz1, N, H, W, st));
    // layer 1: a1 = relu(conv(x, w0) + b0)
    LBM_HIP_TRY(wgrad(L.dz1, 32, x, s->cin, N, H, W, L.gpart, g->w[0], g->b[0], st));
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
    AdamJobs j{};
    j.theta[0] = theta;
    j.m[0] = m;
    j.v[0] = v;
    j.g[0] = grad;
    j.count[0] = count;
    j.bf16[0] = bf16_out;
    LBM_HIP_TRY(launch_adam_many(j, 1, lr, beta1, beta2, eps, t, (hipStream_t)stream));
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
