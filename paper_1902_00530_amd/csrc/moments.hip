// Fields and FP64 observables of the stored state, taken (like step (ii) of
// the algorithm) on its streamed populations: rho, u (eq.
// D2Q7macroscopic_u_disc), the order parameter phi (eq. phi), the mean speed,
// zeta and the banding measure (standard deviation over x of the y-averaged
// density), section "Regime Categorisation in the phase diagram".
//
// Pass 1: each block covers 256 columns x kRowsPerBlock rows; lanes hold
// FP64 sums, reduced across the wavefront with shuffles and across the block
// through LDS, one partial per block; per-column density sums go to a
// [row-block][nx] array.  Pass 2 sums each column over the row blocks (one
// thread per column) and pass 3 (one block) adds the block partials and the
// column means in a fixed order, so the result does not depend on
// scheduling.
#include "device_q9.h"
#include "internal.h"

namespace lbm {

constexpr int kMomBX = 256;
constexpr int kRowsPerBlock = 16;
constexpr int kNPart = 5;  // M, Jx, Jy, sum|j|, nonfinite

static int mom_grid_x(const lbm_params &p) { return (p.nx + kMomBX - 1) / kMomBX; }
static int mom_grid_y(const lbm_params &p) { return (p.ny + kRowsPerBlock - 1) / kRowsPerBlock; }

size_t moments_scratch_doubles(const lbm_params &p)
{
    const size_t blocks = (size_t)mom_grid_x(p) * mom_grid_y(p);
    return blocks * kNPart + (size_t)mom_grid_y(p) * p.nx + (size_t)p.nx;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Block-wide sum of kNPart doubles, fixed order; result valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double v[N], double (*lds)[N])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k)
            lds[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < N; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w)
                s += lds[w][k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// The streamed populations of site (x, y) and their rho, j and finiteness,
// on the triangular (Q = 7) or the square (Q = 9) lattice.
template <int S, int Q>
__device__ __forceinline__ void gathered_moments(const typename Store<S>::T *src, const StepArgs &a, int x, int y,
                                                 float &rho, float &jx, float &jy, bool &finite)
{
    float f[Q];
    if constexpr (Q == 7) {
        const PullSources g_src = pull_sources(a, x, y);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            f[i] = Planes<S>::ld(src, g_src.idx[i], i, a.plane, a);
        site_moments(f, rho, jx, jy);
    } else {
        const Q9Sources g_src = q9_sources(a, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = Store<S>::load(src, i * a.plane + g_src.idx[i], q9_wr(a, i));
        q9_moments(f, rho, jx, jy);
    }
    finite = true;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        finite = finite && isfinite(f[i]);
}

template <int S, int Q>
__global__ __launch_bounds__(kMomBX) void k_moments(const typename Store<S>::T *__restrict__ src, StepArgs a,
                                                    float *__restrict__ rho_out, float *__restrict__ ux_out,
                                                    float *__restrict__ uy_out, double *__restrict__ part,
                                                    double *__restrict__ colpart)
{
    __shared__ double lds[kMomBX / 64][kNPart];
    const int x = blockIdx.x * kMomBX + threadIdx.x;
    const int yb = blockIdx.y * kRowsPerBlock;
    double acc[kNPart] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double col = 0.0;
    if (x < a.nx) {
        const int ye = min(yb + kRowsPerBlock, a.ny);
        for (int y = yb; y < ye; ++y) {
            float rho, jx, jy;
            bool finite;
            gathered_moments<S, Q>(src, a, x, y, rho, jx, jy, finite);
            const double dr = rho, dx = jx, dy = jy;
            acc[0] += dr;
            acc[1] += dx;
            acc[2] += dy;
            acc[3] += sqrt(dx * dx + dy * dy);
            acc[4] += finite ? 0.0 : 1.0;
            col += dr;
            const int64_t o = (int64_t)y * a.nx + x;
            if (rho_out)
                rho_out[o] = rho;
            if (ux_out)
                ux_out[o] = rho != 0.0f ? jx / rho : 0.0f;
            if (uy_out)
                uy_out[o] = rho != 0.0f ? jy / rho : 0.0f;
        }
        colpart[(int64_t)blockIdx.y * a.nx + x] = col;
    }
    block_sum<kNPart>(acc, lds);
    if (threadIdx.x == 0) {
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
        for (int k = 0; k < kNPart; ++k)
            part[b * kNPart + k] = acc[k];
    }
}

// Column means rho_y(x): one thread per column, row blocks in order.
__global__ __launch_bounds__(256) void k_column_means(const double *__restrict__ colpart, int nrowblocks,
                                                      double *__restrict__ colmean, int nx, int ny)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx)
        return;
    double c = 0.0;
#pragma unroll 16
    for (int r = 0; r < nrowblocks; ++r)
        c += colpart[(int64_t)r * nx + x];
    colmean[x] = c / (double)ny;
}

// One block: fixed-order totals of the block partials and of the column
// means, then the variance of the column means over x.
__global__ __launch_bounds__(256) void k_moments_final(const double *__restrict__ part, int nblocks,
                                                       const double *__restrict__ colmean, int nx,
                                                       double *__restrict__ result)
{
    __shared__ double lds[4][kNPart + 1];
    double v[kNPart + 1] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < kNPart; ++k)
            v[k] += part[(int64_t)b * kNPart + k];
    for (int x = threadIdx.x; x < nx; x += blockDim.x)
        v[kNPart] += colmean[x];
    block_sum<kNPart + 1>(v, lds);
    __shared__ double mean_s;
    if (threadIdx.x == 0)
        mean_s = v[kNPart] / (double)nx;
    __syncthreads();
    const double mean = mean_s;
    double q[1] = {0.0};
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        const double d = colmean[x] - mean;
        q[0] += d * d;
    }
    __shared__ double lds1[4][1];
    block_sum<1>(q, lds1);
    if (threadIdx.x == 0) {
        for (int k = 0; k < kNPart; ++k)
            result[k] = v[k];
        result[5] = mean;
        result[6] = q[0] / (double)nx;
        result[7] = 0.0;
    }
}

hipError_t launch_moments(const lbm_params &p, const StepArgs &a, const void *src, float *rho, float *ux,
                          float *uy, double *scratch, double *result, hipStream_t s)
{
    const int gx = mom_grid_x(p), gy = mom_grid_y(p);
    double *part = scratch;
    double *colpart = part + (size_t)gx * gy * kNPart;
    double *colmean = colpart + (size_t)gy * p.nx;
    dim3 grd(gx, gy), blk(kMomBX);
    const bool q9 = p.lattice == LBM_D2Q9;
    switch (p.storage) {
    case kF32:
        if (q9)
            hipLaunchKernelGGL((k_moments<kF32, 9>), grd, blk, 0, s, (const float *)src, a, rho, ux, uy, part, colpart);
        else
            hipLaunchKernelGGL((k_moments<kF32, 7>), grd, blk, 0, s, (const float *)src, a, rho, ux, uy, part, colpart);
        break;
    case kBf16Dev:
        if (q9)
            hipLaunchKernelGGL((k_moments<kBf16Dev, 9>), grd, blk, 0, s, (const uint16_t *)src, a, rho, ux, uy, part,
                               colpart);
        else
            hipLaunchKernelGGL((k_moments<kBf16Dev, 7>), grd, blk, 0, s, (const uint16_t *)src, a, rho, ux, uy, part,
                               colpart);
        break;
    case kF16Dev:
        if (q9)
            hipLaunchKernelGGL((k_moments<kF16Dev, 9>), grd, blk, 0, s, (const _Float16 *)src, a, rho, ux, uy, part,
                               colpart);
        else
            hipLaunchKernelGGL((k_moments<kF16Dev, 7>), grd, blk, 0, s, (const _Float16 *)src, a, rho, ux, uy, part,
                               colpart);
        break;
    case kBf16R32:
        if (q9)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_moments<kBf16R32, 7>), grd, blk, 0, s, (const uint16_t *)src, a, rho, ux, uy, part,
                           colpart);
        break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_column_means, dim3((p.nx + 255) / 256), dim3(256), 0, s, colpart, gy, colmean, p.nx, p.ny);
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(256), 0, s, part, gx * gy, colmean, p.nx, result);
    return hipGetLastError();
}

void finish_obs(const lbm_params &p, const double *r, int64_t step, lbm_obs *o)
{
    o->step = step;
    o->M = r[0];
    o->Jx = r[1];
    o->Jy = r[2];
    o->phi = r[0] != 0.0 ? sqrt(r[1] * r[1] + r[2] * r[2]) / r[0] : 0.0;
    o->mean_speed = r[0] != 0.0 ? r[3] / r[0] : 0.0;
    o->zeta = r[0] != 0.0 ? p.B - r[3] / r[0] : 0.0;
    o->drho = sqrt(r[6]);
    o->nonfinite = (int64_t)r[4];
}

}  // namespace lbm
