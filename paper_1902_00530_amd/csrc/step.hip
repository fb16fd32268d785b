// Fused per-site step of the modified D2Q7 lattice Boltzmann method on
// gfx950, in the order of the algorithm of the appendix "Summary of modified
// lattice Boltzmann model algorithm": (i) stream by gathering population i of
// site r from r - e_i in the source buffer, (ii) rho and j, (iii) the target
// velocity u* and xi(rho, u*), (iv) BGK relaxation, (v) zero-sum noise,
// (vi) negative correction; the seven results are stored at r in the other
// buffer.
//
// The step is bandwidth-bound (7 loads + 7 stores per site, ~100 flops and
// one Philox call), so there is no matrix-core work.  Streaming is a gather
// (x-shifted loads, aligned stores): on MI355X a wavefront's shifted loads
// merge in L2 at no HBM cost, whereas shifted stores leave partial cache
// lines at tile edges, measured 7% slower at 4096^2.
#include "internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Passive and CIL: u* depends on the site alone.  A block is a BX x BY tile
// (BX a multiple of 64 so each wavefront covers 64 consecutive x of one row);
// the grid is laid out in row groups so each row of tiles runs on one XCD.
// Offsets are 32-bit element indices from per-plane base pointers.
// ---------------------------------------------------------------------------
template <int M, int S, int F, int CP>
__global__ __launch_bounds__(256) void k_step_local(const typename Store<S>::T *__restrict__ src,
                                                    typename Store<S>::T *__restrict__ dst, StepArgs a,
                                                    StepClock *__restrict__ clk, int slot)
{
    const uint64_t tt = clock_read(clk, slot);
    const uint32_t t_lo = (uint32_t)(tt & 0xffffffffu), t_hi = (uint32_t)(tt >> 32);
    int txi, tyi;
    row_group_tile(txi, tyi);
    const int x = txi * blockDim.x + threadIdx.x;
    const int y = tyi * blockDim.y + threadIdx.y;
    if (x >= a.nx || y >= a.ny)
        return;
    const uint32_t plane = (uint32_t)a.plane;
    const uint32_t bytes = (uint32_t)Planes<S>::bytes(plane);  // < 2^32: 7 planes < 2^30 elements
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(src, bytes), rd = buffer_rsrc(dst, bytes);
    const PullSources32 g_src = pull_sources32(a, x, y);
    float f[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        f[i] = Planes<S>::load(rs, g_src.idx[i], 0u, i, plane, a);
    float rho, jx, jy, ux, uy;
    site_moments(f, rho, jx, jy);
    local_ustar<M>(a, rho, jx, jy, ux, uy);
    site_collide<F, S>(a, f, rho, ux, uy, (uint32_t)y * (uint32_t)a.nx + (uint32_t)x, t_lo, t_hi);
    const uint32_t own = g_src.idx[0];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        Planes<S>::template store<CP>(rd, own, 0u, i, plane, f[i], a);
    clock_advance(clk, slot, tt);
}

// Same body with 64-bit offsets, for buffers of 2^30 elements per plane set
// or more.
template <int M, int S, int F>
__global__ __launch_bounds__(256) void k_step_local64(const typename Store<S>::T *__restrict__ src,
                                                      typename Store<S>::T *__restrict__ dst, StepArgs a,
                                                      StepClock *__restrict__ clk, int slot)
{
    const uint64_t tt = clock_read(clk, slot);
    const uint32_t t_lo = (uint32_t)(tt & 0xffffffffu), t_hi = (uint32_t)(tt >> 32);
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= a.nx || y >= a.ny)
        return;
    const PullSources g_src = pull_sources(a, x, y);
    float f[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        f[i] = Planes<S>::ld(src, g_src.idx[i], i, a.plane, a);
    float rho, jx, jy, ux, uy;
    site_moments(f, rho, jx, jy);
    local_ustar<M>(a, rho, jx, jy, ux, uy);
    site_collide<F, S>(a, f, rho, ux, uy, (uint32_t)y * (uint32_t)a.nx + (uint32_t)x, t_lo, t_hi);
    const int64_t own = g_src.idx[0];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        Planes<S>::st(dst, own, i, a.plane, f[i], a);
    clock_advance(clk, slot, tt);
}

// ---------------------------------------------------------------------------
// MIPS with 64-bit offsets (lattices of 2^30 elements per plane set or more):
// a 64 x 4 tile stages rho of the tile plus a one-site ring in LDS; ring sites
// gather their seven streamed populations themselves (served from L2).  Every
// LDS slot holds rho at its periodically wrapped lattice site.
// ---------------------------------------------------------------------------
constexpr int kMipsTX = 64, kMipsTY = 4;

template <int S>
__device__ __forceinline__ float rho_at(const typename Store<S>::T *src, const StepArgs &a, int x, int y)
{
    const PullSources g_src = pull_sources(a, x, y);
    float f[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        f[i] = Planes<S>::ld(src, g_src.idx[i], i, a.plane, a);
    return f[0] + ((f[1] + f[4]) + ((f[2] + f[5]) + (f[3] + f[6])));
}

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <int S, int F>
__global__ __launch_bounds__(256) void k_step_mips64(const typename Store<S>::T *__restrict__ src,
                                                   typename Store<S>::T *__restrict__ dst, StepArgs a,
                                                   StepClock *__restrict__ clk, int slot)
{
    const uint64_t tt = clock_read(clk, slot);
    const uint32_t t_lo = (uint32_t)(tt & 0xffffffffu), t_hi = (uint32_t)(tt >> 32);
    constexpr int LX = kMipsTX + 2, LY = kMipsTY + 2;
    __shared__ float srho[LY][LX];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * kMipsTX + tx;
    const int x0 = blockIdx.x * kMipsTX, y0 = blockIdx.y * kMipsTY;
    const int x = x0 + tx, y = y0 + ty;
    const bool live = x < a.nx && y < a.ny;
    const int xw = wrapi(x, a.nx), yw = wrapi(y, a.ny);
    const PullSources g_src = pull_sources(a, xw, yw);
    float f[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        f[i] = Planes<S>::ld(src, g_src.idx[i], i, a.plane, a);
    float rho, jx, jy;
    site_moments(f, rho, jx, jy);
    srho[ty + 1][tx + 1] = rho;
    // ring: 2 LX + 2 kMipsTY = 140 slots
    constexpr int kRing = 2 * LX + 2 * kMipsTY;
    if (tid < kRing) {
        int lx, ly;
        if (tid < LX) {
            lx = tid;
            ly = 0;
        } else if (tid < 2 * LX) {
            lx = tid - LX;
            ly = LY - 1;
        } else if (tid < 2 * LX + kMipsTY) {
            lx = 0;
            ly = tid - 2 * LX + 1;
        } else {
            lx = LX - 1;
            ly = tid - 2 * LX - kMipsTY + 1;
        }
        srho[ly][lx] = rho_at<S>(src, a, wrapi(x0 + lx - 1, a.nx), wrapi(y0 + ly - 1, a.ny));
    }
    __syncthreads();
    if (!live)
        return;
    // neighbour rho along e_1..e_6 in LDS coordinates (row parity of y)
    const int p = y & 1;
    const int cx = tx + 1, cy = ty + 1;
    float nb[7];
    nb[0] = rho;
    nb[1] = srho[cy][cx + 1];
    nb[2] = srho[cy + 1][cx + p];
    nb[3] = srho[cy + 1][cx - 1 + p];
    nb[4] = srho[cy][cx - 1];
    nb[5] = srho[cy - 1][cx - 1 + p];
    nb[6] = srho[cy - 1][cx + p];
    float ux, uy;
    mips_ustar(a, rho, nb, ux, uy);
    site_collide<F, S>(a, f, rho, ux, uy, (uint32_t)y * (uint32_t)a.nx + (uint32_t)x, t_lo, t_hi);
    const int64_t own = g_src.idx[0];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        Planes<S>::st(dst, own, i, a.plane, f[i], a);
    clock_advance(clk, slot, tt);
}

// ---------------------------------------------------------------------------
// MIPS: the 64 x ROWS tile body (mips_tile_step in device.h) on a grid in row
// groups: ROWS = 16, or 4 on lattices too small to fill the GPU with 64 x 16
// tiles (a wave then owns one row, so a launch ends sooner; the per-site
// arithmetic is the same).  Offsets are 32-bit (7 planes below 2^30
// elements); larger lattices take k_step_mips64.
// ---------------------------------------------------------------------------
template <int S, int F, int ROWS, int NW, int CP>
__global__ __launch_bounds__(64 * NW) void k_step_mips(const typename Store<S>::T *__restrict__ src,
                                                   typename Store<S>::T *__restrict__ dst, StepArgs a,
                                                   StepClock *__restrict__ clk, int slot)
{
    const uint64_t tt = clock_read(clk, slot);
    const uint32_t t_lo = (uint32_t)(tt & 0xffffffffu), t_hi = (uint32_t)(tt >> 32);
    __shared__ float srho[mips_tile_lds(ROWS)];
    int txi, tyi;
    row_group_tile(txi, tyi);
    const int x0 = txi * 64, y0 = tyi * ROWS;
    if (y0 >= a.ny)  // padding tile rows of the last group: the whole block
        return;
    const uint32_t bytes = (uint32_t)Planes<S>::bytes(a.plane);  // < 2^32: 7 planes < 2^30 elements
    mips_tile_step<S, F, ROWS, NW, CP>(buffer_rsrc(src, bytes), buffer_rsrc(dst, bytes), a, x0, y0, t_lo, t_hi, srho);
    clock_advance(clk, slot, tt);
}

// 64 x 16 MIPS tiles below this count leave the GPU under-filled (two per CU)
constexpr int64_t kMipsSmallTiles = 512;

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static dim3 local_block(int nx)
{
    int bx = nx >= 256 ? 256 : ((nx + 63) / 64) * 64;
    return dim3(bx, 256 / bx, 1);
}

static bool fits32(const StepArgs &a) { return (uint64_t)a.plane * 7ull < (1ull << 30); }

template <int S, int F, int CP>
static hipError_t launch_step_sfc(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk,
                                  int slot, hipStream_t s)
{
    using T = typename Store<S>::T;
    const T *in = (const T *)src;
    T *out = (T *)dst;
    if (p.model == kMips) {
        if (fits32(a)) {
            const int ntx = (p.nx + 63) / 64, nty = (p.ny + kMipsRows - 1) / kMipsRows;
            if ((int64_t)ntx * nty < kMipsSmallTiles) {
                const int nty4 = (p.ny + 3) / 4;
                dim3 grd(8u * (unsigned)ntx, (unsigned)((nty4 + 7) / 8));
                hipLaunchKernelGGL((k_step_mips<S, F, 4, 4, CP>), grd, dim3(256), 0, s, in, out, a, clk, slot);
            } else {
                dim3 grd(8u * (unsigned)ntx, (unsigned)((nty + 7) / 8));
                hipLaunchKernelGGL((k_step_mips<S, F, kMipsRows, kMipsWaves, CP>), grd, dim3(64 * kMipsWaves), 0, s,
                                   in, out, a, clk, slot);
            }
        } else {
            dim3 blk(kMipsTX, kMipsTY), grd((p.nx + kMipsTX - 1) / kMipsTX, (p.ny + kMipsTY - 1) / kMipsTY);
            hipLaunchKernelGGL((k_step_mips64<S, F>), grd, blk, 0, s, in, out, a, clk, slot);
        }
        return hipGetLastError();
    }
    dim3 blk = local_block(p.nx);
    const int ntx = (p.nx + blk.x - 1) / blk.x, nty = (p.ny + blk.y - 1) / blk.y;
    if (fits32(a)) {
        dim3 grd(8u * (unsigned)ntx, (unsigned)((nty + 7) / 8));
        if (p.model == kCil)
            hipLaunchKernelGGL((k_step_local<kCil, S, F, CP>), grd, blk, 0, s, in, out, a, clk, slot);
        else
            hipLaunchKernelGGL((k_step_local<kPassive, S, F, CP>), grd, blk, 0, s, in, out, a, clk, slot);
    } else {
        dim3 grd(ntx, nty);
        if (p.model == kCil)
            hipLaunchKernelGGL((k_step_local64<kCil, S, F>), grd, blk, 0, s, in, out, a, clk, slot);
        else
            hipLaunchKernelGGL((k_step_local64<kPassive, S, F>), grd, blk, 0, s, in, out, a, clk, slot);
    }
    return hipGetLastError();
}

// stores stream past the caches when the two buffers cannot stay in the
// Infinity Cache (the lattices beyond 2^30 elements take the 64-bit kernels,
// whose stores stay cached)
template <int S, int F>
static hipError_t launch_step_sf(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                                 hipStream_t s)
{
    if (2ull * Planes<S>::bytes(a.plane) > kStreamStateBytes)
        return launch_step_sfc<S, F, kStoreStream>(p, a, src, dst, clk, slot, s);
    return launch_step_sfc<S, F, kStoreCached>(p, a, src, dst, clk, slot, s);
}

int step_flags(const StepArgs &a) { return (a.omega == 1.0f ? kUnitTau : 0) | (a.noisy ? kNoisy : 0); }

template <int S>
static hipError_t launch_step_s(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                                hipStream_t s)
{
    switch (step_flags(a)) {
    case 0: return launch_step_sf<S, 0>(p, a, src, dst, clk, slot, s);
    case kUnitTau: return launch_step_sf<S, kUnitTau>(p, a, src, dst, clk, slot, s);
    case kNoisy: return launch_step_sf<S, kNoisy>(p, a, src, dst, clk, slot, s);
    default: return launch_step_sf<S, kUnitTau | kNoisy>(p, a, src, dst, clk, slot, s);
    }
}

hipError_t launch_step(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                       hipStream_t s)
{
    switch (p.storage) {
    case kF32: return launch_step_s<kF32>(p, a, src, dst, clk, slot, s);
    case kBf16Dev: return launch_step_s<kBf16Dev>(p, a, src, dst, clk, slot, s);
    case kF16Dev: return launch_step_s<kF16Dev>(p, a, src, dst, clk, slot, s);
    case kBf16R32: return launch_step_s<kBf16R32>(p, a, src, dst, clk, slot, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Initial state (appendix "CIL Model: General notes"), evaluated in FP64 and
// rounded once into the storage format.  Per site: Philox4x32-10 with
// counter (site, 0, 0, 1) gives four 32-bit uniforms (w + 1/2) / 2^32: the
// first sets a uniform direction, the second the density within +-spread,
// the last two a Box-Muller normal for the Gaussian-angle variant.  The
// optional population perturbation uses the 16-bit halves of counter
// (site, 0, 0, 2).
// ---------------------------------------------------------------------------
struct InitArgs {
    int32_t mode, model;
    double rho_mean, rho_spread, angle_std, u_mag, pop_noise, A, B;
};

template <int S>
__global__ __launch_bounds__(256) void k_init(typename Store<S>::T *__restrict__ dst, StepArgs a, InitArgs in)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx)
        return;
    const uint32_t site = (uint32_t)y * (uint32_t)a.nx + (uint32_t)x;
    const Philox4 w = philox4x32_10(site, 0u, 0u, 1u, a.key0, a.key1);
    double u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        u[k] = ((double)w.v[k] + 0.5) * (1.0 / 4294967296.0);
    const double two_pi = 6.283185307179586476925;
    double theta;
    if (in.mode == LBM_INIT_GAUSS_DIR)
        theta = in.angle_std * sqrt(-2.0 * log(u[2])) * cos(two_pi * u[3]);
    else
        theta = two_pi * u[0];
    const double r = in.rho_mean * (1.0 + in.rho_spread * (2.0 * u[1] - 1.0));
    double mag = 0.0;
    if (in.u_mag >= 0.0)
        mag = in.u_mag;
    else if (in.model == kCil)
        mag = fmax(in.B - in.A * r * r, 0.0);
    const double vx = mag * cos(theta), vy = mag * sin(theta);
    // xi(r, v) in the pair form
    const double h3 = 0.86602540378443864676;
    const double usq = vx * vx + vy * vy, base = 1.0 - 2.0 * usq;
    const double al[3] = {vx, 0.5 * vx + h3 * vy, -0.5 * vx + h3 * vy};
    double g[7];
    g[0] = 0.5 * r * base;
    for (int k = 0; k < 3; ++k) {
        const double b = base + 8.0 * al[k] * al[k];
        g[k + 1] = (r / 12.0) * (b + 4.0 * al[k]);
        g[k + 4] = (r / 12.0) * (b - 4.0 * al[k]);
    }
    if (in.pop_noise != 0.0) {
        const Philox4 w2 = philox4x32_10(site, 0u, 0u, 2u, a.key0, a.key1);
        for (int i = 0; i < 7; ++i) {
            const uint32_t hw = (i & 1) ? (w2.v[i >> 1] >> 16) : (w2.v[i >> 1] & 0xffffu);
            g[i] += in.pop_noise * (2.0 * (((double)hw + 0.5) * (1.0 / 65536.0)) - 1.0);
        }
    }
    const int64_t own = (int64_t)y * a.pitch + x;
    for (int i = 0; i < 7; ++i)
        Planes<S>::st(dst, own, i, a.plane, (float)g[i], a);
}

template <int S>
__global__ __launch_bounds__(256) void k_add_density(typename Store<S>::T *__restrict__ buf, StepArgs a, float add)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx)
        return;
    const int64_t own = (int64_t)y * a.pitch + x;
    for (int i = 0; i < 7; ++i) {
        const float v = Planes<S>::ld(buf, own, i, a.plane, a);
        Planes<S>::st(buf, own, i, a.plane, v + add, a);
    }
}

hipError_t launch_init(const lbm_params &p, const lbm_init &in, const StepArgs &a, void *dst, hipStream_t s)
{
    InitArgs ia{in.mode, p.model, in.rho_mean, in.rho_spread, in.angle_std, in.u_mag, in.pop_noise, p.A, p.B};
    dim3 blk(256), grd((p.nx + 255) / 256, p.ny);
    switch (p.storage) {
    case kF32: hipLaunchKernelGGL(k_init<kF32>, grd, blk, 0, s, (float *)dst, a, ia); break;
    case kBf16Dev: hipLaunchKernelGGL(k_init<kBf16Dev>, grd, blk, 0, s, (uint16_t *)dst, a, ia); break;
    case kF16Dev: hipLaunchKernelGGL(k_init<kF16Dev>, grd, blk, 0, s, (_Float16 *)dst, a, ia); break;
    case kBf16R32: hipLaunchKernelGGL(k_init<kBf16R32>, grd, blk, 0, s, (uint16_t *)dst, a, ia); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_add_density(const lbm_params &p, const StepArgs &a, void *buf, double drho, hipStream_t s)
{
    const float add = (float)(drho / 7.0);
    dim3 blk(256), grd((p.nx + 255) / 256, p.ny);
    switch (p.storage) {
    case kF32: hipLaunchKernelGGL(k_add_density<kF32>, grd, blk, 0, s, (float *)buf, a, add); break;
    case kBf16Dev: hipLaunchKernelGGL(k_add_density<kBf16Dev>, grd, blk, 0, s, (uint16_t *)buf, a, add); break;
    case kF16Dev: hipLaunchKernelGGL(k_add_density<kF16Dev>, grd, blk, 0, s, (_Float16 *)buf, a, add); break;
    case kBf16R32: hipLaunchKernelGGL(k_add_density<kBf16R32>, grd, blk, 0, s, (uint16_t *)buf, a, add); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
