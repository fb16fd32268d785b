// Fused step of the square-lattice (D2Q9) variant on gfx950: the algorithm
// of the appendix "Summary of modified lattice Boltzmann model algorithm" on
// the D2Q9 velocity set (site body in device_q9.h).  Population i of site r is
// gathered from r - e_i in the source buffer, collided, and stored at r in
// the other buffer: 9 loads and 9 stores, 72 B per site-update in F32.
//
// Each population plane gets its own buffer resource, so element offsets are
// 32-bit within a plane and the lattice may hold up to 2^30 F32 sites per
// plane.  Like the D2Q7 path, the step is bound by HBM bandwidth and has no
// matrix-core work.
#include "device_q9.h"
#include "internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Passive and CIL (u* from the site alone).  A block is a BX x BY tile with
// BX a multiple of 64, laid out in row groups so each row of tiles runs on
// one XCD.
// ---------------------------------------------------------------------------
template <int M, int S, int F, int CP>
__global__ __launch_bounds__(256) void k_q9_step_local(const typename Store<S>::T *__restrict__ src,
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
    q9_site_step<M, S, F, CP>(src, dst, a, x, y, t_lo, t_hi);
    clock_advance(clk, slot, tt);
}

// ---------------------------------------------------------------------------
// MIPS: the 64 x 16 tile body (q9_mips_tile_step in device_q9.h) on a grid
// in row groups.
// ---------------------------------------------------------------------------
template <int S, int F, int CP>
__global__ __launch_bounds__(256) void k_q9_step_mips(const typename Store<S>::T *__restrict__ src,
                                                      typename Store<S>::T *__restrict__ dst, StepArgs a,
                                                      StepClock *__restrict__ clk, int slot)
{
    const uint64_t tt = clock_read(clk, slot);
    const uint32_t t_lo = (uint32_t)(tt & 0xffffffffu), t_hi = (uint32_t)(tt >> 32);
    __shared__ float srho[(kQ9MipsRows + 2) * 66];
    int txi, tyi;
    row_group_tile(txi, tyi);
    const int x0 = txi * 64, y0 = tyi * kQ9MipsRows;
    if (y0 >= a.ny)  // padding tile rows of the last group: the whole block
        return;
    q9_mips_tile_step<S, F, CP>(src, dst, a, x0, y0, t_lo, t_hi, srho);
    clock_advance(clk, slot, tt);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int S, int F, int CP>
static hipError_t launch_q9_sfc(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk,
                                int slot, hipStream_t s)
{
    using T = typename Store<S>::T;
    const T *in = (const T *)src;
    T *out = (T *)dst;
    if (p.model == kMips) {
        const int ntx = (p.nx + 63) / 64, nty = (p.ny + kQ9MipsRows - 1) / kQ9MipsRows;
        dim3 grd(8u * (unsigned)ntx, (unsigned)((nty + 7) / 8));
        hipLaunchKernelGGL((k_q9_step_mips<S, F, CP>), grd, dim3(256), 0, s, in, out, a, clk, slot);
        return hipGetLastError();
    }
    const int bx = p.nx >= 256 ? 256 : ((p.nx + 63) / 64) * 64;
    dim3 blk(bx, 256 / bx);
    const int ntx = (p.nx + blk.x - 1) / blk.x, nty = (p.ny + blk.y - 1) / blk.y;
    dim3 grd(8u * (unsigned)ntx, (unsigned)((nty + 7) / 8));
    if (p.model == kCil)
        hipLaunchKernelGGL((k_q9_step_local<kCil, S, F, CP>), grd, blk, 0, s, in, out, a, clk, slot);
    else
        hipLaunchKernelGGL((k_q9_step_local<kPassive, S, F, CP>), grd, blk, 0, s, in, out, a, clk, slot);
    return hipGetLastError();
}

// stores stream past the caches when the two buffers cannot stay in the
// Infinity Cache
template <int S, int F>
static hipError_t launch_q9_sf(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                               hipStream_t s)
{
    if (2ull * 9ull * (uint64_t)a.plane * sizeof(typename Store<S>::T) > kStreamStateBytes)
        return launch_q9_sfc<S, F, kStoreStream>(p, a, src, dst, clk, slot, s);
    return launch_q9_sfc<S, F, kStoreCached>(p, a, src, dst, clk, slot, s);
}

template <int S>
static hipError_t launch_q9_s(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                              hipStream_t s)
{
    switch (step_flags(a)) {
    case 0: return launch_q9_sf<S, 0>(p, a, src, dst, clk, slot, s);
    case kUnitTau: return launch_q9_sf<S, kUnitTau>(p, a, src, dst, clk, slot, s);
    case kNoisy: return launch_q9_sf<S, kNoisy>(p, a, src, dst, clk, slot, s);
    default: return launch_q9_sf<S, kUnitTau | kNoisy>(p, a, src, dst, clk, slot, s);
    }
}

hipError_t launch_step_q9(const lbm_params &p, const StepArgs &a, const void *src, void *dst, StepClock *clk, int slot,
                          hipStream_t s)
{
    switch (p.storage) {
    case kF32: return launch_q9_s<kF32>(p, a, src, dst, clk, slot, s);
    case kBf16Dev: return launch_q9_s<kBf16Dev>(p, a, src, dst, clk, slot, s);
    case kF16Dev: return launch_q9_s<kF16Dev>(p, a, src, dst, clk, slot, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Initial state (appendix "CIL Model: General notes") in FP64, rounded once
// into the storage: the variates of the D2Q7 initial state (counter
// (site, 0, 0, 1): direction, density, Box-Muller angle) with this lattice's
// steady state; the optional population perturbation takes the nine 14-bit
// draws of counter (site, 0, 0, 2).
// ---------------------------------------------------------------------------
struct Q9InitArgs {
    int32_t mode, model;
    double rho_mean, rho_spread, angle_std, u_mag, pop_noise, A, B;
};

template <int S>
__global__ __launch_bounds__(256) void k_q9_init(typename Store<S>::T *__restrict__ dst, StepArgs a, Q9InitArgs in)
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
    const double theta = in.mode == LBM_INIT_GAUSS_DIR ? in.angle_std * sqrt(-2.0 * log(u[2])) * cos(two_pi * u[3])
                                                       : two_pi * u[0];
    const double r = in.rho_mean * (1.0 + in.rho_spread * (2.0 * u[1] - 1.0));
    double mag = 0.0;
    if (in.u_mag >= 0.0)
        mag = in.u_mag;
    else if (in.model == kCil)
        mag = fmax(in.B - in.A * r * r, 0.0);
    const double vx = mag * cos(theta), vy = mag * sin(theta);
    const double base = 1.0 - 1.5 * (vx * vx + vy * vy);
    const double al[4] = {vx, vy, vx + vy, vy - vx};  // e_1, e_2, e_5, e_6 dotted with v
    const int first[4] = {1, 2, 5, 6};
    double g[9];
    g[0] = (4.0 / 9.0) * r * base;
    for (int k = 0; k < 4; ++k) {
        const double wr = (k < 2 ? 1.0 / 9.0 : 1.0 / 36.0) * r;
        const double b = base + 4.5 * al[k] * al[k];
        g[first[k]] = wr * (b + 3.0 * al[k]);
        g[first[k] + 2] = wr * (b - 3.0 * al[k]);
    }
    if (in.pop_noise != 0.0) {
        float h[9];
        q9_draws(philox4x32_10(site, 0u, 0u, 2u, a.key0, a.key1), h);
        for (int i = 0; i < 9; ++i)
            g[i] += in.pop_noise * (2.0 * (((double)h[i] + 0.5) * (1.0 / 16384.0)) - 1.0);
    }
    const int64_t own = (int64_t)y * a.pitch + x;
    for (int i = 0; i < 9; ++i)
        Store<S>::store(dst, i * a.plane + own, (float)g[i], q9_wr(a, i));
}

template <int S>
__global__ __launch_bounds__(256) void k_q9_add_density(typename Store<S>::T *__restrict__ buf, StepArgs a,
                                                        float add)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx)
        return;
    const int64_t own = (int64_t)y * a.pitch + x;
    for (int i = 0; i < 9; ++i) {
        const float wr = q9_wr(a, i);
        const float v = Store<S>::load(buf, i * a.plane + own, wr);
        Store<S>::store(buf, i * a.plane + own, v + add, wr);
    }
}

hipError_t launch_init_q9(const lbm_params &p, const lbm_init &in, const StepArgs &a, void *dst, hipStream_t s)
{
    Q9InitArgs ia{in.mode, p.model, in.rho_mean, in.rho_spread, in.angle_std, in.u_mag, in.pop_noise, p.A, p.B};
    dim3 blk(256), grd((p.nx + 255) / 256, p.ny);
    switch (p.storage) {
    case kF32: hipLaunchKernelGGL(k_q9_init<kF32>, grd, blk, 0, s, (float *)dst, a, ia); break;
    case kBf16Dev: hipLaunchKernelGGL(k_q9_init<kBf16Dev>, grd, blk, 0, s, (uint16_t *)dst, a, ia); break;
    case kF16Dev: hipLaunchKernelGGL(k_q9_init<kF16Dev>, grd, blk, 0, s, (_Float16 *)dst, a, ia); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_add_density_q9(const lbm_params &p, const StepArgs &a, void *buf, double drho, hipStream_t s)
{
    const float add = (float)(drho / 9.0);
    dim3 blk(256), grd((p.nx + 255) / 256, p.ny);
    switch (p.storage) {
    case kF32: hipLaunchKernelGGL(k_q9_add_density<kF32>, grd, blk, 0, s, (float *)buf, a, add); break;
    case kBf16Dev:
        hipLaunchKernelGGL(k_q9_add_density<kBf16Dev>, grd, blk, 0, s, (uint16_t *)buf, a, add);
        break;
    case kF16Dev:
        hipLaunchKernelGGL(k_q9_add_density<kF16Dev>, grd, blk, 0, s, (_Float16 *)buf, a, add);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
