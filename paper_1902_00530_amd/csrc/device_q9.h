// Device-side building blocks of the square-lattice (D2Q9) variant of the
// modified lattice Boltzmann step: the same algorithm as the D2Q7 site body
// (appendix "Summary of modified lattice Boltzmann model algorithm") on the
// standard square velocity set, whose sound speed is c_s^2 = 1/3.
//
// Directions: 0 rest; 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1); 5 (1,1),
// 6 (-1,1), 7 (-1,-1), 8 (1,-1); weights 4/9, 1/9 (axes), 1/36 (diagonals);
// opposite pairs 1-3, 2-4, 5-7, 6-8.
#pragma once

#include "device.h"

namespace lbm {

constexpr int kQ9 = 9;

// w_i rho_ref of plane i (deviation storages; 0 for F32).
__device__ __forceinline__ float q9_wr(const StepArgs &a, int i) { return i == 0 ? a.wr0 : (i <= 4 ? a.wr1 : a.wr2); }

// rho and j = sum f_i e_i, the momentum over opposite pairs.
__device__ __forceinline__ void q9_moments(const float f[9], float &rho, float &jx, float &jy)
{
    rho = f[0] + (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
    const float d1 = f[1] - f[3], d2 = f[2] - f[4], d5 = f[5] - f[7], d6 = f[6] - f[8];
    jx = d1 + (d5 - d6);
    jy = d2 + (d5 + d6);
}

// MIPS target velocity from the eight neighbour densities nb[i] = rho(r + e_i):
// grad rho = (1/c_s^2) sum_i w_i e_i nb_i, the construction of the paper's
// isotropic stencil on this lattice, then eq. bu_mips and the U_max clamp.
__device__ __forceinline__ void q9_mips_ustar(const StepArgs &a, float rho, const float nb[9], float &ux, float &uy)
{
    const float d5 = nb[5] - nb[7], d6 = nb[6] - nb[8];
    const float gx = (nb[1] - nb[3]) * (1.0f / 3.0f) + (d5 - d6) * (1.0f / 12.0f);
    const float gy = (nb[2] - nb[4]) * (1.0f / 3.0f) + (d5 + d6) * (1.0f / 12.0f);
    mips_from_gradient(a, rho, gx, gy, ux, uy);
}

// 1/9 as an unevaluated float pair (float(1/9) alone would bias the mass of
// every relaxed site); 4/9 and 1/36 follow by exact powers of two.
constexpr float kNinthHi = (float)(1.0 / 9.0);
constexpr float kNinthLo = (float)(1.0 / 9.0 - (double)(float)(1.0 / 9.0));

// Steady state of this lattice in pair form: a_k = e_k.u,
// base = 1 - (3/2)|u|^2, xi_{k, opp} = w_k rho (base + (9/2) a_k^2 +- 3 a_k),
// xi_0 = (4/9) rho base.
__device__ __forceinline__ void q9_equilibrium(float rho, float ux, float uy, float eq[9])
{
    const float usq = ux * ux + uy * uy;
    const float base = 1.0f - 1.5f * usq;
    const float r9 = fmaf(rho, kNinthHi, rho * kNinthLo);
    const float r36 = 0.25f * r9;
    eq[0] = 4.0f * r9 * base;
    const float a1 = ux, a2 = uy, a5 = ux + uy, a6 = uy - ux;
    const float b1 = base + 4.5f * a1 * a1, b2 = base + 4.5f * a2 * a2;
    const float b5 = base + 4.5f * a5 * a5, b6 = base + 4.5f * a6 * a6;
    eq[1] = r9 * (b1 + 3.0f * a1);
    eq[3] = r9 * (b1 - 3.0f * a1);
    eq[2] = r9 * (b2 + 3.0f * a2);
    eq[4] = r9 * (b2 - 3.0f * a2);
    eq[5] = r36 * (b5 + 3.0f * a5);
    eq[7] = r36 * (b5 - 3.0f * a5);
    eq[6] = r36 * (b6 + 3.0f * a6);
    eq[8] = r36 * (b6 - 3.0f * a6);
}

// The nine 14-bit draws of one Philox4x32-10 output: draw i is bits
// 14 i .. 14 i + 13 of the 128-bit word v0 + 2^32 v1 + 2^64 v2 + 2^96 v3.
// Draws that straddle two words take a funnel shift (v_alignbit_b32).
__device__ __forceinline__ void q9_draws(const Philox4 &w, float h[9])
{
    h[0] = (float)(w.v[0] & 0x3fffu);
    h[1] = (float)((w.v[0] >> 14) & 0x3fffu);
    h[2] = (float)(__builtin_amdgcn_alignbit(w.v[1], w.v[0], 28) & 0x3fffu);
    h[3] = (float)((w.v[1] >> 10) & 0x3fffu);
    h[4] = (float)(__builtin_amdgcn_alignbit(w.v[2], w.v[1], 24) & 0x3fffu);
    h[5] = (float)((w.v[2] >> 6) & 0x3fffu);
    h[6] = (float)(__builtin_amdgcn_alignbit(w.v[3], w.v[2], 20) & 0x3fffu);
    h[7] = (float)((w.v[3] >> 2) & 0x3fffu);
    h[8] = (float)((w.v[3] >> 16) & 0x3fffu);
}

// Zero-sum noise (eq. noiseDensityConservation) over nine directions: raw
// draws sigma (2 h_i + 1 - 16384) / 16384, minus their mean, is
// sigma (9 h_i - H) / 73728, H = sum h_i; the integers are exact in float.
__device__ __forceinline__ void q9_add_noise(const StepArgs &a, uint32_t site, uint32_t t_lo, uint32_t t_hi,
                                             float f[9])
{
    float h[9];
    q9_draws(philox4x32_10(site, t_lo, t_hi, 0u, a.key0, a.key1), h);
    const float H = (((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]))) + h[8];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = fmaf(fmaf(h[i], 9.0f, -H), a.noise_scale, f[i]);
}

// BGK relaxation towards xi(rho, u*), noise, and the negative correction
// (closed pair form of the appendix "Negative Correction": a negative rest
// population becomes 0, a pair with a negative member becomes
// (max(d, 0), max(-d, 0)), and a site where a rule fired is rescaled to rho).
template <int F, int S = kF32>
__device__ __forceinline__ void q9_collide(const StepArgs &a, float f[9], float rho, float ux, float uy,
                                           uint32_t site, uint32_t t_lo, uint32_t t_hi)
{
    float eq[9];
    q9_equilibrium(rho, ux, uy, eq);
    if (F & kUnitTau) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = eq[i];
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = f[i] - (f[i] - eq[i]) * a.omega;
    }
    if (F & kNoisy)
        q9_add_noise(a, site, t_lo, t_hi, f);
    // the rest population is rho minus the moving ones (as on D2Q7: float32
    // here; the 16-bit storages below, at sites where no rule fired)
    const bool absorb = (F & kUnitTau) || a.omega != 0.0f;
    if constexpr (S == kF32) {
        if (absorb)
            f[0] = rho - (((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8])));
    }
    constexpr int kNegative = 0x3c;  // -inf, -normal, -denormal, -0 (as in the D2Q7 body)
    bool fired = false;
    if (__builtin_amdgcn_classf(f[0], kNegative)) {
        f[0] = 0.0f;
        fired = true;
    }
    constexpr int kFirst[4] = {1, 2, 5, 6};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = kFirst[q], o = k + 2;
        if (__builtin_amdgcn_classf(f[k], kNegative) | __builtin_amdgcn_classf(f[o], kNegative)) {
            const float d = f[k] - f[o];
            f[k] = fmaxf(d, 0.0f);
            f[o] = fmaxf(-d, 0.0f);
            fired = true;
        }
    }
    if constexpr (S != kF32) {
        if (!fired && absorb) {
            float g[9];
#pragma unroll
            for (int i = 1; i < 9; ++i)
                g[i] = Store<S>::round(f[i], q9_wr(a, i));
            f[0] = rho - (((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8])));
        }
    }
    if (fired) {
        const float s = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
        float q = __builtin_amdgcn_rcpf(s);  // refined by one Newton step (as on D2Q7)
        q = fmaf(fmaf(-s, q, 1.0f), q, q);
        const float r = s > 0.0f ? rho * q : 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] *= r;
    }
}

// Streaming sources (step (i)) with 32-bit element offsets within a plane:
// population i at (x, y) comes from (x, y) - e_i, periodic.
struct Q9Sources {
    uint32_t idx[9];
};

__device__ __forceinline__ Q9Sources q9_sources(const StepArgs &a, int x, int y)
{
    const uint32_t xm = x == 0 ? a.nx - 1 : x - 1;
    const uint32_t xp = x == a.nx - 1 ? 0 : x + 1;
    const uint32_t P = (uint32_t)a.pitch;
    const uint32_t ry = (uint32_t)y * P;
    const uint32_t ru = y == a.ny - 1 ? 0u : ry + P;
    const uint32_t rd = y == 0 ? (uint32_t)(a.ny - 1) * P : ry - P;
    Q9Sources t;
    t.idx[0] = ry + x;
    t.idx[1] = ry + xm;
    t.idx[2] = rd + x;
    t.idx[3] = ry + xp;
    t.idx[4] = ru + x;
    t.idx[5] = rd + xm;
    t.idx[6] = rd + xp;
    t.idx[7] = ru + xp;
    t.idx[8] = ru + xm;
    return t;
}

// One buffer resource per population plane: offsets stay 32-bit for planes
// of up to 2^32 bytes, and each plane's base is a scalar.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t q9_plane_rsrc(const T *base, int i, uint32_t plane)
{
    return buffer_rsrc(base + (size_t)i * plane, plane * (uint32_t)sizeof(T));
}

// One site-update of the local models (passive, CIL) at (x, y): the nine
// streamed populations gathered from their periodic sources, collided, and
// stored at (x, y) in dst.  src and dst are [9][ny][pitch] population buffers.
template <int M, int S, int F, int CP = kStoreCached>
__device__ __forceinline__ void q9_site_step(const typename Store<S>::T *src, typename Store<S>::T *dst,
                                             const StepArgs &a, int x, int y, uint32_t t_lo, uint32_t t_hi)
{
    using T = typename Store<S>::T;
    const uint32_t plane = (uint32_t)a.plane;
    const Q9Sources g = q9_sources(a, x, y);
    float f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = Store<S>::widen(BufIO<T>::load(q9_plane_rsrc(src, i, plane), g.idx[i], 0u), q9_wr(a, i));
    float rho, jx, jy, ux, uy;
    q9_moments(f, rho, jx, jy);
    local_ustar<M>(a, rho, jx, jy, ux, uy);
    q9_collide<F, S>(a, f, rho, ux, uy, (uint32_t)y * (uint32_t)a.nx + (uint32_t)x, t_lo, t_hi);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        BufIO<T>::template store<CP>(q9_plane_rsrc(dst, i, plane), g.idx[0], 0u, Store<S>::narrow(f[i], q9_wr(a, i)));
}

// ---------------------------------------------------------------------------
// MIPS step of one 64 x 16 tile at (x0, y0) (u* needs the streamed density of
// the eight neighbours).  256 threads: wave w owns rows w, w+4, w+8, w+12,
// one column per lane.  rho of the tile and of its one-site ring (rows above
// and below, corners included, and the two edge columns: 164 sites, taken by
// waves 0-2) is staged in LDS (srho, 18 x 66 floats).  The tile's own
// populations stay in registers from the density pass to the collision.  On
// tiles whose sources do not wrap, a row's nine loads share one vector offset
// (the lane) and wave-uniform scalar offsets.  Every LDS slot holds rho at
// its periodically wrapped site, so ragged tiles and lattices narrower than
// a tile need no special case.  The single-lattice and the batched D2Q9 MIPS
// kernels both run this body.
// ---------------------------------------------------------------------------
constexpr int kQ9MipsRows = 16;

template <int S, int F, int CP = kStoreCached>
__device__ __forceinline__ void q9_mips_tile_step(const typename Store<S>::T *src, typename Store<S>::T *dst,
                                                  const StepArgs &a, int x0, int y0, uint32_t t_lo, uint32_t t_hi,
                                                  float *srho)
{
    using T = typename Store<S>::T;
    constexpr int W = 66, H = kQ9MipsRows + 2, RW = kQ9MipsRows / 4;
    constexpr int kRing = 2 * W + 2 * kQ9MipsRows;  // 164
    const uint32_t plane = (uint32_t)a.plane, P = (uint32_t)a.pitch, nx = (uint32_t)a.nx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool interior = x0 >= 1 && x0 + 65 <= a.nx && y0 >= 1 && y0 + kQ9MipsRows + 1 <= a.ny;
    auto load_wrapped = [&](float *g, int x, int y) {
        const Q9Sources q = q9_sources(a, wrap_coord(x, a.nx), wrap_coord(y, a.ny));
#pragma unroll
        for (int i = 0; i < 9; ++i)
            g[i] = Store<S>::widen(BufIO<T>::load(q9_plane_rsrc(src, i, plane), q.idx[i], 0u), q9_wr(a, i));
    };
    float f[RW][9];
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int y = y0 + wv + 4 * k;
        if (interior) {
            const uint32_t c = (uint32_t)y * P + (uint32_t)x0;  // offset of (x0, y)
            const uint32_t e[9] = {c, c - 1u, c - P, c + 1u, c + P, c - P - 1u, c - P + 1u, c + P + 1u, c + P - 1u};
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[k][i] = Store<S>::widen(BufIO<T>::load(q9_plane_rsrc(src, i, plane), lane, e[i]), q9_wr(a, i));
        } else {
            load_wrapped(f[k], x0 + lane, y);
        }
    }
    const int re = wv * 64 + lane;  // this lane's ring site (waves 0-2)
    if (re < kRing) {
        int rlx, rly;
        if (re < W) {
            rlx = re;
            rly = 0;
        } else if (re < 2 * W) {
            rlx = re - W;
            rly = H - 1;
        } else {
            rlx = re < 2 * W + kQ9MipsRows ? 0 : W - 1;
            rly = 1 + (re - 2 * W) % kQ9MipsRows;
        }
        float g[9], jx, jy;
        load_wrapped(g, x0 - 1 + rlx, y0 - 1 + rly);
        q9_moments(g, srho[rly * W + rlx], jx, jy);
    }
    float rho[RW];
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        float jx, jy;
        q9_moments(f[k], rho[k], jx, jy);
        srho[(wv + 4 * k + 1) * W + lane + 1] = rho[k];
    }
    __syncthreads();
    const int x = x0 + lane;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int r = wv + 4 * k, y = y0 + r;
        if (x >= a.nx || y >= a.ny)
            continue;
        const int c = (r + 1) * W + lane + 1;
        float nb[9];
        nb[0] = rho[k];
        nb[1] = srho[c + 1];
        nb[2] = srho[c + W];
        nb[3] = srho[c - 1];
        nb[4] = srho[c - W];
        nb[5] = srho[c + W + 1];
        nb[6] = srho[c + W - 1];
        nb[7] = srho[c - W - 1];
        nb[8] = srho[c - W + 1];
        float ux, uy;
        q9_mips_ustar(a, rho[k], nb, ux, uy);
        q9_collide<F, S>(a, f[k], rho[k], ux, uy, (uint32_t)y * nx + (uint32_t)x, t_lo, t_hi);
        const uint32_t own = (uint32_t)y * P + (uint32_t)x;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            BufIO<T>::template store<CP>(q9_plane_rsrc(dst, i, plane), own, 0u, Store<S>::narrow(f[k][i], q9_wr(a, i)));
    }
}

}  // namespace lbm
