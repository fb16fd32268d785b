// Device-side building blocks of the fused D2Q7 active-LBM step (gfx950).
//
// Everything here runs inside the kernels: the counter-based noise generator,
// the population storage formats, and the per-site collision of the modified
// lattice Boltzmann method (Nesbitt, Pruessner & Lee, arXiv:1902.00530).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum Model : int { kPassive = 0, kMips = 1, kCil = 2 };
enum Storage : int { kF32 = 0, kBf16Dev = 1, kF16Dev = 2, kBf16R32 = 3 };

// Kernel-side copy of the parameters, with derived constants precomputed on
// the host in double and rounded once to float.
struct StepArgs {
    int32_t nx, ny;
    int64_t pitch;      // elements per row
    int64_t plane;      // elements per population plane (ny * pitch)
    float omega;        // 1 / tau (0 for tau = +inf)
    float noise_scale;  // D2Q7: sigma / 229376, eta_i = (7 h_i - sum h) * noise_scale;
                        // D2Q9: sigma / 73728, eta_i = (9 h_i - sum h) * noise_scale
    float noise_h;      // D2Q7: sigma / 32768 = 7 noise_scale, the factor of h_i alone
    float A16, B16;     // CIL A and B times 2^16 (exact), see local_ustar
    float C, rho_star, inv_rho_star, u_max;  // MIPS
    float wr0, wr1, wr2;  // w_i rho_ref (deviation storages): D2Q7 rest, moving;
                          // D2Q9 rest, axes, diagonals
    uint32_t key0, key1;
    int32_t noisy;      // sigma != 0
};

// Step index of the single-lattice step kernels, kept in device memory so a
// captured graph of steps replays with unchanged arguments: a launch reads
// the absolute step index (the noise counter) from slot `slot` and the first
// lane of block (0, 0) stores the next index in the other slot, which only
// the next launch reads.  The slot is the buffer parity of the launch's
// source.  The store comes at the end of the kernel (site (0, 0), which
// every lattice has, so that lane never leaves early), so the read is waited
// on only where the noise needs it, after the population loads are issued.
struct StepClock {
    int64_t t[2];
};

__device__ __forceinline__ uint64_t clock_read(const StepClock *clk, int slot) { return (uint64_t)clk->t[slot]; }

__device__ __forceinline__ void clock_advance(StepClock *clk, int slot, uint64_t t)
{
    if ((blockIdx.x | blockIdx.y | threadIdx.x | threadIdx.y) == 0)
        clk->t[slot ^ 1] = (int64_t)t + 1;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the Philox multipliers, a word permutation and a
// key xor; the key advances by the Weyl increments between rounds.  The key
// and the upper counter words are uniform across the launch, so the
// compiler keeps the key schedule in scalar registers.
// ---------------------------------------------------------------------------
struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per multiplier (a single v_mad_u64_u32 each)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input xor (truth table 0x96) in one v_bitop3_b32
        c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        c1 = (uint32_t)p1;
        c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// Zero-sum noise of one site and step (eq. noiseDensityConservation with
// uniform raw draws).  With 16-bit draws h_i the raw value is sigma (2 h_i -
// 65535) / 65536; subtracting the mean over the seven directions leaves
// sigma (7 h_i - H) / 229376 with H = sum h_i, taken as h_i sigma / 32768 -
// H sigma / 229376 (one product for the site, one fma per direction).  The
// halves are taken as 16-bit values so that each becomes one convert with a
// word select (SDWA), no mask or shift.
__device__ __forceinline__ void site_noise(const StepArgs &a, uint32_t site, uint32_t t_lo, uint32_t t_hi, float nz[7])
{
    const Philox4 w = philox4x32_10(site, t_lo, t_hi, 0u, a.key0, a.key1);
    float h[7];
    h[0] = (float)(uint16_t)w.v[0];
    h[1] = (float)(uint16_t)(w.v[0] >> 16);
    h[2] = (float)(uint16_t)w.v[1];
    h[3] = (float)(uint16_t)(w.v[1] >> 16);
    h[4] = (float)(uint16_t)w.v[2];
    h[5] = (float)(uint16_t)(w.v[2] >> 16);
    h[6] = (float)(uint16_t)w.v[3];
    const float H = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + h[6]);
    const float hs = H * a.noise_scale;
#pragma unroll
    for (int i = 0; i < 7; ++i)
        nz[i] = fmaf(h[i], a.noise_h, -hs);
}

// ---------------------------------------------------------------------------
// Storage formats.  F32 holds f_i; the deviation formats hold
// d_i = f_i - w_i rho_ref rounded to nearest even in bf16 / fp16, and are
// widened to f32 on load.
// ---------------------------------------------------------------------------
template <int S>
struct Store;

template <>
struct Store<kF32> {
    using T = float;
    __device__ __forceinline__ static float load(const T *p, int64_t i, float) { return p[i]; }
    __device__ __forceinline__ static void store(T *p, int64_t i, float v, float) { p[i] = v; }
    __device__ __forceinline__ static float widen(T v, float) { return v; }
    __device__ __forceinline__ static T narrow(float v, float) { return v; }
    // the value a store and a later load give back
    __device__ __forceinline__ static float round(float v, float) { return v; }
};

__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even into bfloat16 bits (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t float_to_bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <>
struct Store<kBf16Dev> {
    using T = uint16_t;
    __device__ __forceinline__ static float load(const T *p, int64_t i, float wr) { return bf16_bits_to_float(p[i]) + wr; }
    __device__ __forceinline__ static void store(T *p, int64_t i, float v, float wr) { p[i] = float_to_bf16_rne(v - wr); }
    __device__ __forceinline__ static float widen(T v, float wr) { return bf16_bits_to_float(v) + wr; }
    __device__ __forceinline__ static T narrow(float v, float wr) { return float_to_bf16_rne(v - wr); }
    __device__ __forceinline__ static float round(float v, float wr) { return widen(narrow(v, wr), wr); }
};

template <>
struct Store<kF16Dev> {
    using T = _Float16;
    __device__ __forceinline__ static float load(const T *p, int64_t i, float wr) { return (float)p[i] + wr; }
    __device__ __forceinline__ static void store(T *p, int64_t i, float v, float wr) { p[i] = (_Float16)(v - wr); }
    __device__ __forceinline__ static float widen(T v, float wr) { return (float)v + wr; }
    __device__ __forceinline__ static T narrow(float v, float wr) { return (_Float16)(v - wr); }
    __device__ __forceinline__ static float round(float v, float wr) { return widen(narrow(v, wr), wr); }
};

// bfloat16 deviations of the six moving populations with the rest population
// in float32: the buffer is the float32 rest plane followed by six bfloat16
// planes; every access goes through Planes<kBf16R32> (below).
template <>
struct Store<kBf16R32> {
    using T = uint16_t;
};

// ---------------------------------------------------------------------------
// Per-site arithmetic.
// ---------------------------------------------------------------------------
constexpr float kHalfSqrt3 = 0.86602540378443864676f;        // sqrt(3)/2
// sqrt(3)/2 - kHalfSqrt3: with both parts, a_2^2 + a_3^2 keeps the lattice
// identity sum_k (e_k.u)^2 = (3/2)|u|^2 to float precision (float(sqrt(3)/2)
// squared is 3.6e-8 below 3/4, which biased every site's mass by about
// 2 rho u_y^2 x 3.6e-8 per step, the same sign at every site)
constexpr float kHalfSqrt3Lo = (float)(0.86602540378443864676 - (double)kHalfSqrt3);
constexpr float kInv2Sqrt3 = 0.28867513459481288225f;        // 1/(2 sqrt 3)
// 1/12 as an unevaluated float pair: float(1/12) is 3e-8 too large, which
// would add a same-signed bias to the mass of every relaxed site; rho * hi +
// rho * lo (one fma) is within an ulp of rho/12 with no systematic sign.
constexpr float kTwelfthHi = (float)(1.0 / 12.0);
constexpr float kTwelfthLo = (float)(1.0 / 12.0 - (double)(float)(1.0 / 12.0));

// rho and j = sum f_i e_i, with the momentum taken over opposite pairs so
// that a pairwise-symmetric site has exactly zero momentum.
__device__ __forceinline__ void site_moments(const float f[7], float &rho, float &jx, float &jy)
{
    rho = f[0] + ((f[1] + f[4]) + ((f[2] + f[5]) + (f[3] + f[6])));
    const float d1 = f[1] - f[4], d2 = f[2] - f[5], d3 = f[3] - f[6];
    jx = d1 + 0.5f * (d2 - d3);
    jy = kHalfSqrt3 * (d2 + d3);
}

// CIL target velocity: u* = U0(rho) j/|j|, U0 = max(B - A rho^2, 0); zero
// where j = 0.  Passive: u* = j/rho (zero where rho = 0).
template <int M>
__device__ __forceinline__ void local_ustar(const StepArgs &a, float rho, float jx, float jy, float &ux, float &uy)
{
    if (M == kCil) {
        // 1/|j| from the hardware reciprocal square root, which flushes
        // denormal inputs: jn2 is taken times 2^32 (exact, and normal for
        // every jn2 > 0 below 2^96), and U0 comes times 2^16 from the
        // pre-scaled A and B (exact), so s = U0 / |j| with no extra rounding
        const float u0s = fmaxf(a.B16 - a.A16 * rho * rho, 0.0f);
        const float jn2 = jx * jx + jy * jy;
        const float s = jn2 > 0.0f ? u0s * __builtin_amdgcn_rsqf(jn2 * 0x1p32f) : 0.0f;
        ux = s * jx;
        uy = s * jy;
    } else {
        const float r = rho != 0.0f ? __builtin_amdgcn_rcpf(rho) : 0.0f;
        ux = jx * r;
        uy = jy * r;
    }
}

// MIPS target velocity (eq. bu_mips) from the density gradient, with the
// U_max clamp that keeps the direction.
__device__ __forceinline__ void mips_from_gradient(const StepArgs &a, float rho, float gx, float gy, float &ux,
                                                   float &uy)
{
    float k = 0.0f;
    if (rho < a.rho_star)
        k = a.C * (1.0f - rho * a.inv_rho_star);
    ux = k * gx;
    uy = k * gy;
    const float un2 = ux * ux + uy * uy;
    if (un2 > a.u_max * a.u_max) {
        const float s = a.u_max * rsqrtf(un2);
        ux *= s;
        uy *= s;
    }
}

// MIPS target velocity from the six neighbour densities (isotropic stencil,
// component form).
__device__ __forceinline__ void mips_ustar(const StepArgs &a, float rho, const float nb[7], float &ux, float &uy)
{
    const float gx = (2.0f * (nb[1] - nb[4]) + (nb[2] + nb[6]) - (nb[3] + nb[5])) * (1.0f / 6.0f);
    const float gy = ((nb[2] + nb[3]) - (nb[5] + nb[6])) * kInv2Sqrt3;
    mips_from_gradient(a, rho, gx, gy, ux, uy);
}

// Steady state xi(rho, u) of eq. fssD2Q7 in pair form: a_k = e_k.u,
// base = 1 - 2|u|^2, xi_{k, k+3} = (rho/12)(base + 8 a_k^2 +- 4 a_k),
// xi_0 = (rho/2) base.
// ADD: eq_i + add_i, each with one rounding of the last product.
template <bool ADD = false>
__device__ __forceinline__ void site_equilibrium(float rho, float ux, float uy, float eq[7],
                                                 const float *add = nullptr)
{
    const float usq = ux * ux + uy * uy;
    const float a1 = ux;
    const float a2 = fmaf(kHalfSqrt3Lo, uy, fmaf(kHalfSqrt3, uy, 0.5f * ux));
    const float a3 = fmaf(kHalfSqrt3Lo, uy, fmaf(kHalfSqrt3, uy, -0.5f * ux));
    const float r12 = fmaf(rho, kTwelfthHi, rho * kTwelfthLo);
    const float base = 1.0f - 2.0f * usq;
    const float b1 = base + 8.0f * a1 * a1, b2 = base + 8.0f * a2 * a2, b3 = base + 8.0f * a3 * a3;
    const float q[7] = {base,           b1 + 4.0f * a1, b2 + 4.0f * a2, b3 + 4.0f * a3,
                        b1 - 4.0f * a1, b2 - 4.0f * a2, b3 - 4.0f * a3};
    const float r0 = 0.5f * rho;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const float r = i == 0 ? r0 : r12;
        eq[i] = ADD ? fmaf(r, q[i], add[i]) : r * q[i];
    }
}

// Compile-time variants (no uniform branches inside the site body).
enum StepFlags : int { kUnitTau = 1, kNoisy = 2 };

// BGK relaxation towards xi(rho, u*) (eq. fssD2Q7), zero-sum noise, and the
// negative correction (pair form, rescale to rho where a rule fired).  The
// relaxation and the noise conserve the site's mass exactly, so the rest
// population is taken as rho minus the six moving ones: the site then keeps
// its mass to one rounding, where the same formula term by term (the rounded
// products of xi) drifted by ~1e-9 of the mass per step, the same sign at
// every site.  In float32 storage that value enters the correction as the
// rest population; in the 16-bit storages (S) it is taken from the moving
// populations as they will be stored, at sites where no rule fired (where
// one fires, the rescale to rho sets the mass); with a float32 rest plane
// (kBf16R32) at every site, after the correction.  tau = +inf keeps the
// populations as they are.
template <int F, int S = kF32>
__device__ __forceinline__ void site_collide(const StepArgs &a, float f[7], float rho, float ux, float uy,
                                             uint32_t site, uint32_t t_lo, uint32_t t_hi)
{
    float nz[7];
    if (F & kNoisy)
        site_noise(a, site, t_lo, t_hi, nz);
    if (F & kUnitTau) {
        // tau = 1 (the paper's CIL runs): the relaxation lands on xi exactly,
        // and the noise is added by the last product of xi
        if (F & kNoisy)
            site_equilibrium<true>(rho, ux, uy, f, nz);
        else
            site_equilibrium(rho, ux, uy, f);
    } else {
        float eq[7];
        site_equilibrium(rho, ux, uy, eq);
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            f[i] = f[i] - (f[i] - eq[i]) * a.omega;
            if (F & kNoisy)
                f[i] += nz[i];
        }
    }
    const bool absorb = (F & kUnitTau) || a.omega != 0.0f;
    if constexpr (S == kF32 || S == kBf16R32) {
        if (absorb)
            f[0] = rho - ((f[1] + f[4]) + ((f[2] + f[5]) + (f[3] + f[6])));
    }
    // f < 0 as a class test (negative infinity, normal, denormal or zero):
    // one compare per population with no NaN canonicalisation, NaN excluded
    // as by the ordered compare.  -0 counts as negative here; the rules then
    // leave the values as they are and only the rescale to rho runs.
    constexpr int kNegative = 0x3c;
    bool fired = false;
    if (__builtin_amdgcn_classf(f[0], kNegative)) {
        f[0] = 0.0f;
        fired = true;
    }
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (__builtin_amdgcn_classf(f[k], kNegative) | __builtin_amdgcn_classf(f[k + 3], kNegative)) {
            const float d = f[k] - f[k + 3];
            f[k] = fmaxf(d, 0.0f);
            f[k + 3] = fmaxf(-d, 0.0f);
            fired = true;
        }
    }
    if constexpr (S == kBf16Dev || S == kF16Dev) {
        if (!fired && absorb) {
            float g[7];
#pragma unroll
            for (int i = 1; i < 7; ++i)
                g[i] = Store<S>::round(f[i], a.wr1);
            f[0] = rho - ((g[1] + g[4]) + ((g[2] + g[5]) + (g[3] + g[6])));
        }
    }
    if (fired) {
        // every f_i >= 0 here, so a zero sum means zero populations and the
        // factor 0 gives them back unchanged
        const float s = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6];
        // the hardware reciprocal refined by one Newton step (within an ulp
        // alone but not unbiased, and this branch runs at every site where a
        // population went negative)
        float q = __builtin_amdgcn_rcpf(s);
        q = fmaf(fmaf(-s, q, 1.0f), q, q);
        const float r = s > 0.0f ? rho * q : 0.0f;
#pragma unroll
        for (int i = 0; i < 7; ++i)
            f[i] *= r;
    }
    if constexpr (S == kBf16R32) {
        // bfloat16 moving populations, float32 rest population: the rest
        // population takes rho minus the moving ones as they will be stored,
        // at every site (corrected ones included), so the stored site holds
        // its mass to one float32 rounding; it stays >= 0 (where the moving
        // roundings exceed a corrected rest population of ~0, that excess is
        // the only mass the step does not keep)
        if (absorb) {
            float g[7];
#pragma unroll
            for (int i = 1; i < 7; ++i)
                g[i] = Store<kBf16Dev>::round(f[i], a.wr1);
            f[0] = fmaxf(rho - ((g[1] + g[4]) + ((g[2] + g[5]) + (g[3] + g[6]))), 0.0f);
        }
    }
}

// Streaming sources (step (i)): after streaming, population i at site r is
// the one that sat at r - e_i.  On offset rows with p = y & 1 those sites are
// e_1: (x-1, y), e_2: (x-1+p, y-1), e_3: (x+p, y-1), e_4: (x+1, y),
// e_5: (x+p, y+1), e_6: (x-1+p, y+1), all periodic.
struct PullSources {
    int64_t idx[7];
};

__device__ __forceinline__ PullSources pull_sources(const StepArgs &a, int x, int y)
{
    const int p = y & 1;
    const int xm = x == 0 ? a.nx - 1 : x - 1;
    const int xp = x == a.nx - 1 ? 0 : x + 1;
    const int yu = y == a.ny - 1 ? 0 : y + 1;
    const int yd = y == 0 ? a.ny - 1 : y - 1;
    const int xr = p ? xp : x;  // x + p
    const int xl = p ? x : xm;  // x - 1 + p
    const int64_t P = a.pitch;
    PullSources t;
    t.idx[0] = (int64_t)y * P + x;
    t.idx[1] = (int64_t)y * P + xm;
    t.idx[2] = (int64_t)yd * P + xl;
    t.idx[3] = (int64_t)yd * P + xr;
    t.idx[4] = (int64_t)y * P + xp;
    t.idx[5] = (int64_t)yu * P + xr;
    t.idx[6] = (int64_t)yu * P + xl;
    return t;
}

// The same with 32-bit element offsets (buffers below 2^30 elements, checked
// on the host).
struct PullSources32 {
    uint32_t idx[7];
};

__device__ __forceinline__ PullSources32 pull_sources32(const StepArgs &a, int x, int y)
{
    const int p = y & 1;
    const uint32_t xm = x == 0 ? a.nx - 1 : x - 1;
    const uint32_t xp = x == a.nx - 1 ? 0 : x + 1;
    const uint32_t P = (uint32_t)a.pitch;
    const uint32_t ry = (uint32_t)y * P;
    const uint32_t ru = y == a.ny - 1 ? 0u : ry + P;
    const uint32_t rd = y == 0 ? (uint32_t)(a.ny - 1) * P : ry - P;
    const uint32_t xr = p ? xp : (uint32_t)x;  // x + p
    const uint32_t xl = p ? (uint32_t)x : xm;  // x - 1 + p
    PullSources32 t;
    t.idx[0] = ry + x;
    t.idx[1] = ry + xm;
    t.idx[2] = rd + xl;
    t.idx[3] = rd + xr;
    t.idx[4] = ry + xp;
    t.idx[5] = ru + xr;
    t.idx[6] = ru + xl;
    return t;
}

// Periodic image of a coordinate c in [-1, n + 65] on a ring of n sites.
__device__ __forceinline__ int wrap_coord(int c, int n)
{
    if (c < 0)
        c += n;
    if (c >= n)
        c -= n;
    if (c >= n)  // rings shorter than the widened tile
        c %= n;
    return c;
}

// Blocks are handed to the eight XCDs round-robin (block b runs on XCD
// b mod 8).  Tiles are therefore taken in groups of 8 rows: with a grid of
// (8 ntx, ceil(nty / 8)) blocks, block (bx, by) covers tile row 8 by + (bx & 7)
// and tile column bx >> 3.  A whole row of tiles then runs on one XCD (the
// x-shifted loads at tile edges hit that XCD's L2 instead of being fetched
// twice, measured +7% read traffic otherwise) while each round of eight
// blocks still touches eight adjacent rows.  Blocks past the last tile row
// exit at once.
__device__ __forceinline__ void row_group_tile(int &tx, int &ty)
{
    ty = 8 * (int)blockIdx.y + (int)(blockIdx.x & 7u);
    tx = (int)(blockIdx.x >> 3);
}

// Element access through a uniform base pointer and a 32-bit byte offset,
// which maps onto the scalar-base + vector-offset global addressing mode.
template <typename T>
__device__ __forceinline__ T ld32(const T *base, uint32_t elem)
{
    return *(const T *)((const char *)base + elem * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T *base, uint32_t elem, T v)
{
    *(T *)((char *)base + elem * (uint32_t)sizeof(T)) = v;
}

// Buffer-resource access (gfx9 raw buffers: stride 0, 32-bit data format in
// the third descriptor word).  One resource spans a whole population buffer;
// the plane offset goes in the scalar offset and the element offset in the
// vector offset, so no per-lane 64-bit address is formed.  Accesses past
// num_records bytes read 0 and write nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// Cache policy of a buffer store (the instruction's auxiliary bits on
// gfx950): kStoreCached keeps the written lines in L2 and the Infinity
// Cache, kStoreStream marks them non-temporal.  A step over a lattice whose
// two buffers cannot stay in the 256 MB Infinity Cache never reads its
// output within the launch, and streaming its stores moved the 4096^2 FP32
// step from 173.8 to 167.9 us; on a cache-resident state they cost 10%.
constexpr int kStoreCached = 0, kStoreStream = 2;
// the two buffers' size above which a single-lattice step streams its
// stores: the budget the batched sweep keeps a lattice group's state within
constexpr uint64_t kStreamStateBytes = 240ull << 20;

template <typename T>
struct BufIO;

template <>
struct BufIO<float> {
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, elem * 4u, first * 4u, 0));
    }
    template <int CP = kStoreCached>
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, elem * 4u, first * 4u, CP);
    }
};

template <>
struct BufIO<uint16_t> {
    __device__ __forceinline__ static uint16_t load(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, elem * 2u, first * 2u, 0);
    }
    template <int CP = kStoreCached>
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first, uint16_t v)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, elem * 2u, first * 2u, CP);
    }
};

template <>
struct BufIO<_Float16> {
    __device__ __forceinline__ static _Float16 load(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first)
    {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, elem * 2u, first * 2u, 0));
    }
    template <int CP = kStoreCached>
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t elem, uint32_t first, _Float16 v)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, elem * 2u, first * 2u, CP);
    }
};

// Population planes of a buffer in storage S, plane i of `plane` elements:
// load / store of element v + s of plane i through a buffer resource (v the
// per-lane part, s the wave-uniform part; stores with cache policy CP), the
// same through a plain pointer
// (ld / st), the value a store and a later load give back (round), and the
// buffer's size in bytes.  One type per buffer except kBf16R32, whose rest
// plane is float32 (two 16-bit planes of room) before six bfloat16 planes.
template <int S>
struct Planes {
    using T = typename Store<S>::T;
    __host__ __device__ static constexpr uint64_t bytes(uint64_t plane) { return 7u * plane * sizeof(T); }
    __device__ __forceinline__ static float wr(int i, const StepArgs &a) { return i == 0 ? a.wr0 : a.wr1; }
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, int i,
                                                 uint32_t plane, const StepArgs &a)
    {
        return Store<S>::widen(BufIO<T>::load(r, v, (uint32_t)i * plane + s), wr(i, a));
    }
    template <int CP = kStoreCached>
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, int i,
                                                 uint32_t plane, float x, const StepArgs &a)
    {
        BufIO<T>::template store<CP>(r, v, (uint32_t)i * plane + s, Store<S>::narrow(x, wr(i, a)));
    }
    __device__ __forceinline__ static float ld(const T *p, int64_t e, int i, int64_t plane, const StepArgs &a)
    {
        return Store<S>::load(p, i * plane + e, wr(i, a));
    }
    __device__ __forceinline__ static void st(T *p, int64_t e, int i, int64_t plane, float x, const StepArgs &a)
    {
        Store<S>::store(p, i * plane + e, x, wr(i, a));
    }
    __device__ __forceinline__ static float round(float x, int i, const StepArgs &a) { return Store<S>::round(x, wr(i, a)); }
};

template <>
struct Planes<kBf16R32> {
    using T = uint16_t;
    __host__ __device__ static constexpr uint64_t bytes(uint64_t plane) { return 16u * plane; }
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, int i,
                                                 uint32_t plane, const StepArgs &a)
    {
        if (i == 0)
            return BufIO<float>::load(r, v, s);
        return Store<kBf16Dev>::widen(BufIO<uint16_t>::load(r, v, (uint32_t)(i + 1) * plane + s), a.wr1);
    }
    template <int CP = kStoreCached>
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, int i,
                                                 uint32_t plane, float x, const StepArgs &a)
    {
        if (i == 0)
            BufIO<float>::store<CP>(r, v, s, x);
        else
            BufIO<uint16_t>::store<CP>(r, v, (uint32_t)(i + 1) * plane + s, Store<kBf16Dev>::narrow(x, a.wr1));
    }
    __device__ __forceinline__ static float ld(const T *p, int64_t e, int i, int64_t plane, const StepArgs &a)
    {
        if (i == 0)
            return ((const float *)p)[e];
        return Store<kBf16Dev>::load(p, (i + 1) * plane + e, a.wr1);
    }
    __device__ __forceinline__ static void st(T *p, int64_t e, int i, int64_t plane, float x, const StepArgs &a)
    {
        if (i == 0)
            ((float *)p)[e] = x;
        else
            Store<kBf16Dev>::store(p, (i + 1) * plane + e, x, a.wr1);
    }
    __device__ __forceinline__ static float round(float x, int i, const StepArgs &a)
    {
        return i == 0 ? x : Store<kBf16Dev>::round(x, a.wr1);
    }
};

// ---------------------------------------------------------------------------
// MIPS step of one 64 x ROWS tile at (x0, y0), ROWS = 4 or 16 (u* needs the
// streamed density of the six neighbours).  256 threads: wave w owns rows w,
// w+4, ..., one column per lane.  rho of the tile and of a one-site ring (the
// rows above and below and the two edge columns: 2 x 66 + 2 ROWS sites, taken
// by waves 0-2) is staged in LDS (srho, mips_tile_lds(ROWS) floats).  The tile's own populations stay
// in registers from the density pass to the collision; every load of a wave
// is issued before any of its sites is computed.  On tiles whose sources do
// not wrap, a row's seven loads share one vector offset (the lane) and
// wave-uniform scalar offsets.  Every LDS slot holds rho at its periodically
// wrapped lattice site, so ragged tiles and lattices narrower than a tile need
// no special case.  rs / rd cover the source and destination population
// buffers ([7][ny][pitch], 32-bit element offsets).  The single-lattice and
// the batched MIPS kernels both run this body.
// ---------------------------------------------------------------------------
constexpr int kMipsRows = 16;
constexpr int kMipsWaves = 8;
constexpr int mips_tile_lds(int rows) { return (rows + 2) * 66; }

template <int S, int F, int ROWS = kMipsRows, int NW = 4, int CP = kStoreCached>
__device__ __forceinline__ void mips_tile_step(__amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rd,
                                               const StepArgs &a, int x0, int y0, uint32_t t_lo, uint32_t t_hi,
                                               float *srho)
{
    constexpr int W = 66, H = ROWS + 2, RW = ROWS / NW;  // RW rows per wave
    constexpr int kRing = 2 * W + 2 * ROWS;
    static_assert(NW % 2 == 0 && ROWS % NW == 0 && kRing <= 64 * NW, "NW waves own the rows and cover the ring");
    const uint32_t plane = (uint32_t)a.plane, P = (uint32_t)a.pitch, nx = (uint32_t)a.nx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool interior = x0 >= 1 && x0 + 65 <= a.nx && y0 >= 1 && y0 + ROWS + 1 <= a.ny;
    // the seven streamed populations of site (x, y), periodically wrapped
    auto load_wrapped = [&](float *g, int x, int y) {
        const PullSources32 q = pull_sources32(a, wrap_coord(x, a.nx), wrap_coord(y, a.ny));
#pragma unroll
        for (int i = 0; i < 7; ++i)
            g[i] = Planes<S>::load(rs, q.idx[i], 0u, i, plane, a);
    };
    float f[RW][7];
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int y = y0 + wv + NW * k;
        if (interior) {
            const uint32_t p = (uint32_t)y & 1u;
            const uint32_t c = (uint32_t)y * P + (uint32_t)x0;  // offset of (x0, y)
            const uint32_t e[7] = {c, c - 1u, c - P - 1u + p, c - P + p, c + 1u, c + P + p, c + P - 1u + p};
#pragma unroll
            for (int i = 0; i < 7; ++i)
                f[k][i] = Planes<S>::load(rs, lane, e[i], i, plane, a);
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
            rlx = re < 2 * W + ROWS ? 0 : W - 1;
            rly = 1 + (re - 2 * W) % ROWS;
        }
        float g[7];
        load_wrapped(g, x0 - 1 + rlx, y0 - 1 + rly);
        srho[rly * W + rlx] = g[0] + ((g[1] + g[4]) + ((g[2] + g[5]) + (g[3] + g[6])));
    }
    float rho[RW];
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        float jx, jy;
        site_moments(f[k], rho[k], jx, jy);
        srho[(wv + NW * k + 1) * W + lane + 1] = rho[k];
    }
    __syncthreads();
    // collisions; row r of the tile has parity r & 1 = wv & 1 (y0 is even)
    const int p = wv & 1;
    const int x = x0 + lane;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        const int r = wv + NW * k, y = y0 + r;
        if (x >= a.nx || y >= a.ny)
            continue;
        const int cx = lane + 1, cy = r + 1;
        float nb[7];
        nb[0] = rho[k];
        nb[1] = srho[cy * W + cx + 1];
        nb[2] = srho[(cy + 1) * W + cx + p];
        nb[3] = srho[(cy + 1) * W + cx - 1 + p];
        nb[4] = srho[cy * W + cx - 1];
        nb[5] = srho[(cy - 1) * W + cx - 1 + p];
        nb[6] = srho[(cy - 1) * W + cx + p];
        float ux, uy;
        mips_ustar(a, rho[k], nb, ux, uy);
        site_collide<F, S>(a, f[k], rho[k], ux, uy, (uint32_t)y * nx + (uint32_t)x, t_lo, t_hi);
        const uint32_t own = (uint32_t)y * P + (uint32_t)x;
#pragma unroll
        for (int i = 0; i < 7; ++i)
            Planes<S>::template store<CP>(rd, own, 0u, i, plane, f[k][i], a);
    }
}

}  // namespace lbm
