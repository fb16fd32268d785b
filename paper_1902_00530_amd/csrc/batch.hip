// Batched sweeps: many independent lattices of different sizes and
// parameters advanced together (one kernel launch per step, or per two steps,
// covers every lattice), with FP64 observables sampled every sample_every
// steps.
//
// Work list.  Each lattice is cut into TX x TY tiles; the list of all tiles
// of all lattices is built on the host.  Within a lattice, tiles are listed
// in groups of eight tile rows, column by column, so that tile list position
// b runs on XCD b mod 8 and a whole row of tiles stays on one XCD (the same
// order as the single-lattice kernel).  A block reads its tile and its
// lattice's descriptor with scalar loads and runs the same site body as the
// single-lattice kernel, so a batch member gives bit-for-bit the result of
// the single-lattice call with the same seed.
//
// Two steps per launch.  The state of step t+1 at a site depends on the state
// of step t at the site and its six neighbours (one streaming move), so the
// state of step t+2 on a 64 x TY tile needs step t+1 on the tile widened by
// one site on every side, which needs step t widened by two.  The two-step
// kernel computes step t+1 on the widened tile into LDS (gathering step t
// from HBM), then step t+2 on the tile from LDS, and writes only that: one
// read and one write of the state per two updates, for about
// (66 (TY + 2)) / (64 TY) - 1 extra site bodies.
//
// Step loop.  One sample period (its step kernels, the sampling kernels, one
// counter update) is captured once in a HIP graph and replayed; the step
// index and the buffer parity come from a small control block in device
// memory that the last node advances, so no kernel arguments change between
// replays and no kernel waits on another workgroup.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "device_q9.h"
#include "internal.h"

namespace lbm {

struct BatchTile {
    int32_t lat;
    int16_t tx, ty;
};

struct LatDesc {
    StepArgs a;
    void *buf[2];
    float B;            // CIL B for zeta
    int32_t mt_begin;   // first moments tile
    int32_t mt_count;   // moments tiles of this lattice
    int32_t nrb;        // moments row blocks
    int64_t col_off;    // offset of this lattice's column partials
    int64_t cm_off;     // offset of this lattice's column means
    float add;          // added to every population after each sample (drho / Q)
    int32_t stream;     // 1: stores streamed past the caches (two buffers beyond the
                        // Infinity Cache budget: the lattice is a group of its own)
};

// A batch kernel's population stores at element v + s of each plane:
// streamed past the caches for a lattice flagged LatDesc::stream (uniform per
// block), cached otherwise, where the next launch or a later lattice group
// reads them from the Infinity Cache.
template <int ST>
__device__ __forceinline__ void batch_store7(bool stream, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s,
                                             uint32_t plane, const float f[7], const StepArgs &a)
{
    if (stream) {
#pragma unroll
        for (int i = 0; i < 7; ++i)
            Planes<ST>::template store<kStoreStream>(r, v, s, i, plane, f[i], a);
    } else {
#pragma unroll
        for (int i = 0; i < 7; ++i)
            Planes<ST>::store(r, v, s, i, plane, f[i], a);
    }
}

__device__ __forceinline__ void batch_store9(bool stream, float *dst, uint32_t plane, uint32_t v, uint32_t s,
                                             const float f[9])
{
    if (stream) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            BufIO<float>::store<kStoreStream>(q9_plane_rsrc(dst, i, plane), v, s, f[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            BufIO<float>::store(q9_plane_rsrc(dst, i, plane), v, s, f[i]);
    }
}

struct MomTile {
    int32_t lat;
    int16_t cx, cy;
};

struct Ctrl {
    int64_t t0;      // absolute step index of the next step
    int64_t k0;      // steps done in this sweep (buffer parity)
    int64_t sample;  // index of the next sample
    int64_t pad;
};

constexpr int kMomRows = 16;

// ---------------------------------------------------------------------------
// Step kernels over the tile list.  step_off: steps of this sample period
// before this launch; launch_off: launches before it (the buffer parity).
// ---------------------------------------------------------------------------
template <int M, int ST, int F>
__global__ __launch_bounds__(256) void k_batch_step(const BatchTile *__restrict__ tiles,
                                                    const LatDesc *__restrict__ lats,
                                                    const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x = tl.tx * blockDim.x + threadIdx.x;
    const int y = tl.ty * blockDim.y + threadIdx.y;
    if (x >= a.nx || y >= a.ny)
        return;
    const uint32_t plane = (uint32_t)a.plane;
    const __amdgpu_buffer_rsrc_t src = buffer_rsrc(L.buf[par], (uint32_t)Planes<ST>::bytes(plane));
    const __amdgpu_buffer_rsrc_t dst = buffer_rsrc(L.buf[par ^ 1], (uint32_t)Planes<ST>::bytes(plane));
    const PullSources32 g_src = pull_sources32(a, x, y);
    float f[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
        f[i] = Planes<ST>::load(src, g_src.idx[i], 0u, i, plane, a);
    float rho, jx, jy, ux, uy;
    site_moments(f, rho, jx, jy);
    local_ustar<M>(a, rho, jx, jy, ux, uy);
    // batch buffers have pitch nx, so the own offset is the site index
    const uint32_t own = g_src.idx[0];
    site_collide<F, ST>(a, f, rho, ux, uy, own, (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32));
    batch_store7<ST>(L.stream != 0, dst, own, 0u, plane, f, a);
}

// MIPS over a list of 64 x ROWS tiles (the tile body of the single-lattice
// MIPS kernel, mips_tile_step), one step per launch.
template <int ST, int F, int ROWS>
__global__ __launch_bounds__(256) void k_batch_step_mips(const BatchTile *__restrict__ tiles,
                                                         const LatDesc *__restrict__ lats,
                                                         const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    __shared__ float srho[mips_tile_lds(ROWS)];
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x0 = tl.tx * 64, y0 = tl.ty * ROWS;
    if (x0 >= a.nx || y0 >= a.ny)  // whole-block exit, before the barrier
        return;
    const uint32_t bytes = (uint32_t)Planes<ST>::bytes(a.plane);
    mips_tile_step<ST, F, ROWS>(buffer_rsrc(L.buf[par], bytes), buffer_rsrc(L.buf[par ^ 1], bytes), a, x0, y0,
                            (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32), srho);
}

// Whole lattices resident in LDS (D2Q7, at most kResidentSites sites each):
// one workgroup of 1024 lanes per lattice runs every step of the launch
// without leaving its CU.  The state is read from HBM once; each step pulls
// every site's populations out of LDS into registers (for MIPS also putting
// each site's density into LDS), waits, collides with the site body of the
// tile kernels and writes the populations back to LDS in place; after the
// last step the state goes to HBM, into the buffer the step count's parity
// names (as after the same number of one-step launches).  A lattice of the
// paper's size (90 x 30) then costs one CU for a whole sample period instead
// of a launch per step.  Results equal the tile kernels' bit for bit.
constexpr int kResidentSites = 4096;
constexpr int kResidentLanes = 1024;
constexpr int kResidentPer = (kResidentSites + kResidentLanes - 1) / kResidentLanes;  // sites per lane

template <int M, int ST, int F>
__global__ __launch_bounds__(kResidentLanes) void k_batch_resident(const LatDesc *__restrict__ lats,
                                                                  const Ctrl *__restrict__ ctrl, int steps)
{
    using T = typename Store<ST>::T;
    __shared__ float st[8 * kResidentSites];  // plane i of the state at i * S, densities at 7 * S
    const LatDesc &L = lats[blockIdx.x];
    const StepArgs a = L.a;  // pitch nx: plane i holds S = nx * ny contiguous elements
    const int S = a.nx * a.ny;
    const int par = (int)(ctrl->k0 & 1);
    const T *__restrict__ src = (const T *)L.buf[par];
    T *__restrict__ dst = (T *)L.buf[par ^ (steps & 1)];
    const int tid = threadIdx.x;
    float *rho_l = st + 7 * S;
    // the state is kept in LDS as stored (16-bit storages: the stored bits),
    // so every step rounds and widens exactly as lbm_step's loads and stores;
    // with a float32 rest plane (kBf16R32) as the values the storage gives
    // back, in float32
    constexpr bool kFloatLds = ST == kBf16R32;
    T *sv = (T *)st;
#pragma unroll
    for (int i = 0; i < 7; ++i)
        for (int e = tid; e < S; e += kResidentLanes) {
            if constexpr (kFloatLds)
                st[i * S + e] = Planes<ST>::ld(src, e, i, a.plane, a);
            else
                sv[i * S + e] = src[(int64_t)i * a.plane + e];
        }
    // this lane's sites s = tid + j * 1024 and their coordinates
    int sx[kResidentPer], sy[kResidentPer];
#pragma unroll
    for (int j = 0; j < kResidentPer; ++j) {
        const int s = tid + j * kResidentLanes;
        sy[j] = s / a.nx;
        sx[j] = s - sy[j] * a.nx;
    }
    __syncthreads();
    const int64_t t0 = ctrl->t0;
    for (int k = 0; k < steps; ++k) {
        const uint64_t t = (uint64_t)(t0 + k);
        const uint32_t tlo = (uint32_t)(t & 0xffffffffu), thi = (uint32_t)(t >> 32);
        float f[kResidentPer][7], rho[kResidentPer], jx[kResidentPer], jy[kResidentPer];
#pragma unroll
        for (int j = 0; j < kResidentPer; ++j) {
            const int s = tid + j * kResidentLanes;
            if (s < S) {
                const PullSources32 q = pull_sources32(a, sx[j], sy[j]);
#pragma unroll
                for (int i = 0; i < 7; ++i) {
                    if constexpr (kFloatLds)
                        f[j][i] = st[i * S + (int)q.idx[i]];
                    else
                        f[j][i] = Store<ST>::widen(sv[i * S + (int)q.idx[i]], i == 0 ? a.wr0 : a.wr1);
                }
                site_moments(f[j], rho[j], jx[j], jy[j]);
                if (M == kMips)
                    rho_l[s] = rho[j];
            }
        }
        __syncthreads();  // every pull done (the state may be overwritten), densities in place
#pragma unroll
        for (int j = 0; j < kResidentPer; ++j) {
            const int s = tid + j * kResidentLanes;
            if (s < S) {
                float ux, uy;
                if (M == kMips) {
                    // density at r + e_i: the pull source of the opposite population
                    const PullSources32 q = pull_sources32(a, sx[j], sy[j]);
                    float nb[7];
                    nb[0] = rho[j];
                    nb[1] = rho_l[q.idx[4]];
                    nb[2] = rho_l[q.idx[5]];
                    nb[3] = rho_l[q.idx[6]];
                    nb[4] = rho_l[q.idx[1]];
                    nb[5] = rho_l[q.idx[2]];
                    nb[6] = rho_l[q.idx[3]];
                    mips_ustar(a, rho[j], nb, ux, uy);
                } else {
                    local_ustar<M>(a, rho[j], jx[j], jy[j], ux, uy);
                }
                site_collide<F, ST>(a, f[j], rho[j], ux, uy, (uint32_t)s, tlo, thi);
#pragma unroll
                for (int i = 0; i < 7; ++i) {
                    if constexpr (kFloatLds)
                        st[i * S + s] = Planes<ST>::round(f[j][i], i, a);
                    else
                        sv[i * S + s] = Store<ST>::narrow(f[j][i], i == 0 ? a.wr0 : a.wr1);
                }
            }
        }
        __syncthreads();  // the step's writes precede the next step's pulls
    }
#pragma unroll
    for (int i = 0; i < 7; ++i)
        for (int e = tid; e < S; e += kResidentLanes) {
            if constexpr (kFloatLds)
                Planes<ST>::st(dst, e, i, a.plane, st[i * S + e], a);
            else
                dst[(int64_t)i * a.plane + e] = sv[i * S + e];
        }
}

// The same for the square lattice (D2Q9): nine planes and the densities, at
// most kResidentSitesQ9 sites (120 KiB of LDS), the site body of the D2Q9
// tile kernels (q9_moments, local_ustar or q9_mips_ustar, q9_collide).
constexpr int kResidentSitesQ9 = 3072;
constexpr int kResidentPerQ9 = (kResidentSitesQ9 + kResidentLanes - 1) / kResidentLanes;

template <int M, int F>
__global__ __launch_bounds__(kResidentLanes) void k_batch_resident_q9(const LatDesc *__restrict__ lats,
                                                                     const Ctrl *__restrict__ ctrl, int steps)
{
    __shared__ float st[10 * kResidentSitesQ9];  // plane i of the state at i * S, densities at 9 * S
    const LatDesc &L = lats[blockIdx.x];
    const StepArgs a = L.a;  // pitch nx: plane i holds S = nx * ny contiguous floats
    const int S = a.nx * a.ny;
    const int par = (int)(ctrl->k0 & 1);
    const float *__restrict__ src = (const float *)L.buf[par];
    float *__restrict__ dst = (float *)L.buf[par ^ (steps & 1)];
    const int tid = threadIdx.x;
    float *rho_l = st + 9 * S;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        for (int e = tid; e < S; e += kResidentLanes)
            st[i * S + e] = src[(int64_t)i * a.plane + e];
    int sx[kResidentPerQ9], sy[kResidentPerQ9];
#pragma unroll
    for (int j = 0; j < kResidentPerQ9; ++j) {
        const int s = tid + j * kResidentLanes;
        sy[j] = s / a.nx;
        sx[j] = s - sy[j] * a.nx;
    }
    __syncthreads();
    const int64_t t0 = ctrl->t0;
    for (int k = 0; k < steps; ++k) {
        const uint64_t t = (uint64_t)(t0 + k);
        const uint32_t tlo = (uint32_t)(t & 0xffffffffu), thi = (uint32_t)(t >> 32);
        float f[kResidentPerQ9][9], rho[kResidentPerQ9], jx[kResidentPerQ9], jy[kResidentPerQ9];
#pragma unroll
        for (int j = 0; j < kResidentPerQ9; ++j) {
            const int s = tid + j * kResidentLanes;
            if (s < S) {
                const Q9Sources q = q9_sources(a, sx[j], sy[j]);
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[j][i] = st[i * S + (int)q.idx[i]];
                q9_moments(f[j], rho[j], jx[j], jy[j]);
                if (M == kMips)
                    rho_l[s] = rho[j];
            }
        }
        __syncthreads();  // every pull done (the state may be overwritten), densities in place
#pragma unroll
        for (int j = 0; j < kResidentPerQ9; ++j) {
            const int s = tid + j * kResidentLanes;
            if (s < S) {
                float ux, uy;
                if (M == kMips) {
                    // density at r + e_i: the pull source of the opposite population
                    const Q9Sources q = q9_sources(a, sx[j], sy[j]);
                    float nb[9];
                    nb[0] = rho[j];
                    nb[1] = rho_l[q.idx[3]];
                    nb[2] = rho_l[q.idx[4]];
                    nb[3] = rho_l[q.idx[1]];
                    nb[4] = rho_l[q.idx[2]];
                    nb[5] = rho_l[q.idx[7]];
                    nb[6] = rho_l[q.idx[8]];
                    nb[7] = rho_l[q.idx[5]];
                    nb[8] = rho_l[q.idx[6]];
                    q9_mips_ustar(a, rho[j], nb, ux, uy);
                } else {
                    local_ustar<M>(a, rho[j], jx[j], jy[j], ux, uy);
                }
                q9_collide<F>(a, f[j], rho[j], ux, uy, (uint32_t)s, tlo, thi);
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    st[i * S + s] = f[j][i];
            }
        }
        __syncthreads();  // the step's writes precede the next step's pulls
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        for (int e = tid; e < S; e += kResidentLanes)
            dst[(int64_t)i * a.plane + e] = st[i * S + e];
}

// The square lattice (D2Q9) over the tile list: the single-lattice site body
// (passive, CIL) and MIPS tile body, one step per launch.
template <int M, int F>
__global__ __launch_bounds__(256) void k_batch_q9_step(const BatchTile *__restrict__ tiles,
                                                       const LatDesc *__restrict__ lats,
                                                       const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x = tl.tx * blockDim.x + threadIdx.x;
    const int y = tl.ty * blockDim.y + threadIdx.y;
    if (x >= a.nx || y >= a.ny)
        return;
    q9_site_step<M, kF32, F>((const float *)L.buf[par], (float *)L.buf[par ^ 1], a, x, y,
                             (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32));
}

template <int F>
__global__ __launch_bounds__(256) void k_batch_q9_step_mips(const BatchTile *__restrict__ tiles,
                                                            const LatDesc *__restrict__ lats,
                                                            const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    __shared__ float srho[(kQ9MipsRows + 2) * 66];
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x0 = tl.tx * 64, y0 = tl.ty * kQ9MipsRows;
    if (x0 >= a.nx || y0 >= a.ny)  // whole-block exit, before the barrier
        return;
    q9_mips_tile_step<kF32, F>((const float *)L.buf[par], (float *)L.buf[par ^ 1], a, x0, y0,
                               (uint32_t)((uint64_t)t & 0xffffffffu), (uint32_t)((uint64_t)t >> 32), srho);
}

// D2Q9, two steps per launch on a 64 x TY tile (the scheme of k_batch_step2
// below on the square lattice).  The second step reads population i of site
// (lx, ly) from the first step's site (lx - e_ix, ly - e_iy), local
// coordinates (lx, ly) = (x - x0 + 1, y - y0 + 1): every plane keeps TY rows
// of the widened tile's 66 columns, starting one row lower (e_iy = 1: planes
// 2, 5, 6), on the tile's rows (e_iy = 0: 0, 1, 3) or one row higher
// (e_iy = -1: 4, 7, 8).  At TY = 16 that is 38,016 bytes, four blocks per CU.
template <int TY>
struct Q9MidLayout {
    static constexpr int W = 66;
    static constexpr int kSize = 9 * TY * W;
    __host__ __device__ static constexpr int row0(int i)
    {
        return (i == 2 || i == 5 || i == 6) ? 0 : (i == 4 || i == 7 || i == 8) ? 2 : 1;
    }
    __device__ static int at(int i, int lx, int ly) { return (i * TY + ly - row0(i)) * W + lx; }
    __device__ static bool kept(int i, int ly)
    {
        const int r = ly - row0(i);
        return r >= 0 && r < TY;
    }
};

template <int M, int F, int TY, int NW>
__global__ __launch_bounds__(64 * NW) void k_batch_q9_step2(const BatchTile *__restrict__ tiles,
                                                            const LatDesc *__restrict__ lats,
                                                            const Ctrl *__restrict__ ctrl, int step_off,
                                                            int launch_off)
{
    using ML = Q9MidLayout<TY>;
    constexpr int W = 66, H = TY + 2;
    static_assert(NW % 2 == 0 && TY % NW == 0 && 2 * (TY + 2) <= 64 * (NW - 2), "rows per wave split evenly; edges fit");
    __shared__ float mid[ML::kSize];
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int64_t t1 = t + 1;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x0 = tl.tx * 64, y0 = tl.ty * TY;
    if (x0 >= a.nx || y0 >= a.ny)  // whole-block exit, before the barrier
        return;
    const uint32_t plane = (uint32_t)a.plane, nx = (uint32_t)a.nx;
    const float *src = (const float *)L.buf[par];
    float *dst = (float *)L.buf[par ^ 1];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const uint32_t ta_lo = (uint32_t)((uint64_t)t & 0xffffffffu), ta_hi = (uint32_t)((uint64_t)t >> 32);
    const uint32_t tb_lo = (uint32_t)((uint64_t)t1 & 0xffffffffu), tb_hi = (uint32_t)((uint64_t)t1 >> 32);
    // sources two sites around the tile do not wrap: wave-uniform row bases
    const bool interior = x0 >= 2 && x0 + 66 <= a.nx && y0 >= 2 && y0 + TY + 2 <= a.ny;
    const bool stream = L.stream != 0;

    // first step on the widened tile, from HBM into LDS (wave w: rows w,
    // w+NW, ...; waves 2 and up take the two edge columns in their last slot)
    constexpr int NR = (H + NW - 1) / NW;
    float f[NR][9];
    uint32_t site[NR];
    auto load_row = [&](float *g, uint32_t &st, int ly, bool in) {
        if (in) {
            const uint32_t c = (uint32_t)(y0 - 1 + ly) * nx + (uint32_t)x0;  // offset of (x0, y)
            const uint32_t e[9] = {c, c - 1u, c - nx, c + 1u, c + nx, c - nx - 1u, c - nx + 1u, c + nx + 1u,
                                   c + nx - 1u};
#pragma unroll
            for (int i = 0; i < 9; ++i)
                g[i] = BufIO<float>::load(q9_plane_rsrc(src, i, plane), lane, e[i]);
            st = c + (uint32_t)lane;
        } else {
            const Q9Sources q = q9_sources(a, wrap_coord(x0 + lane, a.nx), wrap_coord(y0 - 1 + ly, a.ny));
#pragma unroll
            for (int i = 0; i < 9; ++i)
                g[i] = BufIO<float>::load(q9_plane_rsrc(src, i, plane), q.idx[i], 0u);
            st = q.idx[0];  // pitch nx: own offset = site index
        }
    };
    auto compute = [&](float *g, uint32_t st, int lx, int ly) {
        float rho, jx, jy, ux, uy;
        q9_moments(g, rho, jx, jy);
        local_ustar<M>(a, rho, jx, jy, ux, uy);
        q9_collide<F>(a, g, rho, ux, uy, st, ta_lo, ta_hi);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (ML::kept(i, ly))
                mid[ML::at(i, lx, ly)] = g[i];
    };
    if (interior) {
#pragma unroll
        for (int k = 0; k < NR - 1; ++k)
            load_row(f[k], site[k], wv + NW * k, true);
    } else {
#pragma unroll
        for (int k = 0; k < NR - 1; ++k)
            load_row(f[k], site[k], wv + NW * k, false);
    }
    const int e = (wv - 2) * 64 + lane;
    const bool edge = wv >= 2;
    const int elx = edge ? (e < H ? 0 : W - 1) : lane + 1;
    const int ely = edge ? (e < H ? e : e - H) : wv + NW * (NR - 1);
    bool elive = true;
    if (!edge) {
        load_row(f[NR - 1], site[NR - 1], ely, interior);
    } else {
        elive = e < 2 * H;
        if (elive) {
            const Q9Sources q = q9_sources(a, wrap_coord(x0 - 1 + elx, a.nx), wrap_coord(y0 - 1 + ely, a.ny));
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[NR - 1][i] = BufIO<float>::load(q9_plane_rsrc(src, i, plane), q.idx[i], 0u);
            site[NR - 1] = q.idx[0];
        }
    }
#pragma unroll
    for (int k = 0; k < NR - 1; ++k)
        compute(f[k], site[k], lane + 1, wv + NW * k);
    if (elive)
        compute(f[NR - 1], site[NR - 1], elx, ely);
    __syncthreads();

    // second step on the tile, from LDS into HBM
    auto second = [&](int r) {
        const int lx = lane + 1, ly = r + 1;
        float g[9];
        g[0] = mid[ML::at(0, lx, ly)];
        g[1] = mid[ML::at(1, lx - 1, ly)];
        g[2] = mid[ML::at(2, lx, ly - 1)];
        g[3] = mid[ML::at(3, lx + 1, ly)];
        g[4] = mid[ML::at(4, lx, ly + 1)];
        g[5] = mid[ML::at(5, lx - 1, ly - 1)];
        g[6] = mid[ML::at(6, lx + 1, ly - 1)];
        g[7] = mid[ML::at(7, lx + 1, ly + 1)];
        g[8] = mid[ML::at(8, lx - 1, ly + 1)];
        float rho, jx, jy, ux, uy;
        q9_moments(g, rho, jx, jy);
        local_ustar<M>(a, rho, jx, jy, ux, uy);
        const uint32_t row = (uint32_t)(y0 + r) * nx + (uint32_t)x0;  // pitch nx
        q9_collide<F>(a, g, rho, ux, uy, row + (uint32_t)lane, tb_lo, tb_hi);
        batch_store9(stream, dst, plane, (uint32_t)lane, row, g);
    };
    if (interior) {
        for (int r = wv; r < TY; r += NW)
            second(r);
    } else {
        for (int r = wv; r < TY; r += NW)
            if (x0 + lane < a.nx && y0 + r < a.ny)
                second(r);
    }
}

// Step t+1 on the widened tile as the second step reads it, in local
// coordinates (lx, ly) = (x - x0 + 1, y - y0 + 1): population 0 only at the
// tile's own sites (TY rows of 64), 1 and 4 on the tile's rows (ly 1..TY),
// 2 and 3 one row lower (ly 0..TY-1), 5 and 6 one row higher (ly 2..TY+1),
// each TY rows of 66.  At TY = 16 that is 29,440 bytes, so five blocks fit
// in a CU's 160 KB of LDS (all seven planes of all TY+2 rows would not).
template <int TY>
struct MidLayout {
    static constexpr int W = 66;
    static constexpr int kSize = TY * 64 + 6 * TY * W;
    // plane base and first row of plane i
    static constexpr int base(int i)
    {
        return i == 0 ? 0 : TY * 64 + (i == 1 ? 0 : i == 4 ? 1 : i == 2 ? 2 : i == 3 ? 3 : i == 5 ? 4 : 5) * TY * W;
    }
    static constexpr int row0(int i) { return i == 0 || i == 1 || i == 4 ? 1 : (i == 2 || i == 3 ? 0 : 2); }
    __device__ static int at(int i, int lx, int ly)
    {
        return i == 0 ? (ly - 1) * 64 + (lx - 1) : base(i) + (ly - row0(i)) * W + lx;
    }
    // whether the second step reads population i of local site (lx, ly)
    __device__ static bool kept(int i, int lx, int ly)
    {
        const int r = ly - row0(i);
        return r >= 0 && r < TY && (i != 0 || (lx >= 1 && lx <= 64));
    }
};

// Steps t and t+1 on a 64 x TY tile (NW waves: wave w owns rows w, w+NW,
// ...); the first step's results go to LDS in the MidLayout above.
template <int M, int ST, int F, int TY, int NW>
__global__ __launch_bounds__(64 * NW) void k_batch_step2(const BatchTile *__restrict__ tiles,
                                                     const LatDesc *__restrict__ lats,
                                                     const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    using ML = MidLayout<TY>;
    constexpr int W = 66, H = TY + 2;
    static_assert(NW % 2 == 0 && TY % NW == 0 && 2 * (TY + 2) <= 64 * (NW - 2), "rows per wave split evenly; edges fit");
    __shared__ float mid[ML::kSize];
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int64_t t1 = t + 1;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x0 = tl.tx * 64, y0 = tl.ty * TY;
    if (x0 >= a.nx || y0 >= a.ny)  // whole-block exit, before the barrier
        return;
    const uint32_t plane = (uint32_t)a.plane;
    const __amdgpu_buffer_rsrc_t src = buffer_rsrc(L.buf[par], (uint32_t)Planes<ST>::bytes(plane));
    const __amdgpu_buffer_rsrc_t dst = buffer_rsrc(L.buf[par ^ 1], (uint32_t)Planes<ST>::bytes(plane));
    auto ld = [&](uint32_t elem, uint32_t first, int i) { return Planes<ST>::load(src, elem, first, i, plane, a); };
    const uint32_t nx = (uint32_t)a.nx;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const uint32_t ta_lo = (uint32_t)((uint64_t)t & 0xffffffffu), ta_hi = (uint32_t)((uint64_t)t >> 32);
    const uint32_t tb_lo = (uint32_t)((uint64_t)t1 & 0xffffffffu), tb_hi = (uint32_t)((uint64_t)t1 >> 32);
    // A tile whose sources (two sites around it) do not wrap: every offset is
    // a wave-uniform row base plus the lane.
    const bool interior = x0 >= 2 && x0 + 66 <= a.nx && y0 >= 2 && y0 + TY + 2 <= a.ny;
    const bool stream = L.stream != 0;

    // First step on the widened tile, from HBM into LDS.  Wave w takes rows
    // w, w+NW, ... of the H rows; waves 2 and up own one row fewer (H = 2 mod
    // NW) and take the two edge columns (2H sites) in that slot instead.  All
    // of a wave's loads are issued before any of its sites is computed.
    constexpr int NR = (H + NW - 1) / NW;
    float f[NR][7];
    uint32_t site[NR];
    auto load_row = [&](float *g, uint32_t &st, int ly, bool in) {
        if (in) {
            const int yg = y0 - 1 + ly;
            const uint32_t p = (uint32_t)yg & 1u;
            const uint32_t c = (uint32_t)yg * nx + (uint32_t)x0;  // offset of (x0, yg)
            g[0] = ld(lane, c, 0);
            g[1] = ld(lane, c - 1u, 1);
            g[2] = ld(lane, c - nx - 1u + p, 2);
            g[3] = ld(lane, c - nx + p, 3);
            g[4] = ld(lane, c + 1u, 4);
            g[5] = ld(lane, c + nx + p, 5);
            g[6] = ld(lane, c + nx - 1u + p, 6);
            st = c + (uint32_t)lane;
        } else {
            const int xg = wrap_coord(x0 + lane, a.nx), yg = wrap_coord(y0 - 1 + ly, a.ny);
            const PullSources32 q = pull_sources32(a, xg, yg);
#pragma unroll
            for (int i = 0; i < 7; ++i)
                g[i] = ld(q.idx[i], 0u, i);
            st = q.idx[0];  // pitch nx: own offset = site index
        }
    };
    auto compute = [&](float *g, uint32_t st, int lx, int ly) {
        float rho, jx, jy, ux, uy;
        site_moments(g, rho, jx, jy);
        local_ustar<M>(a, rho, jx, jy, ux, uy);
        site_collide<F, ST>(a, g, rho, ux, uy, st, ta_lo, ta_hi);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            if (ML::kept(i, lx, ly))  // the value a store and the next step's load would give
                mid[ML::at(i, lx, ly)] = Planes<ST>::round(g[i], i, a);
    };
    // slots 0 .. NR-2: rows of every wave
    if (interior) {
#pragma unroll
        for (int k = 0; k < NR - 1; ++k)
            load_row(f[k], site[k], wv + NW * k, true);
    } else {
#pragma unroll
        for (int k = 0; k < NR - 1; ++k)
            load_row(f[k], site[k], wv + NW * k, false);
    }
    // slot NR-1: last row of waves 0 and 1, edge sites of waves 2 and up
    const int e = (wv - 2) * 64 + lane;
    const bool edge = wv >= 2;
    const int elx = edge ? (e < H ? 0 : W - 1) : lane + 1;
    const int ely = edge ? (e < H ? e : e - H) : wv + NW * (NR - 1);
    bool elive = true;
    if (!edge) {
        load_row(f[NR - 1], site[NR - 1], ely, interior);
    } else {
        elive = e < 2 * H;
        if (elive) {
            const int xg = wrap_coord(x0 - 1 + elx, a.nx), yg = wrap_coord(y0 - 1 + ely, a.ny);
            const PullSources32 q = pull_sources32(a, xg, yg);
#pragma unroll
            for (int i = 0; i < 7; ++i)
                f[NR - 1][i] = ld(q.idx[i], 0u, i);
            site[NR - 1] = q.idx[0];
        }
    }
#pragma unroll
    for (int k = 0; k < NR - 1; ++k)
        compute(f[k], site[k], lane + 1, wv + NW * k);
    if (elive)
        compute(f[NR - 1], site[NR - 1], elx, ely);
    __syncthreads();

    // second step on the tile, from LDS into HBM; y0 is even, so row r has
    // parity r & 1 = wv & 1
    const int p = wv & 1;
    auto second = [&](int r) {
        const int lx = lane + 1, ly = r + 1;
        float f[7];
        f[0] = mid[ML::at(0, lx, ly)];
        f[1] = mid[ML::at(1, lx - 1, ly)];
        f[2] = mid[ML::at(2, lx - 1 + p, ly - 1)];
        f[3] = mid[ML::at(3, lx + p, ly - 1)];
        f[4] = mid[ML::at(4, lx + 1, ly)];
        f[5] = mid[ML::at(5, lx + p, ly + 1)];
        f[6] = mid[ML::at(6, lx - 1 + p, ly + 1)];
        float rho, jx, jy, ux, uy;
        site_moments(f, rho, jx, jy);
        local_ustar<M>(a, rho, jx, jy, ux, uy);
        const uint32_t row = (uint32_t)(y0 + r) * nx + (uint32_t)x0;  // pitch nx
        site_collide<F, ST>(a, f, rho, ux, uy, row + (uint32_t)lane, tb_lo, tb_hi);
        batch_store7<ST>(stream, dst, (uint32_t)lane, row, plane, f, a);
    };
    if (interior) {
        for (int r = wv; r < TY; r += NW)
            second(r);
    } else {
        for (int r = wv; r < TY; r += NW)
            if (x0 + lane < a.nx && y0 + r < a.ny)
                second(r);
    }
}

// ---------------------------------------------------------------------------
// MIPS, steps t and t+1 on a 64 x TY tile, on either lattice.  u* at a site
// needs the streamed density of its neighbours (eq. bu_mips with the
// isotropic stencil: six on the triangular lattice, eight on the square), so
// the second step on the tile reads the first step's populations on a ring of
// two sites around it (region B) and its densities on a ring of one (C), and
// the first step on B reads densities on a ring of three (A), which gather
// from the stored state on a ring of four.  Four phases, a barrier after each
// of the first three:
//  1. every site of A: its streamed populations from HBM and their density
//     into LDS; B's sites come first and keep their populations in
//     registers, the ring A \ B follows in one more slot, so the collisions
//     of phase 2 fill whole waves;
//  2. every site of B: u* from the densities, collision of step t, the
//     populations into LDS as a store and a later load give them back;
//  3. every site of C: the streamed density of step t+1 from LDS;
//  4. every site of the tile: its streamed populations from LDS, u* from the
//     densities of phase 3, collision of step t+1, store.
// Ring sites are computed at their periodic images with the one-step site
// body, so every site gets the values two one-step launches give it, bit for
// bit.  On the triangular lattice row parity follows the global row (y0 and
// ny are even).
// ---------------------------------------------------------------------------
template <int TY>
struct Mips2Layout {
    static constexpr int WA = 70, HA = TY + 6;  // A: x0-3 .. x0+66, y0-3 .. y0+TY+2
    static constexpr int WB = 68, HB = TY + 4;  // B: x0-2 .. x0+65, y0-2 .. y0+TY+1
    static constexpr int WC = 66, HC = TY + 2;  // C: x0-1 .. x0+64, y0-1 .. y0+TY
    static constexpr int NA = WA * HA, NB = WB * HB, NC = WC * HC;
    static constexpr int kRing = NA - NB;           // A outside B: 2 WA + 2 (HA - 2) sites
    static constexpr int kRho = NA > NC ? NA : NC;  // densities on A (phases 1-2), then on C (3-4)
    // A-local position of ring site e (0 <= e < kRing): the row above B, the
    // row below, then the left and the right column between them
    __device__ static void ring(int e, int &ax, int &ay)
    {
        if (e < WA) {
            ax = e;
            ay = 0;
        } else if (e < 2 * WA) {
            ax = e - WA;
            ay = HA - 1;
        } else {
            const int c = e - 2 * WA;
            ax = c < HA - 2 ? 0 : WA - 1;
            ay = 1 + (c < HA - 2 ? c : c - (HA - 2));
        }
    }
};

// Lattice policies of the two-step MIPS kernel: the streamed populations of a
// global site from the stored state (sources inside the lattice, or at the
// periodic images of a wrapped site), the density, u* from the densities
// around position c of an LDS map of row width W, the collision, the value a
// store and a later load give back, the streamed populations of a site of
// the step-t map (nb sites per plane, row width wb), and the store.
template <int ST>
struct Mips2Q7 {  // offset-row triangular lattice, any storage
    static constexpr int Q = 7;
    const StepArgs &a;
    const __amdgpu_buffer_rsrc_t src, dst;
    const uint32_t plane, nx;
    __device__ Mips2Q7(const StepArgs &a_, const void *s, void *d)
        : a(a_), src(buffer_rsrc(s, (uint32_t)Planes<ST>::bytes(a_.plane))),
          dst(buffer_rsrc(d, (uint32_t)Planes<ST>::bytes(a_.plane))), plane((uint32_t)a_.plane), nx((uint32_t)a_.nx)
    {
    }
    __device__ float ld(uint32_t e, int i) const { return Planes<ST>::load(src, e, 0u, i, plane, a); }
    __device__ void gather_in(float *g, uint32_t &own, int x, int y) const
    {
        const uint32_t p = (uint32_t)y & 1u;
        const uint32_t c = (uint32_t)y * nx + (uint32_t)x;
        g[0] = ld(c, 0);
        g[1] = ld(c - 1u, 1);
        g[2] = ld(c - nx - 1u + p, 2);
        g[3] = ld(c - nx + p, 3);
        g[4] = ld(c + 1u, 4);
        g[5] = ld(c + nx + p, 5);
        g[6] = ld(c + nx - 1u + p, 6);
        own = c;
    }
    __device__ void gather_wrapped(float *g, uint32_t &own, int xg, int yg) const
    {
        const PullSources32 q = pull_sources32(a, xg, yg);
#pragma unroll
        for (int i = 0; i < 7; ++i)
            g[i] = ld(q.idx[i], i);
        own = q.idx[0];
    }
    __device__ static float density(const float *g) { return g[0] + ((g[1] + g[4]) + ((g[2] + g[5]) + (g[3] + g[6]))); }
    template <int W>
    __device__ void ustar(const float *rs, int c, int p, float rho, float &ux, float &uy) const
    {
        float nb[7];
        nb[0] = rho;
        nb[1] = rs[c + 1];
        nb[2] = rs[c + W + p];
        nb[3] = rs[c + W - 1 + p];
        nb[4] = rs[c - 1];
        nb[5] = rs[c - W - 1 + p];
        nb[6] = rs[c - W + p];
        mips_ustar(a, rho, nb, ux, uy);
    }
    template <int F>
    __device__ void collide(float *f, float rho, float ux, float uy, uint32_t site, uint32_t lo, uint32_t hi) const
    {
        site_collide<F, ST>(a, f, rho, ux, uy, site, lo, hi);
    }
    __device__ float round(float v, int i) const { return Planes<ST>::round(v, i, a); }
    template <int NB, int WB>
    __device__ static void pull_mid(float *g, const float *mid, int bx, int by, int p)
    {
        const int m = by * WB + bx;
        g[0] = mid[0 * NB + m];
        g[1] = mid[1 * NB + m - 1];
        g[2] = mid[2 * NB + m - WB - 1 + p];
        g[3] = mid[3 * NB + m - WB + p];
        g[4] = mid[4 * NB + m + 1];
        g[5] = mid[5 * NB + m + WB + p];
        g[6] = mid[6 * NB + m + WB - 1 + p];
    }
    __device__ void store(bool stream, uint32_t row, int lane, const float *g) const
    {
        batch_store7<ST>(stream, dst, (uint32_t)lane, row, plane, g, a);
    }
};

struct Mips2Q9 {  // square lattice, float32 storage; one buffer resource per plane
    static constexpr int Q = 9;
    const StepArgs &a;
    const float *const srcp;
    float *const dstp;
    const uint32_t plane, nx;
    __device__ Mips2Q9(const StepArgs &a_, const void *s, void *d)
        : a(a_), srcp((const float *)s), dstp((float *)d), plane((uint32_t)a_.plane), nx((uint32_t)a_.nx)
    {
    }
    __device__ float ld(uint32_t e, int i) const { return BufIO<float>::load(q9_plane_rsrc(srcp, i, plane), e, 0u); }
    __device__ void gather_in(float *g, uint32_t &own, int x, int y) const
    {
        const uint32_t c = (uint32_t)y * nx + (uint32_t)x;
        const uint32_t e[9] = {c, c - 1u, c - nx, c + 1u, c + nx, c - nx - 1u, c - nx + 1u, c + nx + 1u, c + nx - 1u};
#pragma unroll
        for (int i = 0; i < 9; ++i)
            g[i] = ld(e[i], i);
        own = c;
    }
    __device__ void gather_wrapped(float *g, uint32_t &own, int xg, int yg) const
    {
        const Q9Sources q = q9_sources(a, xg, yg);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            g[i] = ld(q.idx[i], i);
        own = q.idx[0];
    }
    __device__ static float density(const float *g)
    {
        return g[0] + (((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8])));
    }
    template <int W>
    __device__ void ustar(const float *rs, int c, int, float rho, float &ux, float &uy) const
    {
        float nb[9];
        nb[0] = rho;
        nb[1] = rs[c + 1];
        nb[2] = rs[c + W];
        nb[3] = rs[c - 1];
        nb[4] = rs[c - W];
        nb[5] = rs[c + W + 1];
        nb[6] = rs[c + W - 1];
        nb[7] = rs[c - W - 1];
        nb[8] = rs[c - W + 1];
        q9_mips_ustar(a, rho, nb, ux, uy);
    }
    template <int F>
    __device__ void collide(float *f, float rho, float ux, float uy, uint32_t site, uint32_t lo, uint32_t hi) const
    {
        q9_collide<F, kF32>(a, f, rho, ux, uy, site, lo, hi);
    }
    __device__ float round(float v, int) const { return v; }
    template <int NB, int WB>
    __device__ static void pull_mid(float *g, const float *mid, int bx, int by, int)
    {
        const int m = by * WB + bx;
        g[0] = mid[0 * NB + m];
        g[1] = mid[1 * NB + m - 1];
        g[2] = mid[2 * NB + m - WB];
        g[3] = mid[3 * NB + m + 1];
        g[4] = mid[4 * NB + m + WB];
        g[5] = mid[5 * NB + m - WB - 1];
        g[6] = mid[6 * NB + m - WB + 1];
        g[7] = mid[7 * NB + m + WB + 1];
        g[8] = mid[8 * NB + m + WB - 1];
    }
    __device__ void store(bool stream, uint32_t row, int lane, const float *g) const
    {
        batch_store9(stream, dstp, plane, (uint32_t)lane, row, g);
    }
};

template <class LP, int F, int TY, int NW>
__global__ __launch_bounds__(64 * NW) void k_batch_step2_mips(const BatchTile *__restrict__ tiles,
                                                          const LatDesc *__restrict__ lats,
                                                          const Ctrl *__restrict__ ctrl, int step_off, int launch_off)
{
    using ML = Mips2Layout<TY>;
    constexpr int Q = LP::Q, NT = 64 * NW;
    constexpr int KB = (ML::NB + NT - 1) / NT, KR = (ML::kRing + NT - 1) / NT, KC = (ML::NC + NT - 1) / NT;
    static_assert(TY % NW == 0 && TY % 2 == 0, "rows per wave split evenly; tile rows start even");
    __shared__ float lds[Q * ML::NB + ML::kRho];
    float *const mid = lds;               // [Q][HB][WB]
    float *const rs = lds + Q * ML::NB;  // [HA][WA], then [HC][WC]
    const BatchTile tl = tiles[blockIdx.x];
    const LatDesc &L = lats[tl.lat];
    const StepArgs a = L.a;
    const int64_t t = ctrl->t0 + step_off;
    const int64_t t1 = t + 1;
    const int par = (int)((ctrl->k0 + launch_off) & 1);
    const int x0 = tl.tx * 64, y0 = tl.ty * TY;
    if (x0 >= a.nx || y0 >= a.ny)  // whole-block exit, before the barrier
        return;
    const LP lp(a, L.buf[par], L.buf[par ^ 1]);
    const uint32_t nx = (uint32_t)a.nx;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const uint32_t ta_lo = (uint32_t)((uint64_t)t & 0xffffffffu), ta_hi = (uint32_t)((uint64_t)t >> 32);
    const uint32_t tb_lo = (uint32_t)((uint64_t)t1 & 0xffffffffu), tb_hi = (uint32_t)((uint64_t)t1 >> 32);
    // sources four sites around the tile inside the lattice: no wrap at all
    const bool interior = x0 >= 4 && x0 + 68 <= a.nx && y0 >= 4 && y0 + TY + 4 <= a.ny;
    // A's coordinates lie in [-3, n + 65] (x) and [-3, n + TY + 1] (y): one
    // period brings them into the lattice unless it is that small
    const bool once = a.nx >= 66 && a.ny >= TY + 2;
    auto wrap = [&](int c, int n) {
        if (once) {
            c = c < 0 ? c + n : c;
            return c >= n ? c - n : c;
        }
        c %= n;
        return c < 0 ? c + n : c;
    };
    // the Q streamed populations of global site (x, y), unwrapped
    // coordinates; `own` its offset (pitch nx: the site index of the noise)
    auto gather = [&](float *g, uint32_t &own, int x, int y) {
        if (interior)
            lp.gather_in(g, own, x, y);
        else
            lp.gather_wrapped(g, own, wrap(x, a.nx), wrap(y, a.ny));
    };

    // phase 1: every load of the block's sites of A is issued first
    float f[KB][Q], fr[KR][Q];
    uint32_t own[KB], ownr[KR];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int s = tid + k * NT;
        if ((k + 1) * NT <= ML::NB || s < ML::NB)
            gather(f[k], own[k], x0 - 2 + s % ML::WB, y0 - 2 + s / ML::WB);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int e = tid + k * NT;
        if (e < ML::kRing) {
            int ax, ay;
            ML::ring(e, ax, ay);
            gather(fr[k], ownr[k], x0 - 3 + ax, y0 - 3 + ay);
        }
    }
    float rho[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int s = tid + k * NT;
        if ((k + 1) * NT <= ML::NB || s < ML::NB) {
            rho[k] = LP::density(f[k]);
            rs[(s / ML::WB + 1) * ML::WA + s % ML::WB + 1] = rho[k];
        }
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int e = tid + k * NT;
        if (e < ML::kRing) {
            int ax, ay;
            ML::ring(e, ax, ay);
            rs[ay * ML::WA + ax] = LP::density(fr[k]);
        }
    }
    __syncthreads();

    // phase 2: step t on B (row by has parity by & 1: y0 is even)
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int s = tid + k * NT;
        if ((k + 1) * NT <= ML::NB || s < ML::NB) {
            const int by = s / ML::WB, ax = s % ML::WB + 1, ay = by + 1;
            float ux, uy;
            lp.template ustar<ML::WA>(rs, ay * ML::WA + ax, by & 1, rho[k], ux, uy);
            lp.template collide<F>(f[k], rho[k], ux, uy, own[k], ta_lo, ta_hi);
#pragma unroll
            for (int i = 0; i < Q; ++i)
                mid[i * ML::NB + s] = lp.round(f[k][i], i);
        }
    }
    __syncthreads();

    // phase 3: densities of step t+1 on C (row cy has parity (cy + 1) & 1)
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int s = tid + k * NT;
        if ((k + 1) * NT <= ML::NC || s < ML::NC) {
            const int cx = s % ML::WC, cy = s / ML::WC;
            float g[Q];
            LP::template pull_mid<ML::NB, ML::WB>(g, mid, cx + 1, cy + 1, (cy + 1) & 1);
            rs[s] = LP::density(g);
        }
    }
    __syncthreads();

    // phase 4: step t+1 on the tile; wave w takes rows w, w + NW, ...
    for (int r = wv; r < TY; r += NW) {
        const int x = x0 + lane, y = y0 + r;
        if (!interior && (x >= a.nx || y >= a.ny))
            continue;
        float g[Q];
        LP::template pull_mid<ML::NB, ML::WB>(g, mid, lane + 2, r + 2, r & 1);
        const float rh = LP::density(g);
        float ux, uy;
        lp.template ustar<ML::WC>(rs, (r + 1) * ML::WC + lane + 1, r & 1, rh, ux, uy);
        const uint32_t row = (uint32_t)y * nx + (uint32_t)x0;  // pitch nx
        lp.template collide<F>(g, rh, ux, uy, row + (uint32_t)lane, tb_lo, tb_hi);
        lp.store(L.stream != 0, row, lane, g);
    }
}

// ---------------------------------------------------------------------------
// Sampling: per moments tile (256 columns x 16 rows of one lattice) FP64
// partial sums of M, Jx, Jy, sum |j|, nonfinite and per-column density sums
// of the streamed populations; then per lattice the fixed-order totals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bwave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Q = 7 (triangular) or 9 (square lattice, F32 storage only).  Block b
// takes moments tile base + b (a launch may cover one lattice group).
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_batch_moments(const MomTile *__restrict__ mt, const LatDesc *__restrict__ lats,
                                                       const Ctrl *__restrict__ ctrl, int node, int base,
                                                       double *__restrict__ part, double *__restrict__ colpart)
{
    __shared__ double lds[4][5];
    const int tile = base + (int)blockIdx.x;
    const MomTile m = mt[tile];
    const LatDesc &L = lats[m.lat];
    const StepArgs a = L.a;
    const int par = (int)((ctrl->k0 + node) & 1);
    const uint32_t plane = (uint32_t)a.plane;
    const int x = m.cx * 256 + threadIdx.x;
    const int yb = m.cy * kMomRows;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < a.nx) {
        double col = 0.0;
        const int ye = min(yb + kMomRows, a.ny);
        for (int y = yb; y < ye; ++y) {
            float f[Q];
            bool finite = true;
            float rho, jx, jy;
            if constexpr (Q == 7) {
                const __amdgpu_buffer_rsrc_t src = buffer_rsrc(L.buf[par], (uint32_t)Planes<ST>::bytes(plane));
                const PullSources32 g = pull_sources32(a, x, y);
#pragma unroll
                for (int i = 0; i < 7; ++i)
                    f[i] = Planes<ST>::load(src, g.idx[i], 0u, i, plane, a);
                site_moments(f, rho, jx, jy);
            } else {
                const float *src = (const float *)L.buf[par];
                const Q9Sources g = q9_sources(a, x, y);
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[i] = BufIO<float>::load(q9_plane_rsrc(src, i, plane), g.idx[i], 0u);
                q9_moments(f, rho, jx, jy);
            }
#pragma unroll
            for (int i = 0; i < Q; ++i)
                finite = finite && isfinite(f[i]);
            const double dx = jx, dy = jy;
            acc[0] += (double)rho;
            acc[1] += dx;
            acc[2] += dy;
            acc[3] += sqrt(dx * dx + dy * dy);
            acc[4] += finite ? 0.0 : 1.0;
            col += (double)rho;
        }
        colpart[L.col_off + (int64_t)m.cy * a.nx + x] = col;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k)
        acc[k] = bwave_sum(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k)
            lds[w][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k)
            part[(int64_t)tile * 5 + k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
}

// Column means rho_y(x) of every lattice: one thread per column (grid y =
// lattice), the column's row-block partials added in row order.  Many
// blocks, so a sample of a few large lattices does not wait on a handful of
// CUs walking every column.
__global__ __launch_bounds__(256) void k_batch_colmeans(const LatDesc *__restrict__ lats,
                                                        const double *__restrict__ colpart,
                                                        double *__restrict__ colmean)
{
    const LatDesc &L = lats[blockIdx.y];
    const int nx = L.a.nx;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx)
        return;
    const double *cp = colpart + L.col_off + x;
    double c = 0.0;
#pragma unroll 16
    for (int r = 0; r < L.nrb; ++r)
        c += cp[(int64_t)r * nx];
    colmean[L.cm_off + x] = c / (double)L.a.ny;
}

// One block per lattice: totals of its tiles, the mean of its column means
// and their variance; writes 8 doubles {M, Jx, Jy, sum|j|, nonfinite, mean,
// var, step} of sample s.
__global__ __launch_bounds__(256) void k_batch_final(const LatDesc *__restrict__ lats, const Ctrl *__restrict__ ctrl,
                                                     int node, const double *__restrict__ part,
                                                     const double *__restrict__ colmean,
                                                     double *__restrict__ results, int n_samples)
{
    __shared__ double lds[4][6];
    __shared__ double mean_s;
    const LatDesc &L = lats[blockIdx.x];
    const int nx = L.a.nx;
    const double *cm = colmean + L.cm_off;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < L.mt_count; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 5; ++k)
            v[k] += part[(int64_t)(L.mt_begin + b) * 5 + k];
    for (int x = threadIdx.x; x < nx; x += blockDim.x)
        v[5] += cm[x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        v[k] = bwave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 6; ++k)
            lds[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        mean_s = (((lds[0][5] + lds[1][5]) + lds[2][5]) + lds[3][5]) / (double)nx;
    __syncthreads();
    const double mean = mean_s;
    double q = 0.0;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        const double d = cm[x] - mean;
        q += d * d;
    }
    q = bwave_sum(q);
    __shared__ double lq[4];
    if (lane == 0)
        lq[w] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t s = ctrl->sample;
        if (s < n_samples) {
            double *r = results + ((int64_t)blockIdx.x * n_samples + s) * 8;
#pragma unroll
            for (int k = 0; k < 5; ++k)
                r[k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
            r[5] = mean;
            r[6] = (((lq[0] + lq[1]) + lq[2]) + lq[3]) / (double)nx;
            r[7] = (double)(ctrl->t0 + node);
        }
    }
}

// The density change of the paper's protocol (appendix "Simulation procedure
// for results"): every population of lattice l gains drho_l / Q, in the
// buffer that holds the state after this period's steps; per moments tile.
template <int Q, int ST>
__global__ __launch_bounds__(256) void k_batch_add_density(const MomTile *__restrict__ mt,
                                                           const LatDesc *__restrict__ lats,
                                                           const Ctrl *__restrict__ ctrl, int node)
{
    const MomTile m = mt[blockIdx.x];
    const LatDesc &L = lats[m.lat];
    const float add = L.add;
    if (add == 0.0f)
        return;
    const StepArgs &a = L.a;
    const int par = (int)((ctrl->k0 + node) & 1);
    using T = typename Store<ST>::T;
    T *f = (T *)L.buf[par];
    const int x = m.cx * 256 + threadIdx.x;
    if (x >= a.nx)
        return;
    const int ye = min(m.cy * kMomRows + kMomRows, a.ny);
    for (int y = m.cy * kMomRows; y < ye; ++y)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t e = (int64_t)y * a.pitch + x;
            if constexpr (Q == 7) {
                Planes<ST>::st(f, e, i, a.plane, Planes<ST>::ld(f, e, i, a.plane, a) + add, a);
            } else {
                T *p = f + (size_t)i * (size_t)a.plane + (size_t)e;
                *p = Store<ST>::narrow(Store<ST>::widen(*p, 0.0f) + add, 0.0f);
            }
        }
}

__global__ void k_batch_advance(Ctrl *ctrl, int64_t steps, int sampled)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl->t0 += steps;
        ctrl->k0 += steps;
        ctrl->sample += sampled;
    }
}

__global__ void k_batch_set_ctrl(Ctrl *ctrl, int64_t t0)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl->t0 = t0;
        ctrl->k0 = 0;
        ctrl->sample = 0;
        ctrl->pad = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side: layout of the workspace, tile lists, tile-shape tuning.
// ---------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t lat, tiles, mtiles, ctrl, part, colpart, colmean, results, total;
    int64_t n_tiles1, n_tiles2, n_mtiles, colpart_n, colmean_n;
};

// Work-tile shapes: sites across, rows, steps per launch.  Shapes 0..4 serve
// the local models (CIL, passive); MIPS takes the two-step shapes 3 and 4
// (64 x 8, 64 x 16) and, for single steps, shape 6 (D2Q7, 64 x 4) or 5
// (D2Q9, 64 x 16); each model's shapes are tuned among themselves.
struct Shape {
    int tx, ty, steps;
};
constexpr int kNumShapes = 7;
constexpr int kNumTuned = 5;
constexpr int kMipsShape = 5, kMipsShape4 = 6;
static const Shape kShapes[kNumShapes] = {{256, 1, 1}, {128, 2, 1}, {64, 4, 1}, {64, 8, 2},
                                          {64, 16, 2}, {64, 16, 1}, {64, 4, 1}};
constexpr int64_t kChunk = 1024;  // steps per captured graph, at most
// the LDS-resident form (k_batch_resident): no tile list, every step of a
// graph chunk in one launch; a tuning launch runs an odd number of steps, so
// it writes the second buffer like the tile shapes' tuning launches
constexpr int kResident = kNumShapes;
constexpr int kResidentTuneSteps = 63;

static bool resident_fits(const lbm_params *ps, int n)
{
    for (int l = 0; l < n; ++l)
        if ((int64_t)ps[l].nx * ps[l].ny > (ps[l].lattice == LBM_D2Q9 ? kResidentSitesQ9 : kResidentSites))
            return false;
    return true;
}

static int64_t count_tiles(const lbm_params *ps, int n, int tx, int ty)
{
    int64_t c = 0;
    for (int l = 0; l < n; ++l) {
        const int64_t ntx = (ps[l].nx + tx - 1) / tx, nty = (ps[l].ny + ty - 1) / ty;
        c += ntx * ((nty + 7) / 8) * 8;  // rows padded to whole groups of eight
    }
    return c;
}

// Lattices are independent, so a chunk of steps may run lattice group by
// lattice group: every launch of the chunk for the first group, then for the
// next.  A group's two buffers then stay in the 256 MiB Infinity Cache across
// the chunk's launches instead of streaming from HBM every step.  The batch
// takes the fewest groups of at most kCacheGroupBytes (as measured, larger
// groups of fewer launches beat smaller ones down to that size), cut into
// consecutive lattices of about equal bytes.
constexpr uint64_t kCacheGroupBytes = 240ull << 20;

// bytes of a lattice's two population buffers (pitch nx)
static uint64_t state_bytes(const lbm_params &p)
{
    const uint64_t per_site = p.lattice == LBM_D2Q9 ? (p.storage == LBM_F32 ? 36ull : 18ull)
                              : p.storage == LBM_F32        ? 28ull
                              : p.storage == LBM_BF16_DEV_R32 ? 16ull
                                                              : 14ull;
    return 2ull * per_site * (uint64_t)p.nx * p.ny;
}

static std::vector<int> cache_groups(const lbm_params *ps, int n)
{
    std::vector<uint64_t> b(n);
    uint64_t total = 0;
    for (int l = 0; l < n; ++l) {
        b[l] = state_bytes(ps[l]);
        total += b[l];
    }
    const uint64_t ng = (total + kCacheGroupBytes - 1) / kCacheGroupBytes;
    const uint64_t target = (total + ng - 1) / ng;
    std::vector<int> first{0};  // first lattice of each group, then n
    uint64_t cum = 0, in_group = 0;
    for (int l = 0; l < n; ++l) {
        const uint64_t cut = (uint64_t)(first.size()) * target;  // where the next group begins
        if (l > first.back() && (cum >= cut || in_group + b[l] > kCacheGroupBytes)) {
            first.push_back(l);
            in_group = 0;
        }
        cum += b[l];
        in_group += b[l];
    }
    first.push_back(n);
    return first;
}

// [begin, count) of each group's tiles in the list of shape k (build_tiles
// lists each lattice's tiles contiguously, in lattice order)
static std::vector<int64_t> group_ranges(const lbm_params *ps, const std::vector<int> &first, int k)
{
    std::vector<int64_t> r;
    int64_t off = 0;
    for (size_t g = 0; g + 1 < first.size(); ++g) {
        const int64_t c = count_tiles(ps + first[g], first[g + 1] - first[g], kShapes[k].tx, kShapes[k].ty);
        r.push_back(off);
        r.push_back(c);
        off += c;
    }
    return r;
}

static Layout layout(const lbm_params *ps, int n, int64_t n_samples)
{
    Layout L{};
    // room for the list of one single-step shape and one two-step shape
    L.n_tiles1 = 0;
    L.n_tiles2 = 0;
    for (int k = 0; k < kNumShapes; ++k) {
        int64_t &m = kShapes[k].steps == 1 ? L.n_tiles1 : L.n_tiles2;
        m = std::max(m, count_tiles(ps, n, kShapes[k].tx, kShapes[k].ty));
    }
    L.n_mtiles = 0;
    L.colpart_n = 0;
    L.colmean_n = 0;
    for (int l = 0; l < n; ++l) {
        const int64_t cx = (ps[l].nx + 255) / 256, cy = (ps[l].ny + kMomRows - 1) / kMomRows;
        L.n_mtiles += cx * cy;
        L.colpart_n += cy * ps[l].nx;
        L.colmean_n += ps[l].nx;
    }
    size_t off = 0;
    L.lat = off;
    off = align256(off + sizeof(LatDesc) * n);
    L.tiles = off;
    off = align256(off + sizeof(BatchTile) * (L.n_tiles1 + L.n_tiles2));
    L.mtiles = off;
    off = align256(off + sizeof(MomTile) * L.n_mtiles);
    L.ctrl = off;
    off = align256(off + sizeof(Ctrl));
    L.part = off;
    off = align256(off + sizeof(double) * 5 * L.n_mtiles);
    L.colpart = off;
    off = align256(off + sizeof(double) * L.colpart_n);
    L.colmean = off;
    off = align256(off + sizeof(double) * L.colmean_n);
    L.results = off;
    off = align256(off + sizeof(double) * 8 * (size_t)n * (size_t)std::max<int64_t>(n_samples, 1));
    L.total = off;
    return L;
}

// Tile list of one shape, row-group order per lattice; tiles in the padding
// rows of a lattice's last group point past the lattice and exit at once.
static std::vector<BatchTile> build_tiles(const lbm_params *ps, int n, int tx, int ty)
{
    std::vector<BatchTile> v;
    for (int l = 0; l < n; ++l) {
        const int ntx = (ps[l].nx + tx - 1) / tx, nty = (ps[l].ny + ty - 1) / ty;
        for (int g = 0; g < (nty + 7) / 8; ++g)
            for (int c = 0; c < ntx; ++c)
                for (int r = 0; r < 8; ++r)
                    v.push_back(BatchTile{l, (int16_t)c, (int16_t)(8 * g + r)});
    }
    return v;
}

static int sweep_flags(const lbm_params *ps, int n)
{
    const int f = step_flags(make_step_args(ps[0], ps[0].nx));
    for (int l = 1; l < n; ++l)
        if (step_flags(make_step_args(ps[l], ps[l].nx)) != f)
            return -1;
    return f;
}

// Runtime storage and flags to compile-time template arguments.
template <int V>
using IntTag = std::integral_constant<int, V>;

template <class Fn>
static hipError_t with_storage(int storage, Fn &&fn)
{
    switch (storage) {
    case kF32: return fn(IntTag<kF32>{});
    case kBf16Dev: return fn(IntTag<kBf16Dev>{});
    case kF16Dev: return fn(IntTag<kF16Dev>{});
    case kBf16R32: return fn(IntTag<kBf16R32>{});
    }
    return hipErrorInvalidValue;
}

template <class Fn>
static hipError_t with_flags(int flags, Fn &&fn)
{
    switch (flags) {
    case 0: return fn(IntTag<0>{});
    case kUnitTau: return fn(IntTag<kUnitTau>{});
    case kNoisy: return fn(IntTag<kNoisy>{});
    default: return fn(IntTag<kUnitTau | kNoisy>{});
    }
}

template <int M, int ST, int F>
static hipError_t launch_batch_step_mf(int shape, int64_t ntiles, const BatchTile *tiles, const LatDesc *lats,
                                       const Ctrl *ctrl, int step_off, int launch_off, hipStream_t s)
{
    const Shape &sh = kShapes[shape];
    if (sh.steps == 1)
        hipLaunchKernelGGL((k_batch_step<M, ST, F>), dim3((unsigned)ntiles), dim3(sh.tx, sh.ty), 0, s, tiles, lats,
                           ctrl, step_off, launch_off);
    else if (sh.ty == 8)
        hipLaunchKernelGGL((k_batch_step2<M, ST, F, 8, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats, ctrl,
                           step_off, launch_off);
    else
        hipLaunchKernelGGL((k_batch_step2<M, ST, F, 16, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats,
                           ctrl, step_off, launch_off);
    return hipGetLastError();
}

template <int ST, int F>
static hipError_t launch_batch_mips_f(int shape, int64_t ntiles, const BatchTile *tiles, const LatDesc *lats,
                                      const Ctrl *ctrl, int step_off, int launch_off, hipStream_t s)
{
    if (kShapes[shape].steps == 2 && kShapes[shape].ty == 8)
        hipLaunchKernelGGL((k_batch_step2_mips<Mips2Q7<ST>, F, 8, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles,
                           lats, ctrl, step_off, launch_off);
    else if (kShapes[shape].steps == 2)
        hipLaunchKernelGGL((k_batch_step2_mips<Mips2Q7<ST>, F, 16, 8>), dim3((unsigned)ntiles), dim3(512), 0, s,
                           tiles, lats, ctrl, step_off, launch_off);
    else if (shape == kMipsShape4)
        hipLaunchKernelGGL((k_batch_step_mips<ST, F, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats, ctrl,
                           step_off, launch_off);
    else
        hipLaunchKernelGGL((k_batch_step_mips<ST, F, kMipsRows>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles,
                           lats, ctrl, step_off, launch_off);
    return hipGetLastError();
}

// Every lattice of the batch in one CU's LDS (D2Q9: F32 storage only).
static hipError_t launch_resident(int lattice, int model, int storage, int flags, int n, const LatDesc *lats,
                                  const Ctrl *ctrl, int steps, hipStream_t s)
{
    const dim3 grd((unsigned)n), blk(kResidentLanes);
    return with_storage(storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        return with_flags(flags, [&](auto fl) {
            constexpr int F = decltype(fl)::value;
            if (lattice == LBM_D2Q9) {
                if (ST != kF32)
                    return hipErrorInvalidValue;
                if (model == LBM_MIPS)
                    hipLaunchKernelGGL((k_batch_resident_q9<kMips, F>), grd, blk, 0, s, lats, ctrl, steps);
                else if (model == LBM_CIL)
                    hipLaunchKernelGGL((k_batch_resident_q9<kCil, F>), grd, blk, 0, s, lats, ctrl, steps);
                else
                    hipLaunchKernelGGL((k_batch_resident_q9<kPassive, F>), grd, blk, 0, s, lats, ctrl, steps);
            } else if (model == LBM_MIPS) {
                hipLaunchKernelGGL((k_batch_resident<kMips, ST, F>), grd, blk, 0, s, lats, ctrl, steps);
            } else if (model == LBM_CIL) {
                hipLaunchKernelGGL((k_batch_resident<kCil, ST, F>), grd, blk, 0, s, lats, ctrl, steps);
            } else {
                hipLaunchKernelGGL((k_batch_resident<kPassive, ST, F>), grd, blk, 0, s, lats, ctrl, steps);
            }
            return hipGetLastError();
        });
    });
}

template <int M, int F>
static void launch_q9_two(int ty, int64_t ntiles, const BatchTile *tiles, const LatDesc *lats, const Ctrl *ctrl,
                          int step_off, int launch_off, hipStream_t s)
{
    if (ty == 8)
        hipLaunchKernelGGL((k_batch_q9_step2<M, F, 8, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats, ctrl,
                           step_off, launch_off);
    else
        hipLaunchKernelGGL((k_batch_q9_step2<M, F, 16, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats,
                           ctrl, step_off, launch_off);
}

template <int F>
static hipError_t launch_batch_q9_f(int model, int shape, int64_t ntiles, const BatchTile *tiles, const LatDesc *lats,
                                    const Ctrl *ctrl, int step_off, int launch_off, hipStream_t s)
{
    const Shape &sh = kShapes[shape];
    if (model == kMips && sh.steps == 2 && sh.ty == 8)
        hipLaunchKernelGGL((k_batch_step2_mips<Mips2Q9, F, 8, 4>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles,
                           lats, ctrl, step_off, launch_off);
    else if (model == kMips && sh.steps == 2)
        hipLaunchKernelGGL((k_batch_step2_mips<Mips2Q9, F, 16, 8>), dim3((unsigned)ntiles), dim3(512), 0, s, tiles,
                           lats, ctrl, step_off, launch_off);
    else if (model == kMips)
        hipLaunchKernelGGL((k_batch_q9_step_mips<F>), dim3((unsigned)ntiles), dim3(256), 0, s, tiles, lats, ctrl,
                           step_off, launch_off);
    else if (sh.steps == 2 && model == kCil)
        launch_q9_two<kCil, F>(sh.ty, ntiles, tiles, lats, ctrl, step_off, launch_off, s);
    else if (sh.steps == 2)
        launch_q9_two<kPassive, F>(sh.ty, ntiles, tiles, lats, ctrl, step_off, launch_off, s);
    else if (model == kCil)
        hipLaunchKernelGGL((k_batch_q9_step<kCil, F>), dim3((unsigned)ntiles), dim3(sh.tx, sh.ty), 0, s, tiles, lats,
                           ctrl, step_off, launch_off);
    else
        hipLaunchKernelGGL((k_batch_q9_step<kPassive, F>), dim3((unsigned)ntiles), dim3(sh.tx, sh.ty), 0, s, tiles,
                           lats, ctrl, step_off, launch_off);
    return hipGetLastError();
}

// One launch of shape `shape` over a tile list (D2Q9: F32 storage only).
static hipError_t launch_batch_step(int lattice, int model, int storage, int flags, int shape, int64_t ntiles,
                                    const BatchTile *tiles, const LatDesc *lats, const Ctrl *ctrl, int step_off,
                                    int launch_off, hipStream_t s)
{
    return with_flags(flags, [&](auto fl) {
        constexpr int F = decltype(fl)::value;
        if (lattice == LBM_D2Q9)
            return storage == kF32
                       ? launch_batch_q9_f<F>(model, shape, ntiles, tiles, lats, ctrl, step_off, launch_off, s)
                       : hipErrorInvalidValue;
        return with_storage(storage, [&](auto st) {
            constexpr int ST = decltype(st)::value;
            if (model == kMips)
                return launch_batch_mips_f<ST, F>(shape, ntiles, tiles, lats, ctrl, step_off, launch_off, s);
            if (model == kCil)
                return launch_batch_step_mf<kCil, ST, F>(shape, ntiles, tiles, lats, ctrl, step_off, launch_off, s);
            return launch_batch_step_mf<kPassive, ST, F>(shape, ntiles, tiles, lats, ctrl, step_off, launch_off, s);
        });
    });
}

// Tuned tile shape per batch signature (arch + lattice type + multiset of
// lattice sizes + model + flags), kept for the life of the process.
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tuned;

static std::string signature(const lbm_params *ps, int n, int flags)
{
    std::map<std::pair<int, int>, int> hist;
    for (int l = 0; l < n; ++l)
        hist[{ps[l].nx, ps[l].ny}]++;
    std::string s = "gfx950/q" + std::to_string(ps[0].lattice == LBM_D2Q9 ? 9 : 7) + "/m" +
                    std::to_string(ps[0].model) + "/s" + std::to_string(ps[0].storage) + "/f" + std::to_string(flags);
    for (auto &h : hist)
        s += "/" + std::to_string(h.first.first) + "x" + std::to_string(h.first.second) + ":" +
             std::to_string(h.second);
    return s;
}

// Instantiated sample-period graphs, least recently used first out.
struct GraphKey {
    int device;
    const void *tiles_main, *tiles_one, *lat, *ctrl, *mt, *part, *colpart, *colmean, *results;
    int lattice, model, storage, flags, shape;
    int64_t ntiles_main, ntiles_one, nmt, n, n_samples, steps;
    int sample, add, rev;
    std::vector<int64_t> groups;  // tile ranges of the lattice groups
    auto tie() const
    {
        return std::tie(device, tiles_main, tiles_one, lat, ctrl, mt, part, colpart, colmean, results, lattice, model,
                        storage, flags, shape, ntiles_main, ntiles_one, nmt, n, n_samples, steps, sample, add, rev,
                        groups);
    }
    bool operator==(const GraphKey &o) const { return tie() == o.tie(); }
};

// An executable graph, destroyed when the last holder lets go (the cache or
// a call still running it).
// An instantiated graph and an event recorded after its latest launch: a
// sweep returns without waiting for its graphs, so an exec evicted from the
// cache (or released at the end of a call) waits for that launch to finish
// before it is destroyed.
struct GraphExec {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    hipError_t launched(hipStream_t s)
    {
        if (!done) {
            hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
            if (e != hipSuccess) {
                done = nullptr;
                return e;
            }
        }
        return hipEventRecord(done, s);
    }
    ~GraphExec()
    {
        if (done) {
            (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        if (exec)
            (void)hipGraphExecDestroy(exec);
    }
};
using GraphPtr = std::shared_ptr<GraphExec>;

constexpr size_t kGraphCacheSize = 16;
static std::mutex g_graph_mu;
// most recently used last; never destroyed, so no HIP call runs from a static
// destructor after the runtime may have shut down at process exit
static auto &g_graphs = *new std::vector<std::pair<GraphKey, GraphPtr>>();

static GraphPtr graph_cache_get(const GraphKey &k)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size(); ++i)
        if (g_graphs[i].first == k) {
            auto hit = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + (ptrdiff_t)i);
            g_graphs.push_back(hit);
            return hit.second;
        }
    return nullptr;
}

static void graph_cache_put(const GraphKey &k, const GraphPtr &g)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= kGraphCacheSize)
        g_graphs.erase(g_graphs.begin());
    g_graphs.emplace_back(k, g);
}

// What this library last wrote into the tables of a workspace (lattice
// descriptors, moments tiles and the tile list held in each of the two list
// regions), per device and workspace address.  A call with keep_tables set
// takes the record at its word (its caller has not written into the
// workspace since) and uploads only the tables that differ, so a repeated
// sweep of the same batch starts its first kernel without host work.
struct WsTables {
    int lattice = -1;
    std::vector<std::pair<int32_t, int32_t>> sizes;  // (nx, ny) of each lattice, in batch order
    std::vector<LatDesc> lat;
    int region[2] = {-1, -1};  // shape whose list is in the one-step / two-step region
    // lattice groups in reverse order in the next call: each call starts with
    // the group the previous one ended with, whose state is still in the
    // Infinity Cache
    bool rev_next = false;
};
constexpr size_t kWsRecords = 64;
static std::mutex g_ws_mu;
static auto &g_ws = *new std::map<std::pair<int, const void *>, WsTables>();

// Field-by-field equality (bit patterns: +0 and -0 differ), so padding bytes
// play no part.
#define LBM_SAME(f) (memcmp(&x.f, &y.f, sizeof(x.f)) == 0)
static bool same_args(const StepArgs &x, const StepArgs &y)
{
    return LBM_SAME(nx) && LBM_SAME(ny) && LBM_SAME(pitch) && LBM_SAME(plane) && LBM_SAME(omega) &&
           LBM_SAME(noise_scale) && LBM_SAME(noise_h) && LBM_SAME(A16) && LBM_SAME(B16) && LBM_SAME(C) && LBM_SAME(rho_star) &&
           LBM_SAME(inv_rho_star) && LBM_SAME(u_max) && LBM_SAME(wr0) && LBM_SAME(wr1) && LBM_SAME(wr2) &&
           LBM_SAME(key0) && LBM_SAME(key1) && LBM_SAME(noisy);
}
static bool same_desc(const LatDesc &x, const LatDesc &y)
{
    return same_args(x.a, y.a) && LBM_SAME(buf) && LBM_SAME(B) && LBM_SAME(mt_begin) && LBM_SAME(mt_count) &&
           LBM_SAME(nrb) && LBM_SAME(col_off) && LBM_SAME(cm_off) && LBM_SAME(add) && LBM_SAME(stream);
}
#undef LBM_SAME

// Copy a sweep's samples (8 doubles each, lattice-major) to the host after
// the stream's work and turn them into lbm_obs.
static int32_t read_samples(const lbm_params *ps, int n, int64_t n_samples, const double *d_results, hipStream_t s,
                            lbm_obs *out)
{
    std::vector<double> res((size_t)n * n_samples * 8);
    LBM_HIP_TRY(hipMemcpyAsync(res.data(), d_results, sizeof(double) * res.size(), hipMemcpyDeviceToHost, s));
    LBM_HIP_TRY(hipStreamSynchronize(s));
    bool bad = false;
    for (int l = 0; l < n; ++l)
        for (int64_t k = 0; k < n_samples; ++k) {
            const double *r = &res[((size_t)l * n_samples + k) * 8];
            lbm_obs &ob = out[(size_t)l * n_samples + k];
            finish_obs(ps[l], r, (int64_t)r[7], &ob);
            bad = bad || ob.nonfinite;
        }
    if (bad)
        return fail(LBM_ENONFINITE, "non-finite populations in a batch sample");
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

int32_t lbm_sweep_groups(const lbm_params *ps, int32_t n)
{
    if (!ps || n <= 0)
        return fail(LBM_EINVAL, "null parameters or empty batch");
    return (int32_t)cache_groups(ps, n).size() - 1;
}

int32_t lbm_sweep_tile_rows(const lbm_params *ps, int32_t n)
{
    if (!ps || n <= 0)
        return fail(LBM_EINVAL, "null parameters or empty batch");
    const int flags = sweep_flags(ps, n);
    if (flags < 0)
        return 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(signature(ps, n, flags));
    if (it == g_tuned.end())
        return 0;
    return it->second == kResident ? LBM_TILE_RESIDENT : kShapes[it->second].ty;
}

size_t lbm_sweep_workspace_bytes(const lbm_params *ps, int32_t n, int64_t n_samples)
{
    if (!ps || n <= 0 || n_samples < 0)
        return 0;
    return layout(ps, n, n_samples).total;
}

int32_t lbm_sweep_batch(const lbm_params *ps, int32_t n, const lbm_sweep_opts *o, void *const *bufs, void *ws,
                        size_t ws_bytes, void *stream, lbm_obs *out)
{
    if (!ps || n <= 0 || !o || !bufs || !ws)
        return fail(LBM_EINVAL, "null argument or empty batch");
    if (o->n_steps < 0 || o->sample_every < 0 || o->step0 < 0)
        return fail(LBM_EINVAL, "negative step counts");
    if (o->use_graph < 0 || o->use_graph > 2)
        return fail(LBM_EINVAL, "use_graph must be 0, 1 or 2");
    if (o->drho)
        for (int l = 0; l < n; ++l)
            if (!isfinite(o->drho[l]))
                return fail(LBM_EINVAL, "drho must be finite");
    for (int l = 0; l < n; ++l) {
        int32_t rc = validate_params(&ps[l], ps[l].nx);
        if (rc)
            return fail(rc, "lattice " + std::to_string(l) + ": " + lbm_last_error());
        if (ps[l].lattice != ps[0].lattice)
            return fail(LBM_EINVAL, "all lattices of a batch must use the same velocity set");
        if (ps[l].storage != ps[0].storage)
            return fail(LBM_EINVAL, "all lattices of a batch must use the same storage");
        if (ps[l].storage != LBM_F32 && ps[l].lattice == LBM_D2Q9)
            return fail(LBM_EUNSUPPORTED, "batched D2Q9 sweeps take F32 storage");
        if (ps[l].model != ps[0].model)
            return fail(LBM_EINVAL, "all lattices of a batch must use the same model");
        if ((uint64_t)ps[l].nx * ps[l].ny * (ps[l].lattice == LBM_D2Q9 ? 9ull : 7ull) >= (1ull << 30))
            return fail(LBM_EINVAL, "batch lattices must hold fewer than 2^30 populations");
        if (!bufs[2 * l] || !bufs[2 * l + 1] || bufs[2 * l] == bufs[2 * l + 1])
            return fail(LBM_EINVAL, "lattice " + std::to_string(l) + ": null or equal buffers");
        if (ps[l].ny > 32760 || ps[l].nx > 64 * 32760)
            return fail(LBM_EINVAL, "batch lattices need ny <= 32760 and nx <= 2096640 (16-bit tile indices)");
    }
    const int flags = sweep_flags(ps, n);
    if (flags < 0)
        return fail(LBM_EINVAL, "all lattices of a batch must agree on tau == 1 and on sigma == 0");
    const int64_t period = o->sample_every > 0 ? o->sample_every : o->n_steps;
    const int64_t n_samples = o->sample_every > 0 ? o->n_steps / o->sample_every : 1;
    if (o->sample_every > 0 && o->n_steps % o->sample_every != 0)
        return fail(LBM_EINVAL, "n_steps must be a multiple of sample_every");
    const Layout Ly = layout(ps, n, n_samples);
    if (ws_bytes < Ly.total)
        return fail(LBM_EINVAL, "workspace smaller than lbm_sweep_workspace_bytes()");
    if (o->surrogate)
        return surrogate_sweep(ps, n, o, bufs, ws, ws_bytes, (hipStream_t)stream, out);
    // tile shape: caller's choice (tile_rows 1, 2, 4: 256x1, 128x2, 64x4
    // sites, one step per launch; 8, 16: 64x8, 64x16 sites, two steps per
    // launch; MIPS 8, 16 and, D2Q7 only, 4 with one step per launch),
    // else the tuned one for
    // this signature, else tuned below: every tuning launch reads the state
    // in the first buffer of each lattice and writes the second (free until
    // the sweep starts), so the state is unchanged.
    int shape = -1;
    const bool mips = ps[0].model == LBM_MIPS, q9 = ps[0].lattice == LBM_D2Q9;
    // the shapes this model and lattice may take (tuned among themselves):
    // MIPS 64x8 and 64x16 with two steps per launch and, D2Q7 only, 64x4
    // with one; the local models shapes 0..4
    std::vector<int> cands;
    if (mips)
        cands = q9 ? std::vector<int>{3, 4} : std::vector<int>{kMipsShape4, 3, 4};
    else
        for (int k = 0; k < kNumTuned; ++k)
            cands.push_back(k);
    for (int k : cands)
        if (o->tile_rows == kShapes[k].ty)
            shape = k;
    const bool resident_ok = resident_fits(ps, n);
    if (resident_ok)
        cands.push_back(kResident);
    if (o->tile_rows == LBM_TILE_RESIDENT) {
        if (!resident_ok)
            return fail(LBM_EINVAL, "tile_rows LBM_TILE_RESIDENT needs lattices of at most " +
                                        std::to_string(kResidentSites) + " (D2Q7) or " +
                                        std::to_string(kResidentSitesQ9) + " (D2Q9) sites");
        shape = kResident;
    }
    if (shape < 0 && o->tile_rows != 0)
        return fail(LBM_EINVAL, mips ? (q9 ? "D2Q9 MIPS batches take tile_rows 0, 8, 16 or LBM_TILE_RESIDENT"
                                          : "MIPS batches take tile_rows 0, 4, 8, 16 or LBM_TILE_RESIDENT")
                                     : "tile_rows must be 0, 1, 2, 4, 8, 16 or LBM_TILE_RESIDENT");
    const std::string sig = signature(ps, n, flags);
    if (shape < 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(sig);
        if (it != g_tuned.end())
            shape = it->second;
    }
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    LatDesc *d_lat = (LatDesc *)(w + Ly.lat);
    BatchTile *d_tiles = (BatchTile *)(w + Ly.tiles);
    MomTile *d_mt = (MomTile *)(w + Ly.mtiles);
    Ctrl *d_ctrl = (Ctrl *)(w + Ly.ctrl);
    double *d_part = (double *)(w + Ly.part);
    double *d_colpart = (double *)(w + Ly.colpart);
    double *d_colmean = (double *)(w + Ly.colmean);
    double *d_results = (double *)(w + Ly.results);

    // descriptors (and the moments tiles: per lattice, cx x cy tiles of 256
    // columns x kMomRows rows)
    std::vector<LatDesc> lat(n);
    std::vector<std::pair<int32_t, int32_t>> sizes(n);
    int64_t col_off = 0, cm_off = 0, nmt = 0;
    for (int l = 0; l < n; ++l) {
        LatDesc &D = lat[l];
        D.a = make_step_args(ps[l], ps[l].nx);
        D.buf[0] = bufs[2 * l];
        D.buf[1] = bufs[2 * l + 1];
        D.B = (float)ps[l].B;
        D.add = o->drho ? (float)(o->drho[l] / (ps[l].lattice == LBM_D2Q9 ? 9.0 : 7.0)) : 0.0f;
        D.stream = state_bytes(ps[l]) > kCacheGroupBytes ? 1 : 0;
        const int cx = (ps[l].nx + 255) / 256, cy = (ps[l].ny + kMomRows - 1) / kMomRows;
        D.mt_begin = (int32_t)nmt;
        D.mt_count = cx * cy;
        D.nrb = cy;
        D.col_off = col_off;
        D.cm_off = cm_off;
        nmt += (int64_t)cx * cy;
        col_off += (int64_t)cy * ps[l].nx;
        cm_off += ps[l].nx;
        sizes[l] = {ps[l].nx, ps[l].ny};
    }
    // the workspace's record: a copy, written back once the uploads are enqueued
    int dev = 0;
    LBM_HIP_TRY(hipGetDevice(&dev));
    const std::pair<int, const void *> ws_key{dev, ws};
    WsTables rec;
    if (o->keep_tables) {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        auto it = g_ws.find(ws_key);
        if (it != g_ws.end())
            rec = it->second;
    }
    const bool same_sizes = rec.lattice == ps[0].lattice && rec.sizes == sizes;
    if (!same_sizes)
        rec.region[0] = rec.region[1] = -1;
    bool same_lat = same_sizes && rec.lat.size() == lat.size();
    for (int l = 0; l < n && same_lat; ++l)
        same_lat = same_desc(rec.lat[l], lat[l]);
    // host copies of the uploaded tables stay alive until the stream is
    // synchronised at the end of this call
    std::vector<MomTile> mt;
    std::vector<std::vector<BatchTile>> host_lists;
    auto save_record = [&]() {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        if (g_ws.size() >= kWsRecords && !g_ws.count(ws_key))
            g_ws.erase(g_ws.begin());
        g_ws[ws_key] = rec;
    };
    // a failed call leaves the workspace's tables unknown
    auto forget_record = [&]() {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        g_ws.erase(ws_key);
    };

    forget_record();  // until this call has written every table it uses
    const bool uploaded_desc = !same_lat || !same_sizes;
    if (!same_lat)
        LBM_HIP_TRY(hipMemcpyAsync(d_lat, lat.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice, s));
    if (!same_sizes) {
        mt.reserve((size_t)nmt);
        for (int l = 0; l < n; ++l) {
            const int cx = (ps[l].nx + 255) / 256, cy = (ps[l].ny + kMomRows - 1) / kMomRows;
            for (int j = 0; j < cy; ++j)
                for (int i = 0; i < cx; ++i)
                    mt.push_back(MomTile{l, (int16_t)i, (int16_t)j});
        }
        LBM_HIP_TRY(hipMemcpyAsync(d_mt, mt.data(), sizeof(MomTile) * mt.size(), hipMemcpyHostToDevice, s));
    }
    rec.lattice = ps[0].lattice;
    rec.sizes = sizes;
    rec.lat = lat;
    BatchTile *d_tiles1 = d_tiles, *d_tiles2 = d_tiles + Ly.n_tiles1;
    hipError_t up_err = hipSuccess;
    // the tile list of shape k in its region (one-step shapes in the first,
    // two-step shapes in the second), uploaded unless the region holds it
    auto upload = [&](int k) -> std::pair<BatchTile *, int64_t> {
        const int r = kShapes[k].steps == 1 ? 0 : 1;
        BatchTile *d = r == 0 ? d_tiles1 : d_tiles2;
        const int64_t count = count_tiles(ps, n, kShapes[k].tx, kShapes[k].ty);
        if (rec.region[r] == k)
            return {d, count};
        host_lists.push_back(build_tiles(ps, n, kShapes[k].tx, kShapes[k].ty));
        const std::vector<BatchTile> &v = host_lists.back();
        up_err = hipMemcpyAsync(d, v.data(), sizeof(BatchTile) * v.size(), hipMemcpyHostToDevice, s);
        rec.region[r] = up_err == hipSuccess ? k : -1;
        return {up_err == hipSuccess ? d : nullptr, (int64_t)v.size()};
    };
    if (shape < 0) {
        float best = 1e30f;
        struct EventPair {  // destroyed on every exit path
            hipEvent_t a = nullptr, b = nullptr;
            ~EventPair()
            {
                if (a)
                    (void)hipEventDestroy(a);
                if (b)
                    (void)hipEventDestroy(b);
            }
        } ev;
        LBM_HIP_TRY(hipEventCreate(&ev.a));
        LBM_HIP_TRY(hipEventCreate(&ev.b));
        hipEvent_t e0 = ev.a, e1 = ev.b;
        hipLaunchKernelGGL(k_batch_set_ctrl, dim3(1), dim3(64), 0, s, d_ctrl, (int64_t)0);
        // each shape: ten launches captured in a graph (as the sweep runs
        // them), replayed once to warm up and three times timed; the least
        // time per step wins
        for (int k : cands) {
            const bool res = k == kResident;
            std::pair<BatchTile *, int64_t> tl{nullptr, 0};
            if (!res) {
                tl = upload(k);
                if (!tl.first)
                    return hip_fail(up_err, "tile list upload");
            }
            hipStream_t cap;
            LBM_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (res && e == hipSuccess)  // first buffer -> second buffer
                e = launch_resident(ps[0].lattice, ps[0].model, ps[0].storage, flags, n, d_lat, d_ctrl, kResidentTuneSteps, cap);
            // ten launches per lattice group, group after group, as the sweep runs them
            const std::vector<int64_t> gr = res ? std::vector<int64_t>{} : group_ranges(ps, cache_groups(ps, n), k);
            for (size_t g = 0; 2 * g < gr.size(); ++g)
                for (int r10 = 0; r10 < 10 && e == hipSuccess; ++r10)
                    e = launch_batch_step(ps[0].lattice, ps[0].model, ps[0].storage, flags, k, gr[2 * g + 1], tl.first + gr[2 * g],
                                          d_lat, d_ctrl, 0, 0, cap);
            hipError_t ee = hipStreamEndCapture(cap, &g);
            (void)hipStreamDestroy(cap);
            if (e == hipSuccess)
                e = ee;
            hipGraphExec_t ge = nullptr;
            if (e == hipSuccess)
                e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            if (g)
                (void)hipGraphDestroy(g);
            float ms = 1e30f;
            for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    e = hipGraphLaunch(ge, s);
                if (e == hipSuccess)
                    e = hipEventRecord(e1, s);
                if (e == hipSuccess)
                    e = hipEventSynchronize(e1);
                float m = 0.0f;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&m, e0, e1);
                if (rep > 0)  // time per ten steps
                    ms = std::min(ms, res ? m * 10.0f / kResidentTuneSteps : m / (float)kShapes[k].steps);
            }
            if (ge)
                (void)hipGraphExecDestroy(ge);
            if (e != hipSuccess)
                return hip_fail(e, "tile-shape tuning");
            if (ms < best) {
                best = ms;
                shape = k;
            }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[sig] = shape;
    }
    // the chosen list, and for a two-step shape the list of a one-step shape
    // (256x1; MIPS 64x4, D2Q9 MIPS 64x16) for the single steps that keep the launch count's
    // parity equal to the step count's (so the state ends in
    // bufs[2l + (n_steps & 1)])
    const bool resident = shape == kResident;
    const bool two = !resident && kShapes[shape].steps == 2;
    const int one_shape = two ? (mips ? (q9 ? kMipsShape : kMipsShape4) : 0) : shape;
    std::pair<BatchTile *, int64_t> main_list{d_tiles1, 0};
    if (!resident) {
        main_list = upload(shape);
        if (!main_list.first)
            return hip_fail(up_err, "tile list upload");
    }
    std::pair<BatchTile *, int64_t> one_list = main_list;
    if (two) {
        one_list = upload(one_shape);
        if (!one_list.first)
            return hip_fail(up_err, "tile list upload");
    }
    int max_nx = 0;
    for (int l = 0; l < n; ++l)
        max_nx = std::max(max_nx, ps[l].nx);
    hipLaunchKernelGGL(k_batch_set_ctrl, dim3(1), dim3(64), 0, s, d_ctrl, (int64_t)o->step0);
    LBM_HIP_TRY(hipGetLastError());
    // lattice groups that fit the Infinity Cache (one group when resident)
    const std::vector<int> gfirst = resident ? std::vector<int>{0, n} : cache_groups(ps, n);
    const std::vector<int64_t> g_main = resident ? std::vector<int64_t>{0, 0} : group_ranges(ps, gfirst, shape);
    const std::vector<int64_t> g_one = two ? group_ranges(ps, gfirst, one_shape) : g_main;
    std::vector<int64_t> gkey(g_main);
    gkey.insert(gkey.end(), g_one.begin(), g_one.end());

    // the order of the lattice groups in this call, and in the next one
    const bool rev = !resident && gfirst.size() > 2 && rec.rev_next;
    rec.rev_next = o->use_graph == 2 ? rev : (!resident && gfirst.size() > 2 && !rev);
    // moments tiles of each lattice group ([begin, end) in the lattice-ordered list)
    std::vector<int> gmt(gfirst.size(), 0);
    {
        std::vector<int> first_mt(n + 1, 0);
        for (int l = 0; l < n; ++l)
            first_mt[l + 1] = first_mt[l] + ((ps[l].nx + 255) / 256) * ((ps[l].ny + kMomRows - 1) / kMomRows);
        for (size_t g = 0; g < gfirst.size(); ++g)
            gmt[g] = first_mt[gfirst[g]];
    }
    // the sample's moments of lattice group g: right after the group's last
    // launch, while its state is still in the Infinity Cache
    auto group_moments = [&](size_t g, int64_t steps) {
        const int base = gmt[g], cnt = gmt[g + 1] - gmt[g];
        if (cnt <= 0)
            return;
        if (q9)
            hipLaunchKernelGGL((k_batch_moments<9, kF32>), dim3((unsigned)cnt), dim3(256), 0, s, d_mt, d_lat, d_ctrl,
                               (int)steps, base, d_part, d_colpart);
        else
            (void)with_storage(ps[0].storage, [&](auto st) {
                hipLaunchKernelGGL((k_batch_moments<7, decltype(st)::value>), dim3((unsigned)cnt), dim3(256), 0, s,
                                   d_mt, d_lat, d_ctrl, (int)steps, base, d_part, d_colpart);
                return hipSuccess;
            });
    };
    // `steps` steps, then the sample if asked, then the counter update
    auto enqueue = [&](int64_t steps, bool sample) -> hipError_t {
        int64_t done = 0, launches = 0;
        if (resident && steps > 0) {
            hipError_t e = launch_resident(ps[0].lattice, ps[0].model, ps[0].storage, flags, n, d_lat, d_ctrl, (int)steps, s);
            if (e != hipSuccess)
                return e;
            done = steps;
        }
        if (resident && sample)
            group_moments(0, steps);
        // every launch of the chunk for one lattice group, then the next
        const int64_t d0 = done, l0 = launches;
        for (size_t k = 0; k + 1 < gfirst.size() && !resident; ++k) {
            const size_t g = rev ? gfirst.size() - 2 - k : k;
            done = d0;
            launches = l0;
            if (two) {
                int64_t q = steps / 2;
                q -= q & 1;  // an even number of two-step launches
                for (; launches < q; ++launches, done += 2) {
                    hipError_t e = launch_batch_step(ps[0].lattice, ps[0].model, ps[0].storage, flags, shape, g_main[2 * g + 1],
                                                     main_list.first + g_main[2 * g], d_lat, d_ctrl, (int)done,
                                                     (int)launches, s);
                    if (e != hipSuccess)
                        return e;
                }
            }
            for (; done < steps; ++launches, ++done) {
                hipError_t e = launch_batch_step(ps[0].lattice, ps[0].model, ps[0].storage, flags, one_shape, g_one[2 * g + 1],
                                                 one_list.first + g_one[2 * g], d_lat, d_ctrl, (int)done,
                                                 (int)launches, s);
                if (e != hipSuccess)
                    return e;
            }
            if (sample)
                group_moments(g, steps);
        }
        if (sample) {
            const int sto = ps[0].storage;
            hipLaunchKernelGGL(k_batch_colmeans, dim3((unsigned)((max_nx + 255) / 256), (unsigned)n), dim3(256), 0, s,
                               d_lat, d_colpart, d_colmean);
            hipLaunchKernelGGL(k_batch_final, dim3((unsigned)n), dim3(256), 0, s, d_lat, d_ctrl, (int)steps, d_part,
                               d_colmean, d_results, (int)n_samples);
            if (o->drho && q9)
                hipLaunchKernelGGL((k_batch_add_density<9, kF32>), dim3((unsigned)nmt), dim3(256), 0, s, d_mt, d_lat,
                                   d_ctrl, (int)steps);
            else if (o->drho)
                (void)with_storage(sto, [&](auto st) {
                    hipLaunchKernelGGL((k_batch_add_density<7, decltype(st)::value>), dim3((unsigned)nmt), dim3(256),
                                       0, s, d_mt, d_lat, d_ctrl, (int)steps);
                    return hipSuccess;
                });
        }
        hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, d_ctrl, steps, sample ? 1 : 0);
        return hipGetLastError();
    };
    // a sample period runs as `reps` chunks of `chunk` steps and a tail of
    // `tail` steps plus the sample; each of the two pieces is captured once
    // (on a private stream: the caller's may be the legacy null stream, which
    // cannot be captured) and replayed on the caller's stream
    const int64_t chunk = std::min<int64_t>(period, kChunk);
    const int64_t reps = o->n_steps == 0 ? 0 : (period - 1) / chunk;
    const int64_t tail = o->n_steps == 0 ? 0 : period - reps * chunk;
    const int64_t n_periods = o->n_steps == 0 ? 1 : o->n_steps / period;
    auto capture = [&](int64_t steps, bool sample, GraphPtr *ge) -> hipError_t {
        // an instantiated graph bakes in the launch shapes and the workspace
        // addresses it reads (descriptors and tile lists are uploaded again by
        // every call before it runs), so it is kept and replayed by later
        // calls with the same key
        const GraphKey key{dev, (const void *)main_list.first, (const void *)one_list.first, (const void *)d_lat,
                           (const void *)d_ctrl, (const void *)d_mt, (const void *)d_part, (const void *)d_colpart,
                           (const void *)d_colmean, (const void *)d_results, ps[0].lattice, ps[0].model,
                           ps[0].storage, flags,
                           shape,
                           main_list.second, one_list.second, nmt, (int64_t)n, n_samples, steps, sample ? 1 : 0,
                           o->drho ? 1 : 0, rev ? 1 : 0, gkey};
        if ((*ge = graph_cache_get(key)))
            return hipSuccess;
        hipGraph_t g;
        hipStream_t cap;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess)
            return e;
        hipStream_t saved = s;
        s = cap;
        hipError_t be = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        hipError_t ce = be == hipSuccess ? enqueue(steps, sample) : be;
        hipError_t ee = be == hipSuccess ? hipStreamEndCapture(cap, &g) : be;
        s = saved;
        (void)hipStreamDestroy(cap);
        if (ce != hipSuccess)
            return ce;
        if (ee != hipSuccess)
            return ee;
        auto holder = std::make_shared<GraphExec>();
        e = hipGraphInstantiate(&holder->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e == hipSuccess) {
            *ge = holder;
            graph_cache_put(key, holder);
        }
        return e;
    };
    if (o->use_graph) {
        GraphPtr g_chunk, g_tail;
        hipError_t e = reps > 0 ? capture(chunk, false, &g_chunk) : hipSuccess;
        if (e == hipSuccess)
            e = capture(tail, true, &g_tail);
        if (o->use_graph == 2) {  // prepare only: the graphs are cached, nothing runs
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                return hip_fail(e, "lbm_sweep_batch graph");
            save_record();
            return LBM_OK;
        }
        for (int64_t p = 0; p < n_periods && e == hipSuccess; ++p) {
            for (int64_t r = 0; r < reps && e == hipSuccess; ++r)
                e = hipGraphLaunch(g_chunk->exec, s);
            if (e == hipSuccess)
                e = hipGraphLaunch(g_tail->exec, s);
        }
        // no wait here: each exec remembers its latest launch (GraphExec)
        if (e == hipSuccess && g_chunk && reps > 0 && n_periods > 0)
            e = g_chunk->launched(s);
        if (e == hipSuccess)
            e = g_tail->launched(s);
        if (e != hipSuccess)
            return hip_fail(e, "lbm_sweep_batch graph");
    } else {
        for (int64_t p = 0; p < n_periods; ++p) {
            for (int64_t r = 0; r < reps; ++r)
                LBM_HIP_TRY(enqueue(chunk, false));
            LBM_HIP_TRY(enqueue(tail, true));
        }
    }

    const bool uploaded = uploaded_desc || !host_lists.empty();
    if (!out) {
        // enqueue only: the samples stay in the workspace (lbm_sweep_samples);
        // a call that uploaded tables from host vectors waits for those copies
        if (uploaded)
            LBM_HIP_TRY(hipStreamSynchronize(s));
        save_record();
        return LBM_OK;
    }
    int32_t rc = read_samples(ps, n, n_samples, d_results, s, out);
    if (rc != LBM_EHIP)
        save_record();
    return rc;
}

int32_t lbm_sweep_samples(const lbm_params *ps, int32_t n, int64_t n_samples, const void *ws, void *stream,
                          lbm_obs *out)
{
    if (!ps || n <= 0 || n_samples <= 0 || !ws || !out)
        return fail(LBM_EINVAL, "null argument, empty batch or no samples");
    for (int l = 0; l < n; ++l) {
        int32_t rc = validate_params(&ps[l], ps[l].nx);
        if (rc)
            return fail(rc, "lattice " + std::to_string(l) + ": " + lbm_last_error());
    }
    const Layout Ly = layout(ps, n, n_samples);
    return read_samples(ps, n, n_samples, (const double *)((const char *)ws + Ly.results), (hipStream_t)stream,
                        out);
}

}  // extern "C"
