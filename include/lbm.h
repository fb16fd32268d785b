/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the modified lattice
 * Boltzmann method of dense dry polar active fluids (Nesbitt, Pruessner & Lee,
 * arXiv:1902.00530).
 *
 * What it computes.  Populations f_i(t, r), i = 0..6, live on a periodic
 * triangular (D2Q7) lattice of nx x ny sites (section "Dry polar active
 * fluids").  One step is the algorithm of the appendix "Summary of modified
 * lattice Boltzmann model algorithm": densities and velocities (eq.
 * D2Q7macroscopic_u_disc), a target velocity u* (MIPS: eq. bu_mips with the
 * U_max clamp and the isotropic gradient stencil; CIL: eq. bu_CIL with the
 * speed law eq. U0; passive: u* = u), BGK relaxation towards the steady
 * state xi(rho, u*) (eq. fssD2Q7, eq. fevolution2), zero-sum noise (eq.
 * noiseDensityConservation), the negative-population correction (appendix
 * "Negative Correction") and streaming.
 *
 * Conventions shared by every entry point.
 *  - Lattice vectors e_i = (cos((i-1) pi/3), sin((i-1) pi/3)), weights
 *    w_0 = 1/2, w_i = 1/12; opposite pairs 1-4, 2-5, 3-6.
 *  - Storage is offset rows: site (x, y) sits at (x + (y mod 2)/2, y sqrt(3)/2);
 *    ny must be even.  Neighbour along e_1: (x+1, y); e_2: (x+p, y+1);
 *    e_3: (x-1+p, y+1); e_4: (x-1, y); e_5: (x-1+p, y-1); e_6: (x+p, y-1),
 *    p = y mod 2, all indices periodic.
 *  - A population buffer is [7][ny][pitch] elements of the storage type
 *    (plane i, row y, column x), pitch >= nx elements (LBM_BF16_DEV_R32: a
 *    float32 plane, then six 16-bit planes).  The state kept
 *    between steps is the population after the last step of the algorithm
 *    (the negative correction); a step streams it (population i of site r
 *    comes from r - e_i), then collides.  An initial state f^SS is therefore
 *    streamed by the first step, as in the paper.  Fields and observables of
 *    a state are those of its streamed populations (the input of step (ii)).
 *  - Noise: raw draws eta~_i = sigma (2 U_i - 1), U_i = (h_i + 1/2)/65536,
 *    h_i = the i-th 16-bit half (low half first) of Philox4x32-10 with
 *    key (seed lo, seed hi) and counter (y*nx + x, step lo, step hi, 0);
 *    eta_i = eta~_i - mean_j eta~_j.  "step" is the absolute step index.
 *  - Negative correction: a negative rest population is set to 0; an
 *    opposite pair with a negative member becomes (max(d, 0), max(-d, 0)),
 *    d = f_i - f_opp (the paper's rule (ii), in closed form); if either rule
 *    fired, the site is rescaled to this step's density.
 *
 * Square-lattice variant (lattice = LBM_D2Q9).  The same algorithm on the
 * standard D2Q9 velocity set, whose sound speed is c_s^2 = 1/3 (the paper
 * notes that c_s is a property of the lattice, appendix "Chapman-Enskog
 * Expansion"):
 *  - e_0 = 0; e_1..e_4 = (1,0), (0,1), (-1,0), (0,-1); e_5..e_8 = (1,1),
 *    (-1,1), (-1,-1), (1,-1); weights 4/9, 1/9, 1/36; opposite pairs 1-3,
 *    2-4, 5-7, 6-8; site (x, y) at (x, y), periodic; ny may be odd.
 *  - xi_i(rho, u) = w_i rho [1 + 3 e_i.u + (9/2)(e_i.u)^2 - (3/2)|u|^2].
 *  - MIPS gradient: grad rho = 3 sum_i w_i e_i rho(r + e_i), the paper's
 *    construction of its isotropic stencil on this lattice.
 *  - Noise: the raw draw of direction i is sigma (2 U_i - 1),
 *    U_i = (h_i + 1/2)/16384, h_i = bits 14 i .. 14 i + 13 of the 128-bit
 *    Philox4x32-10 output (word 0 lowest; same key and counter as above);
 *    eta_i subtracts the mean of the nine.
 *  - A population buffer is [9][ny][pitch]; every plane must be below 2^32
 *    bytes (ny * pitch < 2^30 for F32, < 2^31 for the 16-bit storages).
 *  - lbm_add_density adds drho/9 to every population.
 *  - Batched sweeps run D2Q9 with one or two steps per launch, or resident
 *    in LDS up to 3072 sites; the coarse-field calls take D2Q7 only
 *    (LBM_EUNSUPPORTED).
 *
 * Memory ownership.  The library never allocates or frees device memory.
 * The caller owns every device buffer passed in (population buffers, field
 * outputs, batch buffers, workspaces, network tensors) and the HIP stream,
 * and keeps them alive until the context that uses them is destroyed.  A
 * context owns a host object and the HIP graphs it captures; its device
 * scratch (step clock, reduction partials) lives in the caller's workspace.
 *
 * Errors.  Every entry point returns an int32_t status: LBM_OK (0) or a
 * negative code.  The message of the last error on the calling thread is
 * returned by lbm_last_error().  No C++ exception crosses this ABI.  Work is
 * enqueued on the caller's stream; an entry point only synchronises the
 * stream where its description says so.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)       /* invalid argument (sizes, parameters, null pointers) */
#define LBM_EHIP (-2)         /* HIP runtime error; message kept */
#define LBM_ENONFINITE (-3)   /* a reduction saw a NaN or infinite population */
#define LBM_EUNSUPPORTED (-4) /* valid request the library does not implement */
#define LBM_ESTATE (-5)       /* call out of order (e.g. destroyed context) */

/* Models: how u* is computed. */
#define LBM_PASSIVE 0 /* u* = u: standard BGK lattice Boltzmann */
#define LBM_MIPS 1    /* u* = C (1 - rho/rho*) grad rho for rho < rho*, |u*| <= U_max */
#define LBM_CIL 2     /* u* = U0(rho) u/|u|, U0 = B - A rho^2 if B >= A rho^2, else 0 */

/* Velocity sets. */
#define LBM_D2Q7 0 /* triangular lattice, offset rows (the paper's) */
#define LBM_D2Q9 1 /* square lattice, c_s^2 = 1/3 */

/* Population storage. */
#define LBM_F32 0      /* float32 populations */
#define LBM_BF16_DEV 1 /* bfloat16 deviations d_i = f_i - r_i (round to nearest even) */
#define LBM_F16_DEV 2  /* IEEE half deviations d_i = f_i - r_i (round to nearest even) */
#define LBM_BF16_DEV_R32 3 /* bfloat16 deviations of the six moving populations, float32 rest population */
/* The reference r_i of plane i is w_i rho_ref rounded to float, then to the
 * storage format, so that f_i = 0 is stored exactly (lbm_deviation_reference
 * returns the values); a population is read back as float(d_i) + r_i in
 * float32.
 * LBM_BF16_DEV_R32 (D2Q7 only): the buffer is the float32 rest plane
 * [ny][pitch] followed by the six bfloat16 deviation planes [6][ny][pitch],
 * 16 bytes per site (the size of [8][ny][pitch] 16-bit elements, the rest
 * plane taking the room of two); r_0 = 0 and f_0 is stored as is.  Each
 * step stores the rest population as the site's density minus its six
 * moving populations as they are stored (kept >= 0), so a site keeps its
 * mass to one float32 rounding, where the bfloat16 rest deviation of
 * LBM_BF16_DEV rounds it at every step. */

/* Initial states (appendix "CIL Model: General notes"). */
#define LBM_INIT_NONE 0        /* caller has filled the first buffer */
#define LBM_INIT_UNIFORM_DIR 1 /* direction uniform on [0, 2 pi), density uniform within +-spread */
#define LBM_INIT_GAUSS_DIR 2   /* direction normal about +x with std angle_std */

typedef struct lbm_params {
    int32_t nx, ny;    /* lattice size; ny <= 65535; nx * ny < 2^32; ny even on D2Q7 */
    int32_t model;     /* LBM_PASSIVE / LBM_MIPS / LBM_CIL */
    int32_t storage;   /* LBM_F32 / LBM_BF16_DEV / LBM_F16_DEV / LBM_BF16_DEV_R32 */
    double tau;        /* relaxation time, >= 1 (appendix "Negative Correction"); +inf = streaming only */
    double sigma;      /* noise half-width, >= 0 */
    double A, B;       /* CIL speed law */
    double C, rho_star;/* MIPS gradient gain and cut-off density */
    double u_max;      /* MIPS clamp */
    double rho_ref;    /* reference density of the deviation storages */
    uint64_t seed;     /* Philox key */
    int32_t lattice;   /* LBM_D2Q7 / LBM_D2Q9 */
    int32_t reserved;  /* 0 */
} lbm_params;

typedef struct lbm_init {
    int32_t mode;      /* LBM_INIT_* */
    int32_t reserved;
    double rho_mean;   /* mean density */
    double rho_spread; /* relative half-width of the density draw (paper: 0.1) */
    double angle_std;  /* LBM_INIT_GAUSS_DIR: standard deviation of the angle */
    double u_mag;      /* |u| of the initial state; < 0 means U0(rho) (CIL), 0 otherwise */
    double pop_noise;  /* half-width of a uniform perturbation added to every f_i */
} lbm_init;

/* Observables of the stored state, accumulated in FP64 (section "Regime
 * Categorisation in the phase diagram"). */
typedef struct lbm_obs {
    int64_t step;      /* absolute step index of the state */
    double M;          /* sum rho */
    double Jx, Jy;     /* sum rho u */
    double phi;        /* |sum rho u| / sum rho (eq. phi) */
    double mean_speed; /* sum rho |u| / sum rho */
    double zeta;       /* sum rho (B - |u|) / sum rho */
    double drho;       /* standard deviation over x of rho_y(x) = mean over y of rho(x, y) */
    int64_t nonfinite; /* number of non-finite populations */
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* Device workspace bytes a context of these parameters needs (its step
 * clock and the reduction scratch of lbm_moments); 0 on invalid
 * parameters. */
size_t lbm_workspace_bytes(const lbm_params *p, int64_t pitch);

/* Create a lattice context on the current HIP device.
 *   p        parameters (copied).
 *   f_a,f_b  two caller-owned device buffers [Q][ny][pitch] of the storage
 *            type (Q = 7 on D2Q7, 9 on D2Q9); the state starts in f_a.
 *   pitch    row pitch in elements, >= nx.
 *   init     initial state written into f_a (NULL or LBM_INIT_NONE: the
 *            caller has filled f_a).
 *   ws       caller-owned device workspace, 256-byte aligned, of ws_bytes >=
 *            lbm_workspace_bytes(p, pitch); used by this context alone until
 *            lbm_destroy.
 *   stream   caller's hipStream_t (NULL: the null stream), cast to void*.
 *   out      receives the context.
 * Enqueues the initial state (if any) and the step clock's start; no sync.
 * Returns LBM_EINVAL for nx < 2, ny < 2 or > 65535 (or odd on D2Q7),
 * nx*ny >= 2^32, pitch < nx, tau < 1, sigma < 0, non-finite or negative model
 * constants, null or equal buffers, a null, misaligned or short workspace,
 * unknown lattice/model/storage/init mode; LBM_EUNSUPPORTED for a D2Q9 plane
 * of 2^32 bytes or more. */
int32_t lbm_create(const lbm_params *p, void *f_a, void *f_b, int64_t pitch, const lbm_init *init, void *ws,
                   size_t ws_bytes, void *stream, lbm_ctx **out);

/* Enqueue n >= 0 steps on the context's stream (no synchronisation), one
 * kernel launch per step.  Runs of 64 steps replay a HIP graph captured on
 * first use (one per starting buffer); the remainder, and every step while
 * the caller is capturing the stream itself, are launched directly.  Every
 * launch reads its step index (the noise counter) from the workspace's step
 * clock, so graphs replay with unchanged arguments.  The state alternates
 * between the two buffers; lbm_current_buffer() tells which holds it
 * afterwards.  Where the two buffers together exceed 240 MiB (more than the
 * 256 MB Infinity Cache keeps) the steps' stores are non-temporal; the values
 * are the same either way. */
int32_t lbm_step(lbm_ctx *c, int64_t n);

/* Fields and observables of the stored state.  rho, ux, uy: caller-owned
 * device arrays [ny][nx] of float, or NULL to skip (u = 0 where rho = 0).
 * obs: host struct, or NULL.  With obs != NULL the call synchronises the
 * stream and returns LBM_ENONFINITE (after filling obs) if a population is
 * NaN or infinite. */
int32_t lbm_moments(lbm_ctx *c, float *rho, float *ux, float *uy, lbm_obs *obs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fields
 * and observables of lbm_moments for a population buffer f ([Q][ny][pitch]
 * of p's storage type, read only) without a context or workspace.  The
 * reduction partials live in a static device array of the library, 12 MiB
 * per GPU, held until the process ends; lattices whose partials need more
 * (moments partials grow as nx * ny / 16 doubles: up to about 5000 x 5000
 * sites) return LBM_EINVAL, and lbm_moments serves them.  step is copied into
 * obs->step.  rho, ux, uy: caller-owned device arrays [ny][nx] or NULL; obs:
 * host struct or NULL (with obs the call synchronises the stream and returns
 * LBM_ENONFINITE after filling obs if a population is not finite).  Calls on
 * one GPU share its array: calls that overlap on one GPU (two streams, two
 * threads) race.  No device memory is allocated or freed. */
int32_t lbm_observe(const lbm_params *p, const void *f, int64_t pitch, int64_t step, float *rho, float *ux,
                    float *uy, void *stream, lbm_obs *obs);

/* 0 if the state is in f_a, 1 if in f_b; negative on error. */
int32_t lbm_current_buffer(const lbm_ctx *c);

/* Absolute step index of the stored state (the Philox counter of the next
 * step); lbm_set_step sets it (checkpoint/resume; enqueued on the stream). */
int64_t lbm_get_step(const lbm_ctx *c);
int32_t lbm_set_step(lbm_ctx *c, int64_t step);

/* Add drho/7 (D2Q9: drho/9) to every population of the stored state (the
 * adiabatic density change of the appendix "CIL Model: General notes"), which
 * raises every site's density by drho.  Enqueued, no sync. */
int32_t lbm_add_density(lbm_ctx *c, double drho);

/* The per-plane references r_i (Q floats: 7 on D2Q7, 9 on D2Q9) the
 * deviation storages of these parameters are stored against (all 0 for
 * F32).  LBM_EINVAL on invalid parameters. */
int32_t lbm_deviation_reference(const lbm_params *p, float *wr);

/* Release the context (waits for its stream first). */
int32_t lbm_destroy(lbm_ctx *c);

/* Message of the last error on this thread ("" if none). */
const char *lbm_last_error(void);

/* ------------------------------------------------------------------------
 * Batched sweeps: n independent lattices of arbitrary sizes and parameters
 * (the paper's repeated runs over a grid of mean density and model constants,
 * appendix "Simulation procedure for results") advanced together: one kernel
 * launch per step (or per two steps) covers every lattice of a lattice group
 * (lbm_sweep_groups), or one launch runs a whole captured chunk of steps with
 * the lattices resident in LDS; a sample period (its steps and the FP64
 * sampling kernels) is captured in HIP graphs of at most 1024 steps and
 * replayed.
 * ---------------------------------------------------------------------- */
/* lbm_sweep_opts.tile_rows value (no tile has that many rows) for the
 * LDS-resident form: each lattice of at most 4096 sites (D2Q7; 3072 on D2Q9)
 * lives in the LDS of one CU (one 1024-lane workgroup per
 * lattice) for all the steps of a captured chunk, one launch per chunk; the
 * state crosses HBM only at the chunk's ends.  For lattices of the paper's
 * size (90 x 30), where one launch per step leaves the GPU bound by launch
 * latency. */
#define LBM_TILE_RESIDENT 1024

struct lbm_surrogate; /* lbm_cnn.h */

typedef struct lbm_sweep_opts {
    int64_t n_steps;      /* steps to run (a multiple of sample_every) */
    int64_t sample_every; /* observables every sample_every steps (0: once, at the end) */
    int64_t step0;        /* absolute step index of the first step (noise counter) */
    int32_t tile_rows;    /* work tile: 1, 2, 4 = 256x1, 128x2, 64x4 sites, one step per
                             launch; 8, 16 = 64x8, 64x16 sites, two steps per launch
                             (the second from LDS); 0 = tuned (every shape timed on the
                             batch itself, cached per batch signature).  MIPS batches
                             take 0 (tuned), 4: 64x4 tiles, one step per launch, or 8,
                             16: 64x8, 64x16 tiles, two steps per launch (the first on
                             a two-site ring, from densities of a three-site ring,
                             all in LDS).  LBM_TILE_RESIDENT (1024):
                             whole lattices in LDS (every lattice at most 4096 sites
                             on D2Q7, 3072 on D2Q9, any model; tuned among the others
                             when the batch qualifies).  D2Q9 batches take 0, 1, 2, 4, 8
                             or 16 (MIPS: 0, 8 or 16, two steps per launch), and
                             LBM_TILE_RESIDENT */
    int32_t use_graph;    /* 0: launch every kernel directly; 1: run each sample period
                             as captured HIP graphs of at most 1024 steps, kept (16 most
                             recent) and replayed by later calls with the same batch,
                             workspace and step counts; 2: prepare only: tune and
                             capture those graphs, run nothing and leave out unwritten */
    const double *drho;   /* NULL, or host array of n density changes: right after each
                             sample, every population of lattice l gains drho[l] / Q
                             (the density ramp of the paper's protocol, appendix
                             "Simulation procedure for results"); finite values only */
    int32_t keep_tables;  /* 0: build and upload the batch's tables (lattice descriptors,
                             tile lists) into ws.  1: the caller promises that ws still
                             holds what the library wrote into it on the last call with
                             this ws (it has not written into ws since, nor freed and
                             reallocated it); tables that this call would write
                             identically are then not rebuilt or uploaded, so a repeated
                             sweep of one batch enqueues its first kernel without host
                             work.  Pass 0 on the first call after allocating ws */
    /* Surrogate sweep (lbm_cnn.h; not part of the paper's method).  With
     * surrogate != NULL the network advances the coarse fields (rho, jx, jy
     * and the lattice's B as a constant channel) of every lattice by k steps
     * per evaluation; every check_every evaluations the method judges each
     * lattice still on the network from the same coarse state (lift to the
     * steady state of each cell, k steps with the sweep's noise counters,
     * coarsen) and a lattice whose relative L2 field error exceeds tol
     * continues from the judge's populations with the method (fallback).  At
     * the end each lattice still on the network is lifted from its coarse
     * fields into bufs[2l + (n_steps & 1)] and sampled like the others.
     * Needs n_steps a multiple of k, sample_every 0 or n_steps, no drho,
     * D2Q7 CIL or passive lattices of (w c) x (h c) sites (the surrogate's
     * coarse grid), n <= max_batch, the surrogate's stream, and ws of
     * lbm_sweep_workspace_bytes(ps, n, 1). */
    int32_t check_every;  /* surrogate: evaluations between checks (>= 1) */
    struct lbm_surrogate *surrogate; /* NULL: the method alone */
    int32_t k;            /* surrogate: steps per network evaluation; must equal its k */
    int32_t reserved;     /* 0 */
    double tol;           /* surrogate: fallback bound on the relative L2 error of (rho, j) */
    float *coarse_out;    /* surrogate, optional: device [n][cin][h][w], final coarse fields */
    int32_t *fallen_out;  /* surrogate, optional: host [n], 1 where the lattice fell back */
    double *check_errors_out; /* surrogate, optional: host [max_checks][n], each check's
                                 errors (NaN for lattices fallen before it) */
    int64_t max_checks;   /* rows of check_errors_out */
    int64_t *n_checks_out; /* surrogate, optional: host, checks made */
} lbm_sweep_opts;

/* Workspace bytes lbm_sweep_batch needs for these n lattices and n_samples
 * samples per lattice (0 on invalid arguments). */
size_t lbm_sweep_workspace_bytes(const lbm_params *ps, int32_t n, int64_t n_samples);

/* Work-tile rows (1, 2, 4, 8 or 16, as in lbm_sweep_opts.tile_rows, or
 * LBM_TILE_RESIDENT) the tuning chose for a batch with these lattices' sizes,
 * model and step variant (MIPS: 4 (D2Q7 only), 8, 16 or LBM_TILE_RESIDENT), 0
 * if not tuned yet in this process; negative on invalid arguments. */
int32_t lbm_sweep_tile_rows(const lbm_params *ps, int32_t n);

/* Lattice groups a sweep of these n lattices runs each captured chunk in
 * (tile forms; the LDS-resident form launches every lattice at once): the
 * lattices are independent, so every launch of a chunk runs for the first
 * group of consecutive lattices, then for the next, each group's two buffers
 * (about equal shares, at most 240 MiB where one lattice is not larger) kept
 * in the 256 MiB Infinity Cache across those launches.  A chunk of s steps
 * therefore makes groups times the launches of one group.  Successive calls on
 * one workspace take the groups in alternating order (last group first on
 * every other call; a prepare-only call keeps the order), so a call starts
 * with the state the previous one left in the cache; results do not depend on
 * the order.  LBM_EINVAL on invalid arguments. */
int32_t lbm_sweep_groups(const lbm_params *ps, int32_t n);

/* Run a batch.  ps[n]: per-lattice parameters; every lattice uses the same
 * velocity set (D2Q7 or D2Q9), the same storage (F32; on D2Q7 also
 * BF16_DEV, F16_DEV or BF16_DEV_R32, each step rounding its results into the storage as
 * lbm_step does), the same model (CIL, MIPS or passive), and agrees on
 * tau == 1 and on sigma == 0; nx*ny*Q < 2^30 (Q = 7 or 9 populations),
 * ny <= 32760.  bufs[2n]: caller-owned device buffers [Q][ny][nx] of the
 * storage type, lattice l's state in bufs[2l] and bufs[2l+1] free.
 * ws: caller-owned device workspace of ws_bytes >=
 * lbm_sweep_workspace_bytes(ps, n, n_samples).  out: host array of
 * n * n_samples lbm_obs, n_samples = n_steps / sample_every (1 if
 * sample_every == 0), sample s of lattice l at out[l * n_samples + s]; or
 * NULL: the call only enqueues the sweep (no synchronisation, unless it had
 * to upload tables from host memory) and the samples stay in ws until
 * lbm_sweep_samples reads them.  The
 * steps of lattice l use its own seed and the noise counters
 * step0 .. step0 + n_steps - 1, so a lattice gives the same result as
 * lbm_step on its own (bit for bit).  Afterwards lattice l's state is in
 * bufs[2l + (n_steps & 1)].  With out != NULL, synchronises the stream at
 * the end.  Errors: LBM_EINVAL for the conditions above, LBM_EUNSUPPORTED for
 * other storages or lattices, LBM_ENONFINITE if a sample saw a non-finite
 * population. */
int32_t lbm_sweep_batch(const lbm_params *ps, int32_t n, const lbm_sweep_opts *o, void *const *bufs, void *ws,
                        size_t ws_bytes, void *stream, lbm_obs *out);

/* The n * n_samples samples a sweep with out == NULL left in ws (same ps, n
 * and n_samples as that call), into out as lbm_sweep_batch would have
 * written them.  Synchronises the stream first.  LBM_ENONFINITE if a sample
 * saw a non-finite population. */
int32_t lbm_sweep_samples(const lbm_params *ps, int32_t n, int64_t n_samples, const void *ws, void *stream,
                          lbm_obs *out);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
