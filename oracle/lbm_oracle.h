/*
 * Reference oracle for the modified lattice Boltzmann method for dense dry
 * polar active fluids (Nesbitt, Pruessner & Lee, arXiv:1902.00530).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * of the paper's method.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may build, load or call it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * Layout: populations are f[i][y][x], i = 0..6, 0 <= x < nx, 0 <= y < ny,
 * contiguous (no pitch), FP64.  The stored state between steps is the
 * population after the last step of the algorithm in the appendix "Summary
 * of modified lattice Boltzmann model algorithm" (the negative correction),
 * so one oracle step is that algorithm in order: stream -> moments -> u* ->
 * f^SS -> collide -> noise -> negative correction.  Fields and observables
 * of a stored state are those of its streamed populations.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#define ORC_PASSIVE 0
#define ORC_MIPS 1
#define ORC_CIL 2

typedef struct {
    int32_t nx, ny;      /* lattice size; ny must be even (offset rows) */
    int32_t model;       /* ORC_PASSIVE / ORC_MIPS / ORC_CIL */
    int32_t pad_;
    double tau;          /* BGK relaxation time, tau >= 1 or +inf */
    double sigma;        /* noise amplitude: eta~ uniform in [-sigma, sigma] */
    double A, B;         /* CIL speed law U0 = B - A rho^2 (clamped at 0) */
    double C, rho_star;  /* MIPS u* = C (1 - rho/rho*) grad rho */
    double u_max;        /* MIPS clamp of |u*| */
    uint64_t seed;       /* Philox key */
} orc_params;

typedef struct {
    int32_t mode;        /* 0 none, 1 uniform direction, 2 Gaussian angle about +x */
    int32_t pad_;
    double rho_mean;     /* mean density */
    double rho_spread;   /* relative half-width of the uniform density draw */
    double angle_std;    /* std of the Gaussian angle (mode 2) */
    double u_mag;        /* |u| of the initial state; < 0 means U0(rho) (CIL) */
    double pop_noise;    /* half-width of a uniform perturbation added to each f_i */
} orc_init;

typedef struct {
    double M, Jx, Jy;    /* total mass and momentum */
    double phi;          /* |sum rho u| / sum rho */
    double mean_speed;   /* sum rho|u| / sum rho */
    double zeta;         /* sum rho (B - |u|) / sum rho */
    double drho;         /* population std over x of the column mean rho_y(x) */
    double nonfinite;    /* number of non-finite populations */
} orc_obs;

/* Philox4x32 with R rounds (Salmon et al., SC'11). */
void orc_philox4x32(int rounds, const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Lattice: neighbour r + e_i of site (x, y) on the offset-row triangular lattice. */
void orc_neighbour(int nx, int ny, int x, int y, int i, int *xn, int *yn);
/* Physical lattice vector e_i and weight w_i of D2Q7. */
void orc_lattice_vector(int i, double *ex, double *ey);
double orc_weight(int i);

/* Steady-state distribution xi_i(rho, u), eq. fssD2Q7. */
void orc_xi(double rho, double ux, double uy, double out[7]);
/* Zeroth and first moments of one site's populations. */
void orc_moments(const double f[7], double *rho, double *jx, double *jy);
/* Target velocity for the CIL and passive models (local rules). */
void orc_ustar_local(const orc_params *p, double rho, double jx, double jy, double *usx, double *usy);
/* MIPS target velocity from the density and its lattice gradient. */
void orc_ustar_mips(const orc_params *p, double rho, double gx, double gy, double *usx, double *usy);
/* Isotropic lattice gradient from the six neighbour densities rho_1..rho_6. */
void orc_gradient(const double rho_nb[7], double *gx, double *gy);
/* Zero-sum noise eta_i for (site, step). */
void orc_noise(const orc_params *p, uint32_t site, int64_t step, double eta[7]);
/* Negative-population correction; returns 1 if any rule fired. */
int orc_correct(double f[7], double rho);

/* One full step of the lattice, f in place.  step = absolute step index. */
int orc_step(const orc_params *p, double *f, int64_t step);
/* n steps starting at absolute step index step0. */
int orc_run(const orc_params *p, double *f, int64_t step0, int64_t n);
/* Initial populations (appendix "CIL Model: General notes"). */
int orc_initialise(const orc_params *p, const orc_init *in, double *f);
/* Streaming (step (i)) of a whole lattice, pull form; out must not alias in. */
void orc_stream(const orc_params *p, const double *in, double *out);
/* Observables and fields (arrays of ny*nx) of the given populations. */
void orc_observables_of(const orc_params *p, const double *f, orc_obs *out);
void orc_fields_of(const orc_params *p, const double *f, double *rho, double *ux, double *uy);
/* Observables and fields of a stored state: those of its streamed populations. */
void orc_observables(const orc_params *p, const double *f, orc_obs *out);
void orc_fields(const orc_params *p, const double *f, double *rho, double *ux, double *uy);

/* Host threads of a step's row loops in the OpenMP build (n <= 0 keeps the
 * current count); returns the count in effect, 1 in the plain build. */
int orc_set_threads(int n);

/* ------------------------------------------------------------------------
 * Square-lattice (D2Q9) variant, lbm_oracle_q9.c: populations f[9][ny][nx];
 * same parameter, init and observable structs; ny may be odd.
 * ---------------------------------------------------------------------- */
void orc9_lattice_vector(int i, double *ex, double *ey);
double orc9_weight(int i);
int orc9_opposite(int i);
void orc9_neighbour(int nx, int ny, int x, int y, int i, int *xn, int *yn);
void orc9_xi(double rho, double ux, double uy, double out[9]);
void orc9_moments(const double f[9], double *rho, double *jx, double *jy);
void orc9_gradient(const double rho_nb[9], double *gx, double *gy);
void orc9_draws(const uint32_t w[4], uint32_t h[9]);
void orc9_noise(const orc_params *p, uint32_t site, int64_t step, double eta[9]);
int orc9_correct(double f[9], double rho);
void orc9_stream(const orc_params *p, const double *in, double *out);
int orc9_step(const orc_params *p, double *f, int64_t step);
int orc9_run(const orc_params *p, double *f, int64_t step0, int64_t n);
int orc9_initialise(const orc_params *p, const orc_init *in, double *f);
void orc9_fields_of(const orc_params *p, const double *f, double *rho, double *ux, double *uy);
void orc9_observables_of(const orc_params *p, const double *f, orc_obs *out);
void orc9_fields(const orc_params *p, const double *f, double *rho, double *ux, double *uy);
void orc9_observables(const orc_params *p, const double *f, orc_obs *out);

#endif
