/*
 * Reference oracle: plain FP64 CPU implementation of the modified lattice
 * Boltzmann method of Nesbitt, Pruessner & Lee (arXiv:1902.00530).
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).  Written for clarity, not
 * speed: every routine is a direct transcription of the equation it cites,
 * evaluated in double precision, one site at a time.  Built with
 * -O2 -ffp-contract=off so that no fused multiply-adds change the rounding.
 *
 * Readings of the paper that this file commits to (each is listed, with the
 * reason, in the design notes of the repository):
 *   - lattice vectors e_i = (cos((i-1) pi/3), sin((i-1) pi/3)) (the printed
 *     pi/6 cannot give a lattice whose opposite pairs are 1-4, 2-5, 3-6);
 *   - offset-row storage of the triangular lattice, odd rows shifted by +1/2;
 *   - the stored state between steps is the population after step (vi)
 *     (correction), so a step is the algorithm's order (i)-(vi) verbatim, and
 *     the initial state f^SS is streamed by the first step;
 *   - observables and fields are those of the streamed populations, from
 *     which step (ii) computes rho and u (eq. D2Q7macroscopic_u_disc);
 *   - the noise subtracts the mean of the raw draws over all seven directions;
 *   - the raw draws come from Philox4x32-10 keyed by the seed, with counter
 *     (site, step lo, step hi, 0), one 16-bit half-word per direction;
 *   - u* = 0 where |u| = 0 (CIL) and u = 0 where rho = 0;
 *   - the rescale of the negative correction uses this step's density and is
 *     applied only at sites where rule (i) or (ii) fired;
 *   - the MIPS clamp keeps the direction of u* and scales its length to U_max.
 *
 * The row loops of a step carry OpenMP pragmas: each row writes only its own
 * sites, so the timing build (-fopenmp, liboracle_omp.so) runs rows on
 * several host threads with the same per-site arithmetic; the plain build
 * ignores the pragmas.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Philox4x32-R (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11, section 3.2).  Each round multiplies counter words
 * 0 and 2 by the two Philox multipliers, swaps the halves and mixes in the
 * round key; the round key is advanced by the two Weyl constants (the golden
 * ratio and sqrt(3) - 1 scaled to 32 bits) between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32(int rounds, const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k[0] += weyl0;
            k[1] += weyl1;
        }
        uint64_t p0 = (uint64_t)mult0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)mult1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------------
 * D2Q7 lattice (section "Dry polar active fluids"; appendix "Conventional
 * Lattice Boltzmann Methods").  e_0 = 0; e_i at angle (i-1) pi/3.
 * ---------------------------------------------------------------------- */
void orc_lattice_vector(int i, double *ex, double *ey)
{
    if (i == 0) {
        *ex = 0.0;
        *ey = 0.0;
        return;
    }
    const double pi = 3.14159265358979323846;
    double ang = (double)(i - 1) * pi / 3.0;
    *ex = cos(ang);
    *ey = sin(ang);
}

double orc_weight(int i) { return i == 0 ? 0.5 : 1.0 / 12.0; }

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Offset-row triangular lattice.  Site (x, y) sits at physical position
 * (x + (y mod 2)/2, y sqrt(3)/2).  The neighbour along e_i is found by
 * moving to the site whose physical position differs by e_i: rows change by
 * the sign of e_i's y-component and the column shift depends on the row
 * parity.  Everything wraps periodically. */
void orc_neighbour(int nx, int ny, int x, int y, int i, int *xn, int *yn)
{
    int par = y & 1;
    int dx = 0, dy = 0;
    switch (i) {
    case 0: dx = 0; dy = 0; break;
    case 1: dx = 1; dy = 0; break;
    case 2: dx = par; dy = 1; break;       /* (+1/2, +sqrt3/2) */
    case 3: dx = par - 1; dy = 1; break;   /* (-1/2, +sqrt3/2) */
    case 4: dx = -1; dy = 0; break;
    case 5: dx = par - 1; dy = -1; break;  /* (-1/2, -sqrt3/2) */
    case 6: dx = par; dy = -1; break;      /* (+1/2, -sqrt3/2) */
    }
    *xn = wrap(x + dx, nx);
    *yn = wrap(y + dy, ny);
}

static int opposite(int i) { return i == 0 ? 0 : ((i - 1 + 3) % 6) + 1; }

/* ------------------------------------------------------------------------
 * Steady state xi_i(rho, u) = w_i rho [1 + 4 e_i.u + 8 (e_i.u)^2 - 2|u|^2]
 * (eq. fssD2Q7 with c = 1; notation xi of the Chapman-Enskog appendix).
 * ---------------------------------------------------------------------- */
void orc_xi(double rho, double ux, double uy, double out[7])
{
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 7; ++i) {
        double ex, ey;
        orc_lattice_vector(i, &ex, &ey);
        double eu = ex * ux + ey * uy;
        out[i] = orc_weight(i) * rho * (1.0 + 4.0 * eu + 8.0 * eu * eu - 2.0 * usq);
    }
}

/* rho = sum_i f_i, rho u = sum_i f_i e_i (eq. D2Q7macroscopic_u_disc).
 * The momentum sum is taken over the three opposite pairs, using
 * e_{i+3} = -e_i, so that a pairwise-symmetric state has exactly zero
 * momentum. */
void orc_moments(const double f[7], double *rho, double *jx, double *jy)
{
    double r = 0.0;
    for (int i = 0; i < 7; ++i)
        r += f[i];
    double sx = 0.0, sy = 0.0;
    for (int i = 1; i <= 3; ++i) {
        double ex, ey;
        orc_lattice_vector(i, &ex, &ey);
        double d = f[i] - f[i + 3];
        sx += d * ex;
        sy += d * ey;
    }
    *rho = r;
    *jx = sx;
    *jy = sy;
}

/* Target velocity u* for the passive limit (u* = u, standard BGK) and the
 * CIL model (eq. bu_CIL with the speed law eq. U0). */
void orc_ustar_local(const orc_params *p, double rho, double jx, double jy, double *usx, double *usy)
{
    *usx = 0.0;
    *usy = 0.0;
    if (p->model == ORC_PASSIVE) {
        if (rho != 0.0) {
            *usx = jx / rho;
            *usy = jy / rho;
        }
        return;
    }
    if (p->model == ORC_CIL) {
        double u0 = (p->B >= p->A * rho * rho) ? (p->B - p->A * rho * rho) : 0.0;
        /* u / |u| equals j / |j| for rho > 0. */
        double jn = sqrt(jx * jx + jy * jy);
        if (jn > 0.0) {
            *usx = u0 * jx / jn;
            *usy = u0 * jy / jn;
        }
        return;
    }
}

/* MIPS target velocity (eq. bu_mips) followed by the clamp |u*| -> min(|u*|, U_max). */
void orc_ustar_mips(const orc_params *p, double rho, double gx, double gy, double *usx, double *usy)
{
    double ux = 0.0, uy = 0.0;
    if (rho < p->rho_star) {
        double k = p->C * (1.0 - rho / p->rho_star);
        ux = k * gx;
        uy = k * gy;
    }
    double un = sqrt(ux * ux + uy * uy);
    if (un > p->u_max) {
        ux = ux * (p->u_max / un);
        uy = uy * (p->u_max / un);
    }
    *usx = ux;
    *usy = uy;
}

/* Isotropic gradient grad rho = (1/3) sum_{k=1..3} (rho_k - rho_{k+3}) e_k
 * with rho_k = rho(r + e_k), Delta x = 1 (section "Motility-Induced Phase
 * Separation", the finite-difference stencil).  rho_nb[k] for k = 1..6. */
void orc_gradient(const double rho_nb[7], double *gx, double *gy)
{
    double sx = 0.0, sy = 0.0;
    for (int k = 1; k <= 3; ++k) {
        double ex, ey;
        orc_lattice_vector(k, &ex, &ey);
        sx += (rho_nb[k] - rho_nb[k + 3]) * ex;
        sy += (rho_nb[k] - rho_nb[k + 3]) * ey;
    }
    *gx = sx / 3.0;
    *gy = sy / 3.0;
}

/* Zero-sum noise (eq. noiseDensityConservation): raw draws eta~_i uniform in
 * [-sigma, sigma], then eta_i = eta~_i - (1/7) sum_j eta~_j.  The uniform
 * variate of direction i is (h_i + 1/2) / 65536 with h_i the i-th 16-bit
 * half-word (low half first) of Philox4x32-10(counter = (site, step lo,
 * step hi, 0), key = seed). */
void orc_noise(const orc_params *p, uint32_t site, int64_t step, double eta[7])
{
    uint32_t ctr[4] = {site, (uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32), 0u};
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    uint32_t w[4];
    orc_philox4x32(10, ctr, key, w);
    double raw[7];
    for (int i = 0; i < 7; ++i) {
        uint32_t word = w[i / 2];
        uint32_t h = (i % 2 == 0) ? (word & 0xffffu) : (word >> 16);
        double u = ((double)h + 0.5) / 65536.0;
        raw[i] = p->sigma * (2.0 * u - 1.0);
    }
    double mean = 0.0;
    for (int i = 0; i < 7; ++i)
        mean += raw[i];
    mean /= 7.0;
    for (int i = 0; i < 7; ++i)
        eta[i] = raw[i] - mean;
}

/* Negative correction (appendix "Negative Correction"), in the order the
 * paper states it: (i) a negative rest population is set to zero; (ii) a
 * negative moving population gives its magnitude to the opposite direction
 * and is set to zero, directions taken in the order 1..6; (iii) the site is
 * rescaled to the density rho.  Returns 1 if (i) or (ii) fired. */
int orc_correct(double f[7], double rho)
{
    int fired = 0;
    if (f[0] < 0.0) {
        f[0] = 0.0;
        fired = 1;
    }
    for (int i = 1; i <= 6; ++i) {
        if (f[i] < 0.0) {
            f[opposite(i)] += fabs(f[i]);
            f[i] = 0.0;
            fired = 1;
        }
    }
    if (fired) {
        double s = 0.0;
        for (int i = 0; i < 7; ++i)
            s += f[i];
        if (s > 0.0) {
            for (int i = 0; i < 7; ++i)
                f[i] = f[i] * (rho / s);
        } else {
            for (int i = 0; i < 7; ++i)
                f[i] = 0.0;
        }
    }
    return fired;
}

static size_t plane(const orc_params *p) { return (size_t)p->nx * (size_t)p->ny; }

static int valid(const orc_params *p)
{
    if (p->nx < 2 || p->ny < 2 || (p->ny & 1))
        return 0;
    if (!(p->tau >= 1.0))
        return 0;
    return 1;
}

/* Streaming, step (i): f*_i(r) = f_i(r - e_i), taken as a pull from the
 * neighbour along the opposite direction.  out must not alias in. */
void orc_stream(const orc_params *p, const double *in, double *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane(p);
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 7; ++i) {
                int xs, ys;
                orc_neighbour(nx, ny, x, y, opposite(i), &xs, &ys);
                out[(size_t)i * n + (size_t)y * nx + x] = in[(size_t)i * n + (size_t)ys * nx + xs];
            }
}

/* One step of the algorithm in the appendix "Summary of modified lattice
 * Boltzmann model algorithm", in its order: (i) streaming of the whole
 * lattice, then at every site (ii) rho and u, (iii) u* and f^SS, (iv) BGK
 * redistribution, (v) noise and (vi) the negative correction. */
int orc_step(const orc_params *p, double *f, int64_t step)
{
    if (!valid(p))
        return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane(p);
    double *rho = (double *)malloc(n * sizeof(double));
    double *fs = (double *)malloc(7 * n * sizeof(double));
    if (!rho || !fs) {
        free(rho);
        free(fs);
        return -2;
    }
    /* (i) streaming */
    orc_stream(p, f, fs);
    /* (ii) densities of the whole streamed lattice (the MIPS gradient needs them) */
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double g[7], r, jx, jy;
            for (int i = 0; i < 7; ++i)
                g[i] = fs[(size_t)i * n + (size_t)y * nx + x];
            orc_moments(g, &r, &jx, &jy);
            rho[(size_t)y * nx + x] = r;
        }
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double g[7], r, jx, jy;
            for (int i = 0; i < 7; ++i)
                g[i] = fs[(size_t)i * n + s];
            orc_moments(g, &r, &jx, &jy);
            /* (iii) u* and f^SS */
            double usx, usy;
            if (p->model == ORC_MIPS) {
                double nb[7];
                nb[0] = r;
                for (int k = 1; k <= 6; ++k) {
                    int xn, yn;
                    orc_neighbour(nx, ny, x, y, k, &xn, &yn);
                    nb[k] = rho[(size_t)yn * nx + xn];
                }
                double gx, gy;
                orc_gradient(nb, &gx, &gy);
                orc_ustar_mips(p, r, gx, gy, &usx, &usy);
            } else {
                orc_ustar_local(p, r, jx, jy, &usx, &usy);
            }
            double fss[7];
            orc_xi(r, usx, usy, fss);
            /* (iv) BGK redistribution */
            double out[7];
            for (int i = 0; i < 7; ++i)
                out[i] = g[i] - (g[i] - fss[i]) / p->tau;
            /* (v) noise */
            double eta[7];
            orc_noise(p, (uint32_t)s, step, eta);
            for (int i = 0; i < 7; ++i)
                out[i] += eta[i];
            /* (vi) negative correction */
            orc_correct(out, r);
            for (int i = 0; i < 7; ++i)
                f[(size_t)i * n + s] = out[i];
        }
    free(rho);
    free(fs);
    return 0;
}

int orc_run(const orc_params *p, double *f, int64_t step0, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        int rc = orc_step(p, f, step0 + t);
        if (rc)
            return rc;
    }
    return 0;
}

/* Initial state (appendix "CIL Model: General notes"): per site, one uniform
 * variate sets the direction of u and another the density, uniform within
 * +-rho_spread of rho_mean; |u| = U0(rho) (CIL) unless u_mag >= 0 is given;
 * the populations are f^SS of that (rho, u).  Mode 2 draws the angle from a
 * normal distribution about +x instead (Box-Muller).  The variates are the
 * four words of Philox4x32-10(counter = (site, 0, 0, 1), key = seed), mapped
 * to (w + 1/2) / 2^32.  An optional uniform perturbation of each population
 * uses the 16-bit halves of Philox4x32-10(counter = (site, 0, 0, 2)). */
int orc_initialise(const orc_params *p, const orc_init *in, double *f)
{
    if (!valid(p))
        return -1;
    if (in->mode == 0)
        return 0;
    const double pi = 3.14159265358979323846;
    const size_t n = plane(p);
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            uint32_t s = (uint32_t)((size_t)y * p->nx + x);
            uint32_t ctr[4] = {s, 0u, 0u, 1u};
            uint32_t w[4];
            orc_philox4x32(10, ctr, key, w);
            double u[4];
            for (int k = 0; k < 4; ++k)
                u[k] = ((double)w[k] + 0.5) / 4294967296.0;
            double theta;
            if (in->mode == 2)
                theta = in->angle_std * sqrt(-2.0 * log(u[2])) * cos(2.0 * pi * u[3]);
            else
                theta = 2.0 * pi * u[0];
            double r = in->rho_mean * (1.0 + in->rho_spread * (2.0 * u[1] - 1.0));
            double mag;
            if (in->u_mag >= 0.0)
                mag = in->u_mag;
            else if (p->model == ORC_CIL)
                mag = (p->B >= p->A * r * r) ? (p->B - p->A * r * r) : 0.0;
            else
                mag = 0.0;
            double fs[7];
            orc_xi(r, mag * cos(theta), mag * sin(theta), fs);
            if (in->pop_noise != 0.0) {
                uint32_t ctr2[4] = {s, 0u, 0u, 2u};
                uint32_t w2[4];
                orc_philox4x32(10, ctr2, key, w2);
                for (int i = 0; i < 7; ++i) {
                    uint32_t word = w2[i / 2];
                    uint32_t h = (i % 2 == 0) ? (word & 0xffffu) : (word >> 16);
                    double v = ((double)h + 0.5) / 65536.0;
                    fs[i] += in->pop_noise * (2.0 * v - 1.0);
                }
            }
            for (int i = 0; i < 7; ++i)
                f[(size_t)i * n + s] = fs[i];
        }
    return 0;
}

void orc_fields_of(const orc_params *p, const double *f, double *rho, double *ux, double *uy)
{
    const size_t n = plane(p);
    for (size_t s = 0; s < n; ++s) {
        double fs[7], r, jx, jy;
        for (int i = 0; i < 7; ++i)
            fs[i] = f[(size_t)i * n + s];
        orc_moments(fs, &r, &jx, &jy);
        if (rho)
            rho[s] = r;
        if (ux)
            ux[s] = (r != 0.0) ? jx / r : 0.0;
        if (uy)
            uy[s] = (r != 0.0) ? jy / r : 0.0;
    }
}

/* Observables of the section "Regime Categorisation in the phase diagram":
 * phi (eq. phi), the banding measure (standard deviation over x of the
 * y-averaged density) and zeta; plus total mass and momentum; of the given
 * populations. */
void orc_observables_of(const orc_params *p, const double *f, orc_obs *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane(p);
    double M = 0.0, Jx = 0.0, Jy = 0.0, speed = 0.0, zsum = 0.0, bad = 0.0;
    double *col = (double *)calloc((size_t)nx, sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double fs[7], r, jx, jy;
            for (int i = 0; i < 7; ++i) {
                fs[i] = f[(size_t)i * n + s];
                if (!isfinite(fs[i]))
                    bad += 1.0;
            }
            orc_moments(fs, &r, &jx, &jy);
            double umag = (r != 0.0) ? sqrt(jx * jx + jy * jy) / r : 0.0;
            M += r;
            Jx += jx;
            Jy += jy;
            speed += r * umag;
            zsum += r * (p->B - umag);
            col[x] += r;
        }
    double mean = 0.0;
    for (int x = 0; x < nx; ++x) {
        col[x] /= (double)ny;
        mean += col[x];
    }
    mean /= (double)nx;
    double var = 0.0;
    for (int x = 0; x < nx; ++x)
        var += (col[x] - mean) * (col[x] - mean);
    var /= (double)nx;
    free(col);
    out->M = M;
    out->Jx = Jx;
    out->Jy = Jy;
    out->phi = (M != 0.0) ? sqrt(Jx * Jx + Jy * Jy) / M : 0.0;
    out->mean_speed = (M != 0.0) ? speed / M : 0.0;
    out->zeta = (M != 0.0) ? zsum / M : 0.0;
    out->drho = sqrt(var);
    out->nonfinite = bad;
}

/* Fields and observables of a stored state: those of its streamed
 * populations, from which step (ii) takes rho and u. */
void orc_fields(const orc_params *p, const double *f, double *rho, double *ux, double *uy)
{
    double *fs = (double *)malloc(7 * plane(p) * sizeof(double));
    if (!fs)
        return;
    orc_stream(p, f, fs);
    orc_fields_of(p, fs, rho, ux, uy);
    free(fs);
}

void orc_observables(const orc_params *p, const double *f, orc_obs *out)
{
    double *fs = (double *)malloc(7 * plane(p) * sizeof(double));
    if (!fs)
        return;
    orc_stream(p, f, fs);
    orc_observables_of(p, fs, out);
    free(fs);
}
