/*
 * Reference oracle, square-lattice (D2Q9) variant of the modified lattice
 * Boltzmann method of Nesbitt, Pruessner & Lee (arXiv:1902.00530).
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).  Plain FP64, one site at a
 * time, built with -ffp-contract=off.
 *
 * The paper states its method on the triangular D2Q7 lattice and notes that
 * the sound speed (and with it every coefficient of the steady state) is a
 * property of the chosen lattice (appendix "Chapman-Enskog Expansion").  This
 * file carries the same algorithm (appendix "Summary of modified lattice
 * Boltzmann model algorithm") over to the standard D2Q9 velocity set; the
 * readings it commits to are:
 *   - e_0 = 0; e_1..e_4 = (1,0), (0,1), (-1,0), (0,-1); e_5..e_8 = (1,1),
 *     (-1,1), (-1,-1), (1,-1); weights 4/9, 1/9, 1/36; c_s^2 = 1/3; opposite
 *     pairs 1-3, 2-4, 5-7, 6-8; square sites at integer (x, y), periodic;
 *   - the steady state is the discretised Maxwellian of this lattice,
 *     xi_i = w_i rho [1 + 3 e_i.u + (9/2)(e_i.u)^2 - (3/2)|u|^2], which is the
 *     paper's D2Q7 form with c_s^2 = 1/3 in place of 1/4;
 *   - the MIPS gradient is the paper's construction on this lattice,
 *     grad rho = (1/c_s^2) sum_i w_i e_i rho(r + e_i) (on D2Q7 this is the
 *     paper's six-neighbour stencil);
 *   - the noise subtracts the mean of nine raw draws; the draw of direction i
 *     is bits 14 i .. 14 i + 13 of the 128-bit Philox4x32-10 output (word 0
 *     lowest), U_i = (h_i + 1/2) / 16384, so one generator call serves all
 *     nine directions;
 *   - the negative correction is the paper's rule with four opposite pairs;
 *   - the density change of the protocol adds drho / 9 to every population;
 *   - u*, the CIL speed law, the MIPS clamp, the BGK step, the stored-state
 *     convention and the observables are those of the D2Q7 oracle.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

#define Q9 9

/* D2Q9 velocity set: the rest vector, the four axis vectors counter-clockwise
 * from +x, then the four diagonals counter-clockwise from (1, 1). */
static const int EX9[Q9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY9[Q9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

void orc9_lattice_vector(int i, double *ex, double *ey)
{
    *ex = (double)EX9[i];
    *ey = (double)EY9[i];
}

double orc9_weight(int i)
{
    if (i == 0)
        return 4.0 / 9.0;
    return i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0;
}

/* The direction j with e_j = -e_i. */
int orc9_opposite(int i)
{
    for (int j = 0; j < Q9; ++j)
        if (EX9[j] == -EX9[i] && EY9[j] == -EY9[i])
            return j;
    return -1;
}

static int wrap9(int a, int n) { return ((a % n) + n) % n; }

void orc9_neighbour(int nx, int ny, int x, int y, int i, int *xn, int *yn)
{
    *xn = wrap9(x + EX9[i], nx);
    *yn = wrap9(y + EY9[i], ny);
}

/* xi_i(rho, u) = w_i rho [1 + e_i.u / c_s^2 + (e_i.u)^2 / (2 c_s^4)
 *                          - |u|^2 / (2 c_s^2)], c_s^2 = 1/3. */
void orc9_xi(double rho, double ux, double uy, double out[9])
{
    const double cs2 = 1.0 / 3.0;
    const double usq = ux * ux + uy * uy;
    for (int i = 0; i < Q9; ++i) {
        double eu = EX9[i] * ux + EY9[i] * uy;
        out[i] = orc9_weight(i) * rho * (1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - usq / (2.0 * cs2));
    }
}

/* rho = sum f_i; rho u = sum f_i e_i, summed over the four opposite pairs
 * (e_opp = -e) so that a pairwise-symmetric site has exactly zero momentum. */
void orc9_moments(const double f[9], double *rho, double *jx, double *jy)
{
    double r = 0.0;
    for (int i = 0; i < Q9; ++i)
        r += f[i];
    double sx = 0.0, sy = 0.0;
    const int first[4] = {1, 2, 5, 6};
    for (int k = 0; k < 4; ++k) {
        int i = first[k];
        double d = f[i] - f[orc9_opposite(i)];
        sx += d * EX9[i];
        sy += d * EY9[i];
    }
    *rho = r;
    *jx = sx;
    *jy = sy;
}

/* grad rho = (1/c_s^2) sum_i w_i e_i rho_i, rho_i = rho(r + e_i). */
void orc9_gradient(const double rho_nb[9], double *gx, double *gy)
{
    double sx = 0.0, sy = 0.0;
    for (int i = 1; i < Q9; ++i) {
        sx += orc9_weight(i) * EX9[i] * rho_nb[i];
        sy += orc9_weight(i) * EY9[i] * rho_nb[i];
    }
    *gx = 3.0 * sx;
    *gy = 3.0 * sy;
}

/* The nine 14-bit fields of the 128-bit word w[0] + 2^32 w[1] + 2^64 w[2]
 * + 2^96 w[3], lowest first. */
void orc9_draws(const uint32_t w[4], uint32_t h[9])
{
    for (int i = 0; i < Q9; ++i) {
        uint32_t v = 0;
        for (int b = 0; b < 14; ++b) {
            int bit = 14 * i + b;
            uint32_t one = (w[bit / 32] >> (bit % 32)) & 1u;
            v |= one << b;
        }
        h[i] = v;
    }
}

/* Zero-sum noise (eq. noiseDensityConservation) over the nine directions. */
void orc9_noise(const orc_params *p, uint32_t site, int64_t step, double eta[9])
{
    uint32_t ctr[4] = {site, (uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32), 0u};
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    uint32_t w[4], h[9];
    orc_philox4x32(10, ctr, key, w);
    orc9_draws(w, h);
    double raw[9], mean = 0.0;
    for (int i = 0; i < Q9; ++i) {
        double u = ((double)h[i] + 0.5) / 16384.0;
        raw[i] = p->sigma * (2.0 * u - 1.0);
        mean += raw[i];
    }
    mean /= 9.0;
    for (int i = 0; i < Q9; ++i)
        eta[i] = raw[i] - mean;
}

/* Negative correction (appendix "Negative Correction") in the paper's order:
 * a negative rest population becomes 0; a negative moving population, taken
 * in the order 1..8, gives its magnitude to the opposite direction and
 * becomes 0; if either rule fired, the site is rescaled to rho. */
int orc9_correct(double f[9], double rho)
{
    int fired = 0;
    if (f[0] < 0.0) {
        f[0] = 0.0;
        fired = 1;
    }
    for (int i = 1; i < Q9; ++i) {
        if (f[i] < 0.0) {
            f[orc9_opposite(i)] += fabs(f[i]);
            f[i] = 0.0;
            fired = 1;
        }
    }
    if (fired) {
        double s = 0.0;
        for (int i = 0; i < Q9; ++i)
            s += f[i];
        for (int i = 0; i < Q9; ++i)
            f[i] = s > 0.0 ? f[i] * (rho / s) : 0.0;
    }
    return fired;
}

static size_t plane9(const orc_params *p) { return (size_t)p->nx * (size_t)p->ny; }

static int valid9(const orc_params *p) { return p->nx >= 2 && p->ny >= 2 && p->tau >= 1.0; }

/* Streaming, step (i): f*_i(r) = f_i(r - e_i). */
void orc9_stream(const orc_params *p, const double *in, double *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane9(p);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < Q9; ++i) {
                int xs = wrap9(x - EX9[i], nx), ys = wrap9(y - EY9[i], ny);
                out[(size_t)i * n + (size_t)y * nx + x] = in[(size_t)i * n + (size_t)ys * nx + xs];
            }
}

/* One step in the order of the appendix "Summary of modified lattice
 * Boltzmann model algorithm": (i) stream, (ii) rho and u, (iii) u* and f^SS,
 * (iv) BGK, (v) noise, (vi) negative correction. */
int orc9_step(const orc_params *p, double *f, int64_t step)
{
    if (!valid9(p))
        return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane9(p);
    double *rho = (double *)malloc(n * sizeof(double));
    double *fs = (double *)malloc(Q9 * n * sizeof(double));
    if (!rho || !fs) {
        free(rho);
        free(fs);
        return -2;
    }
    orc9_stream(p, f, fs);
    for (size_t s = 0; s < n; ++s) {
        double g[9], r, jx, jy;
        for (int i = 0; i < Q9; ++i)
            g[i] = fs[(size_t)i * n + s];
        orc9_moments(g, &r, &jx, &jy);
        rho[s] = r;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double g[9], r, jx, jy;
            for (int i = 0; i < Q9; ++i)
                g[i] = fs[(size_t)i * n + s];
            orc9_moments(g, &r, &jx, &jy);
            double usx, usy;
            if (p->model == ORC_MIPS) {
                double nb[9];
                for (int i = 0; i < Q9; ++i) {
                    int xn, yn;
                    orc9_neighbour(nx, ny, x, y, i, &xn, &yn);
                    nb[i] = rho[(size_t)yn * nx + xn];
                }
                double gx, gy;
                orc9_gradient(nb, &gx, &gy);
                orc_ustar_mips(p, r, gx, gy, &usx, &usy);
            } else {
                orc_ustar_local(p, r, jx, jy, &usx, &usy);
            }
            double fss[9], out[9], eta[9];
            orc9_xi(r, usx, usy, fss);
            for (int i = 0; i < Q9; ++i)
                out[i] = g[i] - (g[i] - fss[i]) / p->tau;
            orc9_noise(p, (uint32_t)s, step, eta);
            for (int i = 0; i < Q9; ++i)
                out[i] += eta[i];
            orc9_correct(out, r);
            for (int i = 0; i < Q9; ++i)
                f[(size_t)i * n + s] = out[i];
        }
    free(rho);
    free(fs);
    return 0;
}

int orc9_run(const orc_params *p, double *f, int64_t step0, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; ++t) {
        int rc = orc9_step(p, f, step0 + t);
        if (rc)
            return rc;
    }
    return 0;
}

/* Initial state as in the D2Q7 oracle (same variates: counter (site, 0, 0, 1),
 * direction, density, Box-Muller angle), with the D2Q9 steady state; the
 * optional population perturbation takes the nine 14-bit fields of counter
 * (site, 0, 0, 2). */
int orc9_initialise(const orc_params *p, const orc_init *in, double *f)
{
    if (!valid9(p))
        return -1;
    if (in->mode == 0)
        return 0;
    const double pi = 3.14159265358979323846;
    const size_t n = plane9(p);
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
            double fs[9];
            orc9_xi(r, mag * cos(theta), mag * sin(theta), fs);
            if (in->pop_noise != 0.0) {
                uint32_t ctr2[4] = {s, 0u, 0u, 2u};
                uint32_t w2[4], h[9];
                orc_philox4x32(10, ctr2, key, w2);
                orc9_draws(w2, h);
                for (int i = 0; i < Q9; ++i)
                    fs[i] += in->pop_noise * (2.0 * (((double)h[i] + 0.5) / 16384.0) - 1.0);
            }
            for (int i = 0; i < Q9; ++i)
                f[(size_t)i * n + s] = fs[i];
        }
    return 0;
}

void orc9_fields_of(const orc_params *p, const double *f, double *rho, double *ux, double *uy)
{
    const size_t n = plane9(p);
    for (size_t s = 0; s < n; ++s) {
        double g[9], r, jx, jy;
        for (int i = 0; i < Q9; ++i)
            g[i] = f[(size_t)i * n + s];
        orc9_moments(g, &r, &jx, &jy);
        if (rho)
            rho[s] = r;
        if (ux)
            ux[s] = (r != 0.0) ? jx / r : 0.0;
        if (uy)
            uy[s] = (r != 0.0) ? jy / r : 0.0;
    }
}

/* Observables of the section "Regime Categorisation in the phase diagram"
 * (the D2Q7 oracle's definitions) of the given populations. */
void orc9_observables_of(const orc_params *p, const double *f, orc_obs *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t n = plane9(p);
    double M = 0.0, Jx = 0.0, Jy = 0.0, speed = 0.0, zsum = 0.0, bad = 0.0;
    double *col = (double *)calloc((size_t)nx, sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double g[9], r, jx, jy;
            for (int i = 0; i < Q9; ++i) {
                g[i] = f[(size_t)i * n + s];
                if (!isfinite(g[i]))
                    bad += 1.0;
            }
            orc9_moments(g, &r, &jx, &jy);
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

void orc9_fields(const orc_params *p, const double *f, double *rho, double *ux, double *uy)
{
    double *fs = (double *)malloc(Q9 * plane9(p) * sizeof(double));
    if (!fs)
        return;
    orc9_stream(p, f, fs);
    orc9_fields_of(p, fs, rho, ux, uy);
    free(fs);
}

void orc9_observables(const orc_params *p, const double *f, orc_obs *out)
{
    double *fs = (double *)malloc(Q9 * plane9(p) * sizeof(double));
    if (!fs)
        return;
    orc9_stream(p, f, fs);
    orc9_observables_of(p, fs, out);
    free(fs);
}
