/* Drives every routine of the C oracle on small lattices (D2Q7 and D2Q9, the
 * three models, noise, corrections that fire, zero-density sites) so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer sees every
 * access.  Exit status 0 and no sanitizer report are the pass criteria. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lbm_oracle.h"

static double *alloc_pop(int q, int nx, int ny)
{
    double *f = (double *)calloc((size_t)q * nx * ny, sizeof(double));
    if (!f)
        exit(2);
    return f;
}

static int run_q7(int model, int nx, int ny, int zero_cols)
{
    orc_params p = {nx, ny, model, 0, model == ORC_MIPS ? 2.0 : 1.0, 0.05, 0.125, 0.3, 6.25, 1.6, 0.3, 77};
    orc_init in = {1, 0, 0.74, 0.1, 0.0, model == ORC_MIPS ? 0.1 : -1.0, 1e-3};
    double *f = alloc_pop(7, nx, ny), *g = alloc_pop(7, nx, ny);
    double *rho = alloc_pop(1, nx, ny), *ux = alloc_pop(1, nx, ny), *uy = alloc_pop(1, nx, ny);
    if (orc_initialise(&p, &in, f))
        return 1;
    for (int i = 0; i < 7; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < zero_cols && x < nx; ++x)
                f[((size_t)i * ny + y) * nx + x] = 0.0;
    if (orc_run(&p, f, 0, 5))
        return 1;
    orc_stream(&p, f, g);
    orc_fields(&p, f, rho, ux, uy);
    orc_fields_of(&p, g, rho, ux, uy);
    orc_obs o;
    orc_observables(&p, f, &o);
    orc_observables_of(&p, g, &o);
    int bad = o.nonfinite != 0.0 || !isfinite(o.M);
    free(f);
    free(g);
    free(rho);
    free(ux);
    free(uy);
    return bad;
}

static int run_q9(int model, int nx, int ny)
{
    orc_params p = {nx, ny, model, 0, 1.0, 0.05, 0.125, 0.3, 6.25, 1.6, 0.3, 78};
    orc_init in = {2, 0, 0.74, 0.1, 0.05, -1.0, 0.0};
    double *f = alloc_pop(9, nx, ny), *g = alloc_pop(9, nx, ny);
    double *rho = alloc_pop(1, nx, ny), *ux = alloc_pop(1, nx, ny), *uy = alloc_pop(1, nx, ny);
    if (orc9_initialise(&p, &in, f) || orc9_run(&p, f, 3, 4))
        return 1;
    orc9_stream(&p, f, g);
    orc9_fields(&p, f, rho, ux, uy);
    orc_obs o;
    orc9_observables(&p, f, &o);
    int bad = o.nonfinite != 0.0;
    free(f);
    free(g);
    free(rho);
    free(ux);
    free(uy);
    return bad;
}

int main(void)
{
    int bad = 0;
    for (int m = ORC_PASSIVE; m <= ORC_CIL; ++m) {
        bad |= run_q7(m, 6, 4, 0);
        bad |= run_q7(m, 9, 6, 3);
        bad |= run_q9(m, 5, 3);
        bad |= run_q9(m, 8, 7);
    }
    /* correction with negatives, noise, Philox, lattice helpers */
    double fc[7] = {-0.1, 0.2, -0.05, 0.1, 0.0, 0.3, -0.2};
    orc_correct(fc, 0.25);
    double f9[9] = {-0.1, 0.2, -0.05, 0.1, 0.0, 0.3, -0.2, 0.01, -0.01};
    orc9_correct(f9, 0.25);
    orc_params p = {8, 8, ORC_CIL, 0, 1.0, 0.05, 0.1, 0.3, 0.0, 1.0, 1.0, 5};
    double eta[9];
    orc_noise(&p, 17u, 3, eta);
    orc9_noise(&p, 17u, 3, eta);
    uint32_t c[4] = {1, 2, 3, 4}, k[2] = {5, 6}, w[4];
    orc_philox4x32(10, c, k, w);
    int xn, yn;
    for (int i = 0; i < 7; ++i)
        orc_neighbour(8, 8, 0, 0, i, &xn, &yn);
    for (int i = 0; i < 9; ++i)
        orc9_neighbour(8, 8, 7, 7, i, &xn, &yn);
    printf(bad ? "oracle sanitizer run: FAILED\n" : "oracle sanitizer run: ok\n");
    return bad;
}
