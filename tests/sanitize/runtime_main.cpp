// Drives the host side of the library (argument validation, workspace
// layouts, lattice groups, the table record of batched sweeps, the surrogate
// handle's checks) with no GPU present, in a build whose host code carries
// AddressSanitizer.  Every call must return an error code or a size, never
// crash, leak or touch memory it does not own.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/lbm_cnn.h"

static lbm_params params(int nx, int ny, int model, int storage = LBM_F32, int lattice = LBM_D2Q7)
{
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.model = model;
    p.storage = storage;
    p.tau = 1.0;
    p.sigma = 0.05;
    p.A = 0.125;
    p.B = 0.3;
    p.C = 6.25;
    p.rho_star = 1.6;
    p.u_max = 0.3;
    p.rho_ref = 0.74;
    p.seed = 7;
    p.lattice = lattice;
    return p;
}

int main()
{
    int bad = 0;
    auto expect = [&](bool ok, const char *what) {
        if (!ok) {
            printf("unexpected: %s (%s)\n", what, lbm_last_error());
            bad = 1;
        }
    };
    // workspace sizes and validation of lbm_create
    lbm_params p = params(1000, 64, LBM_CIL);
    expect(lbm_workspace_bytes(&p, 1000) > 0, "workspace bytes");
    expect(lbm_workspace_bytes(&p, 999) == 0, "pitch < nx");
    lbm_ctx *c = nullptr;
    lbm_params odd = params(64, 63, LBM_CIL);
    expect(lbm_create(&odd, (void *)256, (void *)512, 64, nullptr, (void *)4096, 1 << 20, nullptr, &c) == LBM_EINVAL,
           "odd ny");
    expect(lbm_create(&p, (void *)256, (void *)256, 1000, nullptr, (void *)4096, 1 << 20, nullptr, &c) == LBM_EINVAL,
           "equal buffers");
    expect(lbm_create(&p, (void *)256, (void *)512, 1000, nullptr, (void *)4100, 1 << 20, nullptr, &c) == LBM_EINVAL,
           "misaligned workspace");
    expect(lbm_step(nullptr, 1) == LBM_ESTATE && lbm_moments(nullptr, 0, 0, 0, 0) == LBM_ESTATE, "null context");
    // batched sweeps: sizes, groups, validation (no device work happens)
    std::vector<lbm_params> ps;
    for (int l = 0; l < 40; ++l)
        ps.push_back(params(128 + 64 * (l % 7), 128 + 64 * (l % 5), LBM_CIL));
    expect(lbm_sweep_workspace_bytes(ps.data(), (int)ps.size(), 3) > 0, "sweep workspace");
    expect(lbm_sweep_groups(ps.data(), (int)ps.size()) >= 1, "groups");
    expect(lbm_sweep_tile_rows(ps.data(), (int)ps.size()) == 0, "untuned");
    std::vector<void *> bufs(2 * ps.size());
    for (size_t k = 0; k < bufs.size(); ++k)
        bufs[k] = (void *)(4096 * (k + 1));
    lbm_sweep_opts o;
    memset(&o, 0, sizeof o);
    o.n_steps = 10;
    o.sample_every = 3;  // not a divisor
    std::vector<lbm_obs> out(ps.size() * 4);
    expect(lbm_sweep_batch(ps.data(), (int)ps.size(), &o, bufs.data(), (void *)4096, 1 << 30, nullptr, out.data()) ==
               LBM_EINVAL,
           "sample_every");
    std::vector<lbm_params> mixed = {params(128, 128, LBM_CIL), params(128, 128, LBM_CIL, LBM_BF16_DEV)};
    o.sample_every = 0;
    expect(lbm_sweep_batch(mixed.data(), 2, &o, bufs.data(), (void *)4096, 1 << 30, nullptr, out.data()) ==
               LBM_EINVAL,
           "mixed storage");
    lbm_params q9 = params(64, 64, LBM_CIL, LBM_BF16_DEV, LBM_D2Q9);
    expect(lbm_sweep_batch(&q9, 1, &o, bufs.data(), (void *)4096, 1 << 30, nullptr, out.data()) ==
               LBM_EUNSUPPORTED,
           "D2Q9 16-bit batch");
    expect(lbm_sweep_batch(ps.data(), (int)ps.size(), &o, bufs.data(), (void *)4096, 16, nullptr, out.data()) ==
               LBM_EINVAL,
           "small workspace");
    // surrogate object checks
    lbm_surrogate_desc d = {4, 32, 32, 8, 50, 64};
    expect(lbm_surrogate_param_bytes(&d) > 0 && lbm_surrogate_workspace_bytes(&d) > 0, "surrogate sizes");
    lbm_surrogate *s = nullptr;
    expect(lbm_surrogate_create(&d, (void *)4100, 0, 0, (void *)8192, 1 << 30, nullptr, &s) == LBM_EINVAL,
           "misaligned params");
    expect(lbm_surrogate_predict(nullptr, nullptr, 1, nullptr) == LBM_ESTATE, "null surrogate");
    lbm_observe(&odd, (void *)4096, 64, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
    printf(bad ? "runtime sanitizer run: FAILED\n" : "runtime sanitizer run: ok\n");
    return bad;
}
