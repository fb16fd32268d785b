"""The paper's measurement protocol on the GPU: the batched density ramp
(drho / 7 added to every population right after each sample, inside the
sweep's graphs) against single-lattice runs with lbm_add_density, against
the oracle, and the protocol drivers end to end at reduced size."""
import numpy as np
import pytest

import synth_inputs as SI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from test_parity_gpu import STABLE, _cfg, _gparams, _init32, _oparams, rel_err  # noqa: E402


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_00530_amd as lib
    return lib


def _paper_cfgs(n, rho_means):
    return [_cfg(SI.CIL, 180, 60, tau=1.0, sigma=1 / 70, A=2.0, B=0.3, seed=900 + l) for l in range(n)]


@pytest.mark.parametrize("tile_rows,use_graph", [(16, 1), (1, 0)])
def test_ramp_equals_single_lattice_runs(L, tile_rows, use_graph):
    """Three periods of 7 steps, each followed by a sample and a density
    change of its own size per lattice: bit for bit the single-lattice
    sequence step(7), add_density, ... and the same observables."""
    rhos = [0.09, 0.15, 0.3]
    drho = [0.0025, -0.0025, 0.01]
    cfgs = _paper_cfgs(3, rhos)
    lats = [L.Lattice(_gparams(L, c), init=L.make_init(mode=1, rho_mean=r, rho_spread=0.1)) for c, r in zip(cfgs, rhos)]
    torch.cuda.synchronize()
    b = L.Batch([lat.params for lat in lats])
    for l, lat in enumerate(lats):
        b.set_state(l, lat.state)
    out = b.run(21, sample_every=7, tile_rows=tile_rows, use_graph=use_graph, drho=drho)
    for l, lat in enumerate(lats):
        for k in range(3):
            lat.step(7)
            o = lat.observables()
            assert abs(o["phi"] - out[l][k]["phi"]) <= 1e-12 and abs(o["M"] - out[l][k]["M"]) <= 1e-9 * o["M"]
            lat.add_density(drho[l])
        torch.cuda.synchronize()
        assert torch.equal(b.state(l), lat.state), l
        lat.close()


def test_ramp_matches_oracle(L, orc):
    """A stable ordered state, three periods of 4 steps with a density
    change after each sample, against the oracle doing the same."""
    cfg, ini = STABLE["cil_aligned"]
    f0 = _init32(orc, cfg, ini)
    po = _oparams(orc, cfg)
    b = L.Batch([_gparams(L, cfg)])
    b.set_state(0, torch.from_numpy(f0.astype(np.float32)).cuda())
    out = b.run(12, sample_every=4, drho=0.02)
    f = f0.copy()
    for k in range(3):
        f = orc.run(po, f, 4, step0=4 * k)
        o = orc.observables(po, f)
        assert abs(out[0][k]["M"] - o["M"]) <= 1e-6 * o["M"]
        assert abs(out[0][k]["phi"] - o["phi"]) <= 1e-5
        f = orc.add_density(f, 0.02)
    assert rel_err(b.state(0).double().cpu().numpy(), f) < 1e-5


def test_ramp_adds_the_stated_mass(L):
    """Between consecutive samples the total mass grows by drho x sites
    (the step itself conserves mass up to float rounding)."""
    cfgs = _paper_cfgs(2, [0.2, 0.2])
    lats = [L.Lattice(_gparams(L, c), init=L.make_init(mode=1, rho_mean=0.2, rho_spread=0.1)) for c in cfgs]
    b = L.Batch([lat.params for lat in lats])
    for l, lat in enumerate(lats):
        b.set_state(l, lat.state)
        lat.close()
    out = b.run(50, sample_every=10, drho=[0.005, -0.005])
    sites = 180 * 60
    for l, d in enumerate([0.005, -0.005]):
        m = np.array([o["M"] for o in out[l]])
        assert np.allclose(np.diff(m), d * sites, rtol=1e-4, atol=1e-6 * m[0])


def test_protocol_drivers_at_reduced_size(L):
    """Hysteresis and phase-diagram drivers end to end with few runs and
    short periods: shapes, nominal densities, and regimes from the rule set."""
    from paper_1902_00530_amd import protocol as P
    h = P.hysteresis(repeats=3, rho_lo=0.09, rho_hi=0.14, step=0.01, t_low=40, t_high=20, rho_switch=0.11,
                     init_steps=100, nx=64, ny=32)
    assert np.allclose(h["up"]["rho"], [0.09, 0.10, 0.11, 0.12, 0.13, 0.14])
    assert np.allclose(h["down"]["rho"], [0.14, 0.13, 0.12, 0.11, 0.10, 0.09])
    assert h["up"]["steps"] == 100 + 3 * 40 + 3 * 20
    for d in ("up", "down"):
        assert len(h[d]["phi"]) == 6 and all(0.0 <= p <= 0.3 + 0.05 for p in h[d]["phi"])
        assert set(h[d]["regime"]) <= {"HD", "HO", "B", "RB", "none"}
    pd = P.phase_diagram([0.0, 2.0, 10.0], rho_lo=0.1, rho_hi=0.3, step=0.1, t_sample=30, repeats=2, init_steps=50,
                         nx=64, ny=32)
    assert len(pd["regime"]) == 3 and all(len(r) == 3 for r in pd["regime"])
    # B - A rho^2 <= 0 at A = 10 from rho = sqrt(0.03) ~ 0.173: the last two points have no motion
    assert pd["regime"][2][1:] == ["none", "none"]


def test_hysteresis_regimes_at_the_papers_snapshot_densities(L):
    """The paper's increasing-density protocol at A = 2 (50 runs, t_sample 1500
    up to rho = 0.2 and 500 above, 1e4 relaxation steps): the regime of the
    mean observables at the four densities of its snapshot table.  A smoke
    check of the paper's reported behaviour (stochastic runs, not a pin)."""
    import os
    from paper_1902_00530_amd import protocol as P
    here = os.path.dirname(os.path.abspath(__file__))
    want = [l.split() for l in open(os.path.join(here, "golden", "cil_snapshot_regimes.txt"))
            if l.strip() and l[0] != "#"]
    b = P.cil_batch(50, 0.09, 2.0, [50000 + r for r in range(50)])
    b.run(10000)
    phases = P.ramp_schedule(0.09, 0.35, 0.0025, lambda r: 500 if r > 0.2 + 1e-12 else 1500)
    samples = P.run_ramp(b, phases, 0.0025)
    rho = np.array([o["rho_nominal"] for o in samples[0]])
    for r, regime in want:
        k = int(np.argmin(np.abs(rho - float(r))))
        phi = np.mean([s[k]["phi"] for s in samples])
        band = np.mean([s[k]["drho"] for s in samples])
        zeta = np.mean([s[k]["zeta"] for s in samples])
        assert P.classify_cil(phi, band, zeta, rho[k], 2.0, 0.3) == regime, (r, phi, band, zeta)


def test_mips_regimes_at_the_papers_snapshot_points(L):
    """MIPS at the (density, noise) pairs of the paper's snapshot table, two
    runs each on 90 x 30 sites, 10^5 steps from the random start and 20
    samples every 10^3 steps: the regime of the mean banding measure.  A smoke
    check of the paper's reported behaviour (stochastic runs, not a pin)."""
    import os
    from paper_1902_00530_amd import protocol as P
    here = os.path.dirname(os.path.abspath(__file__))
    want = [l.split() for l in open(os.path.join(here, "golden", "mips_snapshot_regimes.txt"))
            if l.strip() and l[0] != "#"]
    rhos = [float(r) for r, _, _ in want for _ in range(2)]
    b = P.mips_batch(rhos, [7000 + l for l in range(len(rhos))])
    for l, (_, s, _) in enumerate(w for w in want for _ in range(2)):
        b.params[l].sigma = float(s)
    b.run(100000)
    out = b.run(20000, sample_every=1000)
    for k, (r, s, regime) in enumerate(want):
        band = np.mean([o["drho"] for l in (2 * k, 2 * k + 1) for o in out[l]])
        assert P.classify_mips(band) == regime, (r, s, band)


def test_mips_noise_ramp_driver(L):
    """The MIPS ramp driver end to end at reduced length: phase separated at
    sigma = 1/70, homogeneous at 3/70 for a density inside the binodal."""
    from paper_1902_00530_amd import protocol as P
    res = P.mips_noise_ramp(rho_means=(0.125,), repeats=2, sigmas=[1 / 70, 3 / 70], init_steps=100000,
                            relax_steps=20000, sample_every=1000, n_samples=20)
    assert res["regime"] == [["PS", "H"]] and res["sigma_homogeneous"] == [3 / 70]
    assert res["steps"] == 100000 + 2 * (20000 + 20000) and res["lattices"] == 2


def test_phase_diagram_brackets_the_critical_point(L):
    """The (rho, A) diagram at the paper's parameters with four repeats at
    A = 2 and A = 3.5: banded regimes (B or RB) appear at A = 2 and none at
    A = 3.5, on either side of the paper's critical point (A_c ~ 2.75).  A
    smoke check of the paper's reported behaviour (stochastic runs, not a
    pin)."""
    from paper_1902_00530_amd import protocol as P
    pd = P.phase_diagram([2.0, 3.5], repeats=4)
    a2, a35 = pd["regime"]
    assert {"B", "RB"} & set(a2), a2
    assert not ({"B", "RB"} & set(a35)), a35
