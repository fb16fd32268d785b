"""The paper's measurement protocol, host side: the CIL and MIPS regime
rules against the appendix's table (tests/golden/cil_regimes.txt) and the
density-ramp schedules of its simulation-procedure appendix."""
import os

import numpy as np

from paper_1902_00530_amd import protocol as P

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cil_regime_rules_match_the_table():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "cil_regimes.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 10
    for phi, band, zeta, rho, A, B, want in rows:
        got = P.classify_cil(float(phi), float(band), float(zeta), float(rho), float(A), float(B))
        assert got == want, (phi, band, zeta, rho, A, B, got, want)


def test_banding_thresholds_scale_with_density():
    # the banding measure is a density: at lambda = 4 the cut is 4 x 0.012
    assert P.classify_cil(0.2, 0.04, 0.0, 0.8, 0.125, 0.3, density_scale=4.0) == "HO"
    assert P.classify_cil(0.2, 0.05, 0.0, 0.8, 0.125, 0.3, density_scale=4.0) == "B"
    assert P.classify_mips(0.043) == "H" and P.classify_mips(0.0431) == "PS"
    assert P.classify_mips(0.17, density_scale=4.0) == "H" and P.classify_mips(0.18, density_scale=4.0) == "PS"


def test_hysteresis_schedule():
    """Increasing run: 0.09 .. 0.35 in steps of 0.0025, t_sample 1500 up to
    0.2 and 500 above; decreasing run the reverse."""
    t_of = lambda r: 500 if r > 0.2 + 1e-12 else 1500
    up = P.ramp_schedule(0.09, 0.35, 0.0025, t_of)
    down = P.ramp_schedule(0.35, 0.09, 0.0025, t_of)
    assert [t for t, _ in up] == [1500, 500] and [t for t, _ in down] == [500, 1500]
    assert [len(r) for _, r in up] == [45, 60] and [len(r) for _, r in down] == [60, 45]
    flat_up = np.concatenate([r for _, r in up])
    assert np.allclose(flat_up, 0.09 + 0.0025 * np.arange(105)) and abs(flat_up[-1] - 0.35) < 1e-12
    assert np.allclose(np.concatenate([r for _, r in down]), flat_up[::-1])
    # phase diagram: 0.05 .. 0.40 in steps of 0.01, one t_sample
    pd = P.ramp_schedule(0.05, 0.40, 0.01, lambda r: 10000)
    assert len(pd) == 1 and len(pd[0][1]) == 36


def test_mips_noise_schedule():
    """The MIPS ramp of the appendix "Simulation procedure for results":
    sigma from 1/70 to 3/70 in steps of 1/700 (21 noise strengths)."""
    from paper_1902_00530_amd import protocol as P
    s = P.sigma_schedule()
    assert len(s) == 21 and abs(s[0] - 1 / 70) < 1e-15 and abs(s[-1] - 3 / 70) < 1e-15
    assert np.allclose(np.diff(s), 1 / 700, rtol=0, atol=1e-15)
    assert P.classify_mips(0.0431) == "PS" and P.classify_mips(0.0430) == "H"
    assert P.classify_mips(0.1, density_scale=8.0) == "H" and P.classify_mips(0.4, density_scale=8.0) == "PS"
