"""The paper's measurement protocol on batched ensembles (arXiv:1902.00530,
appendix "Simulation procedure for results" and appendix "Regime
Categorisation in the phase diagram").

Every run of the protocol is an independent lattice; all runs of an
experiment advance together in one batch (lbm_sweep_batch), with the
observables sampled every t_sample steps and, right after each sample, the
mean density changed by adding drho / 7 to every population (the paper's
adiabatic density ramp), all inside the captured graphs.

Regimes of the CIL model (the categorisation appendix): HD (homogeneous,
disordered) where the order parameter phi is below 0.024; otherwise HO
(homogeneous, ordered) where the banding measure (standard deviation over x
of the column-mean density) is at most 0.012, and among banded states RB
(reverse banding) where zeta exceeds 0.1, else B (banding).  Points with
B - A rho^2 <= 0 have no motion (the region above the red line of the phase
diagram).  The MIPS model counts as phase separated where the banding
measure exceeds 0.0430 (section "Simulation procedure for results", MIPS
model).  The banding thresholds are densities: a lattice run at densities
scaled by lambda (see synth_inputs) compares against lambda times them.
"""
import math

import numpy as np

from . import Batch, LBM_CIL, LBM_MIPS, Lattice, make_init, make_params

CIL_PHI_THRESHOLD = 0.024
CIL_BANDING_THRESHOLD = 0.012
CIL_ZETA_THRESHOLD = 0.1
MIPS_BANDING_THRESHOLD = 0.0430

# The paper's CIL runs: 180 x 60 sites, B = 0.3, tau = 1, sigma = 1/70.
PAPER_CIL = dict(nx=180, ny=60, B=0.3, tau=1.0, sigma=1.0 / 70.0)
# The paper's MIPS parameter table (tau, C, rho*, U_max); its phase-diagram
# runs use 90 x 30 sites and raise sigma from 1/70 to 3/70 by 1/700.
PAPER_MIPS = dict(tau=2.0, C=50.0, rho_star=0.2, u_max=0.3)


def classify_cil(phi, banding, zeta, rho_mean, A, B, density_scale=1.0):
    """Regime of a CIL sample (or of averaged samples): 'none' (no motion),
    'HD', 'HO', 'B' or 'RB'."""
    if B - A * rho_mean * rho_mean <= 0.0:
        return "none"
    if phi < CIL_PHI_THRESHOLD:
        return "HD"
    if banding <= CIL_BANDING_THRESHOLD * density_scale:
        return "HO"
    return "RB" if zeta > CIL_ZETA_THRESHOLD else "B"


def classify_mips(banding, density_scale=1.0):
    """'PS' (phase separated) or 'H' (homogeneous) for a MIPS sample."""
    return "PS" if banding > MIPS_BANDING_THRESHOLD * density_scale else "H"


def ramp_schedule(rho_start, rho_end, step, t_of_rho):
    """Sample densities from rho_start to rho_end (inclusive, |step| apart)
    grouped into phases of equal t_sample: a list of (t_sample, [densities])."""
    n = int(round(abs(rho_end - rho_start) / abs(step))) + 1
    sgn = 1.0 if rho_end >= rho_start else -1.0
    phases = []
    for k in range(n):
        rho = rho_start + sgn * k * abs(step)
        t = t_of_rho(rho)
        if phases and phases[-1][0] == t:
            phases[-1][1].append(rho)
        else:
            phases.append((t, [rho]))
    return phases


def cil_batch(n, rho_mean, A, seeds, nx=180, ny=60, B=0.3, tau=1.0, sigma=1.0 / 70.0):
    """n CIL lattices in the paper's initial state (directions uniform, density
    within +-10% of the mean, |u| = U0(rho), f = f^SS), one seed each; A and
    rho_mean may be per-lattice sequences."""
    A = [A] * n if np.isscalar(A) else list(A)
    rho_mean = [rho_mean] * n if np.isscalar(rho_mean) else list(rho_mean)
    params = [make_params(nx, ny, LBM_CIL, tau=tau, sigma=sigma, A=A[l], B=B, seed=int(seeds[l])) for l in range(n)]
    b = Batch(params)
    for l in range(n):
        lat = Lattice(params[l], init=make_init(mode=1, rho_mean=rho_mean[l], rho_spread=0.1))
        b.set_state(l, lat.state)
        lat.close()
    return b


def run_ramp(batch, phases, step, tile_rows=0):
    """Advance a batch through a density ramp: for every phase (t_sample,
    densities), len(densities) periods of t_sample steps, each ending with a
    sample and then the density change `step`.  Returns per lattice the list
    of sample dicts with the nominal density added as 'rho_nominal'."""
    out = [[] for _ in range(batch.n)]
    for t, rhos in phases:
        res = batch.run(t * len(rhos), sample_every=t, tile_rows=tile_rows, drho=step)
        for l in range(batch.n):
            for k, o in enumerate(res[l]):
                o["rho_nominal"] = rhos[k]
                out[l].append(o)
    return out


def _mean_over_runs(samples, key):
    v = np.array([[o[key] for o in run] for run in samples])
    return v.mean(axis=0), v.std(axis=0, ddof=1) / math.sqrt(v.shape[0]) if v.shape[0] > 1 else np.zeros(v.shape[1])


def hysteresis(repeats=50, A=2.0, rho_lo=0.09, rho_hi=0.35, step=0.0025, t_low=1500, t_high=500, rho_switch=0.2,
               init_steps=10000, seed_base=50000, nx=180, ny=60, B=0.3, tau=1.0, sigma=1.0 / 70.0):
    """The hysteresis experiment of the paper's order-parameter figure:
    `repeats` independent increasing runs from rho_lo and as many decreasing
    runs from rho_hi, |drho| = step every t_sample steps (t_high above
    rho_switch, t_low otherwise), each run first relaxed for init_steps.
    Returns, per direction, the nominal densities, the mean and standard error
    of phi over the runs, the mean banding measure and zeta, and the regime of
    the mean observables."""
    def t_of(r):
        return t_high if r > rho_switch + 1e-12 else t_low
    res = {}
    for name, start, end, sgn, base in (("up", rho_lo, rho_hi, 1.0, seed_base),
                                        ("down", rho_hi, rho_lo, -1.0, seed_base + 100000)):
        b = cil_batch(repeats, start, A, [base + r for r in range(repeats)], nx, ny, B, tau, sigma)
        b.run(init_steps)
        phases = ramp_schedule(start, end, step, t_of)
        samples = run_ramp(b, phases, sgn * step)
        rho = [o["rho_nominal"] for o in samples[0]]
        phi, phi_se = _mean_over_runs(samples, "phi")
        band, _ = _mean_over_runs(samples, "drho")
        zeta, _ = _mean_over_runs(samples, "zeta")
        res[name] = {"rho": rho, "phi": phi.tolist(), "phi_stderr": phi_se.tolist(), "banding": band.tolist(),
                     "zeta": zeta.tolist(),
                     "regime": [classify_cil(phi[k], band[k], zeta[k], rho[k], A, B) for k in range(len(rho))],
                     "steps": int(init_steps + sum(t * len(r) for t, r in phases))}
    return res


def phase_diagram(A_values, rho_lo=0.05, rho_hi=0.40, step=0.01, t_sample=10000, repeats=10, init_steps=10000,
                  seed_base=70000, nx=180, ny=60, B=0.3, tau=1.0, sigma=1.0 / 70.0):
    """The (rho, A) phase diagram of the paper: for every A, `repeats`
    increasing runs from rho_lo in steps of `step` every t_sample steps, all
    A values and repeats in one batch; phi, the banding measure and zeta are
    averaged over the repeats at each (rho, A) and classified.  Returns the
    densities, A values and per-(A, rho) means and regimes."""
    nA = len(A_values)
    n = nA * repeats
    A_of = [A_values[l // repeats] for l in range(n)]
    b = cil_batch(n, rho_lo, A_of, [seed_base + l for l in range(n)], nx, ny, B, tau, sigma)
    b.run(init_steps)
    phases = ramp_schedule(rho_lo, rho_hi, step, lambda r: t_sample)
    samples = run_ramp(b, phases, step)
    rho = [o["rho_nominal"] for o in samples[0]]
    out = {"rho": rho, "A": list(A_values), "phi": [], "banding": [], "zeta": [], "regime": [],
           "steps": int(init_steps + sum(t * len(r) for t, r in phases)), "lattices": n}
    for a in range(nA):
        grp = samples[a * repeats:(a + 1) * repeats]
        phi, _ = _mean_over_runs(grp, "phi")
        band, _ = _mean_over_runs(grp, "drho")
        zeta, _ = _mean_over_runs(grp, "zeta")
        out["phi"].append(phi.tolist())
        out["banding"].append(band.tolist())
        out["zeta"].append(zeta.tolist())
        out["regime"].append([classify_cil(phi[k], band[k], zeta[k], rho[k], A_values[a], B) for k in range(len(rho))])
    return out


def mips_batch(rho_means, seeds, sigma=1.0 / 70.0, nx=90, ny=30):
    """MIPS lattices with the paper's parameter table, one per (mean density,
    seed): density uniform within +-10% of the mean, a random direction of
    small speed (0.01), f = f^SS."""
    params = [make_params(nx, ny, LBM_MIPS, sigma=sigma, seed=int(seeds[l]), **PAPER_MIPS)
              for l in range(len(rho_means))]
    b = Batch(params)
    for l, p in enumerate(params):
        lat = Lattice(p, init=make_init(mode=1, rho_mean=rho_means[l], rho_spread=0.1, u_mag=0.01))
        b.set_state(l, lat.state)
        lat.close()
    return b


def sigma_schedule(sigma_lo=1.0 / 70.0, sigma_hi=3.0 / 70.0, step=1.0 / 700.0):
    """Noise strengths of the MIPS ramp, sigma_lo to sigma_hi inclusive."""
    n = int(round((sigma_hi - sigma_lo) / step)) + 1
    return [sigma_lo + k * step for k in range(n)]


def mips_noise_ramp(rho_means=(0.06, 0.08, 0.10, 0.125, 0.15, 0.18), repeats=2, sigmas=None, init_steps=200000,
                    relax_steps=50000, sample_every=1000, n_samples=50, seed_base=90000, nx=90, ny=30,
                    progress=None):
    """The MIPS experiment of the paper (section "Simulation procedure for
    results"): each run starts at sigma = sigma_0, relaxes, then for every
    noise strength of the schedule relaxes relax_steps and takes n_samples
    samples every sample_every steps before the noise rises.  All densities
    and repeats run as one batch.  The paper relaxes 10^6 steps after each
    rise and samples 100 times every 10^4 steps; the defaults here are
    shorter.  progress, if given, is called with (sigma, banding per density)
    after each noise strength.  Returns the noise strengths, the densities,
    the banding measure per (density, sigma) averaged over samples and
    repeats, the regime ('PS' / 'H') and, per density, the first sigma of the
    schedule at which it is homogeneous."""
    sigmas = sigma_schedule() if sigmas is None else list(sigmas)
    rhos = [float(r) for r in rho_means for _ in range(repeats)]
    b = mips_batch(rhos, [seed_base + l for l in range(len(rhos))], sigma=sigmas[0], nx=nx, ny=ny)
    b.run(init_steps)
    band = np.zeros((len(rho_means), len(sigmas)))
    for k, sg in enumerate(sigmas):
        for l in range(b.n):
            b.params[l].sigma = sg
        b.run(relax_steps)
        out = b.run(sample_every * n_samples, sample_every=sample_every)
        per_run = np.array([np.mean([o["drho"] for o in out[l]]) for l in range(b.n)])
        band[:, k] = per_run.reshape(len(rho_means), repeats).mean(axis=1)
        if progress is not None:
            progress(sg, band[:, k].tolist())
    regime = [[classify_mips(v) for v in row] for row in band]
    sigma_c = []
    for row in regime:
        hom = [sigmas[k] for k, r in enumerate(row) if r == "H"]
        sigma_c.append(hom[0] if hom else None)
    return {"sigma": sigmas, "rho": list(rho_means), "banding": band.tolist(), "regime": regime,
            "sigma_homogeneous": sigma_c,
            "steps": int(init_steps + len(sigmas) * (relax_steps + sample_every * n_samples)),
            "lattices": b.n}
