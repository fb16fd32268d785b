"""Write precision_obs_256.txt: the FP64 oracle's observables on the matched
256 x 256 runs of the precision workload (CIL, lambda = 4 of the paper's
A = 2, B = 0.3, tau = 1, sigma = 1/70; mean density 0.74, the homogeneous
ordered regime; the paper's initial state: density within +-10%, uniform
random direction, |u| = U0(rho)).

For each seed: phi, zeta and the banding measure averaged over the samples
taken every 100 steps from step 10^4 to 2 x 10^4 (101 samples), and the
relative mass change between step 0 and 2 x 10^4.  Calls the oracle only
(its OpenMP build, bit-identical to the plain one); about a minute per seed
on eight host threads.

    python tests/golden/make_precision_obs.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth_inputs as SI  # noqa: E402

N = 256
SEEDS = [SI.seed_for(4, l) for l in range(8)]
T0, T1, EVERY = 10_000, 20_000, 100


def run(seed, threads):
    cfg = dict(SI.cil_4096(n=N), seed=seed)
    ini = cfg.pop("init")
    p = O.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"], cfg["C"],
                      cfg["rho_star"], cfg["u_max"], cfg["seed"])
    f = O.initialise(p, **ini)
    m0 = O.observables(p, f)["M"]
    O.run_parallel(p, f, T0, threads)
    obs = [O.observables(p, f)]
    for t in range(T0 + EVERY, T1 + 1, EVERY):
        O.run_parallel(p, f, EVERY, threads, step0=t - EVERY)
        obs.append(O.observables(p, f))
    assert len(obs) == (T1 - T0) // EVERY + 1
    phi = np.mean([o["phi"] for o in obs])
    zeta = np.mean([o["zeta"] for o in obs])
    drho = np.mean([o["drho"] for o in obs])
    return phi, zeta, drho, obs[-1]["M"] / m0 - 1.0


def main():
    threads = len(os.sched_getaffinity(0))
    out = os.path.join(HERE, "precision_obs_256.txt")
    lines = ["# FP64 oracle, CIL 256x256 (lambda = 4 of the paper's CIL parameters), mean density 0.74,",
             "# sigma 4/70, tau 1, A 0.125, B 0.3, paper initial state; written by make_precision_obs.py.",
             f"# averages over samples every {EVERY} steps from step {T0} to {T1}; mass drift over {T1} steps",
             "# seed phi zeta drho mass_drift"]
    for s in SEEDS:
        phi, zeta, drho, dm = run(s, threads)
        lines.append(f"{s} {phi:.12e} {zeta:.12e} {drho:.12e} {dm:.6e}")
        print(lines[-1], flush=True)
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
