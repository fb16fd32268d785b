"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the lattice Boltzmann method: it only draws
seeded random arrays and states the workload recipes (lattice sizes, parameter
grids and seeds) that both the oracle side and the GPU side are fed with.

Parameter values follow the paper's runs (tables in the appendix "Simulation
procedure for results"), rescaled by an exact power-of-two density scale
lambda: (f, rho, sigma, rho*, C, A) -> (lambda f, lambda rho, lambda sigma,
lambda rho*, C / lambda, A / lambda^2) leaves u, u*, phi and zeta invariant.
"""
import numpy as np

PASSIVE, MIPS, CIL = 0, 1, 2


def rng(seed):
    return np.random.default_rng(int(seed))


def random_populations(nx, ny, seed, lo=0.01, hi=0.2, dtype=np.float64, q=7):
    """Positive populations [q, ny, nx] (q = 7 triangular, 9 square lattice),
    independent uniform in [lo, hi)."""
    return rng(seed).uniform(lo, hi, size=(q, ny, nx)).astype(dtype)


def symmetric_populations(nx, ny, seed, lo=0.01, hi=0.2):
    """Populations with f_i == f_opp(i) at every site (zero momentum)."""
    f = random_populations(nx, ny, seed, lo, hi)
    for k in (1, 2, 3):
        f[k + 3] = f[k]
    return f


def near_negative_populations(nx, ny, seed, q=7):
    """Small populations so that noise drives some of them negative."""
    return rng(seed).uniform(0.0, 0.02, size=(q, ny, nx))


def seed_for(config_index, lattice_index=0):
    """Seed of lattice l in config k: (1000 + k) xor (l << 32)."""
    return (1000 + int(config_index)) ^ (int(lattice_index) << 32)


# ---------------------------------------------------------------------------
# Workload recipes (paper parameters rescaled by lambda; paper values in the
# comments).
# ---------------------------------------------------------------------------

def mips_small():
    """64 x 64 MIPS lattice: lambda = 8 of tau = 2, C = 50, rho* = 0.2,
    U_max = 0.3, sigma = 1/70 and mean density 0.125."""
    return dict(nx=64, ny=64, model=MIPS, tau=2.0, sigma=8.0 / 70.0, A=0.0, B=0.0, C=6.25,
                rho_star=1.6, u_max=0.3, seed=seed_for(0),
                init=dict(mode=1, rho_mean=1.0, rho_spread=0.0, angle_std=0.0, u_mag=0.1, pop_noise=1e-3))


CIL_DENSITIES = (0.5, 0.75, 1.0, 1.25, 1.5)   # lambda = 4 of 0.125 ... 0.375 at A = 2


def cil_1024(rho_mean, lattice_index=0, n=1024):
    """1024 x 1024 CIL lattice: lambda = 4 of A = 2, B = 0.3, tau = 1,
    sigma = 1/70; Gaussian polarisation noise (std 0.05) about +x."""
    return dict(nx=n, ny=n, model=CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125, B=0.3, C=0.0,
                rho_star=1.0, u_max=1.0, seed=seed_for(1, lattice_index),
                init=dict(mode=2, rho_mean=float(rho_mean), rho_spread=0.1, angle_std=0.05,
                          u_mag=-1.0, pop_noise=0.0))


def cil_4096(n=4096, rho_mean=0.74):
    """Precision run: 4096 x 4096 CIL lattice in the homogeneous ordered
    regime (lambda = 4 of rho = 0.185, A = 2, B = 0.3)."""
    return dict(nx=n, ny=n, model=CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125, B=0.3, C=0.0,
                rho_star=1.0, u_max=1.0, seed=seed_for(3),
                init=dict(mode=1, rho_mean=float(rho_mean), rho_spread=0.1, angle_std=0.0,
                          u_mag=-1.0, pop_noise=0.0))


def q9_cil_4096(n=4096, rho_mean=0.74, mode=2):
    """Square-lattice (D2Q9) CIL run, 4096 x 4096: the CIL parameters and
    the start of cil_1024 (lambda = 4 of A = 2, B = 0.3, tau = 1, sigma =
    1/70; Gaussian polarisation noise, std 0.05, about +x); mode=1 gives the
    disordered start (uniform directions) instead."""
    return dict(nx=n, ny=n, model=CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125, B=0.3, C=0.0,
                rho_star=1.0, u_max=1.0, seed=seed_for(5),
                init=dict(mode=int(mode), rho_mean=float(rho_mean), rho_spread=0.1, angle_std=0.05,
                          u_mag=-1.0, pop_noise=0.0))


def q9_mips_4096(n=4096):
    """Square-lattice (D2Q9) MIPS run, 4096 x 4096: the parameters of
    mips_small (lambda = 8 of tau = 2, C = 50, rho* = 0.2, U_max = 0.3,
    sigma = 1/70, mean density 0.125)."""
    return dict(nx=n, ny=n, model=MIPS, tau=2.0, sigma=8.0 / 70.0, A=0.0, B=0.0, C=6.25,
                rho_star=1.6, u_max=0.3, seed=seed_for(6),
                init=dict(mode=1, rho_mean=1.0, rho_spread=0.0, angle_std=0.0, u_mag=0.1, pop_noise=1e-3))


BATCH_SIDES = (128, 192, 256, 384, 512)


def batch_sweep(n_lattices=256, seed=1003, sides=BATCH_SIDES, grid=16):
    """Batched phase sweep: sizes drawn independently from `sides` for nx and
    ny, a grid x grid table over mean density [0.2, 2.0] (lambda = 4 of
    0.05 ... 0.5) and activity a in [0, 1] (B = 0.3 a), CIL with A = 0.125."""
    r = rng(seed)
    out = []
    for l in range(n_lattices):
        nx = int(r.choice(sides))
        ny = int(r.choice(sides))
        m, a = divmod(l % (grid * grid), grid)
        rho_mean = 0.2 + 1.8 * m / (grid - 1)
        act = a / (grid - 1)
        out.append(dict(nx=nx, ny=ny, model=CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125, B=0.3 * act, C=0.0,
                        rho_star=1.0, u_max=1.0, seed=seed_for(2, l),
                        init=dict(mode=1, rho_mean=rho_mean, rho_spread=0.1, angle_std=0.0,
                                  u_mag=-1.0, pop_noise=0.0)))
    return out


def surrogate_grid(side=256, seed_base=11000, n_rho=8, n_act=8):
    """Lattices for the surrogate: an n_rho x n_act grid of mean density
    0.3 .. 1.8 (lambda = 4 of 0.075 .. 0.45) and activity (B = 0.3 a,
    a = 1/n_act .. 1), CIL with A = 0.125, tau = 1, sigma = 4/70, paper
    initial state; one lattice per grid point, seed seed_base + index."""
    out = []
    for l in range(n_rho * n_act):
        m, a = divmod(l, n_act)
        out.append(dict(nx=side, ny=side, model=CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125,
                        B=0.3 * (a + 1) / n_act, C=0.0, rho_star=1.0, u_max=1.0, seed=seed_base + l,
                        init=dict(mode=1, rho_mean=0.3 + 1.5 * m / max(1, n_rho - 1), rho_spread=0.1,
                                  angle_std=0.0, u_mag=-1.0, pop_noise=0.0)))
    return out
