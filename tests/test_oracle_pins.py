"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula: each compares it with a
closed form, an invariant, a special case, a published known-answer value, or
the linear dispersion of the paper's Chapman-Enskog hydrodynamic equations.
"""
import math
import os

import numpy as np
import pytest

import synth_inputs as SI

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
S3 = math.sqrt(3.0)


# ---------------------------------------------------------------- helpers

def phys_coords(nx, ny):
    """Physical positions of the offset-row triangular lattice sites."""
    y, x = np.mgrid[0:ny, 0:nx]
    return x + 0.5 * (y % 2), y * S3 / 2.0


def mode_amplitude(field, k):
    """Complex Fourier amplitude sum_r field(r) exp(+i k x_phys(r)) / N."""
    ny, nx = field.shape
    xp, _ = phys_coords(nx, ny)
    return (field * np.exp(1j * k * xp)).sum() / field.size


def xi_field(orc, rho, ux, uy):
    ny, nx = rho.shape
    f = np.zeros((7, ny, nx))
    for y in range(ny):
        for x in range(nx):
            f[:, y, x] = orc.xi(rho[y, x], ux[y, x], uy[y, x])
    return f


# ---------------------------------------------------------------- Philox

def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert orc.philox4x32(v[0:4], v[4:6], rounds=10) == v[6:10]


# ---------------------------------------------------------------- lattice

def test_lattice_moments_d2q7(orc):
    """sum w = 1, sum w e = 0, sum w e e = I/4 (c_s^2 = 1/4), the fourth
    moment is isotropic, and the opposite pairs are 1-4, 2-5, 3-6."""
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    w = np.array([orc.weight(i) for i in range(7)])
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * E).sum(0)).max() < 1e-15
    second = np.einsum("i,ia,ib->ab", w, E, E)
    assert np.allclose(second, np.eye(2) / 4.0, atol=1e-15)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, E, E, E, E)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 16.0
    assert np.allclose(fourth, iso, atol=1e-15)
    for k in (1, 2, 3):
        assert np.allclose(E[k] + E[k + 3], 0.0, atol=1e-15)
    assert np.allclose(np.linalg.norm(E[1:], axis=1), 1.0)


def test_neighbour_map_is_the_geometry(orc):
    """Every site has exactly six sites at unit physical distance (minimum
    image), and they are the oracle's neighbours along e_1..e_6."""
    nx, ny = 8, 6
    xp, yp = phys_coords(nx, ny)
    Lx, Ly = nx, ny * S3 / 2
    E = [orc.lattice_vector(i) for i in range(7)]
    for y in range(ny):
        for x in range(nx):
            dx = xp - xp[y, x]
            dy = yp - yp[y, x]
            dx -= Lx * np.round(dx / Lx)
            dy -= Ly * np.round(dy / Ly)
            dist = np.hypot(dx, dy)
            close = set(zip(*np.nonzero(np.abs(dist - 1.0) < 1e-9)))
            assert len(close) == 6
            got = set()
            for i in range(1, 7):
                xn, yn = orc.neighbour(nx, ny, x, y, i)
                assert abs(dx[yn, xn] - E[i][0]) < 1e-9 and abs(dy[yn, xn] - E[i][1]) < 1e-9
                got.add((yn, xn))
            assert got == close
            assert orc.neighbour(nx, ny, x, y, 0) == (x, y)


# ---------------------------------------------------------------- steady state

def test_xi_moments(orc):
    """sum xi = rho, sum xi e = rho u*, sum xi e e = rho (I/4 + u* u*)."""
    r = np.random.default_rng(1)
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    for _ in range(200):
        rho = r.uniform(0.01, 3.0)
        u = r.uniform(-0.4, 0.4, size=2)
        f = orc.xi(rho, u[0], u[1])
        assert abs(f.sum() - rho) <= 4e-16 * rho * 8
        assert np.allclose((f[:, None] * E).sum(0), rho * u, rtol=0, atol=1e-15 * rho * 8)
        assert np.allclose(np.einsum("i,ia,ib->ab", f, E, E), rho * (np.eye(2) / 4 + np.outer(u, u)),
                           rtol=0, atol=1e-14 * rho)


def test_moments_pairwise_symmetric_zero(orc):
    r = np.random.default_rng(2)
    for _ in range(100):
        f = r.uniform(0, 1, 7)
        f[4:7] = f[1:4]
        rho, jx, jy = orc.moments(f)
        assert jx == 0.0 and jy == 0.0
        assert abs(rho - f.sum()) < 1e-15


# ---------------------------------------------------------------- target velocities

def test_ustar_cil(orc):
    p = orc.make_params(8, 8, orc.CIL, A=2.0, B=0.3)
    for rho, j in [(0.2, (0.03, -0.01)), (0.1, (-0.2, 0.5)), (0.38, (1e-3, 2e-3))]:
        ux, uy = orc.ustar_local(p, rho, *j)
        u0 = 0.3 - 2.0 * rho * rho
        assert abs(math.hypot(ux, uy) - u0) < 1e-15
        assert abs(ux * j[1] - uy * j[0]) < 1e-15 and ux * j[0] + uy * j[1] > 0
    assert orc.ustar_local(p, 0.5, 0.1, 0.1) == (0.0, 0.0)      # B < A rho^2: no motion
    assert orc.ustar_local(p, 0.2, 0.0, 0.0) == (0.0, 0.0)      # |u| = 0
    assert orc.ustar_local(p, math.sqrt(0.15), 0.3, 0.0)[0] < 1e-15


def test_ustar_passive(orc):
    p = orc.make_params(8, 8, orc.PASSIVE)
    assert orc.ustar_local(p, 2.0, 0.3, -0.5) == (0.15, -0.25)
    assert orc.ustar_local(p, 0.0, 0.0, 0.0) == (0.0, 0.0)


def test_ustar_mips_and_clamp(orc):
    p = orc.make_params(8, 8, orc.MIPS, C=50.0, rho_star=0.2, u_max=0.3)
    ux, uy = orc.ustar_mips(p, 0.1, 1e-3, -2e-3)
    assert abs(ux - 50 * 0.5 * 1e-3) < 1e-15 and abs(uy + 50 * 0.5 * 2e-3) < 1e-15
    assert orc.ustar_mips(p, 0.2, 1.0, 1.0) == (0.0, 0.0)
    assert orc.ustar_mips(p, 0.3, 1.0, 1.0) == (0.0, 0.0)
    ux, uy = orc.ustar_mips(p, 0.05, 0.3, 0.4)      # |u*| = 18.75 > U_max
    assert abs(math.hypot(ux, uy) - 0.3) < 1e-15 and abs(ux / uy - 0.75) < 1e-14


def test_gradient_plane_wave(orc):
    """On a plane wave exp(i q.r) the stencil (1/3) sum (rho_k - rho_{k+3}) e_k
    gives (2i/3) sum_k sin(q.e_k) e_k exp(i q.r); with real fields, the sine
    wave's gradient is (2/3) sum_k sin(q.e_k) e_k cos(q.r)."""
    nx, ny = 24, 12
    xp, yp = phys_coords(nx, ny)
    E = [np.array(orc.lattice_vector(i)) for i in range(7)]
    for mx, my in [(1, 0), (2, 0), (0, 1), (3, 2)]:
        # wave vector compatible with the periodic box (rows shift with parity)
        qx = 2 * math.pi * mx / nx
        qy = 2 * math.pi * my / (ny * S3 / 2)
        q = np.array([qx, qy])
        rho = np.sin(qx * xp + qy * yp)
        coef = (2.0 / 3.0) * sum(math.sin(q @ E[k]) * E[k] for k in (1, 2, 3))
        for (y, x) in [(0, 0), (3, 5), (7, 11), (11, 23)]:
            nb = np.zeros(7)
            nb[0] = rho[y, x]
            for k in range(1, 7):
                xn, yn = orc.neighbour(nx, ny, x, y, k)
                nb[k] = rho[yn, xn]
            gx, gy = orc.gradient(nb)
            phase = math.cos(qx * xp[y, x] + qy * yp[y, x])
            assert abs(gx - coef[0] * phase) < 1e-13 and abs(gy - coef[1] * phase) < 1e-13


# ---------------------------------------------------------------- noise

def test_noise_zero_sum_and_covariance(orc):
    """sum_i eta_i = 0; h = sum eta_i e_i has <h> = 0, var h_x = var h_y =
    sigma^2 and <h_x h_y> = 0 (section on the fluctuation-induced
    renormalisation); each eta~ is uniform on [-sigma, sigma]."""
    sigma = 0.25
    p = orc.make_params(8, 8, orc.CIL, sigma=sigma, seed=12345)
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    n = 40000
    eta = np.array([orc.noise(p, s, t) for s in range(200) for t in range(n // 200)])
    assert np.abs(eta.sum(1)).max() < 1e-15
    h = eta @ E
    se = sigma ** 2 / math.sqrt(n)
    assert abs(h[:, 0].mean()) < 5 * sigma / math.sqrt(n)
    assert abs(h[:, 1].mean()) < 5 * sigma / math.sqrt(n)
    assert abs(h[:, 0].var() - sigma ** 2) < 6 * se
    assert abs(h[:, 1].var() - sigma ** 2) < 6 * se
    assert abs((h[:, 0] * h[:, 1]).mean()) < 6 * se
    # eta_i = eta~_i - mean: variance sigma^2/3 * 6/7, and never beyond 12/7 sigma
    assert abs(eta.var(0).mean() - sigma ** 2 * 2 / 7) < 6 * se
    assert np.abs(eta).max() <= sigma * 12 / 7 + 1e-15
    # different steps and sites are uncorrelated
    a = np.array([orc.noise(p, 5, t)[1] for t in range(5000)])
    b = np.array([orc.noise(p, 6, t)[1] for t in range(5000)])
    c = np.array([orc.noise(p, 5, t + 1)[1] for t in range(5000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.06 and abs(np.corrcoef(a, c)[0, 1]) < 0.06
    # sigma = 0 gives exactly zero noise
    p0 = orc.make_params(8, 8, orc.CIL, sigma=0.0, seed=12345)
    assert not orc.noise(p0, 3, 4).any()


# ---------------------------------------------------------------- negative correction

def _pair_form(f, rho):
    """Closed form of rules (i)-(iii): rest population clipped at 0; each
    opposite pair (a, b) becomes (max(a - b, 0), max(b - a, 0)) when either
    is negative; then the site is rescaled to rho."""
    g = np.array(f, dtype=float)
    fired = g[0] < 0
    g[0] = max(g[0], 0.0)
    for k in (1, 2, 3):
        if g[k] < 0 or g[k + 3] < 0:
            fired = True
            d = g[k] - g[k + 3]
            g[k], g[k + 3] = max(d, 0.0), max(-d, 0.0)
    if fired:
        s = g.sum()
        g = g * (rho / s) if s > 0 else np.zeros(7)
    return g, fired


def test_correction_cases(orc):
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    r = np.random.default_rng(3)
    for _ in range(20000):
        f = r.uniform(-0.05, 0.2, 7)
        if f.sum() <= 0:
            continue
        rho = f.sum() + r.uniform(0, 0.01)
        out, fired = orc.correct(f, rho)
        ref, rfired = _pair_form(f, rho)
        assert fired == rfired
        assert (out >= 0).all()
        assert np.allclose(out, ref, rtol=1e-14, atol=1e-16)
        if not fired:
            assert (out == f).all()
        else:
            assert abs(out.sum() - rho) < 1e-14
            # rule (ii) keeps the momentum of every pair; (iii) scales it
            g = np.array(f)
            g[0] = max(g[0], 0)
            mom_before = sum((g[k] - g[k + 3]) * E[k] for k in (1, 2, 3))
            s = sum(abs(g[k] - g[k + 3]) if (g[k] < 0 or g[k + 3] < 0) else g[k] + g[k + 3]
                    for k in (1, 2, 3)) + g[0]
            if s > 0:
                assert np.allclose((out[:, None] * E).sum(0), mom_before * rho / s, atol=1e-14)
    # all-zero after clipping: every population becomes 0
    out, fired = orc.correct([-0.1, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0], 0.0)
    assert fired and not out.any()
    # a pair with both negative
    out, _ = orc.correct([0.5, -0.1, 0.1, 0.1, -0.3, 0.1, 0.1], 1.0)
    assert out[1] > 0 and out[4] == 0.0


# ---------------------------------------------------------------- whole step

def test_stream_only_is_the_lattice_translation(orc):
    """tau = +inf and sigma = 0 make a step a pure streaming: after T steps
    f_i(r) equals the initial f_i at the site whose physical position is
    r - T e_i (found from the geometry, not from the neighbour table)."""
    nx, ny, T = 10, 8, 7
    p = orc.make_params(nx, ny, orc.CIL, tau=math.inf, sigma=0.0, A=2.0, B=0.3, seed=9)
    f0 = SI.random_populations(nx, ny, seed=4)
    f = orc.run(p, f0.copy(), T)
    xp, yp = phys_coords(nx, ny)
    Lx, Ly = nx, ny * S3 / 2
    for i in range(7):
        ex, ey = orc.lattice_vector(i)
        ys = np.round(((yp - T * ey) % Ly) / (S3 / 2)).astype(int) % ny
        xs = np.round((xp - T * ex - 0.5 * (ys % 2)) % Lx).astype(int) % nx
        assert (f[i] == f0[i][ys, xs]).all()


def test_mass_conservation(orc):
    """Collision, zero-sum noise and the rescale all conserve mass: relative
    drift of the total over 300 noisy steps stays at rounding level."""
    for cfg in (SI.mips_small(), SI.cil_1024(1.0, n=32)):
        cfg = dict(cfg)
        cfg["nx"] = cfg["ny"] = 32
        p = orc.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"],
                            cfg["C"], cfg["rho_star"], cfg["u_max"], cfg["seed"])
        f = orc.initialise(p, **cfg["init"])
        m0 = f.sum()
        orc.run(p, f, 300)
        assert abs(f.sum() - m0) / m0 < 1e-13
        assert (f >= 0).all()


def test_negative_correction_in_a_step(orc):
    """Strong noise on small populations: corrections fire, populations stay
    non-negative and mass is conserved."""
    nx = ny = 16
    p = orc.make_params(nx, ny, orc.CIL, tau=1.0, sigma=0.05, A=2.0, B=0.3, seed=77)
    f = SI.near_negative_populations(nx, ny, seed=5)
    m0 = f.sum()
    orc.run(p, f, 20)
    assert (f >= 0).all() and abs(f.sum() - m0) / m0 < 1e-13


def test_fixed_points(orc):
    nx, ny = 16, 8
    one = np.ones((ny, nx))
    # passive: uniform equilibrium with a flow
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=1.3)
    f0 = xi_field(orc, 0.7 * one, 0.05 * one, -0.03 * one)
    f = orc.run(p, f0.copy(), 50)
    assert np.abs(f - f0).max() < 1e-14
    # CIL homogeneous ordered state
    A, B, r0 = 2.0, 0.3, 0.2
    u0 = B - A * r0 * r0
    p = orc.make_params(nx, ny, orc.CIL, tau=1.0, A=A, B=B)
    th = 0.4
    f0 = xi_field(orc, r0 * one, u0 * math.cos(th) * one, u0 * math.sin(th) * one)
    f = orc.run(p, f0.copy(), 50)
    assert np.abs(f - f0).max() < 1e-14
    # MIPS: uniform density at rest (zero gradient)
    p = orc.make_params(nx, ny, orc.MIPS, tau=2.0, C=50.0, rho_star=0.2, u_max=0.3)
    f0 = xi_field(orc, 0.1 * one, 0 * one, 0 * one)
    f = orc.run(p, f0.copy(), 50)
    assert np.abs(f - f0).max() < 1e-15


def test_no_motion_relaxation_rate(orc):
    """CIL with U0 = 0 (A rho^2 > B): u* = 0, so a uniform momentum decays by
    exactly (1 - 1/tau) per step (BGK relaxation, eq. fevolution2)."""
    nx, ny = 8, 4
    one = np.ones((ny, nx))
    for tau in (1.0, 2.0, 4.0):
        p = orc.make_params(nx, ny, orc.CIL, tau=tau, A=2.0, B=0.3)
        f = xi_field(orc, 0.5 * one, 0.1 * one, 0.05 * one)
        j0 = orc.observables(p, f)["Jx"]
        orc.run(p, f, 6)
        assert abs(orc.observables(p, f)["Jx"] - j0 * (1 - 1 / tau) ** 6) < 1e-14 * abs(j0) + 1e-300


def test_resume_is_bitwise(orc):
    cfg = SI.mips_small()
    p = orc.make_params(16, 16, cfg["model"], cfg["tau"], cfg["sigma"], 0, 0, cfg["C"], cfg["rho_star"],
                        cfg["u_max"], cfg["seed"])
    f = orc.initialise(p, **cfg["init"])
    a = orc.run(p, f.copy(), 40)
    b = orc.run(p, f.copy(), 17)
    b = orc.run(p, b, 23, step0=17)
    assert (a == b).all()


@pytest.mark.parametrize("model", ["cil", "mips"])
def test_scale_covariance_bitwise(orc, model):
    """(f, rho, sigma, rho*, C, A) -> (4f, 4 rho, 4 sigma, 4 rho*, C/4, A/16):
    every step is covariant and with a power-of-two factor the oracle's result
    scales exactly."""
    nx = ny = 16
    lam = 4.0
    if model == "cil":
        kw = dict(model=orc.CIL, tau=1.0, sigma=1 / 70, A=2.0, B=0.3, C=0, rho_star=1, u_max=1)
        ini = dict(mode=1, rho_mean=0.2, rho_spread=0.1, angle_std=0, u_mag=-1, pop_noise=0)
    else:
        kw = dict(model=orc.MIPS, tau=2.0, sigma=1 / 70, A=0, B=0, C=50.0, rho_star=0.2, u_max=0.3)
        ini = dict(mode=1, rho_mean=0.12, rho_spread=0.1, angle_std=0, u_mag=0.01, pop_noise=0)
    p1 = orc.make_params(nx, ny, seed=31, **kw)
    kw2 = dict(kw)
    kw2.update(sigma=kw["sigma"] * lam, A=kw["A"] / lam ** 2, C=kw["C"] / lam, rho_star=kw["rho_star"] * lam)
    p2 = orc.make_params(nx, ny, seed=31, **kw2)
    f1 = orc.initialise(p1, **ini)
    f2 = f1 * lam
    orc.run(p1, f1, 60)
    orc.run(p2, f2, 60)
    assert (f2 == lam * f1).all()


# ---------------------------------------------------------------- hydrodynamics

def _run_mode(orc, p, f, steps, k, every=1):
    amps = []
    for t in range(0, steps, every):
        rho, ux, uy = orc.fields(p, f)
        amps.append((t, rho, ux, uy))
        orc.run(p, f, every, step0=t)
    return amps


@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_shear_wave_viscosity(orc, tau):
    """Passive limit: a transverse wave u_y ~ sin(k x) decays as exp(-nu k^2 t)
    with nu = (2 tau - 1)/8 = (2 tau - 1) c_s^2 / 2, c_s = 1/2 (viscosity and
    sound speed of the Chapman-Enskog appendix)."""
    nx, ny = 64, 4
    k = 2 * math.pi / nx
    xp, _ = phys_coords(nx, ny)
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=tau)
    f = xi_field(orc, np.ones((ny, nx)), np.zeros((ny, nx)), 1e-4 * np.sin(k * xp))
    nu = (2 * tau - 1) / 8
    T = 400
    orc.run(p, f, 20)
    a0 = abs(mode_amplitude(orc.fields(p, f)[2], k))
    orc.run(p, f, T, step0=20)
    a1 = abs(mode_amplitude(orc.fields(p, f)[2], k))
    rate = -math.log(a1 / a0) / T
    assert abs(rate / (nu * k * k) - 1) < 0.02


def test_sound_wave(orc):
    """Passive limit, longitudinal density wave: s = -nu k^2 +- i k c_s
    sqrt(1 - nu^2 k^2 / c_s^2) with c_s = 1/2 (derived momentum equation with
    P = c_s^2 rho)."""
    nx, ny = 64, 4
    k = 2 * math.pi / nx
    tau = 1.0
    nu = (2 * tau - 1) / 8
    xp, _ = phys_coords(nx, ny)
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=tau)
    f = xi_field(orc, 1 + 1e-5 * np.cos(k * xp), np.zeros((ny, nx)), np.zeros((ny, nx)))
    series = []
    for t in range(400):
        series.append(mode_amplitude(orc.fields(p, f)[0], k).real)
        orc.run(p, f, 1, step0=t)
    series = np.array(series)
    ts = np.arange(len(series))
    omega = k * 0.5 * math.sqrt(1 - nu * nu * k * k / 0.25)
    # fit a e^{-g t} cos(w t + c) by least squares over (g, w)
    best = None
    for w in np.linspace(omega * 0.9, omega * 1.1, 401):
        for g in np.linspace(0, 3 * nu * k * k, 61):
            basis = np.stack([np.exp(-g * ts) * np.cos(w * ts), np.exp(-g * ts) * np.sin(w * ts)], 1)
            coef, res, *_ = np.linalg.lstsq(basis, series, rcond=None)
            r = ((basis @ coef - series) ** 2).sum()
            if best is None or r < best[0]:
                best = (r, w, g)
    _, w, g = best
    assert abs(w / omega - 1) < 0.01
    assert abs(g / (nu * k * k) - 1) < 0.05


def _growth(orc, p, rho0, u0, k, t0, t1, eps=1e-6, every=5):
    """Growth rate and phase rate of the density mode exp(-i k x) started as a
    small sine on a uniform state (rho0, u0 along x).  The phase is unwrapped
    from samples every `every` steps."""
    nx, ny = p.nx, p.ny
    xp, _ = phys_coords(nx, ny)
    rho = rho0 * (1 + eps * np.sin(k * xp))
    f = xi_field(orc, rho, u0 * np.ones((ny, nx)), np.zeros((ny, nx)))
    orc.run(p, f, t0)
    a0 = mode_amplitude(orc.fields(p, f)[0] - rho0, k)
    phase, prev, t = 0.0, a0, t0
    while t < t1:
        n = min(every, t1 - t)
        orc.run(p, f, n, step0=t)
        t += n
        a = mode_amplitude(orc.fields(p, f)[0] - rho0, k)
        phase += np.angle(a / prev)
        prev = a
    dt = t1 - t0
    return math.log(abs(prev) / abs(a0)) / dt, phase / dt


def _von_neumann_mips(orc, rho0, C, rho_star, tau, k):
    """Largest growth rate ln|lambda| of the MIPS step linearised about a
    uniform state at rest, for a plane wave exp(i k x): the perturbation of
    xi is w_i [d rho + 4 rho0 e_i . d u*], d u* = C (1 - rho0/rho*) times the
    stencil's plane-wave gradient, then BGK relaxation and streaming."""
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    w = np.array([orc.weight(i) for i in range(7)])
    q = np.array([k, 0.0])
    G = (2j / 3) * sum(math.sin(q @ E[m]) * E[m] for m in (1, 2, 3))
    W = np.array([[w[i] * (1 + 4 * rho0 * C * (1 - rho0 / rho_star) * (E[i] @ G))] * 7 for i in range(7)])
    M = np.diag(np.exp(-1j * (E @ q))) @ ((1 - 1 / tau) * np.eye(7) + W / tau)
    return np.log(np.abs(np.linalg.eigvals(M))).max()


def test_mips_spinodal_growth_rate(orc):
    """MIPS about a uniform state rho0 < rho*: linearising the derived momentum
    equation with F_MIPS, using the lattice gradient g(k) = (2/3)(sin k +
    sin k/2) along x, gives s^2 + (gamma + 2 nu k^2) s + k^2 c_s^2 - k g(k)
    gamma rho0 C (1 - rho0/rho*) = 0, gamma = 2/(2 tau - 1).  C is chosen so
    that short waves (which grow fastest for the paper's C = 50) stay far
    below the measured mode over the run."""
    tau, C, rs = 2.0, 12.0, 0.2
    nx, ny = 64, 2
    k = 2 * math.pi / nx
    p = orc.make_params(nx, ny, orc.MIPS, tau=tau, C=C, rho_star=rs, u_max=0.3)
    nu, gam, cs2 = (2 * tau - 1) / 8, 2 / (2 * tau - 1), 0.25
    g = (2 / 3) * (math.sin(k) + math.sin(k / 2))
    for rho0, t1 in ((0.05, 1100), (0.195, 400)):
        roots = np.roots([1, gam + 2 * nu * k * k, k * k * cs2 - k * g * gam * rho0 * C * (1 - rho0 / rs)])
        s_th = roots.real.max()
        s, _ = _growth(orc, p, rho0, 0.0, k, 100, t1)
        assert abs(s / s_th - 1) < 0.02, (rho0, s, s_th)
        s_vn = _von_neumann_mips(orc, rho0, C, rs, tau, k)
        assert abs(s / s_vn - 1) < 1e-6, (rho0, s, s_vn)
    assert _growth(orc, p, 0.05, 0.0, k, 100, 1100)[0] > 0 > _growth(orc, p, 0.195, 0.0, k, 100, 400)[0]


def _von_neumann_cil(orc, rho0, A, B, tau, k):
    """Dominant eigenvalue (growth rate, phase rate) of the CIL step
    linearised about the homogeneous ordered state xi(rho0, v0 x^),
    v0 = U0(rho0), for the plane wave exp(-i k x).  d u*_x = U0' d rho and
    d u*_y = d j_y / rho0 (rotation of j^), then BGK relaxation and
    streaming."""
    E = np.array([orc.lattice_vector(i) for i in range(7)])
    w = np.array([orc.weight(i) for i in range(7)])
    v0, du = B - A * rho0 ** 2, -2 * A * rho0
    J = np.zeros((7, 7))
    for i in range(7):
        ex, ey = E[i]
        d_rho = w[i] * (1 + 4 * ex * v0 + 8 * ex * ex * v0 * v0 - 2 * v0 * v0)
        d_ux = w[i] * rho0 * (4 * ex + 16 * ex * ex * v0 - 4 * v0)
        d_uy = w[i] * rho0 * (4 * ey + 16 * ey * ex * v0)
        for j in range(7):
            J[i, j] = d_rho + d_ux * du + d_uy * E[j][1] / rho0
    q = np.array([-k, 0.0])
    M = np.diag(np.exp(-1j * (E @ q))) @ ((1 - 1 / tau) * np.eye(7) + J / tau)
    lam = np.linalg.eigvals(M)
    top = lam[np.argmax(np.abs(lam))]
    return math.log(abs(top)), np.angle(top)


@pytest.mark.parametrize("rho0,k_div,steps", [(0.37, 32, 1000), (0.30, 32, 1000), (0.36, 64, 3000)])
def test_cil_homogeneous_ordered_dispersion(orc, rho0, k_div, steps):
    """CIL about the homogeneous ordered state (v0 = U0(rho0) along x):
    sigma'^2 + (gamma + 2 nu k^2) sigma' + k^2 c_s^2 - i k gamma rho0 U0' = 0,
    s = sigma' + i k v0 for modes exp(s t - i k x) (derived Toner-Tu equations,
    section "Hydrodynamic description of the transitions").  Growth is
    unstable iff 4 A^2 rho0^4 > c_s^2 at small k, with phase speed
    B - 3 A rho0^2 (backward: reverse banding).  The oracle must match the
    exact rate of the linearised discrete scheme tightly, and the paper's
    small-k dispersion relation to its O(k^2) truncation."""
    tau, A, B = 1.0, 2.0, 0.3
    nx, ny = k_div, 2
    k = 2 * math.pi / nx
    p = orc.make_params(nx, ny, orc.CIL, tau=tau, A=A, B=B)
    nu, gam, cs2 = (2 * tau - 1) / 8, 2 / (2 * tau - 1), 0.25
    v0 = B - A * rho0 ** 2
    du = -2 * A * rho0
    roots = np.roots([1, gam + 2 * nu * k * k, k * k * cs2 - 1j * k * gam * rho0 * du])
    sp = roots[np.argmax(roots.real)]
    s_th = sp + 1j * k * v0
    s, w = _growth(orc, p, rho0, v0, k, 40, 40 + steps)
    assert (s > 0) == (4 * A * A * rho0 ** 4 > cs2)
    assert abs(s - s_th.real) < 0.06 * abs(s_th.real), (s, s_th)
    assert abs(w - s_th.imag) < 0.02 * abs(s_th.imag), (w, s_th)
    s_vn, w_vn = _von_neumann_cil(orc, rho0, A, B, tau, k)
    assert abs(s - s_vn) < 1e-6 * abs(s_vn), (s, s_vn)
    assert abs(w - w_vn) < 1e-3 * abs(w_vn), (w, w_vn)
    assert abs(w / k - (B - 3 * A * rho0 ** 2)) < 0.05 * abs(B - 3 * A * rho0 ** 2)


# ---------------------------------------------------------------- observables

def test_observables_closed_forms(orc):
    nx, ny = 32, 8
    A, B, r0 = 2.0, 0.3, 0.2
    u0 = B - A * r0 * r0
    p = orc.make_params(nx, ny, orc.CIL, A=A, B=B)
    one = np.ones((ny, nx))
    f = xi_field(orc, r0 * one, u0 * 0.6 * one, u0 * 0.8 * one)
    o = orc.observables(p, f, streamed=False)
    assert abs(o["phi"] - u0) < 1e-13 and abs(o["zeta"] - A * r0 * r0) < 1e-13 and o["drho"] < 1e-14
    assert abs(o["M"] - r0 * nx * ny) < 1e-12
    # sinusoidal density on offset rows: std of rho_y(x) = eps cos(k/4)/sqrt 2
    eps, k = 0.01, 2 * math.pi * 3 / nx
    xp, _ = phys_coords(nx, ny)
    f = xi_field(orc, r0 + eps * np.sin(k * xp), 0 * one, 0 * one)
    assert abs(orc.observables(p, f, streamed=False)["drho"] - eps * math.cos(k / 4) / math.sqrt(2)) < 1e-14
    # a stored state's observables are those of its streamed populations:
    # streaming xi(rho(x), 0) averages rho over the stencil, which multiplies
    # a density wave along x by sum_i w_i cos(k e_ix) = 1/2 + (cos k + 2 cos(k/2))/6
    damp = 0.5 + (math.cos(k) + 2 * math.cos(k / 2)) / 6
    assert abs(orc.observables(p, f)["drho"] - damp * eps * math.cos(k / 4) / math.sqrt(2)) < 1e-14
    assert abs(orc.observables(p, f)["M"] - orc.observables(p, f, streamed=False)["M"]) < 1e-12


def test_phi_bounded_by_B(orc):
    """With sigma = 0 and tau = 1 the post-collision populations are
    xi(rho, u*) with |u*| <= U0 <= B, so 0 <= phi <= B."""
    nx = ny = 16
    p = orc.make_params(nx, ny, orc.CIL, tau=1.0, sigma=0.0, A=2.0, B=0.3, seed=5)
    f = orc.initialise(p, mode=1, rho_mean=0.2, rho_spread=0.1)
    for _ in range(5):
        orc.run(p, f, 10)
        o = orc.observables(p, f)
        assert 0 <= o["phi"] <= 0.3 + 1e-15 and o["mean_speed"] <= 0.3 + 1e-15


def test_initialisation_statistics(orc):
    nx, ny = 64, 64
    A, B = 2.0, 0.3
    p = orc.make_params(nx, ny, orc.CIL, A=A, B=B, seed=11)
    f = orc.initialise(p, mode=1, rho_mean=0.2, rho_spread=0.1)
    rho, ux, uy = orc.fields(p, f, streamed=False)
    assert rho.min() >= 0.18 and rho.max() <= 0.22
    assert abs(rho.mean() - 0.2) < 3 * 0.2 * 0.1 / math.sqrt(3 * rho.size)
    assert np.allclose(np.hypot(ux, uy), B - A * rho ** 2, atol=1e-15)
    ang = np.arctan2(uy, ux)
    assert abs(np.cos(ang).mean()) < 0.05 and abs(np.sin(ang).mean()) < 0.05
    f2 = orc.initialise(p, mode=2, rho_mean=0.2, rho_spread=0.1, angle_std=0.05)
    _, ux, uy = orc.fields(p, f2, streamed=False)
    ang = np.arctan2(uy, ux)
    assert abs(ang.std() - 0.05) < 0.005 and abs(ang.mean()) < 0.005


# ---------------------------------------------------------------- coarse fields (surrogate's maps)

def _neighbour(x, y, i, nx, ny):
    """Site r + e_i of (x, y) on the offset-row lattice (the table of the
    conventions: odd rows sit half a site to the right)."""
    p = y % 2
    dx, dy = [(0, 0), (1, 0), (p, 1), (p - 1, 1), (-1, 0), (p - 1, -1), (p, -1)][i]
    return (x + dx) % nx, (y + dy) % ny


def test_coarsen_is_the_block_mean_of_the_streamed_moments(orc):
    """A stored state built so that its streamed populations are a planted
    random pattern g (f_i(s) = g_i(s + e_i), by the geometric neighbour table,
    not the oracle's streaming): coarsen must return, block by block, the means
    of rho = sum_i g_i and j = sum_i g_i e_i over the c x c sites of that block
    (row-major blocks [3][ny/c][nx/c], nx != ny so a transposed layout fails)."""
    nx, ny, c = 24, 12, 4
    p = orc.make_params(nx, ny, orc.CIL, A=0.1, B=0.3)
    rng = np.random.default_rng(11)
    g = rng.uniform(0.0, 1.0, size=(7, ny, nx))
    # plant distinct block levels so a misplaced block cannot match by chance
    for by in range(ny // c):
        for bx in range(nx // c):
            g[:, by * c:(by + 1) * c, bx * c:(bx + 1) * c] += 3.0 * by + 0.5 * bx
    f = np.zeros_like(g)
    for y in range(ny):
        for x in range(nx):
            for i in range(7):
                sx, sy = _neighbour(x, y, i, nx, ny)
                f[i, y, x] = g[i, sy, sx]
    E = np.array([[0.0, 0.0]] + [[math.cos(k * math.pi / 3), math.sin(k * math.pi / 3)] for k in range(6)])
    got = orc.coarsen(p, f, c)
    assert got.shape == (3, ny // c, nx // c)
    for by in range(ny // c):
        for bx in range(nx // c):
            blk = g[:, by * c:(by + 1) * c, bx * c:(bx + 1) * c]
            rho = blk.sum(axis=0).mean()
            jx = np.einsum("i,iyx->yx", E[:, 0], blk).mean()
            jy = np.einsum("i,iyx->yx", E[:, 1], blk).mean()
            assert abs(got[0, by, bx] - rho) < 1e-13 * rho
            assert abs(got[1, by, bx] - jx) < 1e-13 * rho
            assert abs(got[2, by, bx] - jy) < 1e-13 * rho


def test_lift_gives_each_block_its_own_fields(orc):
    """lift puts the steady state xi of block (by, bx) on exactly the c x c
    sites of that block: the unstreamed fields of the lifted state return each
    block's rho and u = j / rho (Sigma xi = rho, Sigma xi e = rho u), and a
    block with rho <= 0 lifts to empty sites."""
    nx, ny, c = 20, 8, 4
    p = orc.make_params(nx, ny, orc.CIL, A=0.1, B=0.3)
    rng = np.random.default_rng(12)
    hb, wb = ny // c, nx // c
    coarse = np.zeros((3, hb, wb))
    coarse[0] = rng.uniform(0.5, 2.0, size=(hb, wb))
    u = rng.uniform(-0.2, 0.2, size=(2, hb, wb))
    coarse[1] = coarse[0] * u[0]
    coarse[2] = coarse[0] * u[1]
    coarse[0, 1, 3] = 0.0
    coarse[:, 0, 2] = (-0.4, 0.1, -0.2)  # negative density: treated as 0
    f = orc.lift(p, coarse, c)
    rho, ux, uy = orc.fields(p, f, streamed=False)
    for y in range(ny):
        for x in range(nx):
            by, bx = y // c, x // c
            r = coarse[0, by, bx]
            if r <= 0.0:
                assert np.all(f[:, y, x] == 0.0) and rho[y, x] == 0.0
                assert ux[y, x] == 0.0 and uy[y, x] == 0.0
                continue
            assert abs(rho[y, x] - r) < 1e-14 * r
            assert abs(ux[y, x] - coarse[1, by, bx] / r) < 1e-14
            assert abs(uy[y, x] - coarse[2, by, bx] / r) < 1e-14


def test_parallel_build_equals_the_plain_build(orc):
    """The OpenMP build (the CPU baseline's host-core timing) runs the rows of
    a step on several threads; every row writes only its own sites, so the
    state after a run equals the plain build's bit for bit (CIL and MIPS)."""
    for model, kw, ini in ((orc.CIL, dict(tau=1.0, sigma=4 / 70, A=0.125, B=0.3), dict(rho_mean=0.74)),
                           (orc.MIPS, dict(tau=2.0, sigma=8 / 70, C=6.25, rho_star=1.6, u_max=0.3),
                            dict(rho_mean=1.0, u_mag=0.1, pop_noise=1e-3))):
        p = orc.make_params(96, 34, model, seed=9, **kw)
        f = orc.initialise(p, mode=1, **ini)
        a = orc.run(p, f.copy(), 7)
        b = f.copy()
        assert orc.run_parallel(p, b, 7, 4) >= 1
        assert np.array_equal(a, b)
