"""Pins of the square-lattice (D2Q9) oracle against what the mathematics fixes.

The paper works on the triangular D2Q7 lattice and notes that the sound speed
depends on the lattice (appendix "Chapman-Enskog Expansion").  The D2Q9
variant carries the same algorithm over to the standard square velocity set
(c_s^2 = 1/3).  None of these tests re-types the oracle: they check lattice
isotropy, the moments of the steady state, closed forms of the gradient
stencil, symmetries of the square lattice (quarter turns and mirrors), exact
translations, conservation laws, fixed points, and the linear dispersion of
the derived hydrodynamic equations with this lattice's c_s^2 and viscosity.
"""
import math

import numpy as np
import pytest

import synth_inputs as SI

Q = 9
# quarter turn (x, y) -> (-y, x) and mirror x -> -x as direction maps,
# found from the vectors in the tests below
ROT_EXPECT = [0, 2, 3, 4, 1, 6, 7, 8, 5]


@pytest.fixture(scope="module")
def q9(orc):
    from oracle import q9
    q9.lib()
    return q9


def vecs(q9):
    return np.array([q9.lattice_vector(i) for i in range(Q)])


def xi_field(q9, rho, ux, uy):
    ny, nx = rho.shape
    f = np.zeros((Q, ny, nx))
    for y in range(ny):
        for x in range(nx):
            f[:, y, x] = q9.xi(rho[y, x], ux[y, x], uy[y, x])
    return f


def mode_amplitude(field, k):
    ny, nx = field.shape
    x = np.arange(nx)[None, :]
    return (field * np.exp(1j * k * x)).sum() / field.size


def direction_map(E, M):
    """Index map i -> j with M e_i = e_j."""
    out = []
    for i in range(Q):
        t = M @ E[i]
        out.append(int(np.argmin(np.abs(E - t).sum(1))))
        assert np.allclose(E[out[-1]], t)
    return out


def transform_state(f, site_map, dir_map):
    """g[dir_map[i]][site_map(y, x)] = f[i][y, x]."""
    q, ny, nx = f.shape
    g = np.empty_like(f)
    for y in range(ny):
        for x in range(nx):
            y2, x2 = site_map(y, x)
            for i in range(q):
                g[dir_map[i], y2, x2] = f[i, y, x]
    return g


# ---------------------------------------------------------------- lattice

def test_lattice_isotropy(q9):
    """sum w = 1, sum w e = 0, sum w e e = I/3, sum w e e e = 0, the fourth
    moment is isotropic (I I + perms)/9, opposite vectors pair up and the
    speeds are 0, 1 and sqrt 2."""
    E = vecs(q9)
    w = np.array([q9.weight(i) for i in range(Q)])
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * E).sum(0)).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, E, E), np.eye(2) / 3.0, atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, E, E, E)).max() < 1e-16
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, E, E, E, E), iso, atol=1e-16)
    for i in range(Q):
        assert np.allclose(E[q9.opposite(i)], -E[i])
    assert sorted(np.round(np.linalg.norm(E, axis=1) ** 2).astype(int)) == [0, 1, 1, 1, 1, 2, 2, 2, 2]


def test_neighbour_map_is_the_geometry(q9):
    """The eight neighbours of a site are the sites at distance 1 and sqrt 2
    (minimum image), each at its lattice vector."""
    nx, ny = 7, 5
    E = vecs(q9)
    for y in range(ny):
        for x in range(nx):
            got = set()
            for i in range(Q):
                xn, yn = q9.neighbour(nx, ny, x, y, i)
                dx = (xn - x + nx // 2) % nx - nx // 2
                dy = (yn - y + ny // 2) % ny - ny // 2
                assert (dx, dy) == tuple(E[i].astype(int))
                got.add((xn, yn))
            assert len(got) == 9


# ---------------------------------------------------------------- steady state

def test_xi_moments(q9):
    """sum xi = rho, sum xi e = rho u, sum xi e e = rho (I/3 + u u): the
    discretised Maxwellian of this lattice reproduces the first three moments
    exactly."""
    r = np.random.default_rng(1)
    E = vecs(q9)
    for _ in range(200):
        rho = r.uniform(0.01, 3.0)
        u = r.uniform(-0.4, 0.4, size=2)
        f = q9.xi(rho, u[0], u[1])
        assert abs(f.sum() - rho) <= 1e-15 * rho * 8
        assert np.allclose((f[:, None] * E).sum(0), rho * u, rtol=0, atol=1e-15 * rho * 8)
        assert np.allclose(np.einsum("i,ia,ib->ab", f, E, E), rho * (np.eye(2) / 3 + np.outer(u, u)),
                           rtol=0, atol=1e-14 * rho)
    # at rest xi is the weights times rho
    assert np.allclose(q9.xi(2.0, 0.0, 0.0), 2.0 * np.array([q9.weight(i) for i in range(Q)]), atol=1e-16)


def test_moments_pairwise_symmetric_zero(q9):
    r = np.random.default_rng(2)
    for _ in range(100):
        f = r.uniform(0, 1, Q)
        for i in (1, 2, 5, 6):
            f[q9.opposite(i)] = f[i]
        rho, jx, jy = q9.moments(f)
        assert jx == 0.0 and jy == 0.0 and abs(rho - f.sum()) < 1e-15


# ---------------------------------------------------------------- gradient

def test_gradient_closed_forms(q9):
    """The stencil is exact on polynomials up to degree two, and on a plane
    wave exp(i k.r) it gives i [(2/3) sin kx + (1/3) sin kx cos ky,
    (2/3) sin ky + (1/3) sin ky cos kx]."""
    E = vecs(q9)
    r = np.random.default_rng(3)
    for _ in range(50):
        c = r.normal(size=6)
        fn = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
        x0, y0 = r.normal(size=2)
        nb = [fn(x0 + E[i][0], y0 + E[i][1]) for i in range(Q)]
        gx, gy = q9.gradient(nb)
        assert abs(gx - (c[1] + 2 * c[3] * x0 + c[4] * y0)) < 1e-12
        assert abs(gy - (c[2] + c[4] * x0 + 2 * c[5] * y0)) < 1e-12
    for kx, ky in ((0.3, 0.0), (0.7, -1.1), (math.pi, 0.5)):
        re = [math.cos(kx * E[i][0] + ky * E[i][1]) for i in range(Q)]
        im = [math.sin(kx * E[i][0] + ky * E[i][1]) for i in range(Q)]
        gxr, gyr = q9.gradient(re)
        gxi, gyi = q9.gradient(im)
        assert abs(gxr) < 1e-15 and abs(gyr) < 1e-15
        assert abs(gxi - (2 / 3 * math.sin(kx) + 1 / 3 * math.sin(kx) * math.cos(ky))) < 1e-15
        assert abs(gyi - (2 / 3 * math.sin(ky) + 1 / 3 * math.sin(ky) * math.cos(kx))) < 1e-15


# ---------------------------------------------------------------- noise

def test_draws_use_each_bit_once(q9):
    """The nine 14-bit draws are a bijection of bits 0..125 of the generator
    output: flipping one input bit flips exactly one bit of one draw, each
    draw bit comes from exactly one input bit, and bits 126-127 are unused."""
    r = np.random.default_rng(4)
    for _ in range(5):
        w = [int(v) for v in r.integers(0, 2 ** 32, size=4)]
        h0 = q9.draws(w)
        assert all(0 <= v < 2 ** 14 for v in h0)
        seen = set()
        for bit in range(128):
            w2 = list(w)
            w2[bit // 32] ^= 1 << (bit % 32)
            h = q9.draws(w2)
            diff = [(i, h[i] ^ h0[i]) for i in range(9) if h[i] != h0[i]]
            if bit >= 126:
                assert diff == []
                continue
            assert len(diff) == 1 and bin(diff[0][1]).count("1") == 1
            seen.add((diff[0][0], diff[0][1].bit_length() - 1))
        assert len(seen) == 126
    # the lowest bits land in the first draw, in order
    assert q9.draws([1, 0, 0, 0])[0] == 1 and q9.draws([1 << 14, 0, 0, 0])[1] == 1


def test_noise_zero_sum_and_covariance(q9, orc):
    """sum_i eta_i = 0 (eq. noiseDensityConservation); 9 * 8192 eta_i / sigma
    is the integer 9 h_i - sum h of the draws of counter (site, step, 0);
    h = sum eta_i e_i has zero mean and variance sigma^2/3 * sum_i e_ix^2 =
    2 sigma^2 per component; var eta_i = (8/9) sigma^2 / 3."""
    sigma = 0.25
    p = orc.make_params(8, 8, orc.CIL, sigma=sigma, seed=12345)
    E = vecs(q9)
    n = 40000
    eta = np.array([q9.noise(p, s, t) for s in range(200) for t in range(n // 200)])
    assert np.abs(eta.sum(1)).max() < 1e-15
    hvec = eta @ E
    se = sigma ** 2 / math.sqrt(n)
    assert abs(hvec[:, 0].mean()) < 5 * math.sqrt(2) * sigma / math.sqrt(n)
    assert abs(hvec[:, 0].var() - 2 * sigma ** 2) < 12 * se
    assert abs(hvec[:, 1].var() - 2 * sigma ** 2) < 12 * se
    assert abs((hvec[:, 0] * hvec[:, 1]).mean()) < 12 * se
    assert abs(eta.var(0).mean() - sigma ** 2 * 8 / 27) < 6 * se
    assert np.abs(eta).max() <= sigma * 16 / 9 + 1e-15
    for site, step in ((0, 0), (17, 5), (3, 2 ** 33 + 7)):
        h = q9.draws(orc.philox4x32([site, step & 0xFFFFFFFF, step >> 32, 0], [12345, 0]))
        e = q9.noise(p, site, step)
        ints = [9 * v - sum(h) for v in h]
        assert np.allclose(e * 9 * 8192 / sigma, ints, rtol=0, atol=1e-9)


# ---------------------------------------------------------------- correction

def _pair_form(q9, f, rho):
    g = np.array(f, dtype=float)
    fired = g[0] < 0
    g[0] = max(g[0], 0.0)
    for k in (1, 2, 5, 6):
        o = q9.opposite(k)
        if g[k] < 0 or g[o] < 0:
            fired = True
            d = g[k] - g[o]
            g[k], g[o] = max(d, 0.0), max(-d, 0.0)
    if fired:
        s = g.sum()
        g = g * (rho / s) if s > 0 else np.zeros(Q)
    return g, fired


def test_correction_cases(q9):
    """The paper's sequential rule equals the closed pair form
    (max(d, 0), max(-d, 0)) and the rescale to rho."""
    r = np.random.default_rng(5)
    for _ in range(20000):
        f = r.uniform(-0.05, 0.2, Q)
        if f.sum() <= 0:
            continue
        rho = f.sum() + r.uniform(0, 0.01)
        out, fired = q9.correct(f, rho)
        ref, rfired = _pair_form(q9, f, rho)
        assert fired == rfired and (out >= 0).all()
        assert np.allclose(out, ref, rtol=1e-14, atol=1e-16)
        if not fired:
            assert (out == f).all()
        else:
            assert abs(out.sum() - rho) < 1e-14
    out, fired = q9.correct([-0.1] + [0.0] * 8, 0.0)
    assert fired and not out.any()


# ---------------------------------------------------------------- symmetries

def _cases(orc):
    return [
        ("passive", orc.make_params(8, 8, orc.PASSIVE, tau=1.3)),
        ("cil", orc.make_params(8, 8, orc.CIL, tau=1.0, A=0.125, B=0.3)),
        ("mips", orc.make_params(8, 8, orc.MIPS, tau=2.0, C=6.25, rho_star=1.6, u_max=0.3)),
    ]


@pytest.mark.parametrize("which", ["passive", "cil", "mips"])
def test_quarter_turn_and_mirror_covariance(q9, orc, which):
    """Without noise the step commutes with the square lattice's quarter turn
    (x, y) -> (-y, x) and the mirror x -> -x (directions permuted as their
    vectors): a wrong neighbour, weight, sign or index in any stage breaks
    this."""
    p = dict(_cases(orc))[which]
    n = p.nx
    E = vecs(q9)
    R = direction_map(E, np.array([[0, -1], [1, 0]]))
    assert R == ROT_EXPECT
    Mx = direction_map(E, np.array([[-1, 0], [0, 1]]))
    f0 = SI.random_populations(n, n, seed=6, q=Q)
    # a large-amplitude state: the CIL and MIPS rules and the correction fire
    f0 = f0 * 1.0
    for dmap, smap in ((R, lambda y, x: (x, (-y) % n)), (Mx, lambda y, x: (y, (-x) % n))):
        a = q9.run(p, f0.copy(), 6)
        b = q9.run(p, transform_state(f0, smap, dmap), 6)
        assert np.abs(transform_state(a, smap, dmap) - b).max() < 1e-13


def test_stream_only_is_the_translation(q9, orc):
    """tau = +inf, sigma = 0: after T steps f_i(r) = f_i(r - T e_i) of the
    initial state (a periodic roll)."""
    nx, ny, T = 10, 7, 5
    p = orc.make_params(nx, ny, orc.CIL, tau=math.inf, sigma=0.0, A=2.0, B=0.3, seed=9)
    f0 = SI.random_populations(nx, ny, seed=4, q=Q)
    f = q9.run(p, f0.copy(), T)
    E = vecs(q9).astype(int)
    for i in range(Q):
        assert (f[i] == np.roll(f0[i], (T * E[i][1], T * E[i][0]), axis=(0, 1))).all()


# ---------------------------------------------------------------- conservation, fixed points

def test_mass_conservation_with_noise_and_corrections(q9, orc):
    for p in (orc.make_params(16, 12, orc.CIL, tau=1.0, sigma=0.05, A=2.0, B=0.3, seed=77),
              orc.make_params(16, 12, orc.MIPS, tau=2.0, sigma=0.05, C=6.25, rho_star=1.6, u_max=0.3, seed=78)):
        f = SI.near_negative_populations(p.nx, p.ny, seed=5, q=Q)
        m0 = f.sum()
        q9.run(p, f, 30)
        assert (f >= 0).all() and abs(f.sum() - m0) / m0 < 1e-13


def test_fixed_points(q9, orc):
    nx, ny = 12, 6
    one = np.ones((ny, nx))
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=1.3)
    f0 = xi_field(q9, 0.7 * one, 0.05 * one, -0.03 * one)
    assert np.abs(q9.run(p, f0.copy(), 50) - f0).max() < 1e-14
    A, B, r0 = 2.0, 0.3, 0.2
    u0 = B - A * r0 * r0
    p = orc.make_params(nx, ny, orc.CIL, tau=1.0, A=A, B=B)
    f0 = xi_field(q9, r0 * one, u0 * math.cos(0.4) * one, u0 * math.sin(0.4) * one)
    assert np.abs(q9.run(p, f0.copy(), 50) - f0).max() < 1e-14
    p = orc.make_params(nx, ny, orc.MIPS, tau=2.0, C=50.0, rho_star=0.2, u_max=0.3)
    f0 = xi_field(q9, 0.1 * one, 0 * one, 0 * one)
    assert np.abs(q9.run(p, f0.copy(), 50) - f0).max() < 1e-15


def test_no_motion_relaxation_rate(q9, orc):
    """U0 = 0 (A rho^2 > B): u* = 0 and a uniform momentum decays by exactly
    (1 - 1/tau) per step."""
    one = np.ones((4, 8))
    for tau in (1.0, 2.0, 4.0):
        p = orc.make_params(8, 4, orc.CIL, tau=tau, A=2.0, B=0.3)
        f = xi_field(q9, 0.5 * one, 0.1 * one, 0.05 * one)
        j0 = q9.observables(p, f)["Jx"]
        q9.run(p, f, 6)
        assert abs(q9.observables(p, f)["Jx"] - j0 * (1 - 1 / tau) ** 6) < 1e-14 * abs(j0) + 1e-300


@pytest.mark.parametrize("model", ["cil", "mips"])
def test_scale_covariance_bitwise(q9, orc, model):
    """(f, rho, sigma, rho*, C, A) -> (4f, 4 rho, 4 sigma, 4 rho*, C/4, A/16)
    scales the result exactly (no absolute constants in the method)."""
    lam = 4.0
    if model == "cil":
        kw = dict(model=orc.CIL, tau=1.0, sigma=1 / 70, A=2.0, B=0.3, C=0, rho_star=1, u_max=1)
        ini = dict(mode=1, rho_mean=0.2, rho_spread=0.1, angle_std=0, u_mag=-1, pop_noise=0)
    else:
        kw = dict(model=orc.MIPS, tau=2.0, sigma=1 / 70, A=0, B=0, C=50.0, rho_star=0.2, u_max=0.3)
        ini = dict(mode=1, rho_mean=0.12, rho_spread=0.1, angle_std=0, u_mag=0.01, pop_noise=0)
    p1 = orc.make_params(16, 16, seed=31, **kw)
    kw2 = dict(kw)
    kw2.update(sigma=kw["sigma"] * lam, A=kw["A"] / lam ** 2, C=kw["C"] / lam, rho_star=kw["rho_star"] * lam)
    p2 = orc.make_params(16, 16, seed=31, **kw2)
    f1 = q9.initialise(p1, **ini)
    f2 = f1 * lam
    q9.run(p1, f1, 60)
    q9.run(p2, f2, 60)
    assert (f2 == lam * f1).all()


# ---------------------------------------------------------------- hydrodynamics (c_s^2 = 1/3)

@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_shear_wave_viscosity(q9, orc, tau):
    """Passive: u_y ~ sin(k x) decays as exp(-nu k^2 t), nu = c_s^2 (tau - 1/2)
    = (2 tau - 1)/6 on this lattice."""
    nx, ny = 64, 2
    k = 2 * math.pi / nx
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=tau)
    f = xi_field(q9, np.ones((ny, nx)), np.zeros((ny, nx)), 1e-4 * np.sin(k * x))
    nu = (2 * tau - 1) / 6
    T = 400
    q9.run(p, f, 20)
    a0 = abs(mode_amplitude(q9.fields(p, f)[2], k))
    q9.run(p, f, T, step0=20)
    a1 = abs(mode_amplitude(q9.fields(p, f)[2], k))
    assert abs(-math.log(a1 / a0) / T / (nu * k * k) - 1) < 0.02


def test_sound_wave(q9, orc):
    """Passive, longitudinal density wave: s = -nu k^2 +- i k c_s sqrt(1 -
    nu^2 k^2 / c_s^2) with c_s = 1/sqrt 3."""
    nx, ny = 64, 2
    k = 2 * math.pi / nx
    tau = 1.0
    nu, cs2 = (2 * tau - 1) / 6, 1 / 3
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    p = orc.make_params(nx, ny, orc.PASSIVE, tau=tau)
    f = xi_field(q9, 1 + 1e-5 * np.cos(k * x), np.zeros((ny, nx)), np.zeros((ny, nx)))
    series = []
    for t in range(300):
        series.append(mode_amplitude(q9.fields(p, f)[0], k).real)
        q9.run(p, f, 1, step0=t)
    series = np.array(series)
    ts = np.arange(len(series))
    omega = k * math.sqrt(cs2) * math.sqrt(1 - nu * nu * k * k / cs2)
    best = None
    for w in np.linspace(omega * 0.9, omega * 1.1, 401):
        for g in np.linspace(0, 3 * nu * k * k, 61):
            basis = np.stack([np.exp(-g * ts) * np.cos(w * ts), np.exp(-g * ts) * np.sin(w * ts)], 1)
            coef, *_ = np.linalg.lstsq(basis, series, rcond=None)
            res = ((basis @ coef - series) ** 2).sum()
            if best is None or res < best[0]:
                best = (res, w, g)
    _, w, g = best
    assert abs(w / omega - 1) < 0.01
    assert abs(g / (nu * k * k) - 1) < 0.05


def _growth(q9, p, rho0, u0, k, t0, t1, eps=1e-6, every=5):
    nx, ny = p.nx, p.ny
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    f = xi_field(q9, rho0 * (1 + eps * np.sin(k * x)), u0 * np.ones((ny, nx)), np.zeros((ny, nx)))
    q9.run(p, f, t0)
    a0 = mode_amplitude(q9.fields(p, f)[0] - rho0, k)
    phase, prev, t = 0.0, a0, t0
    while t < t1:
        n = min(every, t1 - t)
        q9.run(p, f, n, step0=t)
        t += n
        a = mode_amplitude(q9.fields(p, f)[0] - rho0, k)
        phase += np.angle(a / prev)
        prev = a
    return math.log(abs(prev) / abs(a0)) / (t1 - t0), phase / (t1 - t0)


def _von_neumann(M_coll, E, q, tau):
    M = np.diag(np.exp(-1j * (E @ q))) @ ((1 - 1 / tau) * np.eye(Q) + M_coll / tau)
    lam = np.linalg.eigvals(M)
    top = lam[np.argmax(np.abs(lam))]
    return math.log(abs(top)), np.angle(top)


def test_mips_spinodal_growth_rate(q9, orc):
    """MIPS about rho0 < rho* at rest: s^2 + (gamma + 2 nu k^2) s + k^2 c_s^2
    - k g(k) gamma rho0 C (1 - rho0/rho*) = 0 with c_s^2 = 1/3, nu = (2 tau -
    1)/6, gamma = 2/(2 tau - 1) and this stencil's g(k) = sin k along x; the
    oracle also matches the exact rate of the linearised discrete scheme."""
    tau, C, rs = 2.0, 16.0, 0.2
    nx, ny = 64, 2
    k = 2 * math.pi / nx
    p = orc.make_params(nx, ny, orc.MIPS, tau=tau, C=C, rho_star=rs, u_max=0.3)
    nu, gam, cs2 = (2 * tau - 1) / 6, 2 / (2 * tau - 1), 1 / 3
    E = vecs(q9)
    w = np.array([q9.weight(i) for i in range(Q)])
    G = np.array([1j * math.sin(k), 0.0])
    signs = []
    for rho0, t1 in ((0.05, 1100), (0.195, 400)):
        roots = np.roots([1, gam + 2 * nu * k * k, k * k * cs2 - k * math.sin(k) * gam * rho0 * C * (1 - rho0 / rs)])
        s_th = roots.real.max()
        s, _ = _growth(q9, p, rho0, 0.0, k, 100, t1)
        assert abs(s / s_th - 1) < 0.02, (rho0, s, s_th)
        kk = 3 * rho0 * C * (1 - rho0 / rs)
        W = np.array([[w[i] * (1 + kk * (E[i] @ G))] * Q for i in range(Q)])
        s_vn, _ = _von_neumann(W, E, np.array([k, 0.0]), tau)
        assert abs(s / s_vn - 1) < 1e-6, (rho0, s, s_vn)
        signs.append(s > 0)
    assert signs == [True, False]


@pytest.mark.parametrize("rho0,B,k_div,steps", [(0.40, 0.34, 32, 1000), (0.35, 0.27, 32, 1000)])
def test_cil_homogeneous_ordered_dispersion(q9, orc, rho0, B, k_div, steps):
    """CIL about the homogeneous ordered state: sigma'^2 + (gamma + 2 nu k^2)
    sigma' + k^2 c_s^2 - i k gamma rho0 U0' = 0, s = sigma' + i k v0, with
    c_s^2 = 1/3: unstable iff 4 A^2 rho0^4 > 1/3 at small k; the oracle
    matches the linearised discrete scheme tightly."""
    tau, A = 1.0, 2.0
    nx, ny = k_div, 2
    k = 2 * math.pi / nx
    p = orc.make_params(nx, ny, orc.CIL, tau=tau, A=A, B=B)
    nu, gam, cs2 = (2 * tau - 1) / 6, 2 / (2 * tau - 1), 1 / 3
    v0, du = B - A * rho0 ** 2, -2 * A * rho0
    roots = np.roots([1, gam + 2 * nu * k * k, k * k * cs2 - 1j * k * gam * rho0 * du])
    s_th = roots[np.argmax(roots.real)] + 1j * k * v0
    s, wr = _growth(q9, p, rho0, v0, k, 40, 40 + steps)
    assert (s > 0) == (4 * A * A * rho0 ** 4 > cs2)
    assert abs(s - s_th.real) < 0.06 * abs(s_th.real), (s, s_th)
    assert abs(wr - s_th.imag) < 0.02 * abs(s_th.imag), (wr, s_th)
    E = vecs(q9)
    w = np.array([q9.weight(i) for i in range(Q)])
    J = np.zeros((Q, Q))
    for i in range(Q):
        ex, ey = E[i]
        d_rho = w[i] * (1 + 3 * ex * v0 + 4.5 * ex * ex * v0 * v0 - 1.5 * v0 * v0)
        d_ux = w[i] * rho0 * (3 * ex + 9 * ex * ex * v0 - 3 * v0)
        d_uy = w[i] * rho0 * (3 * ey + 9 * ey * ex * v0)
        for j in range(Q):
            J[i, j] = d_rho + d_ux * du + d_uy * E[j][1] / rho0
    s_vn, w_vn = _von_neumann(J, E, np.array([-k, 0.0]), tau)
    assert abs(s - s_vn) < 1e-6 * abs(s_vn), (s, s_vn)
    assert abs(wr - w_vn) < 1e-3 * abs(w_vn), (wr, w_vn)


# ---------------------------------------------------------------- observables, init

def test_observables_closed_forms(q9, orc):
    nx, ny = 32, 8
    A, B, r0 = 2.0, 0.3, 0.2
    u0 = B - A * r0 * r0
    p = orc.make_params(nx, ny, orc.CIL, A=A, B=B)
    one = np.ones((ny, nx))
    f = xi_field(q9, r0 * one, u0 * 0.6 * one, u0 * 0.8 * one)
    o = q9.observables(p, f, streamed=False)
    assert abs(o["phi"] - u0) < 1e-13 and abs(o["zeta"] - A * r0 * r0) < 1e-13 and o["drho"] < 1e-14
    assert abs(o["M"] - r0 * nx * ny) < 1e-12
    # density wave sin(k x): std over x of the column means is eps / sqrt 2;
    # streaming xi(rho(x), 0) multiplies it by sum_i w_i cos(k e_ix) = 2/3 + cos(k)/3
    eps, k = 0.01, 2 * math.pi * 3 / nx
    x = np.arange(nx)[None, :] * one
    f = xi_field(q9, r0 + eps * np.sin(k * x), 0 * one, 0 * one)
    assert abs(q9.observables(p, f, streamed=False)["drho"] - eps / math.sqrt(2)) < 1e-14
    damp = 2 / 3 + math.cos(k) / 3
    assert abs(q9.observables(p, f)["drho"] - damp * eps / math.sqrt(2)) < 1e-14
    # the protocol's density change raises every site's density by drho
    g = q9.add_density(f, 0.09)
    assert np.allclose(q9.fields(p, g, streamed=False)[0], q9.fields(p, f, streamed=False)[0] + 0.09, atol=1e-15)


def test_initialisation_statistics(q9, orc):
    A, B = 2.0, 0.3
    p = orc.make_params(64, 64, orc.CIL, A=A, B=B, seed=11)
    f = q9.initialise(p, mode=1, rho_mean=0.2, rho_spread=0.1)
    rho, ux, uy = q9.fields(p, f, streamed=False)
    assert rho.min() >= 0.18 and rho.max() <= 0.22
    assert np.allclose(np.hypot(ux, uy), B - A * rho ** 2, atol=1e-15)
    ang = np.arctan2(uy, ux)
    assert abs(np.cos(ang).mean()) < 0.05 and abs(np.sin(ang).mean()) < 0.05
    # the same variates as the triangular lattice's initial state
    r7, ux7, uy7 = orc.fields(p, orc.initialise(p, mode=1, rho_mean=0.2, rho_spread=0.1), streamed=False)
    assert np.allclose(rho, r7, atol=1e-15) and np.allclose(ux, ux7, atol=1e-15) and np.allclose(uy, uy7, atol=1e-15)
