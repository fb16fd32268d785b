"""FP64 oracle of the square-lattice (D2Q9) variant (``lbm_oracle_q9.c``).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  Same calling
conventions as the D2Q7 functions of ``oracle``: populations are float64
arrays [9, ny, nx]; parameters come from ``oracle.make_params``.
"""
import ctypes

import numpy as np

from . import Init, Obs, Params, lib as _lib0

Q = 9
_ready = False


def lib():
    global _ready
    L = _lib0()
    if not _ready:
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        pp = ctypes.POINTER(Params)
        L.orc9_lattice_vector.argtypes = [ctypes.c_int, dp, dp]
        L.orc9_weight.argtypes = [ctypes.c_int]
        L.orc9_weight.restype = ctypes.c_double
        L.orc9_opposite.argtypes = [ctypes.c_int]
        L.orc9_opposite.restype = ctypes.c_int
        L.orc9_neighbour.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_int)] * 2
        L.orc9_xi.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc9_moments.argtypes = [dp, dp, dp, dp]
        L.orc9_gradient.argtypes = [dp, dp, dp]
        L.orc9_draws.argtypes = [u32p, u32p]
        L.orc9_noise.argtypes = [pp, ctypes.c_uint32, ctypes.c_int64, dp]
        L.orc9_correct.argtypes = [dp, ctypes.c_double]
        L.orc9_correct.restype = ctypes.c_int
        L.orc9_stream.argtypes = [pp, dp, dp]
        L.orc9_step.argtypes = [pp, dp, ctypes.c_int64]
        L.orc9_step.restype = ctypes.c_int
        L.orc9_run.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_int64]
        L.orc9_run.restype = ctypes.c_int
        L.orc9_initialise.argtypes = [pp, ctypes.POINTER(Init), dp]
        L.orc9_initialise.restype = ctypes.c_int
        for name in ("orc9_fields", "orc9_fields_of"):
            getattr(L, name).argtypes = [pp, dp, dp, dp, dp]
        for name in ("orc9_observables", "orc9_observables_of"):
            getattr(L, name).argtypes = [pp, dp, ctypes.POINTER(Obs)]
        _ready = True
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice_vector(i):
    ex, ey = ctypes.c_double(), ctypes.c_double()
    lib().orc9_lattice_vector(i, ctypes.byref(ex), ctypes.byref(ey))
    return ex.value, ey.value


def weight(i):
    return lib().orc9_weight(i)


def opposite(i):
    return lib().orc9_opposite(i)


def neighbour(nx, ny, x, y, i):
    xn, yn = ctypes.c_int(), ctypes.c_int()
    lib().orc9_neighbour(nx, ny, x, y, i, ctypes.byref(xn), ctypes.byref(yn))
    return xn.value, yn.value


def xi(rho, ux, uy):
    out = np.zeros(Q)
    lib().orc9_xi(rho, ux, uy, _dp(out))
    return out


def moments(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    r, jx, jy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc9_moments(_dp(f), ctypes.byref(r), ctypes.byref(jx), ctypes.byref(jy))
    return r.value, jx.value, jy.value


def gradient(rho_nb):
    a = np.ascontiguousarray(rho_nb, dtype=np.float64)
    gx, gy = ctypes.c_double(), ctypes.c_double()
    lib().orc9_gradient(_dp(a), ctypes.byref(gx), ctypes.byref(gy))
    return gx.value, gy.value


def draws(words):
    w = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in words])
    h = (ctypes.c_uint32 * 9)()
    lib().orc9_draws(w, h)
    return [int(v) for v in h]


def noise(p, site, step):
    out = np.zeros(Q)
    lib().orc9_noise(ctypes.byref(p), site, step, _dp(out))
    return out


def correct(f, rho):
    a = np.array(f, dtype=np.float64)
    fired = lib().orc9_correct(_dp(a), rho)
    return a, bool(fired)


def run(p, f, nsteps, step0=0):
    """Advance f (float64 [9, ny, nx], modified in place) by nsteps."""
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (Q, p.ny, p.nx)
    rc = lib().orc9_run(ctypes.byref(p), _dp(f), int(step0), int(nsteps))
    if rc:
        raise ValueError(f"oracle run failed rc={rc}")
    return f


def initialise(p, mode=1, rho_mean=1.0, rho_spread=0.1, angle_std=0.0, u_mag=-1.0, pop_noise=0.0):
    f = np.zeros((Q, p.ny, p.nx), dtype=np.float64)
    ini = Init(mode, 0, float(rho_mean), float(rho_spread), float(angle_std), float(u_mag), float(pop_noise))
    rc = lib().orc9_initialise(ctypes.byref(p), ctypes.byref(ini), _dp(f))
    if rc:
        raise ValueError(f"oracle init failed rc={rc}")
    return f


def stream(p, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    lib().orc9_stream(ctypes.byref(p), _dp(f), _dp(out))
    return out


def observables(p, f, streamed=True):
    f = np.ascontiguousarray(f, dtype=np.float64)
    o = Obs()
    fn = lib().orc9_observables if streamed else lib().orc9_observables_of
    fn(ctypes.byref(p), _dp(f), ctypes.byref(o))
    return {k: getattr(o, k) for k, _ in Obs._fields_}


def fields(p, f, streamed=True):
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = p.nx * p.ny
    rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
    fn = lib().orc9_fields if streamed else lib().orc9_fields_of
    fn(ctypes.byref(p), _dp(f), _dp(rho), _dp(ux), _dp(uy))
    sh = (p.ny, p.nx)
    return rho.reshape(sh), ux.reshape(sh), uy.reshape(sh)


def add_density(f, drho):
    """The protocol's density change on this lattice: drho / 9 added to
    every population, which raises the mean density by drho."""
    return np.asarray(f, dtype=np.float64) + drho / 9.0
