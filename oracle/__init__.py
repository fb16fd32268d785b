"""FP64 CPU oracle of the modified lattice Boltzmann method (arXiv:1902.00530).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it, and it shares no code with the GPU path.

The C part (``lbm_oracle.c``) holds the lattice Boltzmann method; this module
only marshals numpy arrays into it.  ``cnn`` holds the FP64 reference of the
surrogate network.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PASSIVE, MIPS, CIL = 0, 1, 2
INIT_NONE, INIT_UNIFORM_DIR, INIT_GAUSS_DIR = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("A", ctypes.c_double), ("B", ctypes.c_double), ("C", ctypes.c_double),
                ("rho_star", ctypes.c_double), ("u_max", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Init(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("pad_", ctypes.c_int32), ("rho_mean", ctypes.c_double),
                ("rho_spread", ctypes.c_double), ("angle_std", ctypes.c_double),
                ("u_mag", ctypes.c_double), ("pop_noise", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("Jx", ctypes.c_double), ("Jy", ctypes.c_double),
                ("phi", ctypes.c_double), ("mean_speed", ctypes.c_double), ("zeta", ctypes.c_double),
                ("drho", ctypes.c_double), ("nonfinite", ctypes.c_double)]


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load(_build.LIB)
    return _lib


def lib_parallel():
    """The OpenMP build of the same sources (host-core timing only)."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _load(_build.LIB_OMP)
    return _lib_omp


def _load(path):
    if not os.path.exists(path):
        _build.build()
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    L.orc_philox4x32.argtypes = [ctypes.c_int, u32p, u32p, u32p]
    L.orc_neighbour.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_int)] * 2
    L.orc_lattice_vector.argtypes = [ctypes.c_int, dp, dp]
    L.orc_weight.argtypes = [ctypes.c_int]
    L.orc_weight.restype = ctypes.c_double
    L.orc_xi.argtypes = [ctypes.c_double] * 3 + [dp]
    L.orc_moments.argtypes = [dp, dp, dp, dp]
    L.orc_ustar_local.argtypes = [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, dp, dp]
    L.orc_ustar_mips.argtypes = [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, dp, dp]
    L.orc_gradient.argtypes = [dp, dp, dp]
    L.orc_noise.argtypes = [ctypes.POINTER(Params), ctypes.c_uint32, ctypes.c_int64, dp]
    L.orc_correct.argtypes = [dp, ctypes.c_double]
    L.orc_correct.restype = ctypes.c_int
    L.orc_step.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int64]
    L.orc_step.restype = ctypes.c_int
    L.orc_run.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_int64, ctypes.c_int64]
    L.orc_run.restype = ctypes.c_int
    L.orc_initialise.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Init), dp]
    L.orc_initialise.restype = ctypes.c_int
    L.orc_observables.argtypes = [ctypes.POINTER(Params), dp, ctypes.POINTER(Obs)]
    L.orc_fields.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp]
    L.orc_observables_of.argtypes = [ctypes.POINTER(Params), dp, ctypes.POINTER(Obs)]
    L.orc_fields_of.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp]
    L.orc_stream.argtypes = [ctypes.POINTER(Params), dp, dp]
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = ctypes.c_int
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, model, tau=1.0, sigma=0.0, A=0.0, B=0.0, C=0.0, rho_star=1.0, u_max=1.0, seed=0):
    return Params(nx, ny, model, 0, float(tau), float(sigma), float(A), float(B), float(C),
                  float(rho_star), float(u_max), int(seed) & 0xFFFFFFFFFFFFFFFF)


def philox4x32(ctr, key, rounds=10):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32(rounds, c, k, o)
    return [int(v) for v in o]


def neighbour(nx, ny, x, y, i):
    xn, yn = ctypes.c_int(), ctypes.c_int()
    lib().orc_neighbour(nx, ny, x, y, i, ctypes.byref(xn), ctypes.byref(yn))
    return xn.value, yn.value


def lattice_vector(i):
    ex, ey = ctypes.c_double(), ctypes.c_double()
    lib().orc_lattice_vector(i, ctypes.byref(ex), ctypes.byref(ey))
    return ex.value, ey.value


def weight(i):
    return lib().orc_weight(i)


def xi(rho, ux, uy):
    out = np.zeros(7)
    lib().orc_xi(rho, ux, uy, _dp(out))
    return out


def moments(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    r, jx, jy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_moments(_dp(f), ctypes.byref(r), ctypes.byref(jx), ctypes.byref(jy))
    return r.value, jx.value, jy.value


def ustar_local(p, rho, jx, jy):
    ux, uy = ctypes.c_double(), ctypes.c_double()
    lib().orc_ustar_local(ctypes.byref(p), rho, jx, jy, ctypes.byref(ux), ctypes.byref(uy))
    return ux.value, uy.value


def ustar_mips(p, rho, gx, gy):
    ux, uy = ctypes.c_double(), ctypes.c_double()
    lib().orc_ustar_mips(ctypes.byref(p), rho, gx, gy, ctypes.byref(ux), ctypes.byref(uy))
    return ux.value, uy.value


def gradient(rho_nb):
    a = np.ascontiguousarray(rho_nb, dtype=np.float64)
    gx, gy = ctypes.c_double(), ctypes.c_double()
    lib().orc_gradient(_dp(a), ctypes.byref(gx), ctypes.byref(gy))
    return gx.value, gy.value


def noise(p, site, step):
    out = np.zeros(7)
    lib().orc_noise(ctypes.byref(p), site, step, _dp(out))
    return out


def correct(f, rho):
    a = np.array(f, dtype=np.float64)
    fired = lib().orc_correct(_dp(a), rho)
    return a, bool(fired)


def run(p, f, nsteps, step0=0):
    """Advance f (float64 [7, ny, nx], modified in place) by nsteps."""
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (7, p.ny, p.nx)
    rc = lib().orc_run(ctypes.byref(p), _dp(f), int(step0), int(nsteps))
    if rc:
        raise ValueError(f"oracle run failed rc={rc}")
    return f


def run_parallel(p, f, nsteps, threads, step0=0):
    """run() with a step's rows on `threads` host threads (the OpenMP build);
    returns the thread count in effect."""
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (7, p.ny, p.nx)
    L = lib_parallel()
    used = L.orc_set_threads(int(threads))
    rc = L.orc_run(ctypes.byref(p), _dp(f), int(step0), int(nsteps))
    if rc:
        raise ValueError(f"oracle run failed rc={rc}")
    return used


def initialise(p, mode=INIT_UNIFORM_DIR, rho_mean=1.0, rho_spread=0.1, angle_std=0.0, u_mag=-1.0,
               pop_noise=0.0):
    f = np.zeros((7, p.ny, p.nx), dtype=np.float64)
    ini = Init(mode, 0, float(rho_mean), float(rho_spread), float(angle_std), float(u_mag), float(pop_noise))
    rc = lib().orc_initialise(ctypes.byref(p), ctypes.byref(ini), _dp(f))
    if rc:
        raise ValueError(f"oracle init failed rc={rc}")
    return f


def observables(p, f, streamed=True):
    """Observables of a stored state (of its streamed populations), or with
    streamed=False of the populations exactly as given."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    o = Obs()
    fn = lib().orc_observables if streamed else lib().orc_observables_of
    fn(ctypes.byref(p), _dp(f), ctypes.byref(o))
    return {k: getattr(o, k) for k, _ in Obs._fields_}


def fields(p, f, streamed=True):
    """rho, ux, uy [ny, nx] of a stored state (of its streamed populations),
    or with streamed=False of the populations exactly as given."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = p.nx * p.ny
    rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
    fn = lib().orc_fields if streamed else lib().orc_fields_of
    fn(ctypes.byref(p), _dp(f), _dp(rho), _dp(ux), _dp(uy))
    sh = (p.ny, p.nx)
    return rho.reshape(sh), ux.reshape(sh), uy.reshape(sh)


def stream(p, f):
    """Streaming step (i) of a whole lattice: returns f*_i(r) = f_i(r - e_i)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    lib().orc_stream(ctypes.byref(p), _dp(f), _dp(out))
    return out


def coarsen(p, f, c):
    """Coarse fields [3, ny/c, nx/c]: means over c x c blocks of rho, jx, jy
    of the streamed populations of a stored state."""
    rho, ux, uy = fields(p, f)
    out = np.stack([rho, rho * ux, rho * uy])
    return out.reshape(3, p.ny // c, c, p.nx // c, c).mean(axis=(2, 4))


def lift(p, coarse, c):
    """Stored state whose sites in each c x c block hold xi(rho, j/rho) of
    the block (negative rho treated as 0)."""
    ch, cw = coarse.shape[1], coarse.shape[2]
    f = np.zeros((7, p.ny, p.nx))
    for cy in range(ch):
        for cx in range(cw):
            r = max(coarse[0, cy, cx], 0.0)
            ux = coarse[1, cy, cx] / r if r > 0 else 0.0
            uy = coarse[2, cy, cx] / r if r > 0 else 0.0
            f[:, cy * c:(cy + 1) * c, cx * c:(cx + 1) * c] = xi(r, ux, uy)[:, None, None]
    return f


def add_density(f, drho):
    """The density change of the paper's protocol (appendix "Simulation
    procedure for results"): drho / 7 added to every population of every site,
    which raises the mean density by drho."""
    return np.asarray(f, dtype=np.float64) + drho / 7.0
