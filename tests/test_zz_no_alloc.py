"""The allocation-free observables call lbm_observe against lbm_moments.

lbm_observe runs lbm_moments' kernels with the reduction partials in the
library's static device scratch instead of a context's workspace, so its
fields and observables must equal lbm_moments' bit for bit.  Two calls in a
row, the second on a smaller lattice (the static array keeps the first call's
partials, which the second must not pick up), then the same for D2Q9 and a
16-bit storage, and the size limit as a clean error."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _observe(L, lat, rho=None, ux=None, uy=None):
    fn = L._lib.lbm_observe
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.POINTER(L.lbm_params), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(L.lbm_obs)]
    obs = L.lbm_obs()
    ptr = lambda t: t.data_ptr() if t is not None else None
    rc = fn(ctypes.byref(lat.params), lat.state.data_ptr(), lat.pitch, lat.step_index, ptr(rho), ptr(ux), ptr(uy),
            lat.stream.cuda_stream, ctypes.byref(obs))
    return rc, obs.as_dict()


def _check_equal(L, lat):
    import torch
    rho, ux, uy, ref = lat.fields()
    r2, u2, v2 = (torch.full_like(rho, float("nan")) for _ in range(3))
    rc, got = _observe(L, lat, r2, u2, v2)
    torch.cuda.synchronize()
    assert rc == L.LBM_OK, L.lbm_last_error()
    for k in ref:
        assert np.array_equal(np.float64(got[k]), np.float64(ref[k])), (k, got[k], ref[k])
    assert torch.equal(r2, rho) and torch.equal(u2, ux) and torch.equal(v2, uy)
    # observables only, no fields
    rc, got2 = _observe(L, lat)
    assert rc == L.LBM_OK and got2 == got


@pytest.mark.parametrize("lattice,storage", [(0, 0), (1, 0), (0, 1)])
def test_observe_equals_moments_twice_second_smaller(lattice, storage):
    import torch
    import paper_1902_00530_amd as L
    torch.cuda.set_device(0)
    for k, (nx, ny, pitch) in enumerate(((520, 70, 576), (130, 18, 130))):
        p = L.make_params(nx, ny, L.LBM_CIL, tau=1.0, sigma=4.0 / 70.0, A=0.125, B=0.3, seed=77 + k,
                          storage=storage, rho_ref=0.74 if storage else 0.0, lattice=lattice)
        lat = L.Lattice(p, init=L.make_init(mode=L.LBM_INIT_UNIFORM_DIR, rho_mean=0.74), pitch=pitch)
        lat.step(3 + k)
        _check_equal(L, lat)
        lat.close()


def test_observe_rejects_lattices_beyond_its_scratch():
    import torch
    import paper_1902_00530_amd as L
    torch.cuda.set_device(0)
    p = L.make_params(8192, 8192, L.LBM_CIL, A=0.125, B=0.3)
    fn = L._lib.lbm_observe
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.POINTER(L.lbm_params), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(L.lbm_obs)]
    rc = fn(ctypes.byref(p), ctypes.c_void_p(4096), 8192, 0, None, None, None, None, None)
    assert rc == L.LBM_EINVAL and "static scratch" in L.lbm_last_error()
    rc = fn(ctypes.byref(p), None, 8192, 0, None, None, None, None, None)
    assert rc == L.LBM_EINVAL
