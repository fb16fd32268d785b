"""MI355X-native library for the modified lattice Boltzmann method of dense dry
polar active fluids (Nesbitt, Pruessner & Lee, arXiv:1902.00530).

This module is a thin ctypes binding of the C ABI in ``include/lbm.h``: the
functions below carry the same names and marshal arguments only.  Every step
of the method runs in the HIP kernels of ``liblbm.so``; there is no CPU
fallback, and importing this package fails if the library is not built.
PyTorch tensors provide device memory and streams.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENONFINITE, LBM_EUNSUPPORTED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_PASSIVE, LBM_MIPS, LBM_CIL = 0, 1, 2
LBM_F32, LBM_BF16_DEV, LBM_F16_DEV, LBM_BF16_DEV_R32 = 0, 1, 2, 3
LBM_D2Q7, LBM_D2Q9 = 0, 1
LBM_TILE_RESIDENT = 1024  # tile_rows of the LDS-resident batch form (<= 4096 sites on D2Q7, 3072 on D2Q9)
LBM_INIT_NONE, LBM_INIT_UNIFORM_DIR, LBM_INIT_GAUSS_DIR = 0, 1, 2


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("model", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("A", ctypes.c_double), ("B", ctypes.c_double), ("C", ctypes.c_double),
                ("rho_star", ctypes.c_double), ("u_max", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("lattice", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lbm_init(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved", ctypes.c_int32), ("rho_mean", ctypes.c_double),
                ("rho_spread", ctypes.c_double), ("angle_std", ctypes.c_double), ("u_mag", ctypes.c_double),
                ("pop_noise", ctypes.c_double)]


class lbm_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("M", ctypes.c_double), ("Jx", ctypes.c_double),
                ("Jy", ctypes.c_double), ("phi", ctypes.c_double), ("mean_speed", ctypes.c_double),
                ("zeta", ctypes.c_double), ("drho", ctypes.c_double), ("nonfinite", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_sweep_opts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int64), ("sample_every", ctypes.c_int64), ("step0", ctypes.c_int64),
                ("tile_rows", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("drho", ctypes.POINTER(ctypes.c_double)), ("keep_tables", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("surrogate", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tol", ctypes.c_double), ("coarse_out", ctypes.c_void_p),
                ("fallen_out", ctypes.POINTER(ctypes.c_int32)), ("check_errors_out", ctypes.POINTER(ctypes.c_double)),
                ("max_checks", ctypes.c_int64), ("n_checks_out", ctypes.POINTER(ctypes.c_int64))]


class lbm_surrogate_view(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p * 6), ("m", ctypes.c_void_p * 6), ("v", ctypes.c_void_p * 6),
                ("count", ctypes.c_int64 * 6), ("w_bf16", ctypes.c_void_p * 3), ("norm", ctypes.c_void_p),
                ("adam_steps", ctypes.c_int64)]


class lbm_surrogate_desc(ctypes.Structure):
    _fields_ = [("cin", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("coarse", ctypes.c_int32),
                ("k", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class lbm_cnn_shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("cin", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("cout", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32)]


class lbm_cnn_params(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * 3), ("b", ctypes.c_void_p * 3)]


class lbm_cnn_grads(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * 3), ("b", ctypes.c_void_p * 3)]


class LbmError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where} failed ({code}): {lbm_last_error()}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run python paper_1902_00530_amd/build.py (hipcc, gfx950)")

# torch first: it loads its own HIP and HSA runtimes (sonames libamdhip64.so.7
# and libhsa-runtime64.so.1), which the library's dependencies then resolve
# to, so the process holds one runtime.  Loaded the other way round, torch
# would bring a second copy beside the system one and the library's first
# HIP call would find no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_P = ctypes.POINTER

_SIGS = {
    "lbm_workspace_bytes": (ctypes.c_size_t, [_P(lbm_params), ctypes.c_int64]),
    "lbm_deviation_reference": (ctypes.c_int32, [_P(lbm_params), _P(ctypes.c_float)]),
    "lbm_create": (ctypes.c_int32, [_P(lbm_params), _vp, _vp, ctypes.c_int64, _P(lbm_init), _vp, ctypes.c_size_t,
                                    _vp, _P(_vp)]),
    "lbm_step": (ctypes.c_int32, [_vp, ctypes.c_int64]),
    "lbm_moments": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _P(lbm_obs)]),
    "lbm_observe": (ctypes.c_int32, [_P(lbm_params), _vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp, _vp, _vp,
                                     _P(lbm_obs)]),
    "lbm_current_buffer": (ctypes.c_int32, [_vp]),
    "lbm_get_step": (ctypes.c_int64, [_vp]),
    "lbm_set_step": (ctypes.c_int32, [_vp, ctypes.c_int64]),
    "lbm_add_density": (ctypes.c_int32, [_vp, ctypes.c_double]),
    "lbm_destroy": (ctypes.c_int32, [_vp]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_sweep_workspace_bytes": (ctypes.c_size_t, [_P(lbm_params), ctypes.c_int32, ctypes.c_int64]),
    "lbm_sweep_tile_rows": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32]),
    "lbm_sweep_groups": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32]),
    "lbm_sweep_batch": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32, _P(lbm_sweep_opts), _P(_vp), _vp,
                                         ctypes.c_size_t, _vp, _P(lbm_obs)]),
    "lbm_sweep_samples": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32, ctypes.c_int64, _vp, _vp,
                                           _P(lbm_obs)]),
    "lbm_cnn_workspace_bytes": (ctypes.c_size_t, [_P(lbm_cnn_shape)]),
    "lbm_cnn_forward": (ctypes.c_int32, [_P(lbm_cnn_shape), _P(lbm_cnn_params), _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_size_t, _vp]),
    "lbm_cnn_backward": (ctypes.c_int32, [_P(lbm_cnn_shape), _P(lbm_cnn_params), _vp, _vp, _vp, _vp, _vp,
                                          _P(lbm_cnn_grads), _vp, _vp, ctypes.c_size_t, _vp]),
    "lbm_cnn_adam": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_int64, _vp, _vp]),
    "lbm_channel_affine": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                            _vp, _vp, _vp]),
    "lbm_coarsen": (ctypes.c_int32, [_P(lbm_params), _vp, ctypes.c_int32, _vp, _vp]),
    "lbm_field_error": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                         _vp, _vp]),
    "lbm_channel_stats_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "lbm_channel_stats": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp]),
    "lbm_fill_channel": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _vp,
                                          _vp]),
    "lbm_lift": (ctypes.c_int32, [_P(lbm_params), _vp, ctypes.c_int32, _vp, _vp]),
    "lbm_coarsen_many": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                          _vp]),
    "lbm_lift_many": (ctypes.c_int32, [_P(lbm_params), ctypes.c_int32, _vp, ctypes.c_int64, ctypes.c_int32, _vp,
                                       _vp]),
    "lbm_surrogate_param_bytes": (ctypes.c_size_t, [_P(lbm_surrogate_desc)]),
    "lbm_surrogate_workspace_bytes": (ctypes.c_size_t, [_P(lbm_surrogate_desc)]),
    "lbm_surrogate_create": (ctypes.c_int32, [_P(lbm_surrogate_desc), _vp, ctypes.c_int32, ctypes.c_uint64, _vp,
                                              ctypes.c_size_t, _vp, _P(_vp)]),
    "lbm_surrogate_fit_normalisation": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32]),
    "lbm_surrogate_train_step": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, _vp]),
    "lbm_surrogate_predict": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp]),
    "lbm_surrogate_destroy": (ctypes.c_int32, [_vp]),
    "lbm_surrogate_view_of": (ctypes.c_int32, [_vp, _P(lbm_surrogate_view)]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def lbm_last_error():
    return _lib.lbm_last_error().decode()


def _check(rc, where):
    if rc != LBM_OK:
        raise LbmError(rc, where)
    return rc


# ----------------------------------------------------------------- raw ABI

def lbm_deviation_reference(params):
    """The per-plane references r_i of the deviation storages (numpy float32
    array of Q values): a stored 16-bit d_i reads back as float(d_i) + r_i."""
    out = (ctypes.c_float * 9)()
    _check(_lib.lbm_deviation_reference(ctypes.byref(params), out), "lbm_deviation_reference")
    return np.array(out[:n_populations(params)], dtype=np.float32)


def lbm_workspace_bytes(params, pitch):
    return _lib.lbm_workspace_bytes(ctypes.byref(params), int(pitch))


def lbm_create(params, f_a, f_b, pitch, init, ws, ws_bytes, stream):
    ctx = _vp()
    _check(_lib.lbm_create(ctypes.byref(params), f_a, f_b, int(pitch),
                           ctypes.byref(init) if init is not None else None, ws, int(ws_bytes), stream,
                           ctypes.byref(ctx)),
           "lbm_create")
    return ctx


def lbm_step(ctx, n):
    return _check(_lib.lbm_step(ctx, int(n)), "lbm_step")


def lbm_moments(ctx, rho=None, ux=None, uy=None, want_obs=True, check=True):
    obs = lbm_obs() if want_obs else None
    rc = _lib.lbm_moments(ctx, rho, ux, uy, ctypes.byref(obs) if obs is not None else None)
    if check and rc not in (LBM_OK,):
        raise LbmError(rc, "lbm_moments")
    return obs, rc


def lbm_observe(params, f, pitch, step, rho=None, ux=None, uy=None, stream=None, want_obs=True, check=True):
    """Fields and observables of a population buffer with no context or
    workspace (the library's static scratch; for callers that cannot
    allocate)."""
    obs = lbm_obs() if want_obs else None
    rc = _lib.lbm_observe(ctypes.byref(params), f, int(pitch), int(step), rho, ux, uy, stream,
                          ctypes.byref(obs) if obs is not None else None)
    if check and rc != LBM_OK:
        raise LbmError(rc, "lbm_observe")
    return obs, rc


def lbm_current_buffer(ctx):
    r = _lib.lbm_current_buffer(ctx)
    if r < 0:
        raise LbmError(r, "lbm_current_buffer")
    return r


def lbm_get_step(ctx):
    return _lib.lbm_get_step(ctx)


def lbm_set_step(ctx, step):
    return _check(_lib.lbm_set_step(ctx, int(step)), "lbm_set_step")


def lbm_add_density(ctx, drho):
    return _check(_lib.lbm_add_density(ctx, float(drho)), "lbm_add_density")


def lbm_destroy(ctx):
    return _check(_lib.lbm_destroy(ctx), "lbm_destroy")


def lbm_sweep_workspace_bytes(params_array, n, n_samples):
    return _lib.lbm_sweep_workspace_bytes(params_array, int(n), int(n_samples))


def lbm_sweep_tile_rows(params_array, n):
    return _lib.lbm_sweep_tile_rows(params_array, int(n))


def lbm_sweep_groups(params_array, n):
    """Lattice groups each captured chunk of a tiled sweep runs in."""
    return _lib.lbm_sweep_groups(params_array, int(n))


def lbm_sweep_batch(params_array, n, opts, bufs, ws, ws_bytes, stream, out):
    return _check(_lib.lbm_sweep_batch(params_array, int(n), ctypes.byref(opts), bufs, ws, int(ws_bytes), stream,
                                       out), "lbm_sweep_batch")


def lbm_sweep_samples(params_array, n, n_samples, ws, stream, out):
    return _check(_lib.lbm_sweep_samples(params_array, int(n), int(n_samples), ws, stream, out),
                  "lbm_sweep_samples")


def lbm_cnn_workspace_bytes(shape):
    return _lib.lbm_cnn_workspace_bytes(ctypes.byref(shape))


def lbm_cnn_forward(shape, params, x, a1, a2, y, ws, ws_bytes, stream):
    return _check(_lib.lbm_cnn_forward(ctypes.byref(shape), ctypes.byref(params), x, a1, a2, y, ws, int(ws_bytes),
                                       stream), "lbm_cnn_forward")


def lbm_cnn_backward(shape, params, x, a1, a2, y, target, grads, loss, ws, ws_bytes, stream):
    return _check(_lib.lbm_cnn_backward(ctypes.byref(shape), ctypes.byref(params), x, a1, a2, y, target,
                                        ctypes.byref(grads), loss, ws, int(ws_bytes), stream), "lbm_cnn_backward")


def lbm_cnn_adam(theta, m, v, grad, count, lr, beta1, beta2, eps, t, bf16_out, stream):
    return _check(_lib.lbm_cnn_adam(theta, m, v, grad, int(count), float(lr), float(beta1), float(beta2),
                                    float(eps), int(t), bf16_out, stream), "lbm_cnn_adam")


def lbm_channel_affine(x, n, c, nc, hw, scale, shift, stream):
    return _check(_lib.lbm_channel_affine(x, int(n), int(c), int(nc), int(hw), scale, shift, stream),
                  "lbm_channel_affine")


def lbm_coarsen(params, f, c, out, stream):
    return _check(_lib.lbm_coarsen(ctypes.byref(params), f, int(c), out, stream), "lbm_coarsen")


def lbm_field_error(a, b, n, c, nc, hw, out, stream):
    return _check(_lib.lbm_field_error(a, b, int(n), int(c), int(nc), int(hw), out, stream), "lbm_field_error")


def lbm_channel_stats_workspace_bytes(c):
    return _lib.lbm_channel_stats_workspace_bytes(int(c))


def lbm_channel_stats(x, n, c, hw, mean, stdev, ws, ws_bytes, stream):
    return _check(_lib.lbm_channel_stats(x, int(n), int(c), int(hw), mean, stdev, ws, int(ws_bytes), stream),
                  "lbm_channel_stats")


def lbm_fill_channel(x, n, c, ch, hw, values, stream):
    return _check(_lib.lbm_fill_channel(x, int(n), int(c), int(ch), int(hw), values, stream), "lbm_fill_channel")


def lbm_lift(params, coarse, c, f, stream):
    return _check(_lib.lbm_lift(ctypes.byref(params), coarse, int(c), f, stream), "lbm_lift")


def lbm_coarsen_many(params, n, bufs, c, out, out_stride, stream):
    return _check(_lib.lbm_coarsen_many(ctypes.byref(params), int(n), bufs, int(c), out, int(out_stride), stream),
                  "lbm_coarsen_many")


def lbm_lift_many(params, n, coarse, in_stride, c, bufs, stream):
    return _check(_lib.lbm_lift_many(ctypes.byref(params), int(n), coarse, int(in_stride), int(c), bufs, stream),
                  "lbm_lift_many")


def lbm_surrogate_param_bytes(desc):
    return _lib.lbm_surrogate_param_bytes(ctypes.byref(desc))


def lbm_surrogate_workspace_bytes(desc):
    return _lib.lbm_surrogate_workspace_bytes(ctypes.byref(desc))


def lbm_surrogate_create(desc, params, init, seed, ws, ws_bytes, stream):
    h = _vp()
    _check(_lib.lbm_surrogate_create(ctypes.byref(desc), params, int(init), int(seed) & 0xFFFFFFFFFFFFFFFF, ws,
                                     int(ws_bytes), stream, ctypes.byref(h)), "lbm_surrogate_create")
    return h


def lbm_surrogate_fit_normalisation(h, x, n):
    return _check(_lib.lbm_surrogate_fit_normalisation(h, x, int(n)), "lbm_surrogate_fit_normalisation")


def lbm_surrogate_train_step(h, x, target, idx, n, lr, loss):
    return _check(_lib.lbm_surrogate_train_step(h, x, target, idx, int(n), float(lr), loss),
                  "lbm_surrogate_train_step")


def lbm_surrogate_predict(h, x, n, y):
    return _check(_lib.lbm_surrogate_predict(h, x, int(n), y), "lbm_surrogate_predict")


def lbm_surrogate_view_of(h):
    v = lbm_surrogate_view()
    _check(_lib.lbm_surrogate_view_of(h, ctypes.byref(v)), "lbm_surrogate_view_of")
    return v


def lbm_surrogate_destroy(h):
    return _check(_lib.lbm_surrogate_destroy(h), "lbm_surrogate_destroy")


class Batch:
    """n lattices with torch-owned buffers, advanced by lbm_sweep_batch."""

    def __init__(self, params_list, device="cuda"):
        import torch
        self.n = len(params_list)
        self.params = (lbm_params * self.n)(*params_list)
        self.buffers = [torch.zeros((storage_planes(p), p.ny, p.nx), dtype=storage_dtype(p.storage), device=device)
                        for p in params_list for _ in range(2)]
        self.bufs = (ctypes.c_void_p * (2 * self.n))(*[b.data_ptr() for b in self.buffers])
        # device arrays of the n buffer pointers of each parity (for the
        # many-lattice field maps)
        self.dev_ptrs = [torch.tensor([self.buffers[2 * l + k].data_ptr() for l in range(self.n)],
                                      dtype=torch.int64, device=device) for k in (0, 1)]
        self.current = [0] * self.n
        self.step_index = 0
        self._ws = None
        self._ws_written = False

    def state(self, l):
        return self.buffers[2 * l + self.current[l]]

    def set_state(self, l, f):
        self.buffers[2 * l].copy_(f)
        self.current[l] = 0

    def run(self, n_steps, sample_every=0, tile_rows=0, use_graph=1, stream=None, subset=None, drho=None,
            fetch=True):
        """Advance every lattice (or only the lattices listed in subset) by
        n_steps; returns a list (per advanced lattice) of sample dicts.
        use_graph=2 only prepares the launch plan for such a call (tuning,
        captured graphs) and advances nothing.  drho (a number, or one per
        advanced lattice): right after each sample every population gains
        drho / Q (Q = 7 or 9 populations), the density ramp of the paper's
        protocol.  fetch=False only enqueues the sweep (no synchronisation)
        and returns None; samples() reads its samples afterwards."""
        import torch
        idx = list(range(self.n)) if subset is None else [int(i) for i in subset]
        m = len(idx)
        if m == 0:
            return []
        # the sweep expects each state in the first buffer of its pair
        for l in idx:
            if self.current[l]:
                self.buffers[2 * l].copy_(self.buffers[2 * l + 1])
                self.current[l] = 0
        if subset is None:
            params, bufs = self.params, self.bufs
        else:
            params = (lbm_params * m)(*[self.params[l] for l in idx])
            bufs = (ctypes.c_void_p * (2 * m))(*[self.bufs[2 * l + k] for l in idx for k in (0, 1)])
        n_samples = n_steps // sample_every if sample_every else 1
        need = lbm_sweep_workspace_bytes(params, m, n_samples)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.buffers[0].device)
            self._ws_written = False
        out = (lbm_obs * (m * n_samples))() if fetch else None
        opts = lbm_sweep_opts(int(n_steps), int(sample_every), int(self.step_index), int(tile_rows), int(use_graph))
        # the workspace is this object's alone: after the first call with it,
        # the library may keep the tables it wrote there
        opts.keep_tables = 1 if self._ws_written else 0
        if drho is not None:
            vals = [float(drho)] * m if np.isscalar(drho) else [float(v) for v in drho]
            if len(vals) != m:
                raise ValueError("drho needs one value per advanced lattice")
            dr = (ctypes.c_double * m)(*vals)
            opts.drho = dr
        st = stream if stream is not None else torch.cuda.current_stream()
        try:
            lbm_sweep_batch(params, m, opts, bufs, self._ws.data_ptr(), need, st.cuda_stream, out)
        finally:
            self._ws_written = True
        if use_graph == 2:  # prepared the launch plan only; no step ran
            return []
        if subset is None:
            self.step_index += n_steps
        for l in idx:
            self.current[l] = n_steps & 1
        self._last = (params, m, n_samples)
        if not fetch:
            return None
        return [[out[q * n_samples + s].as_dict() for s in range(n_samples)] for q in range(m)]

    def surrogate_sweep(self, sur, n_steps, check_every, tol, tile_rows=0, coarse_out=None):
        """Advance every lattice by n_steps with the surrogate sur (network
        evaluations of k steps, checks by the method every check_every
        evaluations, fallback where the check error exceeds tol), in one
        lbm_sweep_batch call on the surrogate's stream.  Returns (samples of
        the final states, fallen flags, per-check error arrays with NaN for
        lattices fallen before the check)."""
        import torch
        for l in range(self.n):
            if self.current[l]:
                self.buffers[2 * l].copy_(self.buffers[2 * l + 1])
                self.current[l] = 0
        n = self.n
        need = lbm_sweep_workspace_bytes(self.params, n, 1)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.buffers[0].device)
            self._ws_written = False
        out = (lbm_obs * n)()
        opts = lbm_sweep_opts(int(n_steps), 0, int(self.step_index), int(tile_rows), 1)
        opts.surrogate = sur.handle
        opts.k = sur.k
        opts.check_every = int(check_every)
        opts.tol = float(tol)
        max_checks = n_steps // sur.k // max(1, int(check_every)) + 1
        fallen = (ctypes.c_int32 * n)()
        errs = (ctypes.c_double * (n * max_checks))()
        nchk = ctypes.c_int64(0)
        opts.fallen_out = fallen
        opts.check_errors_out = errs
        opts.max_checks = max_checks
        opts.n_checks_out = ctypes.pointer(nchk)
        opts.coarse_out = coarse_out.data_ptr() if coarse_out is not None else None
        try:
            lbm_sweep_batch(self.params, n, opts, self.bufs, self._ws.data_ptr(), need, sur.stream.cuda_stream, out)
        finally:
            self._ws_written = True
        self.step_index += n_steps
        for l in range(n):
            self.current[l] = n_steps & 1
        e = np.ctypeslib.as_array(errs)[: nchk.value * n].reshape(nchk.value, n).copy()
        return [out[l].as_dict() for l in range(n)], np.ctypeslib.as_array(fallen).astype(bool), list(e)

    def samples(self, stream=None):
        """Samples of the last run(..., fetch=False) (synchronises the stream)."""
        import torch
        params, m, n_samples = self._last
        out = (lbm_obs * (m * n_samples))()
        st = stream if stream is not None else torch.cuda.current_stream()
        lbm_sweep_samples(params, m, n_samples, self._ws.data_ptr(), st.cuda_stream, out)
        return [[out[q * n_samples + s].as_dict() for s in range(n_samples)] for q in range(m)]


# ----------------------------------------------------------------- helpers

def make_params(nx, ny, model, tau=1.0, sigma=0.0, A=0.0, B=0.0, C=0.0, rho_star=1.0, u_max=1.0, seed=0,
                storage=LBM_F32, rho_ref=0.0, lattice=LBM_D2Q7):
    return lbm_params(int(nx), int(ny), int(model), int(storage), float(tau), float(sigma), float(A), float(B),
                      float(C), float(rho_star), float(u_max), float(rho_ref), int(seed) & 0xFFFFFFFFFFFFFFFF,
                      int(lattice), 0)


def n_populations(params):
    """Populations per site: 7 on the triangular lattice, 9 on the square one."""
    return 9 if params.lattice == LBM_D2Q9 else 7


def make_init(mode=LBM_INIT_UNIFORM_DIR, rho_mean=1.0, rho_spread=0.1, angle_std=0.0, u_mag=-1.0, pop_noise=0.0):
    return lbm_init(int(mode), 0, float(rho_mean), float(rho_spread), float(angle_std), float(u_mag),
                    float(pop_noise))


def storage_dtype(storage):
    import torch
    # LBM_BF16_DEV_R32 buffers mix a float32 plane and bfloat16 planes: held
    # as raw 16-bit words (int16), so that comparisons are bitwise
    return {LBM_F32: torch.float32, LBM_BF16_DEV: torch.bfloat16, LBM_F16_DEV: torch.float16,
            LBM_BF16_DEV_R32: torch.int16}[storage]


def storage_planes(params):
    """Planes of storage_dtype in a population buffer: Q, or 8 for
    LBM_BF16_DEV_R32 (its float32 rest plane takes the room of planes 0 and 1
    as one [ny][pitch] float32 array, the six bfloat16 planes follow)."""
    return 8 if params.storage == LBM_BF16_DEV_R32 else n_populations(params)


class Lattice:
    """One lattice with torch-owned population buffers [Q, ny, pitch] on the
    current device (Q = 7 on D2Q7, 9 on D2Q9); every operation is a call of
    the C ABI."""

    def __init__(self, params, init=None, pitch=None, stream=None, device="cuda"):
        import torch
        self.params = params
        self.pitch = int(pitch or params.nx)
        if params.storage == LBM_BF16_DEV_R32 and self.pitch != params.nx:
            # state views slice planes by column, which the float32 rest plane's bytes do not follow
            raise ValueError("LBM_BF16_DEV_R32 lattices take pitch == nx in this binding")
        dt = storage_dtype(params.storage)
        q = storage_planes(params)
        self.buffers = [torch.zeros((q, params.ny, self.pitch), dtype=dt, device=device) for _ in range(2)]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nws = lbm_workspace_bytes(params, self.pitch)
        if nws == 0:
            raise LbmError(LBM_EINVAL, "lbm_workspace_bytes")
        self.workspace = torch.empty(nws, dtype=torch.uint8, device=device)
        self.ctx = lbm_create(params, self.buffers[0].data_ptr(), self.buffers[1].data_ptr(), self.pitch, init,
                              self.workspace.data_ptr(), nws, self.stream.cuda_stream)

    def step(self, n=1):
        lbm_step(self.ctx, n)

    @property
    def state(self):
        return self.buffers[lbm_current_buffer(self.ctx)]

    def set_state(self, f):
        """Copy populations [Q, ny, nx] (storage dtype) into the current buffer."""
        self.state[:, :, : self.params.nx].copy_(f)

    def fields(self):
        import torch
        dev = self.buffers[0].device
        rho = torch.empty((self.params.ny, self.params.nx), dtype=torch.float32, device=dev)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        obs, _ = lbm_moments(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(), want_obs=True, check=False)
        return rho, ux, uy, obs.as_dict()

    def observables(self, check=True):
        obs, rc = lbm_moments(self.ctx, None, None, None, want_obs=True, check=check)
        return obs.as_dict()

    @property
    def step_index(self):
        return lbm_get_step(self.ctx)

    def set_step(self, t):
        lbm_set_step(self.ctx, t)

    def add_density(self, drho):
        lbm_add_density(self.ctx, drho)

    def close(self):
        if self.ctx:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
