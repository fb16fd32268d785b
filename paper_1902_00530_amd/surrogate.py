"""Learned surrogate for phase-diagram sweeps: a small convolutional network
that advances the coarse density and momentum fields of a lattice by k
lattice Boltzmann steps, trained on pairs the method itself generates and
judged by it.

Every arithmetic step runs in the library's HIP kernels behind its C ABI
(lbm_cnn.h, lbm.h): the lattice Boltzmann steps (lbm_sweep_batch),
coarse-graining and lifting (lbm_coarsen_many, lbm_lift_many), and the
surrogate object (lbm_surrogate_create / _fit_normalisation / _train_step /
_predict / _destroy: normalisation, forward and backward passes, Adam).  A
surrogate sweep with its checks and fallbacks is one lbm_sweep_batch call
(lbm_sweep_opts.surrogate).  This module orders those calls and owns the
tensors.

Fields: X = (rho, jx, jy, B) on the coarse grid, with B the lattice's
activity constant as a fourth, constant channel (the dynamics depend on it).
A training pair is (X_t, X'): X_t the coarse fields of a lattice Boltzmann
state, X' the coarse fields after lifting X_t to populations (f^SS of each
coarse cell) and running k steps -- exactly the map the surrogate replaces
inside a sweep, and the check it is judged by.
"""
import ctypes

import math

import numpy as np

from . import (Batch, lbm_coarsen_many, lbm_field_error, lbm_fill_channel, lbm_lift_many, lbm_surrogate_create,
               lbm_surrogate_desc, lbm_surrogate_destroy, lbm_surrogate_fit_normalisation,
               lbm_surrogate_param_bytes, lbm_surrogate_predict, lbm_surrogate_train_step,
               lbm_surrogate_workspace_bytes)

CIN, HIDDEN, COUT = 4, 32, 3


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Surrogate:
    """The library's surrogate object (lbm_surrogate_*): its parameter block
    (weights, Adam moments, normalisation) and workspace are torch tensors
    owned here, its work runs on one stream."""

    def __init__(self, h, w, coarse, k, max_batch, cin=CIN, seed=0, device="cuda", stream=None):
        import torch
        self.desc = lbm_surrogate_desc(int(cin), int(h), int(w), int(coarse), int(k), int(max_batch))
        self.k, self.coarse, self.max_batch, self.cin = int(k), int(coarse), int(max_batch), int(cin)
        pb, wb = lbm_surrogate_param_bytes(self.desc), lbm_surrogate_workspace_bytes(self.desc)
        if not pb or not wb:
            raise ValueError("invalid surrogate description")
        self.params = torch.zeros(pb, dtype=torch.uint8, device=device)
        self.ws = torch.empty(wb, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = lbm_surrogate_create(self.desc, self.params.data_ptr(), 1, seed, self.ws.data_ptr(), wb,
                                           self.stream.cuda_stream)

    def fit_normalisation(self, X):
        """Per-channel normalisation from the mean and spread of samples X."""
        lbm_surrogate_fit_normalisation(self.handle, X.data_ptr(), X.shape[0])

    def train_step(self, X, T, idx, lr):
        """One Adam step on the samples idx (device int32) of X and T; returns
        the loss tensor (device)."""
        lbm_surrogate_train_step(self.handle, X.data_ptr(), T.data_ptr(), idx.data_ptr(), idx.numel(), lr,
                                 self.loss.data_ptr())
        return self.loss

    def predict(self, X):
        """The network's coarse fields k steps after X (constant channels
        carried over), in chunks of max_batch samples."""
        import torch
        Y = torch.empty_like(X)
        for s in range(0, X.shape[0], self.max_batch):
            m = min(self.max_batch, X.shape[0] - s)
            lbm_surrogate_predict(self.handle, X[s:s + m].data_ptr(), m, Y[s:s + m].data_ptr())
        return Y

    def close(self):
        if self.handle:
            lbm_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Data from the lattice Boltzmann method itself
# ---------------------------------------------------------------------------

def _state_ptrs(batch):
    """Device array of the pointers to every lattice's current state."""
    import torch
    par = set(batch.current)
    if len(par) == 1:
        return batch.dev_ptrs[par.pop()]
    return torch.tensor([batch.state(l).data_ptr() for l in range(batch.n)], dtype=torch.int64,
                        device=batch.buffers[0].device)


def coarse_fields(batch, shape_params, c, act, out, stream):
    """out (n, CIN, h, w): channels 0..2 the coarse fields of every lattice of
    the batch (one launch), channel 3 the activity act (device, n floats)."""
    n, h, w = batch.n, shape_params.ny // c, shape_params.nx // c
    if tuple(out.shape) != (n, CIN, h, w) or not out.is_contiguous():
        raise ValueError(f"coarse field tensor must be a contiguous {(n, CIN, h, w)} tensor")
    ptrs = _state_ptrs(batch)
    lbm_coarsen_many(shape_params, n, _ptr(ptrs), c, _ptr(out), CIN * h * w, stream)
    lbm_fill_channel(_ptr(out), n, CIN, 3, h * w, _ptr(act), stream)


class FieldSampler:
    """A batch of lattices of one shape that produces coarse-field pairs
    (X_t, X') and judges coarse states with the lattice Boltzmann method."""

    def __init__(self, params_list, coarse, k, device="cuda"):
        import torch
        self.params = params_list
        self.c = coarse
        self.k = k
        self.batch = Batch(params_list, device=device)
        self.judge = Batch(params_list, device=device)
        self.h = params_list[0].ny // coarse
        self.w = params_list[0].nx // coarse
        for p in params_list:
            if (p.nx, p.ny) != (params_list[0].nx, params_list[0].ny):
                raise ValueError("all lattices of a sampler share one shape")
        self.device = device
        self.act = torch.tensor([p.B for p in params_list], dtype=torch.float32, device=device)
        self.ws = None  # workspace of the sweep's own batched calls

    def set_states(self, states):
        for l, f in enumerate(states):
            self.batch.set_state(l, f)

    def advance(self, steps):
        self.batch.run(steps)

    def coarse_fields(self, batch, out, stream):
        coarse_fields(batch, self.params[0], self.c, self.act, out, stream)

    def judge_from(self, X, stream):
        """Lift coarse fields X (n, CIN, h, w) to populations, run k steps
        with the lattice Boltzmann method (noise counters continuing the
        sampler's) and return the coarse fields X' (n, CIN, h, w)."""
        import torch
        n = len(self.params)
        if tuple(X.shape) != (n, CIN, self.h, self.w) or not X.is_contiguous():
            raise ValueError(f"coarse fields must be a contiguous {(n, CIN, self.h, self.w)} tensor")
        lbm_lift_many(self.params[0], n, _ptr(X), CIN * self.h * self.w, self.c, _ptr(self.judge.dev_ptrs[0]),
                      stream)
        self.judge.current = [0] * n
        self.judge.step_index = self.batch.step_index
        self.judge.run(self.k)
        out = torch.empty_like(X)
        self.coarse_fields(self.judge, out, stream)
        return out


def relative_l2(a, b, stream, channels=COUT):
    """Per-sample relative L2 error of the first `channels` field channels of
    a against b (float64, computed on the device), as a numpy array."""
    import torch
    if a.shape != b.shape or not (a.is_contiguous() and b.is_contiguous()):
        raise ValueError("relative_l2 needs two contiguous tensors of one shape")
    out = torch.empty(a.shape[0], dtype=torch.float64, device=a.device)
    lbm_field_error(_ptr(a), _ptr(b), a.shape[0], a.shape[1], channels, a.shape[2] * a.shape[3], _ptr(out), stream)
    return out.cpu().numpy()


def predict(net, X, stream=None):
    """Surrogate prediction of X' for coarse fields X (unnormalised)."""
    return net.predict(X)


def generate_pairs(sampler, rounds, warmup, stream):
    """rounds x n pairs (X_t, X') after warmup steps; between rounds the
    underlying trajectories advance by k steps."""
    import torch
    n = len(sampler.params)
    X = torch.empty((rounds * n, CIN, sampler.h, sampler.w), device=sampler.device)
    T = torch.empty_like(X)
    sampler.advance(warmup)
    for r in range(rounds):
        xs = X[r * n:(r + 1) * n]
        sampler.coarse_fields(sampler.batch, xs, stream)
        T[r * n:(r + 1) * n] = sampler.judge_from(xs, stream)
        sampler.advance(sampler.k)
    return X, T


def fit_normalisation(net, X, stream=None):
    """Per-channel mean and standard deviation of the training inputs."""
    net.fit_normalisation(X)


def train(net, X, T, epochs, batch, lr, stream=None, seed=0, log=None):
    """Adam on the pairs (inputs and targets share the channel normalisation,
    so the residual connection predicts the change), one library call per
    mini-batch of sample indices, with the step size taken down from lr to
    lr/20 over the epochs on a half cosine (the targets carry the method's own
    noise, so a constant step leaves the weights wandering at the end)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    losses = []
    for ep in range(epochs):
        lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs))))
        perm = torch.randperm(n, generator=g).to(dtype=torch.int32).to(X.device)
        tot = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            loss = net.train_step(X, T, perm[s:s + batch], lr_ep)
            tot += float(loss.item()) if (nb % 16 == 0) else 0.0
            nb += 1
        losses.append(tot / max(1, (nb + 15) // 16))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses


def sweep(net, sampler, jumps, check_every, tol, stream=None):
    """Surrogate sweep with checks and fallback: one lbm_sweep_batch call
    (lbm_sweep_opts.surrogate) over the sampler's lattices.  Every jump
    advances every lattice by k steps: lattices on the surrogate by one
    network evaluation of their coarse fields, lattices that have fallen back
    by k lattice Boltzmann steps of their own populations.  Every check_every
    jumps the method judges the surrogate lattices from the same coarse state
    (lift, k steps, coarsen); a lattice whose relative L2 error exceeds tol
    takes the judge's result and continues from the judge's populations with
    the method.  Returns the final coarse fields, the fallback flags and the
    errors of each check (for the lattices still on the surrogate then)."""
    import torch
    n = len(sampler.params)
    X = torch.empty((n, CIN, sampler.h, sampler.w), device=sampler.device)
    _, fallen, errs = sampler.batch.surrogate_sweep(net, jumps * sampler.k, check_every, tol, coarse_out=X)
    net.stream.synchronize()
    return X, fallen, [e[~np.isnan(e)] for e in errs]


# ---------------------------------------------------------------------------
# The whole recipe: data, training, evaluation, sweep.
# ---------------------------------------------------------------------------

def sampler_from(cfgs, coarse, k, warmup, device="cuda"):
    """A FieldSampler over lattices given as workload dicts (with an 'init'
    entry), initialised by the library's init kernel and warmed up."""
    import torch
    from . import Lattice, make_init, make_params
    ps, states = [], []
    for c in cfgs:
        p = make_params(c["nx"], c["ny"], c["model"], c["tau"], c["sigma"], c["A"], c["B"], c["C"], c["rho_star"],
                        c["u_max"], c["seed"])
        lat = Lattice(p, init=make_init(**c["init"]))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
        ps.append(p)
    smp = FieldSampler(ps, coarse, k, device=device)
    smp.set_states(states)
    if warmup:
        smp.advance(warmup)
    return smp


def noise_floor(cfgs, coarse, k, warmup, other_counters=7919):
    """The method's own run-to-run spread at coarse cells of coarse x coarse
    sites: the mean relative L2 error of (rho, j) between two runs of k steps
    from the same lifted coarse state with different noise counters.  No
    predictor checked against one run of the method can be expected below
    about floor / sqrt(2)."""
    import torch
    st = torch.cuda.current_stream().cuda_stream
    hs = sampler_from(cfgs, coarse, k, warmup)
    X = torch.empty((len(cfgs), CIN, hs.h, hs.w), device=hs.device)
    hs.coarse_fields(hs.batch, X, st)
    T1 = hs.judge_from(X, st)
    hs.batch.step_index += other_counters
    T2 = hs.judge_from(X, st)
    return float(relative_l2(T2, T1, st).mean())


def recipe(train_cfgs, test_cfgs, sweep_cfgs, coarse=8, k=50, warmup=2000, rounds=320, epochs=30, batch=64,
           lr=1e-3, jumps=20, check_every=4, tol_abs=1e-2, tol_floor_factor=1.5, log=None):
    """Generate rounds x len(train_cfgs) training pairs, train, measure the
    held-out error against the persistence baseline (X' = X), the untrained
    network and the method's own run-to-run spread (same coarse state, other
    noise counters), then run surrogate sweeps with a fixed bound and with a
    bound relative to that spread, timed against the plain method."""
    import time
    import torch
    st = torch.cuda.current_stream().cuda_stream
    res = {}
    t0 = time.perf_counter()
    smp = sampler_from(train_cfgs, coarse, k, warmup)
    X, T = generate_pairs(smp, rounds, 0, st)
    torch.cuda.synchronize()
    res["pairs"] = int(X.shape[0])
    res["field_shape"] = list(X.shape[1:])
    res["generate_s"] = round(time.perf_counter() - t0, 3)
    hs = sampler_from(test_cfgs, coarse, k, warmup)
    Xh = torch.empty((len(test_cfgs), CIN, hs.h, hs.w), device=hs.device)
    hs.coarse_fields(hs.batch, Xh, st)
    Th = hs.judge_from(Xh, st)
    hs.batch.step_index += 7919   # other noise counters, same coarse state
    Th2 = hs.judge_from(Xh, st)
    hs.batch.step_index -= 7919
    net = Surrogate(smp.h, smp.w, coarse, k, max(batch, len(test_cfgs), len(sweep_cfgs)), seed=0)
    fit_normalisation(net, X, st)
    floor = float(relative_l2(Th2, Th, st).mean())
    res["persistence_error"] = float(relative_l2(Xh, Th, st).mean())
    res["noise_floor"] = floor
    res["ideal_error"] = floor / np.sqrt(2.0)
    res["untrained_error"] = float(relative_l2(predict(net, Xh, st), Th, st).mean())
    t0 = time.perf_counter()
    losses = train(net, X, T, epochs, batch, lr, st, log=log)
    torch.cuda.synchronize()
    res["train_s"] = round(time.perf_counter() - t0, 3)
    res["train_loss_first_last"] = [losses[0], losses[-1]]
    res["trained_error"] = float(relative_l2(predict(net, Xh, st), Th, st).mean())
    # per-jump cost: network vs k lattice Boltzmann steps on the same lattices
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        predict(net, Xh, st)
    torch.cuda.synchronize()
    res["network_jump_ms"] = round((time.perf_counter() - t0) / 10 * 1e3, 3)
    t0 = time.perf_counter()
    for _ in range(3):
        hs.batch.run(k)
    torch.cuda.synchronize()
    res["lbm_jump_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
    # untimed warm-up of every code path of a sweep (first launches load kernels)
    warm = sampler_from(sweep_cfgs[:max(2, len(sweep_cfgs) // 8)], coarse, k, 0)
    sweep(net, warm, 3, 1, 0.0, st)
    torch.cuda.synchronize()
    sweeps = []
    # the two bounds with checks every check_every jumps, and the bound
    # relative to the noise floor with checks half as often (the checks are
    # most of a sweep's cost; fewer checks verify less)
    for name, tol, ce in (("fixed", tol_abs, check_every),
                          ("relative_to_noise_floor", tol_floor_factor * floor, check_every),
                          ("relative_to_noise_floor", tol_floor_factor * floor, 2 * check_every)):
        sw = sampler_from(sweep_cfgs, coarse, k, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, fallen, errs = sweep(net, sw, jumps, ce, tol, st)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        # the method alone over the same jumps: batched with its tuned tile
        # (two steps per launch) and in the plain one-step form
        times = []
        for rows in (0, 1):
            pl = sampler_from(sweep_cfgs, coarse, k, warmup)
            pl.batch.run(jumps * k, tile_rows=rows, use_graph=2)  # launch plan, untimed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl.batch.run(jumps * k, tile_rows=rows)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tp, tp1 = times
        e = np.concatenate(errs) if errs else np.zeros(0)
        sweeps.append({"bound": name, "tol": tol, "check_every": ce, "sweep_ms": round(ts * 1e3, 2),
                       "plain_lbm_ms": round(tp * 1e3, 2),
                       "speedup": round(tp / ts, 3), "plain_one_step_lbm_ms": round(tp1 * 1e3, 2),
                       "speedup_vs_one_step": round(tp1 / ts, 3), "fallback_rate": float(fallen.mean()),
                       "mean_check_error": float(e.mean()) if e.size else None})
    res["sweeps"] = sweeps
    res["network"] = net
    return res
