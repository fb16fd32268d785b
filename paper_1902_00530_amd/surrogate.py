"""Learned surrogate for phase-diagram sweeps: a small convolutional network
that advances the coarse density and momentum fields of a lattice by k
lattice Boltzmann steps, trained on pairs the method itself generates and
judged by it.

Every arithmetic step runs in the library's HIP kernels (lbm_cnn.h, lbm.h):
the lattice Boltzmann steps (lbm_sweep_batch), coarse-graining and lifting
(lbm_coarsen, lbm_lift), normalisation (lbm_channel_affine), the network's
forward and backward passes (lbm_cnn_forward / lbm_cnn_backward) and Adam
(lbm_cnn_adam).  This module orders those calls and owns the tensors.

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

from . import (Batch, lbm_channel_affine, lbm_channel_stats, lbm_cnn_adam, lbm_cnn_backward, lbm_cnn_forward,
               lbm_cnn_grads, lbm_cnn_params, lbm_cnn_shape, lbm_cnn_workspace_bytes, lbm_coarsen_many,
               lbm_field_error, lbm_fill_channel, lbm_lift_many, lbm_obs, lbm_params, lbm_sweep_batch,
               lbm_sweep_opts, lbm_sweep_workspace_bytes)

CIN, HIDDEN, COUT = 4, 32, 3


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Network:
    """Weights (bf16 copies + float32 masters), Adam state and per-channel
    normalisation of the surrogate network."""

    def __init__(self, seed=0, device="cuda"):
        import torch
        rng = np.random.default_rng(seed)
        shapes = [(HIDDEN, CIN, 3, 3), (HIDDEN, HIDDEN, 3, 3), (COUT, HIDDEN, 3, 3)]
        fan = [9 * CIN, 9 * HIDDEN, 9 * HIDDEN]
        self.master_w, self.w, self.b = [], [], []
        for k, (sh, fi) in enumerate(zip(shapes, fan)):
            lim = np.sqrt(6.0 / fi) * (0.1 if k == 2 else 1.0)
            m = torch.from_numpy(rng.uniform(-lim, lim, size=sh)).float().to(device)
            self.master_w.append(m)
            self.w.append(m.to(torch.bfloat16))
            self.b.append(torch.zeros(sh[0], device=device))
        self.tensors = [self.master_w[0], self.b[0], self.master_w[1], self.b[1], self.master_w[2], self.b[2]]
        self.m = [torch.zeros_like(t) for t in self.tensors]
        self.v = [torch.zeros_like(t) for t in self.tensors]
        self.grads = [torch.zeros_like(t) for t in self.tensors]
        self.t = 0
        self.scale = torch.ones(CIN, device=device)
        self.shift = torch.zeros(CIN, device=device)
        self.inv_scale = torch.ones(CIN, device=device)
        self.inv_shift = torch.zeros(CIN, device=device)
        self.device = device
        self._buf = {}

    def params(self):
        return lbm_cnn_params((ctypes.c_void_p * 3)(*[w.data_ptr() for w in self.w]),
                              (ctypes.c_void_p * 3)(*[b.data_ptr() for b in self.b]))

    def grad_struct(self):
        g = self.grads
        return lbm_cnn_grads((ctypes.c_void_p * 3)(g[0].data_ptr(), g[2].data_ptr(), g[4].data_ptr()),
                             (ctypes.c_void_p * 3)(g[1].data_ptr(), g[3].data_ptr(), g[5].data_ptr()))

    def set_normalisation(self, mean, std):
        """Inputs are mapped to (x - mean)/std per channel (float arrays of CIN)."""
        import torch
        std = np.where(np.asarray(std) > 0, std, 1.0)
        self.scale = torch.tensor(1.0 / std, dtype=torch.float32, device=self.device)
        self.shift = torch.tensor(-np.asarray(mean) / std, dtype=torch.float32, device=self.device)
        self.inv_scale = torch.tensor(std, dtype=torch.float32, device=self.device)
        self.inv_shift = torch.tensor(mean, dtype=torch.float32, device=self.device)

    def _buffers(self, n, h, w):
        import torch
        key = (n, h, w)
        if key not in self._buf:
            shape = lbm_cnn_shape(n, CIN, HIDDEN, COUT, h, w)
            self._buf[key] = dict(
                shape=shape,
                a1=torch.empty((n, HIDDEN, h, w), device=self.device),
                a2=torch.empty((n, HIDDEN, h, w), device=self.device),
                y=torch.empty((n, COUT, h, w), device=self.device),
                ws=torch.empty(lbm_cnn_workspace_bytes(shape), dtype=torch.uint8, device=self.device),
                loss=torch.empty(1, device=self.device))
        return self._buf[key]

    def normalise(self, x, stream, channels=CIN):
        lbm_channel_affine(_ptr(x), x.shape[0], x.shape[1], channels, x.shape[2] * x.shape[3], _ptr(self.scale),
                           _ptr(self.shift), stream)

    def denormalise(self, y, stream):
        lbm_channel_affine(_ptr(y), y.shape[0], y.shape[1], COUT, y.shape[2] * y.shape[3], _ptr(self.inv_scale),
                           _ptr(self.inv_shift), stream)

    def forward_normalised(self, xn, stream):
        """Network output for normalised inputs (n, CIN, h, w); returns the
        (reused) output tensor in normalised units."""
        n, _, h, w = xn.shape
        B = self._buffers(n, h, w)
        lbm_cnn_forward(B["shape"], self.params(), _ptr(xn), _ptr(B["a1"]), _ptr(B["a2"]), _ptr(B["y"]),
                        _ptr(B["ws"]), B["ws"].numel(), stream)
        return B["y"]

    def train_step(self, xn, tn, lr, stream, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on a normalised batch; returns the loss tensor (device)."""
        n, _, h, w = xn.shape
        B = self._buffers(n, h, w)
        p = self.params()
        lbm_cnn_forward(B["shape"], p, _ptr(xn), _ptr(B["a1"]), _ptr(B["a2"]), _ptr(B["y"]), _ptr(B["ws"]),
                        B["ws"].numel(), stream)
        lbm_cnn_backward(B["shape"], p, _ptr(xn), _ptr(B["a1"]), _ptr(B["a2"]), _ptr(B["y"]), _ptr(tn),
                         self.grad_struct(), _ptr(B["loss"]), _ptr(B["ws"]), B["ws"].numel(), stream)
        self.t += 1
        for k, (th, m, v, g) in enumerate(zip(self.tensors, self.m, self.v, self.grads)):
            out = _ptr(self.w[k // 2]) if k % 2 == 0 else None
            lbm_cnn_adam(_ptr(th), _ptr(m), _ptr(v), _ptr(g), th.numel(), lr, beta1, beta2, eps, self.t, out,
                         stream)
        return B["loss"]


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


def predict(net, X, stream):
    """Surrogate prediction of X' for coarse fields X (unnormalised)."""
    xn = X.clone()
    net.normalise(xn, stream)
    y = net.forward_normalised(xn, stream).clone()
    net.denormalise(y, stream)
    out = X.clone()
    out[:, :COUT] = y
    return out


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


def fit_normalisation(net, X, stream):
    """Per-channel mean and standard deviation of the training inputs."""
    import torch
    mean = torch.empty(CIN, dtype=torch.float64, device=X.device)
    std = torch.empty(CIN, dtype=torch.float64, device=X.device)
    lbm_channel_stats(_ptr(X), X.shape[0], CIN, X.shape[2] * X.shape[3], _ptr(mean), _ptr(std), stream)
    net.set_normalisation(mean.cpu().numpy(), std.cpu().numpy())


def train(net, X, T, epochs, batch, lr, stream, seed=0, log=None):
    """Adam on normalised pairs (inputs and targets share the channel
    normalisation so the residual connection predicts the change), with the
    step size taken down from lr to lr/20 over the epochs on a half cosine
    (the targets carry the method's own noise, so a constant step leaves the
    weights wandering at the end)."""
    import torch
    Xn = X.clone()
    Tn = T.clone()
    net.normalise(Xn, stream)
    net.normalise(Tn, stream, channels=COUT)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    losses = []
    for ep in range(epochs):
        lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs))))
        perm = torch.randperm(n, generator=g).to(X.device)
        tot = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            loss = net.train_step(Xn[idx].contiguous(), Tn[idx, :COUT].contiguous(), lr_ep, stream)
            tot += float(loss.item()) if (nb % 16 == 0) else 0.0
            nb += 1
        losses.append(tot / max(1, (nb + 15) // 16))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses


def _advance_lattices(sampler, idx, from_judge, stream):
    """One lattice Boltzmann call advancing lattices idx by k steps, each from
    its fine state (sampler.batch) or, where from_judge[l], from the judge's
    lifted state; the noise counters continue the sampler's.  Returns the
    coarse fields (n, CIN, h, w) of every lattice's advanced state (rows of
    lattices not in idx are left as they are)."""
    import torch
    lbm, judge = sampler.batch, sampler.judge
    k = sampler.k
    srcs = []
    for l in idx:
        b = judge if from_judge[l] else lbm
        if b.current[l]:  # every state in the first buffer of its pair
            b.buffers[2 * l].copy_(b.buffers[2 * l + 1])
            b.current[l] = 0
        srcs.append(b)
    m = len(idx)
    params = (lbm_params * m)(*[sampler.params[l] for l in idx])
    bufs = (ctypes.c_void_p * (2 * m))(*[srcs[q].bufs[2 * l + h] for q, l in enumerate(idx) for h in (0, 1)])
    need = lbm_sweep_workspace_bytes(params, m, 1)
    if sampler.ws is None or sampler.ws.numel() < need:
        sampler.ws = torch.empty(need, dtype=torch.uint8, device=sampler.device)
    out = (lbm_obs * m)()
    # a fixed two-step tile: every new subset would otherwise be tuned
    opts = lbm_sweep_opts(int(k), 0, int(lbm.step_index), 16, 1)
    lbm_sweep_batch(params, m, opts, bufs, _ptr(sampler.ws), need, stream, out)
    for q, l in enumerate(idx):
        srcs[q].current[l] = k & 1
    ptrs = torch.tensor([(judge if from_judge[l] else lbm).state(l).data_ptr() for l in range(len(sampler.params))],
                        dtype=torch.int64, device=sampler.device)
    F = torch.empty((len(sampler.params), CIN, sampler.h, sampler.w), device=sampler.device)
    hw = sampler.h * sampler.w
    lbm_coarsen_many(sampler.params[0], len(sampler.params), _ptr(ptrs), sampler.c, _ptr(F), CIN * hw, stream)
    lbm_fill_channel(_ptr(F), len(sampler.params), CIN, 3, hw, _ptr(sampler.act), stream)
    return F


def sweep(net, sampler, jumps, check_every, tol, stream):
    """Surrogate sweep with checks and fallback.  Every jump advances every
    lattice by k steps: lattices on the surrogate by one network evaluation
    of their coarse fields, lattices that have fallen back by k lattice
    Boltzmann steps of their own populations.  Every check_every jumps the
    lattice Boltzmann method judges the surrogate lattices from the same
    coarse state (lift, k steps, coarsen); a lattice whose relative L2 error
    exceeds tol takes the judge's result and continues from the judge's
    populations with the lattice Boltzmann method.  The fallen lattices and,
    at a check, the judged ones run in one batched call.  Returns the final
    coarse fields, the fallback flags and the check errors of each check."""
    import torch
    n = len(sampler.params)
    X = torch.empty((n, CIN, sampler.h, sampler.w), device=sampler.device)
    sampler.coarse_fields(sampler.batch, X, stream)
    fallen = np.zeros(n, dtype=bool)
    errors = []
    lbm, judge = sampler.batch, sampler.judge
    for j in range(jumps):
        Y = predict(net, X, stream)
        check = (j + 1) % check_every == 0 and not fallen.all()
        if check:
            lbm_lift_many(sampler.params[0], n, _ptr(X), CIN * sampler.h * sampler.w, sampler.c,
                          _ptr(judge.dev_ptrs[0]), stream)
            judge.current = [0] * n
        idx = [l for l in range(n) if fallen[l] or check]
        if idx:
            F = _advance_lattices(sampler, idx, [check and not fallen[l] for l in range(n)], stream)
            if fallen.any():
                fb = torch.from_numpy(np.nonzero(fallen)[0]).to(sampler.device)
                Y[fb] = F[fb]
            if check:
                e = relative_l2(Y, F, stream)
                errors.append(e[~fallen])
                newly = (e > tol) & ~fallen
                for i in np.nonzero(newly)[0]:
                    lbm.buffers[2 * i].copy_(judge.state(i))
                    lbm.current[i] = 0
                if newly.any():
                    nw = torch.from_numpy(np.nonzero(newly)[0]).to(sampler.device)
                    Y[nw] = F[nw]
                    fallen |= newly
        lbm.step_index += sampler.k
        X = Y
    return X, fallen, errors


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
    net = Network(seed=0)
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
