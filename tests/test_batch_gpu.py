"""Batched sweeps (lbm_sweep_batch) against single-lattice runs and the oracle.

A batch member runs the same site body as the single-lattice kernel with its
own seed and noise counters, so its state after the sweep must equal the
single-lattice result bit for bit, for every work-tile shape (one or two steps
per launch) and with or without graph replay; the FP64 samples use the same reduction tree as
lbm_moments and must agree with it to rounding of the final divisions.
"""
import numpy as np
import pytest

import synth_inputs as SI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from test_parity_gpu import _cfg, _oparams, _gparams, _self_sensitivity, rel_err  # noqa: E402


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_00530_amd as lib
    return lib


def small_batch():
    sizes = [(128, 192), (192, 128), (256, 256), (128, 128), (384, 130)]
    cfgs = []
    for l, (nx, ny) in enumerate(sizes):
        cfgs.append(_cfg(SI.CIL, nx, ny, tau=1.0, sigma=4 / 70, A=0.125, B=0.3 * (0.2 + 0.2 * l),
                         seed=SI.seed_for(2, l)))
    return cfgs


def init_states(L, cfgs):
    states = []
    for l, c in enumerate(cfgs):
        lat = L.Lattice(_gparams(L, c), init=L.make_init(mode=1, rho_mean=0.3 + 0.3 * l, rho_spread=0.1))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    return states


def single_runs(L, cfgs, states, steps, sample_every=0):
    finals, samples = [], []
    for c, f0 in zip(cfgs, states):
        lat = L.Lattice(_gparams(L, c))
        lat.set_state(f0)
        obs = []
        if sample_every:
            for _ in range(steps // sample_every):
                lat.step(sample_every)
                obs.append(lat.observables())
        else:
            lat.step(steps)
            obs.append(lat.observables())
        finals.append(lat.state.clone())
        samples.append(obs)
        lat.close()
    return finals, samples


@pytest.mark.parametrize("tile_rows,use_graph,steps", [(1, 1, 37), (2, 1, 37), (4, 0, 37), (0, 1, 37),
                                                      (8, 1, 37), (16, 1, 38), (16, 0, 37), (8, 0, 6),
                                                      (16, 1, 39)])
def test_batch_member_equals_single_run(L, tile_rows, use_graph, steps):
    cfgs = small_batch()
    states = init_states(L, cfgs)
    every = 0
    finals, samples = single_runs(L, cfgs, states, steps)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(steps, sample_every=every, tile_rows=tile_rows, use_graph=use_graph)
    torch.cuda.synchronize()
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), l
        o, s = out[l][0], samples[l][0]
        assert o["step"] == steps
        for k in ("M", "Jx", "Jy", "phi", "mean_speed", "zeta", "drho"):
            assert abs(o[k] - s[k]) <= 1e-12 * max(1.0, abs(s[k])), (l, k, o[k], s[k])


@pytest.mark.parametrize("tile_rows", [0, 16])
def test_batch_samples_and_resume(L, tile_rows):
    cfgs = small_batch()
    states = init_states(L, cfgs)
    finals, samples = single_runs(L, cfgs, states, 40, sample_every=10)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out1 = b.run(20, sample_every=10, tile_rows=tile_rows)
    out2 = b.run(20, sample_every=10, tile_rows=tile_rows)   # continues the noise counters
    for l in range(len(cfgs)):
        got = out1[l] + out2[l]
        assert [o["step"] for o in got] == [10, 20, 30, 40]
        for o, s in zip(got, samples[l]):
            assert abs(o["phi"] - s["phi"]) <= 1e-12 and abs(o["M"] - s["M"]) <= 1e-9 * s["M"]
        assert torch.equal(b.state(l), finals[l])


def test_batch_member_matches_oracle(L, orc):
    cfgs = small_batch()[:2]
    states = init_states(L, cfgs)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    b.run(3)
    for l, c in enumerate(cfgs):
        ref = orc.run(_oparams(orc, c), states[l].double().cpu().numpy(), 3)
        assert rel_err(b.state(l).double().cpu().numpy(), ref) < 3e-6


def test_batch_zero_steps_samples_initial_state(L):
    cfgs = small_batch()[:2]
    states = init_states(L, cfgs)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(0)
    for l, c in enumerate(cfgs):
        lat = L.Lattice(_gparams(L, c))
        lat.set_state(states[l])
        o = lat.observables()
        lat.close()
        assert out[l][0]["step"] == 0 and abs(out[l][0]["M"] - o["M"]) <= 1e-9 * o["M"]


@pytest.mark.parametrize("tile_rows", [1, 8, 16])
def test_batch_small_lattices_and_long_period(L, tile_rows):
    """Lattices narrower and shorter than a work tile (the widened two-step
    tile wraps around them more than once) over a sample period longer than
    one captured chunk (2100 steps: two chunks and a tail)."""
    sizes = [(2, 2), (40, 6), (66, 18), (64, 16), (130, 34)]
    cfgs = [_cfg(SI.CIL, nx, ny, tau=1.0, sigma=4 / 70, A=0.125, B=0.3, seed=SI.seed_for(4, l))
            for l, (nx, ny) in enumerate(sizes)]
    states = init_states(L, cfgs)
    steps = 2100
    finals, samples = single_runs(L, cfgs, states, steps)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(steps, tile_rows=tile_rows)
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), (l, sizes[l])
        assert out[l][0]["step"] == steps
        assert abs(out[l][0]["M"] - samples[l][0]["M"]) <= 1e-12 * samples[l][0]["M"]



def test_batch_repeated_calls_replay_cached_graphs(L):
    """Later calls with the same batch and step counts replay the graphs the
    first call instantiated (the descriptors are uploaded again each time);
    the states must still follow the single-lattice runs bit for bit, also
    when a call with other counts comes in between."""
    cfgs = small_batch()
    states = init_states(L, cfgs)
    finals, _ = single_runs(L, cfgs, states, 3 * 37 + 20)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    assert b.run(37, tile_rows=16, use_graph=2) == []   # prepares only: the state stays
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), states[l])
    b.run(37, tile_rows=16)
    b.run(20, sample_every=10, tile_rows=16)
    b.run(37, tile_rows=16)
    b.run(37, tile_rows=16)
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), l


def test_full_size_two_step_batch_matches_oracle(L, orc):
    """The benchmark's workload and launch configuration (five 1024 x 1024
    CIL lattices, 64 x 16 two-step tiles, graphs): four steps (two two-step
    launches) against the oracle on the whole of one lattice, and the other
    lattices against single-lattice runs bit for bit."""
    cfgs = [SI.cil_1024(r, l) for l, r in enumerate(SI.CIL_DENSITIES)]
    inits = [c.pop("init") for c in cfgs]
    lats = [L.Lattice(_gparams(L, c), init=L.make_init(**ini)) for c, ini in zip(cfgs, inits)]
    torch.cuda.synchronize()
    states = [lat.state.clone() for lat in lats]
    for lat in lats:
        lat.step(4)
    torch.cuda.synchronize()
    singles = [lat.state.clone() for lat in lats]
    for lat in lats:
        lat.close()
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    b.run(4, tile_rows=16)
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), singles[l]), l
    l = 2
    po = _oparams(orc, cfgs[l])
    f0 = states[l].double().cpu().numpy()
    ref = orc.run(po, f0.copy(), 4)
    got = b.state(l).double().cpu().numpy()
    d = got - ref
    assert np.sqrt((d * d).mean() / (ref * ref).mean()) < 1e-6
    # chaotic start: the max-norm bound follows the oracle's own amplification
    # of a 1e-7 perturbation over the same steps (as for the one-step path)
    amp = _self_sensitivity(orc, po, f0, 4) / 1e-7
    assert rel_err(got, ref) < 2e-6 * max(amp, 1.0)


# ---------------------------------------------------------------- MIPS batches

def mips_batch():
    """MIPS lattices (the 64^2 workload's parameters) of uneven sizes, some
    narrower or shorter than the 64 x 16 tile, with their own seeds."""
    sizes = [(2, 2), (40, 6), (66, 18), (128, 192), (200, 70), (130, 34)]
    return [_cfg(SI.MIPS, nx, ny, tau=2.0, sigma=8 / 70, C=6.25, rho_star=1.6, u_max=0.3, seed=SI.seed_for(7, l))
            for l, (nx, ny) in enumerate(sizes)]


def mips_states(L, cfgs):
    states = []
    for l, c in enumerate(cfgs):
        lat = L.Lattice(_gparams(L, c), init=L.make_init(mode=1, rho_mean=0.8 + 0.1 * l, rho_spread=0.1,
                                                         u_mag=0.1, pop_noise=1e-3))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    return states


@pytest.mark.parametrize("tile_rows,use_graph,steps", [(16, 1, 37), (16, 0, 38), (8, 1, 37), (8, 0, 2),
                                                      (4, 0, 37), (0, 1, 1100), (4, 1, 1100), (16, 1, 1100)])
def test_mips_batch_member_equals_single_run(L, tile_rows, use_graph, steps):
    """The batched MIPS kernels (one step per launch on 64 x 4 tiles with the
    single-lattice MIPS tile body; two steps per launch on 64 x 8 and 64 x 16
    tiles, odd step counts ending with a one-step launch): every member,
    lattices smaller than a tile and ragged ones included, equals its
    lbm_step run bit for bit (1100 steps cross a captured chunk), and the
    tuned shape is one of the three."""
    cfgs = mips_batch()
    states = mips_states(L, cfgs)
    finals, samples = single_runs(L, cfgs, states, steps)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(steps, tile_rows=tile_rows, use_graph=use_graph)
    torch.cuda.synchronize()
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), l
        o, s = out[l][0], samples[l][0]
        for k in ("M", "phi", "drho"):
            assert abs(o[k] - s[k]) <= 1e-12 * max(1.0, abs(s[k])), (l, k)
    if tile_rows == 0:
        assert L.lbm_sweep_tile_rows(b.params, b.n) in (4, 8, 16)


def test_mips_batch_samples_density_ramp_and_oracle(L, orc):
    """Samples every 10 steps with the protocol's density change after each,
    against single runs with lbm_add_density (bit for bit), and three steps
    (one two-step launch and one one-step launch where the tile takes two)
    against the oracle."""
    cfgs = mips_batch()[2:5]
    states = mips_states(L, cfgs)
    drho = [0.01, -0.02, 0.03]
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(30, sample_every=10, drho=drho)
    for l, c in enumerate(cfgs):
        lat = L.Lattice(_gparams(L, c))
        lat.set_state(states[l])
        obs = []
        for _ in range(3):
            lat.step(10)
            obs.append(lat.observables())
            lat.add_density(drho[l])
        assert torch.equal(b.state(l), lat.state), l
        lat.close()
        for o, s in zip(out[l], obs):
            assert abs(o["M"] - s["M"]) <= 1e-12 * s["M"] and abs(o["drho"] - s["drho"]) <= 1e-12
    for rows in (0, 8, 16):  # tuned, and both two-step MIPS tiles against the oracle directly
        b2 = L.Batch([_gparams(L, c) for c in cfgs[:2]])
        for l in range(2):
            b2.set_state(l, states[l])
        b2.run(3, tile_rows=rows)
        for l, c in enumerate(cfgs[:2]):
            ref = orc.run(_oparams(orc, c), states[l].double().cpu().numpy(), 3)
            assert rel_err(b2.state(l).double().cpu().numpy(), ref) < 3e-6, (rows, l)


# ---------------------------------------------------------------- lattices resident in LDS

RESIDENT_SIZES = [(2, 2), (40, 6), (90, 30), (66, 18), (64, 64), (130, 30), (7, 100)]
RESIDENT_KW = {
    "cil": (SI.CIL, dict(tau=1.0, sigma=4 / 70, A=0.125, B=0.3)),
    "mips": (SI.MIPS, dict(tau=2.0, sigma=8 / 70, C=6.25, rho_star=1.6, u_max=0.3)),
    "passive": (SI.PASSIVE, dict(tau=1.3, sigma=0.01)),
    "passive_quiet": (SI.PASSIVE, dict(tau=1.3, sigma=0.0)),
}


def resident_batch(name):
    """Lattices of at most 4096 sites (the paper's 90 x 30 MIPS lattice and
    the 64 x 64 limit among them, some narrower than a wave), each with its
    own seed."""
    model, kw = RESIDENT_KW[name]
    return [_cfg(model, nx, ny, seed=SI.seed_for(9, l), **kw) for l, (nx, ny) in enumerate(RESIDENT_SIZES)]


def resident_states(L, cfgs):
    states = []
    for l, c in enumerate(cfgs):
        mips = c["model"] == SI.MIPS
        ini = dict(mode=1, rho_mean=0.6 + 0.1 * l, rho_spread=0.1, u_mag=0.1 if mips else 0.05,
                   pop_noise=1e-3 if mips else 0.0)
        if c["model"] == SI.CIL:
            ini["u_mag"] = -1.0
        lat = L.Lattice(_gparams(L, c), init=L.make_init(**ini))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    return states


@pytest.mark.parametrize("name,use_graph,steps", [("mips", 1, 1100), ("mips", 0, 37), ("cil", 1, 38),
                                                  ("cil", 0, 1), ("passive", 1, 37), ("passive_quiet", 1, 2)])
def test_resident_member_equals_single_run(L, name, use_graph, steps):
    """Whole lattices in LDS (LBM_TILE_RESIDENT, every step of a captured chunk
    in one launch): every member equals its lbm_step run bit for bit, for each
    model and step variant (tau = 1 or not, noise on or off), with odd and even
    step counts (the state ends in the buffer the parity names) and across a
    captured chunk (1100 steps)."""
    cfgs = resident_batch(name)
    states = resident_states(L, cfgs)
    finals, samples = single_runs(L, cfgs, states, steps)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(steps, tile_rows=L.LBM_TILE_RESIDENT, use_graph=use_graph)
    torch.cuda.synchronize()
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), l
        o, s = out[l][0], samples[l][0]
        for k in ("M", "phi", "drho"):
            assert abs(o[k] - s[k]) <= 1e-12 * max(1.0, abs(s[k])), (l, k)


def test_resident_samples_density_ramp_and_oracle(L, orc):
    """The protocol's pattern on LDS-resident MIPS lattices: samples every 10
    steps with a density change after each, against single runs with
    lbm_add_density (bit for bit); then three steps against the oracle."""
    cfgs = resident_batch("mips")
    states = resident_states(L, cfgs)
    drho = [0.01 * (l - 3) for l in range(len(cfgs))]
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(30, sample_every=10, drho=drho, tile_rows=L.LBM_TILE_RESIDENT)
    for l, c in enumerate(cfgs):
        lat = L.Lattice(_gparams(L, c))
        lat.set_state(states[l])
        obs = []
        for _ in range(3):
            lat.step(10)
            obs.append(lat.observables())
            lat.add_density(drho[l])
        assert torch.equal(b.state(l), lat.state), l
        lat.close()
        for o, s in zip(out[l], obs):
            assert abs(o["M"] - s["M"]) <= 1e-12 * s["M"] and abs(o["drho"] - s["drho"]) <= 1e-12
    b2 = L.Batch([_gparams(L, c) for c in cfgs])
    for l in range(len(cfgs)):
        b2.set_state(l, states[l])
    b2.run(3, tile_rows=L.LBM_TILE_RESIDENT)
    for l in (2, 4):
        ref = orc.run(_oparams(orc, cfgs[l]), states[l].double().cpu().numpy(), 3)
        assert rel_err(b2.state(l).double().cpu().numpy(), ref) < 3e-6, l


def test_resident_is_tuned_for_paper_sized_lattices(L):
    """Twelve 90 x 30 MIPS lattices (the paper's noise-ramp batch): the tuning
    picks among the two-step 64 x 16 and 64 x 8, the one-step 64 x 4 and the
    LDS-resident forms, and the tuned run equals single runs bit for bit."""
    model, kw = RESIDENT_KW["mips"]
    cfgs = [_cfg(model, 90, 30, seed=SI.seed_for(10, l), **kw) for l in range(12)]
    states = resident_states(L, cfgs)
    finals, _ = single_runs(L, cfgs, states, 200)
    b = L.Batch([_gparams(L, c) for c in cfgs])
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    b.run(200)
    torch.cuda.synchronize()
    assert L.lbm_sweep_tile_rows(b.params, b.n) in (4, 8, 16, L.LBM_TILE_RESIDENT)
    for l in range(len(cfgs)):
        assert torch.equal(b.state(l), finals[l]), l


def test_lattice_groups_with_samples_and_density_ramp(L):
    """The benchmark's five 1024 x 1024 lattices run as two lattice groups
    (each group's state sized for the Infinity Cache): samples every 10 steps
    with a density change after each, two steps per launch, equal to
    single-lattice runs with lbm_add_density bit for bit; then three more
    calls (the groups' order alternates from call to call), with graphs and
    with direct launches, still equal to the single runs."""
    cfgs = [SI.cil_1024(r, l) for l, r in enumerate(SI.CIL_DENSITIES)]
    inits = [c.pop("init") for c in cfgs]
    params = [_gparams(L, c) for c in cfgs]
    arr = (L.lbm_params * len(params))(*params)
    assert L.lbm_sweep_groups(arr, len(params)) == 2
    states = []
    for p, ini in zip(params, inits):
        lat = L.Lattice(p, init=L.make_init(**ini))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    drho = [0.01, -0.01, 0.02, -0.02, 0.005]
    b = L.Batch(params)
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(40, sample_every=10, drho=drho, tile_rows=16)
    for l, p in enumerate(params):
        lat = L.Lattice(p)
        lat.set_state(states[l])
        obs = []
        for _ in range(4):
            lat.step(10)
            obs.append(lat.observables())
            lat.add_density(drho[l])
        assert torch.equal(b.state(l), lat.state), l
        lat.close()
        for o, s in zip(out[l], obs):
            for k in ("M", "phi", "drho"):
                assert abs(o[k] - s[k]) <= 1e-12 * max(1.0, abs(s[k])), (l, k)
    finals = [b.state(l).clone() for l in range(len(params))]
    b.run(20, tile_rows=16)
    b.run(20, tile_rows=16, use_graph=0)
    out = b.run(20, tile_rows=16)
    for l, p in enumerate(params):
        lat = L.Lattice(p)
        lat.set_state(finals[l])
        lat.set_step(40)
        lat.step(60)
        assert torch.equal(b.state(l), lat.state), l
        o, s = out[l][0], lat.observables()
        assert abs(o["M"] - s["M"]) <= 1e-12 * max(1.0, abs(s["M"])), l
        lat.close()


def _raw_sweep(L, params, bufs, ws, steps, keep, tile_rows=16, sample_every=0):
    import ctypes
    n = len(params)
    pa = (L.lbm_params * n)(*params)
    bp = (ctypes.c_void_p * (2 * n))(*[t.data_ptr() for t in bufs])
    ns = steps // sample_every if sample_every else 1
    out = (L.lbm_obs * (n * ns))()
    o = L.lbm_sweep_opts(steps, sample_every, 0, tile_rows, 1)
    o.keep_tables = keep
    L.lbm_sweep_batch(pa, n, o, bp, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream, out)
    return [out[k].as_dict() for k in range(n * ns)]


def test_keep_tables_reuses_only_what_still_holds(L):
    """keep_tables = 1 skips rebuilding and uploading the tables a workspace
    already holds.  One workspace serves, in turn: a batch (tables written),
    the same batch again (tables kept), the same sizes with other seeds and
    buffers (descriptors differ: uploaded again), other sizes (everything
    uploaded again) and a batch of a two-step shape after a one-step one (the
    other tile list region).  Every call's states equal single-lattice runs
    bit for bit."""
    cfgs = small_batch()
    states = init_states(L, cfgs)
    ws = torch.empty(1 << 26, dtype=torch.uint8, device="cuda")
    steps = 21

    def make_bufs(states_):
        return [t for f in states_ for t in (torch.empty_like(f), torch.empty_like(f))]

    def run(cfgs_, states_, bufs, keep, tile_rows):
        for l, f in enumerate(states_):  # same buffers (descriptors unchanged), fresh start
            bufs[2 * l].copy_(f)
            bufs[2 * l + 1].zero_()
        _raw_sweep(L, [_gparams(L, c) for c in cfgs_], bufs, ws, steps, keep, tile_rows)
        torch.cuda.synchronize()
        finals, _ = single_runs(L, cfgs_, states_, steps)
        for l in range(len(cfgs_)):
            assert torch.equal(bufs[2 * l + (steps & 1)], finals[l]), (l, keep, tile_rows)

    bufs = make_bufs(states)
    run(cfgs, states, bufs, 0, 16)
    run(cfgs, states, bufs, 1, 16)  # every table kept
    reseeded = [dict(c, seed=c["seed"] + 99) for c in cfgs]
    run(reseeded, states, bufs, 1, 16)  # descriptors uploaded, tile lists kept
    run(cfgs, states, make_bufs(states), 1, 16)  # other buffers: descriptors uploaded
    other_bufs = make_bufs(states[1:4])
    run(cfgs[1:4], states[1:4], other_bufs, 1, 1)  # other sizes: every table uploaded
    run(cfgs[1:4], states[1:4], other_bufs, 1, 16)
    run(cfgs, states, bufs, 1, 1)
    run(cfgs, states, bufs, 1, 16)


def test_enqueue_only_sweep_and_later_samples(L):
    """A sweep called with out == NULL only enqueues its work; its samples
    stay in the workspace until lbm_sweep_samples reads them, and equal the
    synchronous call's samples, with the same final states."""
    cfgs = small_batch()
    states = init_states(L, cfgs)
    res = []
    for fetch in (True, False):
        b = L.Batch([_gparams(L, c) for c in cfgs])
        for l, f0 in enumerate(states):
            b.set_state(l, f0)
        b.run(8)  # tables written (and a second call that keeps them)
        out = b.run(24, sample_every=8, tile_rows=16, fetch=fetch)
        if not fetch:
            assert out is None
            out = b.samples()
        torch.cuda.synchronize()
        res.append((out, [b.state(l).clone() for l in range(len(cfgs))]))
    (o1, s1), (o2, s2) = res
    assert o1 == o2 and len(o1[0]) == 3
    for a, b_ in zip(s1, s2):
        assert torch.equal(a, b_)


@pytest.mark.parametrize("storage", [1, 2, 3])
@pytest.mark.parametrize("tile_rows,use_graph", [(1, 1), (16, 1), (0, 1), (8, 0)])
def test_16bit_batch_member_equals_single_run(L, storage, tile_rows, use_graph):
    """BF16 / FP16 deviation storage (and BF16 with the float32 rest plane,
    storage 3) in batched sweeps: every step rounds its results into the
    storage as lbm_step's store does (the two-step kernel rounds its first
    step's results in LDS the same way), so members equal lbm_step runs bit
    for bit, samples and density ramp included."""
    cfgs = small_batch()[:4]
    rr = [0.3 + 0.3 * l for l in range(len(cfgs))]
    gp = [L.make_params(c["nx"], c["ny"], c["model"], c["tau"], c["sigma"], c["A"], c["B"], c["C"], c["rho_star"],
                        c["u_max"], c["seed"], storage=storage, rho_ref=rr[l]) for l, c in enumerate(cfgs)]
    states = []
    for l, p in enumerate(gp):
        lat = L.Lattice(p, init=L.make_init(mode=1, rho_mean=rr[l], rho_spread=0.1))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    steps, every = 14, 7
    finals, samples = [], []
    for p, f0 in zip(gp, states):
        lat = L.Lattice(p)
        lat.set_state(f0)
        obs = []
        for _ in range(steps // every):
            lat.step(every)
            obs.append(lat.observables())
            lat.add_density(0.01)
        finals.append(lat.state.clone())
        samples.append(obs)
        lat.close()
    b = L.Batch(gp)
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    out = b.run(steps, sample_every=every, tile_rows=tile_rows, use_graph=use_graph, drho=0.01)
    torch.cuda.synchronize()
    for l in range(len(gp)):
        assert b.state(l).dtype == f0.dtype
        assert torch.equal(b.state(l), finals[l]), l
        for s_b, s_l in zip(out[l], samples[l]):
            assert abs(s_b["M"] - s_l["M"]) <= 1e-9 * abs(s_l["M"])
            assert abs(s_b["phi"] - s_l["phi"]) <= 1e-12


@pytest.mark.parametrize("storage", [1, 2, 3])
def test_16bit_mips_and_resident_batches(L, storage):
    """MIPS (two steps per launch on 64 x 16 and 64 x 8 tiles, one on 64 x 4)
    and the LDS-resident form in 16-bit storage (the resident form keeps storage 3 as the float32 values the
    storage gives back) equal lbm_step runs bit for bit."""
    import synth_inputs as SI_
    cfgs = [dict(nx=90, ny=30, model=SI_.MIPS, tau=2.0, sigma=1.0 / 70.0, A=0.0, B=0.0, C=50.0, rho_star=0.2,
                 u_max=0.3, seed=SI_.seed_for(9, l)) for l in range(3)]
    rr = [0.10, 0.125, 0.15]
    gp = [L.make_params(c["nx"], c["ny"], c["model"], c["tau"], c["sigma"], c["A"], c["B"], c["C"], c["rho_star"],
                        c["u_max"], c["seed"], storage=storage, rho_ref=rr[l]) for l, c in enumerate(cfgs)]
    states = []
    for l, p in enumerate(gp):
        lat = L.Lattice(p, init=L.make_init(mode=1, rho_mean=rr[l], rho_spread=0.1, u_mag=0.01))
        torch.cuda.synchronize()
        states.append(lat.state.clone())
        lat.close()
    steps = 41
    finals = []
    for p, f0 in zip(gp, states):
        lat = L.Lattice(p)
        lat.set_state(f0)
        lat.step(steps)
        finals.append(lat.state.clone())
        lat.close()
    for rows in (16, 8, 4, L.LBM_TILE_RESIDENT):
        b = L.Batch(gp)
        for l, f0 in enumerate(states):
            b.set_state(l, f0)
        b.run(steps, tile_rows=rows)
        torch.cuda.synchronize()
        for l in range(len(gp)):
            assert torch.equal(b.state(l), finals[l]), (rows, l)
