"""Parity at the full 4096 x 4096 size of the precision workload, in the launch
configurations the benchmark times at that size: the plain FP32 step (one
lbm_step launch per step), the BF16 / FP16 deviation storages, MIPS, and the
batched two-step path.

The CIL workload starts disordered (uniform polarisation directions) with
the paper-scaled noise, so a few sites sit at discontinuities of the method:
u* = U0 j/|j| where |j| is near 0, and the negative-population correction
where a population crosses 0.  There the oracle's own result moves by O(1)
under a 1e-7 relative input perturbation, and no max-norm comparison means
anything.  Every entry is therefore held to the tight bound of the arithmetic
(the FP32 step error, 1e-6 of the population scale, plus one rounding of the
storage format), except at most 1e-5 of them; those few are counted and
printed, next to the number of entries where the oracle's own perturbed run
moves by more than the tight bound (measured, of 117,440,512 entries: FP32 82
against the oracle's 3,257; BF16 114 against 123; FP16 0 against 59; MIPS 0
against 0).  The lattice-wide relative RMS error is bounded as well: 2e-7 in
FP32 (a few roundings at 2^-24), half the format's unit roundoff in BF16 and
FP16.
"""
import numpy as np
import pytest

import synth_inputs as SI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from test_parity_gpu import _gparams, _oparams, dev_ref, rel_err, storage_bound  # noqa: E402

W = np.array([0.5] + [1.0 / 12.0] * 6)
U = {1: 2.0 ** -8, 2: 2.0 ** -11}


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_00530_amd as lib
    return lib


def _host(state, nx):
    return state[:, :, :nx].double().cpu().numpy()


def _rms(got, ref):
    d = got - ref
    return float(np.sqrt((d * d).mean() / (ref * ref).mean()))


def _perturbed(g0):
    """The input perturbed by 1e-7 relative (uniform, seeded)."""
    r = np.random.default_rng(0)
    return g0 * (1 + 1e-7 * r.uniform(-1, 1, g0.shape))


def _check_one_step(orc, po, g0, got, label, storage=0, wr=None):
    ref = orc.run(po, g0.copy(), 1)
    scale = np.abs(ref).max()
    tight = 1e-6 * scale + (storage_bound(ref, wr, U[storage]) + 2.0 ** -25 if storage else 0.0)
    bad = np.abs(got - ref) > tight
    n_bad = int(bad.sum())
    sens = np.abs(orc.run(po, _perturbed(g0), 1) - ref)
    n_sens = int((sens > tight).sum())
    rms = _rms(got, ref)
    print(f"{label}: one step, max rel err {rel_err(got, ref):.2e}, rms {rms:.2e}, entries over the tight "
          f"bound {n_bad} of {ref.size} (oracle's own perturbed run: {n_sens})", flush=True)
    assert n_bad <= 1e-5 * ref.size
    assert rms < (2e-7 if storage == 0 else U[storage] / 2)


def test_cil_4096_fp32(L, orc):
    """GPU init and one lbm_step launch against the oracle on the whole
    lattice."""
    cfg = SI.cil_4096()
    ini = cfg.pop("init")
    po = _oparams(orc, cfg)
    f0 = orc.initialise(po, **ini)
    lat = L.Lattice(_gparams(L, cfg), init=L.make_init(**ini))
    torch.cuda.synchronize()
    g0 = _host(lat.state, cfg["nx"])
    assert rel_err(g0, f0) < 2e-7
    del f0
    lat.step(1)
    got = _host(lat.state, cfg["nx"])
    lat.close()
    _check_one_step(orc, po, g0, got, "CIL 4096^2 FP32")


@pytest.mark.parametrize("storage", [1, 2])
def test_cil_4096_deviation_storage(L, orc, storage):
    """BF16 / FP16 deviations from w_i rho_ref (rho_ref = the mean density, as
    the benchmark sets it): the initial state within two roundings of the
    oracle's, and one step from the stored (dequantised) state within one
    rounding of the format plus the FP32 step error."""
    cfg = SI.cil_4096()
    ini = cfg.pop("init")
    rho_ref = ini["rho_mean"]
    po = _oparams(orc, cfg)
    f0 = orc.initialise(po, **ini)
    lat = L.Lattice(_gparams(L, cfg, storage=storage, rho_ref=rho_ref), init=L.make_init(**ini))
    torch.cuda.synchronize()
    wr = dev_ref(L, _gparams(L, cfg, storage=storage, rho_ref=rho_ref))
    g0 = _host(lat.state, cfg["nx"]) + wr
    assert (np.abs(g0 - f0) <= 2 * U[storage] * np.abs(f0 - wr) + 1e-7).all()
    del f0
    lat.step(1)
    got = _host(lat.state, cfg["nx"]) + wr
    lat.close()
    _check_one_step(orc, po, g0, got, f"CIL 4096^2 storage {storage}", storage, wr)


def test_mips_4096_fp32(L, orc):
    """MIPS with the 64 x 64 workload's parameters at 4096 x 4096 (the
    benchmark's large MIPS lattice): GPU init and one step on the whole
    lattice."""
    cfg = dict(SI.mips_small(), nx=4096, ny=4096)
    ini = cfg.pop("init")
    po = _oparams(orc, cfg)
    f0 = orc.initialise(po, **ini)
    lat = L.Lattice(_gparams(L, cfg), init=L.make_init(**ini))
    torch.cuda.synchronize()
    g0 = _host(lat.state, cfg["nx"])
    assert rel_err(g0, f0) < 2e-7
    del f0
    lat.step(1)
    got = _host(lat.state, cfg["nx"])
    lat.close()
    _check_one_step(orc, po, g0, got, "MIPS 4096^2 FP32")


@pytest.mark.parametrize("tile_rows", [16, 8])
def test_cil_4096_two_step_batch_equals_single(L, tile_rows):
    """The batched path at 4096^2 with two steps per launch (the benchmark's
    tuned shapes): four steps, two two-step launches, equal bit for bit to
    four lbm_step launches, whose one-step parity with the oracle is checked
    above."""
    cfg = SI.cil_4096()
    ini = cfg.pop("init")
    lat = L.Lattice(_gparams(L, cfg), init=L.make_init(**ini))
    torch.cuda.synchronize()
    s0 = lat.state[:, :, : cfg["nx"]].clone()
    lat.step(4)
    torch.cuda.synchronize()
    single = lat.state[:, :, : cfg["nx"]].clone()
    lat.close()
    b = L.Batch([_gparams(L, cfg)])
    b.set_state(0, s0)
    b.run(4, tile_rows=tile_rows)
    torch.cuda.synchronize()
    assert torch.equal(b.state(0), single)


@pytest.mark.parametrize("tile_rows", [16, 8])
def test_mips_4096_two_step_batch_equals_single(L, tile_rows):
    """MIPS at 4096^2 with two steps per launch (64 x 16 and 64 x 8 tiles,
    densities of a three-site ring recomputed in LDS): five steps, two
    two-step launches and one one-step launch, equal bit for bit to five
    lbm_step launches, whose one-step parity with the oracle is checked
    above."""
    cfg = dict(SI.mips_small(), nx=4096, ny=4096)
    ini = cfg.pop("init")
    lat = L.Lattice(_gparams(L, cfg), init=L.make_init(**ini))
    torch.cuda.synchronize()
    s0 = lat.state[:, :, : cfg["nx"]].clone()
    lat.step(5)
    torch.cuda.synchronize()
    single = lat.state[:, :, : cfg["nx"]].clone()
    lat.close()
    b = L.Batch([_gparams(L, cfg)])
    b.set_state(0, s0)
    b.run(5, tile_rows=tile_rows)
    torch.cuda.synchronize()
    assert torch.equal(b.state(0), single)


def test_batch_mixing_streamed_and_cached_stores(L):
    """One 4096^2 lattice (its two buffers exceed the Infinity Cache budget:
    a lattice group of its own, stores streamed past the caches) batched with
    two small lattices (cached stores): five steps with two steps
    per launch, each member equal bit for bit to its lbm_step run."""
    big = SI.cil_4096()
    cfgs = [big, dict(big, nx=200, ny=70, seed=SI.seed_for(21)), dict(big, nx=130, ny=34, seed=SI.seed_for(22))]
    inits = [c.pop("init") for c in cfgs]
    params = [_gparams(L, c) for c in cfgs]
    arr = (L.lbm_params * 3)(*params)
    assert L.lbm_sweep_groups(arr, 3) >= 2  # the big lattice in a group of its own
    states, singles = [], []
    for c, p, ini in zip(cfgs, params, inits):
        lat = L.Lattice(p, init=L.make_init(**ini))
        torch.cuda.synchronize()
        states.append(lat.state[:, :, : c["nx"]].clone())
        lat.step(5)
        torch.cuda.synchronize()
        singles.append(lat.state[:, :, : c["nx"]].clone())
        lat.close()
    b = L.Batch(params)
    for l, f0 in enumerate(states):
        b.set_state(l, f0)
    b.run(5, tile_rows=16)
    torch.cuda.synchronize()
    for l in range(3):
        assert torch.equal(b.state(l), singles[l]), l
