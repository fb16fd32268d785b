"""The surrogate object of the C ABI (lbm_surrogate_*) and the surrogate form
of lbm_sweep_batch.

Prediction and one training step go through the handle and are compared with
the FP64 network oracle (oracle/cnn.py) on the same bfloat16-rounded weights
and normalisation (1e-5 of each tensor's scale, as for the bare network
kernels).  The sweep's check and fallback decision runs behind the ABI: with
a zero bound every lattice falls back at the first check, after which the
sweep is the method itself from the lifted start, so its final states equal a
plain sweep from that start bit for bit; with an infinite bound no lattice
falls back and every final state is the lift of its final coarse fields.
"""
import ctypes

import numpy as np
import pytest

import synth_inputs as SI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import cnn as ocnn  # noqa: E402


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_00530_amd as lib
    return lib



def _write(base, ptr, values, dtype):
    """Copy values into the parameter block tensor base at device address ptr."""
    t = torch.from_numpy(np.ascontiguousarray(values)).to(dtype).cuda().view(torch.uint8).reshape(-1)
    off = ptr - base.data_ptr()
    assert 0 <= off and off + t.numel() <= base.numel()
    base[off:off + t.numel()].copy_(t)


def _read(base, ptr, count, dtype):
    nbytes = count * torch.tensor([], dtype=dtype).element_size()
    off = ptr - base.data_ptr()
    assert 0 <= off and off + nbytes <= base.numel()
    return base[off:off + nbytes].view(dtype).double().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def test_predict_and_train_step_match_the_oracle(L):
    from paper_1902_00530_amd import surrogate as S
    torch.cuda.set_device(0)
    cin, h, w, N = 4, 20, 24, 3
    net = S.Surrogate(h, w, 2, 4, max_batch=2, cin=cin, seed=3)
    v = L.lbm_surrogate_view_of(net.handle)
    r = np.random.default_rng(5)
    p = list(ocnn.init_params(cin, 32, 3, r))
    for k in (1, 3, 5):
        p[k] = r.normal(size=p[k].shape) * 0.1
    p[4] = p[4] * 10
    for k in (0, 2, 4):
        p[k] = torch.from_numpy(p[k]).float().to(torch.bfloat16).double().numpy()
    for k in range(6):
        _write(net.params, v.theta[k], p[k].reshape(-1), torch.float32)
    for k in range(3):
        _write(net.params, v.w_bf16[k], p[2 * k].reshape(-1), torch.bfloat16)
    scale = r.uniform(0.5, 2.0, size=cin)
    shift = r.uniform(-0.5, 0.5, size=cin)
    norm = np.concatenate([scale, shift, 1.0 / scale, -shift / scale]).astype(np.float32).astype(np.float64)
    _write(net.params, v.norm, norm, torch.float32)
    sc, sh, isc, ish = norm[:cin], norm[cin:2 * cin], norm[2 * cin:3 * cin], norm[3 * cin:]
    x = r.normal(size=(N, cin, h, w)).astype(np.float32).astype(np.float64)
    t = r.normal(size=(N, cin, h, w)).astype(np.float32).astype(np.float64)
    X, T = torch.from_numpy(x).float().cuda(), torch.from_numpy(t).float().cuda()

    # prediction: normalise, network (residual on the fields), back to field units
    Y = net.predict(X[:2]).double().cpu().numpy()
    xn = x[:2] * sc[None, :, None, None] + sh[None, :, None, None]
    yo = ocnn.forward(xn, tuple(p))[-1]
    ref = yo * isc[None, :3, None, None] + ish[None, :3, None, None]
    assert _rel(Y[:, :3], ref) < 1e-5
    assert np.array_equal(Y[:, 3], x[:2, 3])

    # one Adam step on samples (2, 0): first moments are 0.1 x the gradients
    idx = torch.tensor([2, 0], dtype=torch.int32, device="cuda")
    loss = net.train_step(X, T, idx, 1e-3)
    torch.cuda.synchronize()
    xs = x[[2, 0]] * sc[None, :, None, None] + sh[None, :, None, None]
    ts = t[[2, 0], :3] * sc[None, :3, None, None] + sh[None, :3, None, None]
    oloss, grads = ocnn.backward(xs, tuple(p), ts)
    assert abs(float(loss.item()) - oloss) < 1e-5 * abs(oloss)
    for k in range(6):
        m = _read(net.params, v.m[k], int(v.count[k]), torch.float32)
        assert _rel(m, 0.1 * grads[k].reshape(-1)) < 1e-5, k
    assert L.lbm_surrogate_view_of(net.handle).adam_steps == 1
    net.close()


def test_fit_normalisation(L):
    from paper_1902_00530_amd import surrogate as S
    net = S.Surrogate(8, 8, 2, 4, max_batch=4)
    r = np.random.default_rng(1)
    x = r.normal(loc=[3.0, -1.0, 0.5, 2.0], scale=[0.5, 2.0, 1.0, 1e-9], size=(50, 8, 8, 4)).transpose(0, 3, 1, 2)
    x = np.ascontiguousarray(x).astype(np.float32)
    x[:, 3] = 2.0  # a constant channel keeps scale 1
    net.fit_normalisation(torch.from_numpy(x).cuda())
    v = L.lbm_surrogate_view_of(net.handle)
    norm = _read(net.params, v.norm, 16, torch.float32)
    xd = x.astype(np.float64)
    mean = xd.mean(axis=(0, 2, 3))
    sd = xd.std(axis=(0, 2, 3))
    sd[3] = 1.0
    assert np.allclose(norm[:4], 1.0 / sd, rtol=1e-6) and np.allclose(norm[4:8], -mean / sd, rtol=1e-6, atol=1e-7)
    assert np.allclose(norm[8:12], sd, rtol=1e-6) and np.allclose(norm[12:], mean, rtol=1e-6)
    net.close()


def _sampler(S, cfgs, warmup):
    return S.sampler_from(cfgs, 8, 10, warmup)


def test_sweep_zero_bound_is_the_method_from_the_lift(L):
    """tol = 0: at the first check every lattice falls back, having been judged
    from the lift of its initial coarse fields; from there it runs the method.
    The final states equal a plain sweep of the same steps (same noise
    counters) from those lifted states, bit for bit."""
    from paper_1902_00530_amd import surrogate as S
    cfgs = SI.surrogate_grid(side=64, seed_base=500, n_rho=2, n_act=2)
    net = S.Surrogate(8, 8, 8, 10, max_batch=len(cfgs), seed=1)
    sw = _sampler(S, cfgs, 30)
    ref = _sampler(S, cfgs, 30)
    n = len(cfgs)
    X0 = torch.empty((n, S.CIN, 8, 8), device="cuda")
    ref.coarse_fields(ref.batch, X0, torch.cuda.current_stream().cuda_stream)
    L.lbm_lift_many(ref.params[0], n, X0.data_ptr(), S.CIN * 64, 8, ref.batch.dev_ptrs[0].data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    ref.batch.current = [0] * n
    samples, fallen, errs = sw.batch.surrogate_sweep(net, 40, 1, 0.0)
    ref_out = ref.batch.run(40)
    torch.cuda.synchronize()
    assert fallen.all() and len(errs) == 1 and np.all(errs[0] > 0)
    for l in range(n):
        assert torch.equal(sw.batch.state(l), ref.batch.state(l)), l
        assert samples[l]["M"] == ref_out[l][0]["M"]
    net.close()


def test_sweep_infinite_bound_keeps_every_lattice(L):
    """tol = inf: no lattice falls back, every check is recorded, and each
    final state is the lift of its final coarse fields."""
    from paper_1902_00530_amd import surrogate as S
    cfgs = SI.surrogate_grid(side=64, seed_base=600, n_rho=2, n_act=2)
    n = len(cfgs)
    net = S.Surrogate(8, 8, 8, 10, max_batch=n, seed=2)
    sw = _sampler(S, cfgs, 30)
    Xf = torch.empty((n, S.CIN, 8, 8), device="cuda")
    samples, fallen, errs = sw.batch.surrogate_sweep(net, 60, 2, float("inf"), coarse_out=Xf)
    torch.cuda.synchronize()
    assert not fallen.any() and len(errs) == 3 and np.isfinite(np.stack(errs)).all()
    lifted = [torch.empty_like(sw.batch.state(l)) for l in range(n)]
    ptrs = torch.tensor([t.data_ptr() for t in lifted], dtype=torch.int64, device="cuda")
    L.lbm_lift_many(sw.params[0], n, Xf.data_ptr(), S.CIN * 64, 8, ptrs.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for l in range(n):
        assert torch.equal(sw.batch.state(l), lifted[l]), l
        assert np.isfinite(samples[l]["M"])
    net.close()
