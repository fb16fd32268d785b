"""Surrogate-network kernels against the FP64 oracle (oracle/cnn.py).

The oracle is given the same bfloat16-rounded weights the GPU stores, so the
comparison isolates the GPU's float32 arithmetic: a few hundred float32
operations per output (relative error ~1e-7 each) allow 1e-5 of each
tensor's scale for the forward pass and the gradients.
"""
import ctypes

import numpy as np
import pytest

import synth_inputs as SI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import cnn as ocnn  # noqa: E402
from test_parity_gpu import _cfg, _oparams, _gparams  # noqa: E402


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_00530_amd as lib
    return lib


def bf16_round(a):
    return torch.from_numpy(a).float().to(torch.bfloat16).double().numpy()


def setup(L, n=2, cin=4, h=20, w=24, seed=0, spread=0.0):
    r = np.random.default_rng(seed)
    x = r.normal(size=(n, cin, h, w))
    if spread:  # magnitudes over 10^-spread .. 10^spread
        x *= 10.0 ** r.uniform(-spread, spread, size=x.shape)
    t = r.normal(size=(n, 3, h, w))
    p = list(ocnn.init_params(cin, 32, 3, r))
    p[1] = r.normal(size=32) * 0.1
    p[3] = r.normal(size=32) * 0.1
    p[5] = r.normal(size=3) * 0.1
    p[4] = p[4] * 10
    for k in (0, 2, 4):
        p[k] = bf16_round(p[k])
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    dev = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    g = dict(x=dev(x), t=dev(t), w=[dev(p[k], torch.bfloat16) for k in (0, 2, 4)],
             b=[dev(p[k]) for k in (1, 3, 5)])
    shape = L.lbm_cnn_shape(n, cin, 32, 3, h, w)
    params = L.lbm_cnn_params((ctypes.c_void_p * 3)(*[a.data_ptr() for a in g["w"]]),
                              (ctypes.c_void_p * 3)(*[a.data_ptr() for a in g["b"]]))
    ws = torch.empty(L.lbm_cnn_workspace_bytes(shape), dtype=torch.uint8, device="cuda")
    return x, t, tuple(p), g, shape, params, ws


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


# (n, cin, h, w): ragged 16 x 8 tiles; an odd reduction length (cin 3);
# fields smaller than a tile, whose halo wraps more than once; every input
# channel the kernels take (cin 32)
SHAPES = [(2, 4, 20, 24), (3, 3, 9, 17), (1, 5, 5, 7), (2, 32, 16, 32)]


@pytest.mark.parametrize("shp", SHAPES)
def test_forward_matches_oracle(L, shp):
    n, cin, h, w = shp
    _forward_case(L, setup(L, n=n, cin=cin, h=h, w=w))


def test_forward_inputs_over_six_decades(L):
    """The convolutions split each float32 activation into three bf16 parts
    (what is left is below 2^-24 of the value): with input magnitudes spread
    over six decades, every first-layer output is within float32 rounding of
    the FP64 value relative to the sum of the magnitudes of its terms (4e-6:
    a few dozen float32 accumulations; a split that dropped its third part
    would err by ~2^-16, its second by ~2^-8), and the tensors keep the 1e-5
    agreement."""
    case = setup(L, n=2, cin=5, h=12, w=20, seed=3, spread=3.0)
    a1 = _forward_case(L, case)
    x, p = case[0], case[2]
    ra1 = ocnn.forward(x, p)[0]
    scale = ocnn.forward(np.abs(x), tuple(np.abs(q) for q in p))[0]  # sum of |term|, per output
    assert (np.abs(a1 - ra1) <= 4e-6 * scale + 1e-30).all()


def _forward_case(L, case):
    x, t, p, g, shape, params, ws = case
    n, h, w = shape.n, shape.h, shape.w
    a1 = torch.empty((n, 32, h, w), device="cuda")
    a2 = torch.empty_like(a1)
    y = torch.empty((n, 3, h, w), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    L.lbm_cnn_forward(shape, params, g["x"].data_ptr(), a1.data_ptr(), a2.data_ptr(), y.data_ptr(),
                      ws.data_ptr(), ws.numel(), s)
    ra1, ra2, ry = ocnn.forward(x, p)
    assert rel(a1.double().cpu().numpy(), ra1) < 1e-5
    assert rel(a2.double().cpu().numpy(), ra2) < 1e-5
    assert rel(y.double().cpu().numpy(), ry) < 1e-5
    return a1.double().cpu().numpy()


@pytest.mark.parametrize("shp", SHAPES)
def test_backward_matches_oracle(L, shp):
    n, cin, h, w = shp
    x, t, p, g, shape, params, ws = setup(L, n=n, cin=cin, h=h, w=w, seed=1)
    n, h, w = shape.n, shape.h, shape.w
    a1 = torch.empty((n, 32, h, w), device="cuda")
    a2 = torch.empty_like(a1)
    y = torch.empty((n, 3, h, w), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    L.lbm_cnn_forward(shape, params, g["x"].data_ptr(), a1.data_ptr(), a2.data_ptr(), y.data_ptr(),
                      ws.data_ptr(), ws.numel(), s)
    gw = [torch.empty(a.shape, device="cuda") for a in g["w"]]
    gb = [torch.empty(a.shape, device="cuda") for a in g["b"]]
    grads = L.lbm_cnn_grads((ctypes.c_void_p * 3)(*[a.data_ptr() for a in gw]),
                            (ctypes.c_void_p * 3)(*[a.data_ptr() for a in gb]))
    loss = torch.empty(1, device="cuda")
    L.lbm_cnn_backward(shape, params, g["x"].data_ptr(), a1.data_ptr(), a2.data_ptr(), y.data_ptr(),
                       g["t"].data_ptr(), grads, loss.data_ptr(), ws.data_ptr(), ws.numel(), s)
    rl, rg = ocnn.backward(x, p, t)
    assert abs(loss.item() - rl) < 1e-5 * rl
    got = [gw[0], gb[0], gw[1], gb[1], gw[2], gb[2]]
    for k in range(6):
        assert rel(got[k].double().cpu().numpy(), rg[k]) < 1e-5, k


def test_adam_matches_oracle(L):
    r = np.random.default_rng(5)
    theta = r.normal(size=1000).astype(np.float32).astype(np.float64)
    m = np.zeros(1000)
    v = np.zeros(1000)
    dth = torch.from_numpy(theta).float().cuda()
    dm = torch.zeros(1000, device="cuda")
    dv = torch.zeros(1000, device="cuda")
    out = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for t in range(1, 8):
        g = r.normal(size=1000).astype(np.float32).astype(np.float64)
        dg = torch.from_numpy(g).float().cuda()
        L.lbm_cnn_adam(dth.data_ptr(), dm.data_ptr(), dv.data_ptr(), dg.data_ptr(), 1000, 1e-2, 0.9, 0.999, 1e-8, t,
                       out.data_ptr(), s)
        theta, m, v = ocnn.adam_step(theta, g, m, v, t, 1e-2)
    assert np.abs(dth.double().cpu().numpy() - theta).max() < 1e-5
    assert torch.equal(out, dth.to(torch.bfloat16))


def test_channel_affine(L):
    x = torch.randn(3, 4, 5, 6, device="cuda")
    ref = x.clone()
    sc = torch.tensor([2.0, -1.0, 0.5], device="cuda")
    sh = torch.tensor([1.0, 0.0, -3.0], device="cuda")
    L.lbm_channel_affine(x.data_ptr(), 3, 4, 3, 30, sc.data_ptr(), sh.data_ptr(), torch.cuda.current_stream().cuda_stream)
    exp = ref.clone()
    exp[:, :3] = ref[:, :3] * sc[None, :, None, None] + sh[None, :, None, None]
    assert torch.allclose(x, exp, atol=1e-6)


def test_coarsen_and_lift_match_oracle(L, orc):
    cfg = _cfg(SI.CIL, 64, 32, tau=1.0, sigma=4 / 70, A=0.125, B=0.3)
    po = _oparams(orc, cfg)
    f = orc.initialise(po, mode=1, rho_mean=0.74, rho_spread=0.1).astype(np.float32).astype(np.float64)
    gp = _gparams(L, cfg)
    s = torch.cuda.current_stream().cuda_stream
    df = torch.from_numpy(f).float().cuda()
    out = torch.empty((3, 8, 16), device="cuda")
    L.lbm_coarsen(gp, df.data_ptr(), 4, out.data_ptr(), s)
    ref = orc.coarsen(po, f, 4)
    assert np.abs(out.double().cpu().numpy() - ref).max() < 1e-6
    # lifting: every site of a block at xi of the block's fields
    lifted = torch.empty((7, 32, 64), device="cuda")
    L.lbm_lift(gp, out.data_ptr(), 4, lifted.data_ptr(), s)
    ref_l = orc.lift(po, out.double().cpu().numpy(), 4)
    assert np.abs(lifted.double().cpu().numpy() - ref_l).max() < 1e-6
    # mass and momentum survive lift -> coarsen (streaming conserves the totals)
    back = orc.coarsen(po, lifted.double().cpu().numpy(), 4)
    assert np.allclose(back.sum(axis=(1, 2)), out.double().cpu().numpy().sum(axis=(1, 2)), rtol=1e-5, atol=1e-6)
