"""ABI contract checks that need no GPU: the library loads, exports every
function that include/*.h declares, and rejects invalid arguments before any
device work."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(lbm_[A-Za-z0-9_]+)\s*\(", text,
                             flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lbm_create", "lbm_step", "lbm_moments", "lbm_sweep_batch", "lbm_destroy", "lbm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1902_00530_amd as L
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = declared_functions() - exported
    assert not missing, missing
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in declared_functions():
        assert getattr(lib, n) is not None


def _create(L, p, pitch=None, a=1, b=2, init=None, ws=4096, ws_bytes=1 << 40):
    ctx = ctypes.c_void_p()
    rc = L._lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(a), ctypes.c_void_p(b),
                           p.nx if pitch is None else pitch, init, ctypes.c_void_p(ws), ws_bytes, None,
                           ctypes.byref(ctx))
    return rc, ctx


@pytest.mark.parametrize("field,value,msg", [
    ("ny", 63, "even"), ("nx", 1, ">= 2"), ("ny", 0, ">= 2"), ("tau", 0.5, "tau"),
    ("tau", float("nan"), "tau"), ("sigma", -0.1, "sigma"), ("sigma", float("inf"), "sigma"),
    ("A", -1.0, "A, B"), ("B", float("nan"), "A, B"), ("model", 7, "model"), ("storage", 9, "storage"),
    ("lattice", 2, "lattice"), ("lattice", -1, "lattice"),
])
def test_create_rejects_invalid_parameters(field, value, msg):
    import paper_1902_00530_amd as L
    p = L.make_params(64, 64, L.LBM_CIL, A=0.1, B=0.3)
    setattr(p, field, value)
    rc, ctx = _create(L, p)
    assert rc == L.LBM_EINVAL and not ctx.value
    assert msg in L.lbm_last_error()


def test_create_rejects_bad_buffers_and_pitch():
    import paper_1902_00530_amd as L
    p = L.make_params(64, 64, L.LBM_CIL)
    assert _create(L, p, pitch=63)[0] == L.LBM_EINVAL
    assert _create(L, p, a=0)[0] == L.LBM_EINVAL
    assert _create(L, p, a=5, b=5)[0] == L.LBM_EINVAL
    big = L.make_params(131072, 32768, L.LBM_CIL)
    assert _create(L, big)[0] == L.LBM_EINVAL
    mips = L.make_params(64, 64, L.LBM_MIPS, rho_star=0.0)
    assert _create(L, mips)[0] == L.LBM_EINVAL
    bad_init = L.make_init(mode=9)
    assert L._lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(1), ctypes.c_void_p(2), 64, ctypes.byref(bad_init),
                             ctypes.c_void_p(4096), 1 << 40, None, ctypes.byref(ctypes.c_void_p())) == L.LBM_EINVAL


def test_create_rejects_bad_workspace():
    """The context's device scratch is the caller's workspace: null,
    misaligned or shorter than lbm_workspace_bytes() is refused before any
    device call; the size covers the step clock, the sample's result and the
    reduction partials (5 per 256 x 16 block, one per column and row block,
    one mean per column)."""
    import paper_1902_00530_amd as L
    p = L.make_params(1000, 64, L.LBM_CIL)
    need = L.lbm_workspace_bytes(p, 1000)
    blocks = 4 * 4
    doubles = blocks * 5 + 4 * 1000 + 1000
    assert need == 512 + ((doubles * 8 + 255) // 256) * 256
    assert _create(L, p, ws=0)[0] == L.LBM_EINVAL and "workspace" in L.lbm_last_error()
    assert _create(L, p, ws=4096 + 8)[0] == L.LBM_EINVAL and "aligned" in L.lbm_last_error()
    assert _create(L, p, ws_bytes=need - 1)[0] == L.LBM_EINVAL and "lbm_workspace_bytes" in L.lbm_last_error()
    bad = L.make_params(64, 63, L.LBM_CIL)
    assert L.lbm_workspace_bytes(bad, 64) == 0
    assert L.lbm_workspace_bytes(p, 999) == 0


def test_square_lattice_validation():
    """D2Q9 takes odd ny (its checks pass and the call reaches the device: a
    HIP error without a GPU, a context with one), rejects planes of 2^32
    bytes or more, is refused by the coarse-field calls, and in batched
    sweeps takes every tile shape on the local models (64 x 16 only on
    MIPS) and no mixing with D2Q7."""
    import paper_1902_00530_amd as L

    def passes_validation(p):
        rc, ctx = _create(L, p)  # no init: nothing is launched on the buffers
        if rc == L.LBM_OK:
            L._lib.lbm_destroy(ctx)
        return rc in (L.LBM_OK, L.LBM_EHIP)

    assert passes_validation(L.make_params(64, 63, L.LBM_CIL, A=0.1, B=0.3, lattice=L.LBM_D2Q9))
    p7 = L.make_params(64, 63, L.LBM_CIL, A=0.1, B=0.3)
    assert _create(L, p7)[0] == L.LBM_EINVAL
    big = L.make_params(32768, 32768, L.LBM_CIL, lattice=L.LBM_D2Q9)
    assert _create(L, big)[0] == L.LBM_EUNSUPPORTED and "2^32" in L.lbm_last_error()
    assert passes_validation(L.make_params(32768, 32768, L.LBM_CIL, lattice=L.LBM_D2Q9, storage=L.LBM_BF16_DEV,
                                           rho_ref=1.0))
    q9 = L.make_params(128, 128, L.LBM_CIL, tau=1.0, sigma=0.05, A=0.1, B=0.3, lattice=L.LBM_D2Q9)
    q7 = L.make_params(128, 128, L.LBM_CIL, tau=1.0, sigma=0.05, A=0.1, B=0.3)
    assert _sweep(L, [q9, q7]) == L.LBM_EINVAL and "velocity set" in L.lbm_last_error()
    for rows in (1, 2, 4, 8, 16):  # the local models take every tile shape, two-step ones included
        assert _sweep(L, [q9], tile_rows=rows) in (L.LBM_OK, L.LBM_EHIP)
    assert _sweep(L, [q9], tile_rows=32) == L.LBM_EINVAL
    q9m = L.make_params(128, 128, L.LBM_MIPS, tau=2.0, rho_star=1.0, lattice=L.LBM_D2Q9)
    for rows in (1, 2, 4):  # D2Q9 MIPS: 8, 16 (two steps per launch) or resident
        assert _sweep(L, [q9m], tile_rows=rows) == L.LBM_EINVAL and "D2Q9" in L.lbm_last_error()
    assert _sweep(L, [q9], tile_rows=L.LBM_TILE_RESIDENT) == L.LBM_EINVAL  # 16384 sites: too large for LDS
    q9h = L.make_params(128, 128, L.LBM_CIL, storage=L.LBM_BF16_DEV, rho_ref=1.0, lattice=L.LBM_D2Q9)
    assert _sweep(L, [q9h]) == L.LBM_EUNSUPPORTED
    assert L._lib.lbm_coarsen(ctypes.byref(q9), ctypes.c_void_p(16), 4, ctypes.c_void_p(32), None) == \
        L.LBM_EUNSUPPORTED
    assert L._lib.lbm_lift(ctypes.byref(q9), ctypes.c_void_p(16), 4, ctypes.c_void_p(32), None) == \
        L.LBM_EUNSUPPORTED


def test_resident_form_validation():
    """LBM_TILE_RESIDENT takes lattices of at most 4096 sites (D2Q7) or 3072
    (D2Q9), any model (the call then reaches the device: a HIP error without
    a GPU); a larger lattice anywhere in the batch is refused before any HIP
    call."""
    import paper_1902_00530_amd as L
    R = L.LBM_TILE_RESIDENT
    small = L.make_params(64, 64, L.LBM_MIPS, tau=2.0, rho_star=1.0)
    big = L.make_params(128, 34, L.LBM_MIPS, tau=2.0, rho_star=1.0)
    assert _sweep(L, [small], tile_rows=R) in (L.LBM_OK, L.LBM_EHIP)
    assert _sweep(L, [L.make_params(90, 30, L.LBM_CIL, A=0.1, B=0.3)], tile_rows=R) in (L.LBM_OK, L.LBM_EHIP)
    assert _sweep(L, [small, big], tile_rows=R) == L.LBM_EINVAL and "4096" in L.lbm_last_error()
    over = L.make_params(2050, 2, L.LBM_CIL, A=0.1, B=0.3)  # 4100 sites, one row pair
    assert _sweep(L, [over], tile_rows=R) == L.LBM_EINVAL
    assert _sweep(L, [L.make_params(2048, 2, L.LBM_CIL, A=0.1, B=0.3)], tile_rows=R) in (L.LBM_OK, L.LBM_EHIP)
    # D2Q9: nine planes and the densities, at most 3072 sites
    q9 = dict(lattice=L.LBM_D2Q9, A=0.1, B=0.3)
    assert _sweep(L, [L.make_params(64, 48, L.LBM_CIL, **q9)], tile_rows=R) in (L.LBM_OK, L.LBM_EHIP)
    assert _sweep(L, [L.make_params(62, 50, L.LBM_CIL, **q9)], tile_rows=R) == L.LBM_EINVAL
    assert _sweep(L, [big], tile_rows=3) == L.LBM_EINVAL and "LBM_TILE_RESIDENT" in L.lbm_last_error()


def test_sweep_groups():
    """The lattice groups a tiled sweep runs each chunk in: the fewest groups
    whose two buffers stay within 240 MiB, in about equal shares of
    consecutive lattices (host logic only, no GPU)."""
    import synth_inputs as SI
    import paper_1902_00530_amd as L

    def groups(plist):
        arr = (L.lbm_params * len(plist))(*plist)
        return L.lbm_sweep_groups(arr, len(plist))
    five = [L.make_params(1024, 1024, L.LBM_CIL, A=0.125, B=0.3, seed=l) for l in range(5)]
    assert groups(five) == 2  # 294 MB of state: 176 + 117 MB
    assert groups(five[:4]) == 1  # 235 MB fits
    assert groups([L.make_params(1024, 1024, L.LBM_CIL, lattice=L.LBM_D2Q9) for _ in range(5)]) == 2
    assert groups([L.make_params(4096, 4096, L.LBM_CIL)]) == 1  # one lattice larger than the budget
    sweep = [L.make_params(c["nx"], c["ny"], c["model"], A=c["A"], B=c["B"]) for c in SI.batch_sweep()]
    assert groups(sweep) == 5
    assert L._lib.lbm_sweep_groups(None, 1) == L.LBM_EINVAL


def test_null_context_is_a_state_error():
    import paper_1902_00530_amd as L
    assert L._lib.lbm_step(None, 1) == L.LBM_ESTATE
    assert L._lib.lbm_moments(None, None, None, None, None) == L.LBM_ESTATE
    assert L._lib.lbm_destroy(None) == L.LBM_ESTATE
    assert L._lib.lbm_current_buffer(None) == L.LBM_ESTATE


def _sweep(L, plist, n_steps=10, every=0, ws_bytes=None, tile_rows=0, use_graph=1):
    n = len(plist)
    arr = (L.lbm_params * n)(*plist)
    bufs = (ctypes.c_void_p * (2 * n))(*[ctypes.c_void_p(16 * (k + 1)) for k in range(2 * n)])
    need = L._lib.lbm_sweep_workspace_bytes(arr, n, max(1, n_steps // every if every else 1))
    opts = L.lbm_sweep_opts(n_steps, every, 0, tile_rows, use_graph)
    out = (L.lbm_obs * (n * 4))()
    return L._lib.lbm_sweep_batch(arr, n, ctypes.byref(opts), bufs, ctypes.c_void_p(64),
                                  need if ws_bytes is None else ws_bytes, None, out)


def test_sweep_batch_rejects_invalid_batches():
    import paper_1902_00530_amd as L
    good = L.make_params(128, 128, L.LBM_CIL, tau=1.0, sigma=0.05, A=0.1, B=0.3)
    assert _sweep(L, [good, L.make_params(128, 128, L.LBM_CIL, tau=2.0, sigma=0.05)]) == L.LBM_EINVAL
    assert "tau" in L.lbm_last_error()
    assert _sweep(L, [good, L.make_params(64, 64, L.LBM_CIL, tau=1.0, sigma=0.0)]) == L.LBM_EINVAL
    mips = L.make_params(128, 128, L.LBM_MIPS, tau=2.0, rho_star=1.0)
    assert _sweep(L, [mips], tile_rows=2) == L.LBM_EINVAL and "MIPS" in L.lbm_last_error()
    mips9 = L.make_params(128, 128, L.LBM_MIPS, tau=2.0, rho_star=1.0, lattice=L.LBM_D2Q9)
    assert _sweep(L, [mips9], tile_rows=4) == L.LBM_EINVAL and "D2Q9 MIPS" in L.lbm_last_error()
    assert _sweep(L, [mips, good]) == L.LBM_EINVAL   # one model per batch
    # 16-bit storages: D2Q7 only, one storage per batch
    assert _sweep(L, [L.make_params(128, 128, L.LBM_CIL, storage=L.LBM_BF16_DEV, lattice=L.LBM_D2Q9)]) == \
        L.LBM_EUNSUPPORTED
    assert _sweep(L, [good, L.make_params(128, 128, L.LBM_CIL, tau=1.0, sigma=0.05, storage=L.LBM_F16_DEV)]) == \
        L.LBM_EINVAL and "storage" in L.lbm_last_error()
    assert _sweep(L, [good, L.make_params(128, 128, L.LBM_PASSIVE, tau=1.0, sigma=0.05)]) == L.LBM_EINVAL
    assert _sweep(L, [good], n_steps=10, every=3) == L.LBM_EINVAL
    assert _sweep(L, [good], ws_bytes=100) == L.LBM_EINVAL
    assert _sweep(L, [L.make_params(128, 127, L.LBM_CIL)]) == L.LBM_EINVAL
    assert _sweep(L, [good], use_graph=3) == L.LBM_EINVAL and "use_graph" in L.lbm_last_error()
    assert _sweep(L, [good], use_graph=-1) == L.LBM_EINVAL
    assert L._lib.lbm_sweep_workspace_bytes(None, 1, 1) == 0


def test_sweep_workspace_grows_with_samples():
    import paper_1902_00530_amd as L
    arr = (L.lbm_params * 2)(L.make_params(128, 128, L.LBM_CIL), L.make_params(256, 192, L.LBM_CIL))
    a = L._lib.lbm_sweep_workspace_bytes(arr, 2, 1)
    b = L._lib.lbm_sweep_workspace_bytes(arr, 2, 100)
    assert 0 < a < b and b - a >= 2 * 99 * 8 * 8 - 256


def test_surrogate_descriptions_and_create_validation():
    """The surrogate object: sizes of its parameter block and workspace, and
    create's checks before any device work (cin 3 or 4, coarse 1 or even,
    k >= 1, 1 <= max_batch <= 65535, 256-byte aligned caller buffers, a large
    enough workspace)."""
    import paper_1902_00530_amd as L
    good = L.lbm_surrogate_desc(4, 32, 32, 8, 50, 64)
    pb, wb = L.lbm_surrogate_param_bytes(good), L.lbm_surrogate_workspace_bytes(good)
    nparam = 32 * 4 * 9 + 32 + 32 * 32 * 9 + 32 + 3 * 32 * 9 + 3
    assert pb >= 3 * nparam * 4 + (32 * 4 * 9 + 32 * 32 * 9 + 3 * 32 * 9) * 2 and pb % 256 == 0
    assert wb >= 64 * (4 + 3 + 32 + 32 + 3 + 3 * 4) * 32 * 32 * 4
    for bad in (L.lbm_surrogate_desc(5, 32, 32, 8, 50, 64), L.lbm_surrogate_desc(4, 32, 32, 3, 50, 64),
                L.lbm_surrogate_desc(4, 32, 32, 8, 0, 64), L.lbm_surrogate_desc(4, 32, 32, 8, 50, 0),
                L.lbm_surrogate_desc(4, 0, 32, 8, 50, 64), L.lbm_surrogate_desc(4, 32, 32, 8, 50, 70000)):
        assert L.lbm_surrogate_param_bytes(bad) == 0 and L.lbm_surrogate_workspace_bytes(bad) == 0
    h = ctypes.c_void_p()
    create = L._lib.lbm_surrogate_create
    assert create(ctypes.byref(L.lbm_surrogate_desc(5, 32, 32, 8, 50, 64)), ctypes.c_void_p(4096), 0, 0,
                  ctypes.c_void_p(8192), wb, None, ctypes.byref(h)) == L.LBM_EINVAL
    assert create(ctypes.byref(good), ctypes.c_void_p(4096 + 4), 0, 0, ctypes.c_void_p(8192), wb, None,
                  ctypes.byref(h)) == L.LBM_EINVAL and "aligned" in L.lbm_last_error()
    assert create(ctypes.byref(good), ctypes.c_void_p(4096), 0, 0, ctypes.c_void_p(8192), wb - 1, None,
                  ctypes.byref(h)) == L.LBM_EINVAL and "workspace" in L.lbm_last_error()
    assert L._lib.lbm_surrogate_train_step(None, None, None, None, 1, ctypes.c_float(1e-3), None) == L.LBM_ESTATE
    assert L._lib.lbm_surrogate_predict(None, None, 1, None) == L.LBM_ESTATE


def test_float32_rest_plane_storage_references_and_validation():
    """LBM_BF16_DEV_R32: the rest population is stored as is (r_0 = 0), the
    moving ones as bfloat16 deviations from w_i rho_ref rounded to bfloat16
    (the references of LBM_BF16_DEV); D2Q7 only; storages past it are
    unknown."""
    import numpy as np
    import paper_1902_00530_amd as L
    p = L.make_params(64, 64, L.LBM_CIL, storage=L.LBM_BF16_DEV_R32, rho_ref=0.74)
    wr = L.lbm_deviation_reference(p)
    wb = L.lbm_deviation_reference(L.make_params(64, 64, L.LBM_CIL, storage=L.LBM_BF16_DEV, rho_ref=0.74))
    assert wr[0] == 0.0 and (wr[1:] == wb[1:]).all()
    # bfloat16-representable: the low 16 bits of the float32 pattern are zero
    assert (wr[1:].view(np.uint32) & 0xFFFF == 0).all() and abs(wr[1] - 0.74 / 12) < 2 ** -8 * 0.74 / 12
    assert L.storage_planes(p) == 8
    q9 = L.make_params(64, 64, L.LBM_CIL, storage=L.LBM_BF16_DEV_R32, rho_ref=0.74, lattice=L.LBM_D2Q9)
    assert L._lib.lbm_deviation_reference(ctypes.byref(q9), (ctypes.c_float * 9)()) == L.LBM_EUNSUPPORTED
    bad = L.make_params(64, 64, L.LBM_CIL, storage=4, rho_ref=0.74)
    assert L._lib.lbm_deviation_reference(ctypes.byref(bad), (ctypes.c_float * 9)()) == L.LBM_EINVAL
    assert "storage" in L.lbm_last_error()
