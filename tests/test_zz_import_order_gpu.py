"""The binding works when it is imported before torch: a fresh interpreter
imports the package first and runs one step (one HIP runtime per process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_package_imported_before_torch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    code = ("import paper_1902_00530_amd as L\n"
            "lat = L.Lattice(L.make_params(64, 8, L.LBM_CIL, A=0.125, B=0.3, sigma=0.01),"
            " init=L.make_init(mode=1, rho_mean=0.7))\n"
            "lat.step(3)\n"
            "o = lat.observables()\n"
            "assert o['step'] == 3 and o['nonfinite'] == 0\n"
            "print('ok', o['M'])\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-2000:]
