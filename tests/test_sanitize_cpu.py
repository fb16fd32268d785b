"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, gcc) and driven through every routine on small lattices
(tests/sanitize/oracle_main.c): no out-of-bounds access, leak, or undefined
behaviour, and a clean exit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    srcs = [os.path.join(ROOT, "oracle", "lbm_oracle.c"), os.path.join(ROOT, "oracle", "lbm_oracle_q9.c"),
            os.path.join(ROOT, "tests", "sanitize", "oracle_main.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", exe, *srcs, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_address_sanitizer(tmp_path):
    """The library built with AddressSanitizer on its host code (device code
    unchanged), driven with no GPU through argument validation, workspace
    layouts, lattice groups, batch checks and the surrogate handle's checks
    (tests/sanitize/runtime_main.cpp): every call returns a code or a size,
    with no memory error or leak."""
    import concurrent.futures as cf
    import glob
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1902_00530_amd", "csrc", "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *common, "-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "liblbm_asan.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-o", lib, *objs], check=True, capture_output=True)
    exe = str(tmp_path / "runtime_asan")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-I",
                    os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "runtime_main.cpp"),
                    "-L" + str(tmp_path), "-llbm_asan", "-Wl,-rpath," + str(tmp_path), "-o", exe], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime sanitizer run: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr
