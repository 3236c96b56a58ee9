"""Host code of libsp2 under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the library with the sanitizers on its host side only (the device
code is unchanged), links tests/host/sanitize_driver.cpp against it and runs
the driver: argument checks, workspace sizes, status strings and the learned
model's create / coefficients / save / load / destroy, including the text
parser on malformed files.  No GPU call is made.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_paths_under_asan_and_ubsan(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_2401_13772_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    lib = tmp_path / "libsp2_san.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san, "-I", inc, "-I", csrc,
                    "-o", str(lib), *srcs], check=True, capture_output=True)
    drv = tmp_path / "driver"
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", *san, "-I", inc, "-x", "c++",
                    os.path.join(HERE, "host", "sanitize_driver.cpp"), "-L", str(tmp_path), "-lsp2_san",
                    f"-Wl,-rpath,{tmp_path}", "-o", str(drv)], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(drv), str(tmp_path)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized host checks passed" in r.stdout
