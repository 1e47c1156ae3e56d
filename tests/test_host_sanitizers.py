"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the library is
rebuilt with host-side instrumentation only (device code is not instrumented) and driven from C
through its CPU-reachable paths, including context and batch creation failing for lack of a
device, so that their error and clean-up paths run too."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2101_07163_amd", "csrc")
SOURCES = ["snowlb_kernels.hip", "snowlb_io.hip", "snowlb_adjoint.hip", "snowlb_api.cpp"]


@pytest.mark.slow
def test_host_paths_clean_under_sanitizers(tmp_path):
    if not shutil.which("hipcc") or not shutil.which("clang"):
        pytest.skip("hipcc / clang not available")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("the creation checks expect no visible device")
    except ImportError:
        pass
    lib = tmp_path / "libsnowlb_asan.so"
    subprocess.check_call(
        ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]
        + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", str(lib)],
        stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    exe = tmp_path / "drv"
    subprocess.check_call(["clang", "-g", "-fsanitize=address,undefined", "-I" + os.path.join(ROOT, "include"),
                           os.path.join(HERE, "asan_driver.c"), "-o", str(exe), "-L" + str(tmp_path),
                           "-lsnowlb_asan", "-Wl,-rpath," + str(tmp_path)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out
    assert "stencil 3: -1 stencil must be 2, 4, 6 or 8" in out
    assert "create valid (no GPU): -3 ctx=(nil)" in out
    assert "batch mixed: -1" in out and "batch valid (no GPU): -3" in out
