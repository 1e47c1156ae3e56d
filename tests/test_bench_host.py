"""Host-side logic of bench.py (CPU only): the one-GPU contract, the algorithmic bytes per update, the
freshness check that ties committed counter summaries to the kernel source, and the tip measurement
of the four-fold set-up."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused_with_a_message(argv, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bytes_per_update():
    # algorithmic: 23 (flow) or 14 populations read and written, phi_prev read and written (FP32)
    assert bench.bytes_per_update(True, "fp32") == 23 * 4 * 2 + 8 == 192
    assert bench.bytes_per_update(False, "fp32") == 14 * 4 * 2 + 8 == 120
    assert bench.bytes_per_update(True, "fp16") == 23 * 2 * 2 + 8 == 100
    assert bench.bytes_per_update(False, "bf16") == 14 * 2 * 2 + 8 == 64
    # this implementation's 16-bit storage also reads and writes the 16-bit references (U, and rho,
    # jx, jy with flow)
    assert bench.impl_bytes_per_update(True, "fp32") == 192
    assert bench.impl_bytes_per_update(True, "fp16") == 100 + 4 * 2 * 2 == 116
    assert bench.impl_bytes_per_update(False, "bf16") == 64 + 1 * 2 * 2 == 68


@pytest.fixture
def tree_copy(tmp_path, monkeypatch):
    """A copy of the kernel sources and profiles that bench's freshness check reads."""
    src = os.path.join(ROOT, "paper_2101_07163_amd", "csrc")
    dst = tmp_path / "paper_2101_07163_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("snowlb_kernels.hip", "snowlb_device.h", "snowlb_internal.h"):
        shutil.copy(os.path.join(src, name), dst / name)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_source_hash_ignores_comments_but_not_code(tree_copy):
    h0 = bench.kernel_source_sha()
    k = tree_copy / "paper_2101_07163_amd" / "csrc" / "snowlb_kernels.hip"
    text = k.read_text()
    k.write_text(text + "\n// a comment only\n\n")
    assert bench.kernel_source_sha() == h0
    k.write_text(text.replace("const int npar = 1 - par;", "const int npar = 1 - par;  // same code"))
    assert bench.kernel_source_sha() == h0
    k.write_text(text + "\nstatic int unused_marker = 0;\n")
    assert bench.kernel_source_sha() != h0


def test_traffic_only_from_a_summary_of_the_current_kernel(tree_copy):
    p = tree_copy / "profiles" / "k_step_wl_fp32_traffic.txt"
    assert bench.load_traffic("wl", "fp32") is None  # no summary
    p.write_text("# counters\nkernel_source_sha: %s\nhbm_bytes_per_launch: 1234.0\n" % bench.kernel_source_sha())
    assert bench.load_traffic("wl", "fp32") == 1234.0
    p.write_text("kernel_source_sha: 0000000000000000\nhbm_bytes_per_launch: 1234.0\n")
    assert bench.load_traffic("wl", "fp32") is None  # taken on another kernel
    # a summary names its launch; another tile shape or grid mode does not use it
    p.write_text("kernel_source_sha: %s\ntile: 64x4\ngrid_mode: 0\nhbm_bytes_per_launch: 99.0\n" % bench.kernel_source_sha())
    assert bench.load_traffic("wl", "fp32", "64x4", 0) == 99.0
    assert bench.load_traffic("wl", "fp32", "64x4", 1) is None
    assert bench.load_traffic("wl", "fp32", "128x2", 0) is None
    assert bench.load_traffic("wl", "fp32", "64x4", 2) is None  # strip order: its own summary
    (tree_copy / "profiles" / "k_step_wl_fp32_strips_traffic.txt").write_text(
        "kernel_source_sha: %s\ntile: 64x4\ngrid_mode: 2\nhbm_bytes_per_launch: 98.0\n" % bench.kernel_source_sha())
    assert bench.load_traffic("wl", "fp32", "64x4", 2) == 98.0


def test_committed_traffic_summary_names_its_kernel_hash():
    p = os.path.join(ROOT, "profiles", "k_step_c3_ventilated_2048_fp32_traffic.txt")
    kv = dict(line.split(":", 1) for line in open(p) if ":" in line and not line.startswith("#"))
    assert len(kv["kernel_source_sha"].strip()) == 16
    assert float(kv["hbm_bytes_per_launch"]) > 0


def test_axis_tip_on_a_tanh_profile():
    x = np.arange(300) - 150.0
    for R in (37.3, 80.0, 101.75):
        phi = np.tile(np.tanh((R - np.abs(x)) / 1.4), (300, 1))
        assert abs(bench.axis_tip(phi, 150, 150) - R) < 0.05
