"""The stored oracle crops used by the full-length GPU parity tests: shape, provenance fields and
physical ranges (CPU only; the values themselves are written by tests/golden/make_oracle_crop.py,
which calls only the oracle)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

import make_oracle_crop as M  # noqa: E402


@pytest.mark.parametrize("name", sorted(M.CASES))
def test_stored_crop_matches_its_recipe(name):
    cfg, ((r0, r1), (c0, c1)), fname = M.CASES[name]
    d = np.load(os.path.join(ROOT, "tests", "golden", fname))
    assert int(d["steps"]) == cfg["steps"]
    assert list(d["rows"]) == [r0, r1] and list(d["cols"]) == [c0, c1]
    sx, sy = cfg["seed"][:2]
    assert r0 <= sy < r1 and c0 <= sx < c1  # the crop holds the crystal's seed
    for k in ("phi", "U", "rho", "ux", "uy"):
        a = d[k]
        assert a.shape == (r1 - r0, c1 - c0) and a.dtype == np.float32 and np.isfinite(a).all(), k
    phi = d["phi"]
    assert phi.min() >= -1.0 - 1e-3 and phi.max() <= 1.0 + 1e-3
    assert (phi > 0).sum() > 100  # a grown crystal inside the crop
    assert abs(float(d["rho"].mean()) - cfg["rho0"]) < 1e-2
    assert 0.0 < float(d["ux"].max()) < 0.1  # inflow-driven, low Mach


def test_stored_adjoint_matches_its_recipe():
    """The oracle's discrete adjoint of the 512^2 adjoint workload (tests/golden/make_oracle_adjoint.py):
    shapes, the run length, a grown target shape, and the identity dL/dU0 = sum dL/dU_init."""
    import make_oracle_adjoint as A
    from paper_2101_07163_amd import workloads as W
    d = np.load(A.OUT)
    cfg = W.C5
    assert int(d["steps"]) == cfg["steps"]
    assert d["target"].shape == (cfg["ny"], cfg["nx"]) and d["target"].dtype == np.float64
    assert d["dU"].shape == (cfg["ny"], cfg["nx"]) and d["dU"].dtype == np.float32
    assert np.isfinite(d["dU"]).all() and np.isfinite(d["target"]).all()
    assert (d["target"] > 0).sum() > 1000  # the target crystal grew well beyond the seed
    assert float(d["L"]) > 0
    assert abs(float(d["dU"].astype(np.float64).sum()) / float(d["dU0"]) - 1) < 1e-6
