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


def test_stored_3d_box_matches_its_recipe():
    """The 3D oracle's fields after the full 3D workload (tests/golden/make_oracle3d_crop.py): the run
    length, a box inside the lattice that holds the seed and every cell of the crystal (phi > -0.9)
    with the stated margin, float32 fields of the box's shape, a grown crystal and an inflow-driven
    velocity."""
    import make_oracle3d_crop as C
    from paper_2101_07163_amd import workloads as W
    cfg = W.F4_3D
    d = np.load(C.OUT)
    assert int(d["steps"]) == cfg["steps"]
    (z0, z1), (y0, y1), (x0, x1) = (tuple(int(v) for v in r) for r in d["box"])
    assert 0 <= z0 < z1 <= cfg["nz"] and 0 <= y0 < y1 <= cfg["ny"] and 0 <= x0 < x1 <= cfg["nx"]
    sx, sy, sz = cfg["seed"][:3]
    assert x0 <= sx < x1 and y0 <= sy < y1 and z0 <= sz < z1
    for k in ("phi", "U", "ux"):
        a = d[k]
        assert a.shape == (z1 - z0, y1 - y0, x1 - x0) and a.dtype == np.float32 and np.isfinite(a).all(), k
    phi = d["phi"]
    inside = phi > -0.9
    assert inside.sum() > 1000  # grown from the R = 8 seed (about 2100 cells)
    zs, ys, xs = np.nonzero(inside)
    for lo, hi, n in ((zs.min(), zs.max(), phi.shape[0]), (ys.min(), ys.max(), phi.shape[1]), (xs.min(), xs.max(), phi.shape[2])):
        assert lo == C.PAD and hi == n - 1 - C.PAD  # the crystal plus the margin, nothing clipped
    assert 0.0 < float(d["ux"].max()) < 0.1


def test_stored_oracle_spreads_match_their_recipe():
    """The oracle's own phase-field spread under one-ulp noise per value and step
    (tests/golden/make_oracle_spread.py): the recorded noise recipe, spreads that grow with the run
    length, and for the 64-crystal sweep members whose stored boxes, parameters and fields agree with
    the sweep's draws (members are stored as the script reaches them)."""
    import json

    import make_oracle_spread as P
    from paper_2101_07163_amd import workloads as W
    d = json.load(open(P.JSON))
    for case in ("v512", "c2"):
        c = d[case]
        assert c["sigma_per_step"] == P.SIGMA and c["every"] == P.EVERY
        steps = sorted(int(k) for k in c["spread_phi"])
        vals = [c["spread_phi"][str(k)] for k in steps]
        assert all(0 < a < b for a, b in zip(vals, vals[1:])), (case, vals)
    if "c3" in d:
        assert 0 < d["c3"]["spread_phi"]["10000"] < 1e-2
    if "c4" in d:
        cfgs = W.c4_domains()
        arrays = np.load(P.C4_NPZ)
        for m in d["c4"]["members"]:
            i = m["i"]
            cfg = cfgs[i]
            assert m["nx"] == cfg["nx"] and abs(m["eps"] - cfg["eps"]) < 1e-12 and abs(m["U0"] - cfg["U0"]) < 1e-12
            (r0, r1), (c0, c1) = m["box"]
            assert list(arrays["box_%d" % i]) == [r0, r1, c0, c1]
            for k in ("phi", "U"):
                a = arrays["%s_%d" % (k, i)]
                assert a.shape == (r1 - r0, c1 - c0) and a.dtype == np.float32 and np.isfinite(a).all()
            assert m["spread_phi"] > 0
            if m["spread_phi"] > 1e-2:  # the chaotic members also carry their crystal areas
                assert m["area_ref"] == int((arrays["phi_%d" % i] > 0).sum()) and m["area_perturbed"] > 0
