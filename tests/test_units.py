"""The physical-unit front end (paper_2101_07163_amd.units) against the numbers the paper prints
(tests/golden/paper_numbers.json) and the oracle package's own sharp-interface relations (CPU only)."""
import json
import math
import os

import pytest

from oracle import sharp_interface as si
from paper_2101_07163_amd import units, workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NUMS = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))


def test_asymptotic_constants():
    a = NUMS["asymptotics"]
    assert abs(units.A1 - a["a1"]) < 5e-5 and units.A2 == a["a2"]


def test_supersaturation_of_table2_densities():
    pr = NUMS["plate_regime"]
    for row in pr["table2"]:
        assert abs(units.supersaturation(row["rho0"], pr["rho_sat_I"]) - row["U0"]) < 1e-12
    with pytest.raises(ValueError):
        units.supersaturation(1.0, 0.0)


def test_table2_rows_match_the_paper():
    rows = NUMS["plate_regime"]["table2"]
    assert [(r["nr"], r["shape"], r["U0"], r["L_sat"]) for r in rows] == list(W.TABLE2)


def test_capillary_lengths():
    m = NUMS["plate_regime"]["material"]
    d0 = units.capillary_length_of_material(m["gamma"], m["T_m"], m["c_p"], m["L"])
    assert abs(d0 - si.capillary_length_material(m["gamma"], m["T_m"], m["c_p"], m["L"])) < 1e-24
    assert 2.6e-9 < d0 < 2.7e-9   # printed as "about 2 nm"
    assert abs(units.capillary_length(1.25, 3.0) - si.capillary_length(1.25, 3.0)) < 1e-15


def test_zero_kinetic_coefficient():
    """beta vanishes for D = a2 lambda W0^2 / tau0; the validation set-up of Sec. 3.1.2 (W0 = tau0 = 1,
    lambda = 6.3826) recovers its kappa = 4."""
    for lam, W0, tau0 in ((3.0, 1.25, 20.0), (6.3826, 1.0, 1.0), (10.0, 1.25, 10.4)):
        D = units.diffusivity_for_zero_beta(lam, W0, tau0)
        assert abs(units.kinetic_coefficient(tau0, W0, lam, D)) < 1e-13
        assert abs(si.kinetic_coefficient(tau0, W0, lam, D)) < 1e-13
        assert abs(si.tau0_for_zero_beta(lam, W0, D) - tau0) < 1e-12 * tau0
    v = NUMS["four_fold_validation"]
    assert abs(units.diffusivity_for_zero_beta(v["lambda"], v["W0"], v["tau0"]) - v["kappa"]) < 1e-4


def test_plate_regime_setup():
    """Table 2 runs in lattice units: W0 = 1.25, tau0 = 20, lambda = 3, eps = 0.05 on 400^2, with the
    vapour relaxation time of the zero-beta diffusivity, tau = 1/2 + 3 D."""
    c = units.plate_regime(0.5, 1.6)
    D = si.A2 * 3.0 * 1.25 ** 2 / 20.0
    assert abs(c["tau_vap"] - (0.5 + 3.0 * D)) < 1e-14
    assert (c["nx"], c["ny"], c["W0"], c["tau0"], c["lam"], c["eps"]) == (400, 400, 1.25, 20.0, 3.0, 0.05)
    assert (c["U0"], c["L_sat"], c["flow"], c["symmetric"]) == (0.5, 1.6, 0, 0)
    with pytest.raises(ValueError):
        units.relaxation_time(0.0)


def test_lattice_conversions():
    # Sec. 3.1.3: u = 1 with dx = 0.4, dt = 0.008 is 0.02 in lattice units
    assert abs(units.lattice_velocity(1.0, 0.4, 0.008) - si.lattice_velocity(1.0, 0.4, 0.008)) < 1e-15
    assert abs(units.lattice_diffusivity(1.152e-6, 4.8e-6, 2e-7) - si.lattice_viscosity(1.152e-6, 4.8e-6, 2e-7)) < 1e-15
    assert abs(units.lattice_diffusivity(1.0, 0.01, 1.5e-5) - 0.15) < 1e-12   # the stencil study's kappa
