"""Parameter relations of the phase-field model (Tan et al., arXiv:2101.07163, Sec. 2.1, 3.1.2, 3.2).

TEST INFRASTRUCTURE ONLY (part of the oracle package).  Plain closed forms that map between
phase-field parameters (W0, tau0, lambda, D) and sharp-interface ones (capillary length d0, kinetic
coefficient beta), the supersaturation of a vapour density, and physical -> lattice units.
"""
from __future__ import annotations

import math

# Matched-asymptotics constants for g(phi) = phi - 2 phi^3/3 + phi^5/5 (Sec. 2.1).  a1 follows from
# the solvability integral of a flat front, a1 = 5 sqrt(2)/8; a2 is the printed value.
A1 = 5.0 * math.sqrt(2.0) / 8.0
A2 = 0.6267
# Excess free-energy integral of the tanh profile, gamma0 = I W0 H (Sec. 2.1).
I_TANH = 2.0 * math.sqrt(2.0) / 3.0


def capillary_length(W0: float, lam: float) -> float:
    """d0 = a1 W0 / lambda."""
    return A1 * W0 / lam


def kinetic_coefficient(tau0: float, W0: float, lam: float, D: float) -> float:
    """beta = a1 (tau0 / (W0 lambda) - a2 W0 / D)."""
    return A1 * (tau0 / (W0 * lam) - A2 * W0 / D)


def tau0_for_zero_beta(lam: float, W0: float, D: float) -> float:
    """tau0 = a2 lambda W0^2 / D makes beta vanish."""
    return A2 * lam * W0 * W0 / D


def lambda_for_zero_beta(tau0: float, W0: float, D: float) -> float:
    """lambda = tau0 D / (a2 W0^2) makes beta vanish."""
    return tau0 * D / (A2 * W0 * W0)


def capillary_length_material(gamma: float, T_m: float, c_p: float, L: float) -> float:
    """Thermal capillary length d0 = gamma T_M c_p / L^2 (Sec. 2.1)."""
    return gamma * T_m * c_p / (L * L)


def supersaturation(rho: float, rho_sat_ice: float) -> float:
    """U = (rho - rho_sat^I) / rho_sat^I (Sec. 3.2.1)."""
    return (rho - rho_sat_ice) / rho_sat_ice


def lattice_velocity(u: float, dx: float, dt: float) -> float:
    return u * dt / dx


def lattice_viscosity(nu: float, dx: float, dt: float) -> float:
    return nu * dt / (dx * dx)
