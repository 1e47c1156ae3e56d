"""Physical-unit front end: phase-field and sharp-interface parameters, vapour supersaturation, and
the conversion of a physical set-up to lattice units (Tan et al., arXiv:2101.07163, Sec. 2.1, 3.2.1).

Host-side parameter arithmetic only; the step itself runs in the HIP library.  The relations:

* capillary length from the material, d0 = gamma T_M c_p / L^2, and from the phase-field parameters,
  d0 = a1 W0 / lambda (matched asymptotics, Sec. 2.1);
* kinetic coefficient beta = a1 (tau0 / (W0 lambda) - a2 W0 / D), which vanishes for
  tau0 = a2 lambda W0^2 / D, i.e. for a vapour diffusivity D = a2 lambda W0^2 / tau0;
* supersaturation of a vapour density over ice, U = (rho - rho_sat^I) / rho_sat^I (Sec. 3.2.1);
* lattice units with grid spacing dx and time step dt: lengths / dx, times / dt, diffusivities and
  viscosities * dt / dx^2, velocities * dt / dx; an LB relaxation time tau = 1/2 + D_lu / cs^2.
"""
from __future__ import annotations

import math

# a1 of the solvability integral for g(phi) = phi - 2 phi^3/3 + phi^5/5 (the printed value 0.8839 is
# 5 sqrt(2)/8 rounded); a2 as printed (Sec. 2.1).
A1 = 5.0 * math.sqrt(2.0) / 8.0
A2 = 0.6267
CS2 = 1.0 / 3.0


def supersaturation(rho: float, rho_sat_ice: float) -> float:
    """U = (rho - rho_sat^I) / rho_sat^I for a vapour density rho (any consistent unit)."""
    if rho_sat_ice <= 0:
        raise ValueError("rho_sat_ice must be > 0")
    return (rho - rho_sat_ice) / rho_sat_ice


def capillary_length_of_material(gamma: float, T_m: float, c_p: float, L: float) -> float:
    """d0 = gamma T_M c_p / L^2 (surface tension, melting temperature, volumetric heat capacity,
    volumetric latent heat; SI units give metres)."""
    return gamma * T_m * c_p / (L * L)


def capillary_length(W0: float, lam: float) -> float:
    """d0 = a1 W0 / lambda."""
    return A1 * W0 / lam


def kinetic_coefficient(tau0: float, W0: float, lam: float, D: float) -> float:
    """beta = a1 (tau0 / (W0 lambda) - a2 W0 / D)."""
    return A1 * (tau0 / (W0 * lam) - A2 * W0 / D)


def diffusivity_for_zero_beta(lam: float, W0: float, tau0: float) -> float:
    """The D that makes beta vanish for given lambda, W0, tau0: D = a2 lambda W0^2 / tau0."""
    return A2 * lam * W0 * W0 / tau0


def relaxation_time(D_lattice: float) -> float:
    """BGK relaxation time of an LB diffusion solver with diffusivity D (lattice units)."""
    if D_lattice <= 0:
        raise ValueError("the diffusivity must be > 0")
    return 0.5 + D_lattice / CS2


def lattice_diffusivity(D: float, dx: float, dt: float) -> float:
    return D * dt / (dx * dx)


def lattice_velocity(u: float, dx: float, dt: float) -> float:
    return u * dt / dx


def plate_regime(U0: float, L_sat: float, n: int = 400, W0: float = 1.25, tau0: float = 20.0, lam: float = 3.0,
                 eps: float = 0.05, seed_r: float = 10.0) -> dict:
    """Lattice set-up of the plate-regime habit runs (Sec. 3.2.1, Table 2): an n x n periodic box
    without flow, W0 = 1.25 dx, tau0 = 20 dt, lambda = 3, eps = 0.05, and the vapour diffusivity that
    makes the kinetic coefficient vanish (the paper fixes W0, tau0 and lambda but not D in lattice
    units).  A circular seed of radius seed_r (width W0) sits at the centre."""
    D = diffusivity_for_zero_beta(lam, W0, tau0)
    return dict(nx=n, ny=n, flow=0, inout=0, n_fold=6, eps=eps, W0=W0, tau0=tau0, lam=lam, L_sat=L_sat,
                tau_vap=relaxation_time(D), tau_f=0.6, h_drag=2.757, kappa_N=1.0, rho0=1.0, u_in=0.0, U_in=0.0,
                grad_eps2=1e-10, U0=U0, seed=(n / 2.0, n / 2.0, seed_r), w_init=W0, stencil=4, symmetric=0)
