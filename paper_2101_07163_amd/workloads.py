"""Seeded synthetic workloads for the coupled ice-growth step.

This module holds parameter sets and seeded random draws only -- none of the method's arithmetic.
It is the one module that feeds both the GPU library (through the binding) and the FP64 oracle
(through the tests), so that both see identical inputs.

Every workload is synthetic: a circular ice seed in uniformly supersaturated vapour, optionally
ventilated by a uniform inflow, as in the paper's set-ups (Sec. 3.1.2, 3.1.3, 3.2.1, 3.2.2).  The
paper uses no dataset.  Parameter names follow the paper's symbols (``lam`` is lambda).
"""
from __future__ import annotations

import math

import numpy as np

# Parameters shared by all workloads (lattice units).  W0^2/tau0 = D_vap = 0.1: phase and vapour
# diffusivities equal, as in the stencil study of Sec. 3.1.1 (W0^2/tau0 = kappa there).
# lambda = 3 as in Sec. 3.2.1; L_sat = 1.6 is the most frequent value of Table 2; h = 2.757 (Sec. 2.2.1).
COMMON = dict(
    n_fold=6, eps=0.05, W0=1.0, tau0=10.0, lam=3.0, L_sat=1.6, tau_vap=0.8, tau_f=0.6,
    h_drag=2.757, kappa_N=1.0, rho0=1.0, u_in=0.0, U_in=0.0, grad_eps2=1e-10,
)


def _cfg(**kw):
    d = dict(COMMON)
    d.update(kw)
    return d


# C1: 128^2 periodic, no flow, seed R = 5 at the centre, U0 = 0.5, 2000 steps.
C1 = _cfg(name="c1_plain_128", nx=128, ny=128, flow=0, inout=0, seed=(64.0, 64.0, 5.0), w_init=1.0,
          U0=0.5, steps=2000)

# C2: 1024^2 ventilated: inlet u = 0.02 at x = 0, outlet at x = nx-1, periodic in y,
# tau_f = 0.6, tau_vap = 0.8, inflow U = 0.6, seed R = 8 at (300, 512), 20000 steps.
C2 = _cfg(name="c2_ventilated_1024", nx=1024, ny=1024, flow=1, inout=1, u_in=0.02, U_in=0.6, U0=0.6,
          seed=(300.0, 512.0, 8.0), w_init=1.0, steps=20000)

# C3: 2048^2, C2 physics with u_in = 0.01, seed at (300, 1024); storage fp32 / fp16 / bf16
# deviations; 10000 steps; FP64 comparison on the 512^2 crop [44, 556) x [768, 1280).
C3 = _cfg(name="c3_ventilated_2048", nx=2048, ny=2048, flow=1, inout=1, u_in=0.01, U_in=0.6, U0=0.6,
          seed=(300.0, 1024.0, 8.0), w_init=1.0, steps=10000, crop=((768, 1280), (44, 556)))

# C5: adjoint workload, 512^2 periodic, no flow, seed R = 6 at the centre.
C5 = _cfg(name="c5_adjoint_512", nx=512, ny=512, flow=0, inout=0, seed=(256.0, 256.0, 6.0),
          w_init=1.0, steps=5000, eps_target=0.06, U0_target=0.55, eps_start=0.04, U0_start=0.5,
          U_noise=0.02, rng_seed=2101)
C5["eps"] = C5["eps_start"]
C5["U0"] = C5["U0_start"]

# Stencil study of Sec. 3.1.1 in lattice units: a hexagonal crystal grown by the symmetric thermal
# model on 800^2 with dx = 0.01, dt = 1.5e-5, i.e. W0 = 0.0125/dx = 1.25, tau0 = 1.5625e-4/dt,
# kappa = 1 -> D = kappa dt/dx^2 = 0.15 (tau_vap = 1/2 + 3 D = 0.95, so W0^2/tau0 = D), lambda = 10,
# eps = 0.05, undercooling Delta = 0.3, seed R = 10 at (400, 400), 1e5 steps.  The reduced
# temperature u enters as U = -u (undercooling U0 = Delta) with latent heat L_sat = 1 and the
# diffusivity q = 1 in both phases.  Set "stencil" to 2, 4, 6 or 8.
F1 = _cfg(name="f1_stencil_study_800", nx=800, ny=800, flow=0, inout=0, W0=1.25, tau0=1.5625e-4 / 1.5e-5,
          tau_vap=0.95, lam=10.0, eps=0.05, L_sat=1.0, U0=0.3, symmetric=1, stencil=4,
          seed=(400.0, 400.0, 10.0), w_init=1.25, steps=100000)

# The four-fold validation set-up of Sec. 3.1.2 in lattice units: W0 = tau0 = 1 with dx = 0.4 W0 and
# dt = 0.008 tau0, i.e. W0 = 2.5, tau0 = 125 (W0^2/tau0 = 0.05); kappa = 4 -> D = 4 dt/dx^2 = 0.2
# (tau_vap = 1/2 + 3 D = 1.1); lambda = tau0 kappa / (a2 W0^2) = 6.3826 in the set-up's own units, which
# makes the kinetic coefficient vanish; eps = 0.05 with four-fold symmetry; the symmetric thermal model
# (q = 1, L_sat = 1, undercooling U0); seed R = 10 at the centre with interface width W0.  U0 = 0.3
# runs on 1000^2 for 1.3e5 steps, U0 = 0.55 on 500^2 (run length not stated; 1.8e4 steps, 144 tau0,
# bring its tips to about 185 cells, inside the box).  The dimensionless tip velocity is V d0 / D
# with d0 = a1 W0 / lambda, all in lattice units.
FOURFOLD = _cfg(name="f1_fourfold_1000", nx=1000, ny=1000, flow=0, inout=0, n_fold=4, W0=2.5, tau0=125.0,
                tau_vap=1.1, lam=4.0 / 0.6267, eps=0.05, L_sat=1.0, U0=0.3, symmetric=1, stencil=4,
                seed=(500.0, 500.0, 10.0), w_init=2.5, steps=130000)
FOURFOLD_055 = dict(FOURFOLD, name="f1_fourfold_500", nx=500, ny=500, U0=0.55, seed=(250.0, 250.0, 10.0),
                    steps=18000)


# Table 2 (Sec. 3.2.1): the seven plate-regime morphologies, (number, name, U0, L_sat).  The lattice
# set-up of each row is units.plate_regime(U0, L_sat).
TABLE2 = (
    (1, "solid plate", 0.4, 2.0),
    (2, "stellar plate I", 0.5, 1.8),
    (3, "sectored plate", 0.5, 1.6),
    (4, "stars", 0.6, 1.0),
    (5, "fern dendrite", 0.8, 1.6),
    (6, "fernlike stellar", 0.7, 1.6),
    (7, "stellar plate II", 0.5, 1.2),
)

SIDES = (256, 384, 512, 768, 1024)


def c4_domains(n: int = 64, seed: int = 7163, side_choices=SIDES) -> list[dict]:
    """C4: ``n`` independent ventilated crystals of uneven size and growth conditions.

    side ~ U{256..1024}, eps ~ U[0.02, 0.08], U0 ~ U[0.2, 0.9], u_in ~ U[0, 0.02], U_in = U0,
    seed radius 6 at the domain centre, inflow/outflow in x.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        side = int(rng.choice(side_choices))
        eps = float(rng.uniform(0.02, 0.08))
        U0 = float(rng.uniform(0.2, 0.9))
        u_in = float(rng.uniform(0.0, 0.02))
        out.append(_cfg(name="c4_%02d" % i, nx=side, ny=side, flow=1, inout=1, eps=eps, U0=U0,
                        U_in=U0, u_in=u_in, seed=(side / 2.0, side / 2.0, 6.0), w_init=1.0,
                        steps=5000))
    return out


def c5_U_init(cfg: dict = C5) -> np.ndarray:
    """Gaussian-perturbed initial supersaturation U0 + sigma * xi, xi ~ N(0, 1) i.i.d. per cell."""
    rng = np.random.default_rng(cfg["rng_seed"])
    xi = rng.standard_normal((cfg["ny"], cfg["nx"]))
    return cfg["U0"] + cfg["U_noise"] * xi


def random_state(nx: int, ny: int, seed: int, flow: bool = True, amp: float = 0.02,
                 n_blobs: int = 3, well_conditioned: bool = False) -> dict:
    """A seeded, smooth, arbitrary population state [q, y, x] (float64) for one-step parity tests.

    The phase populations are spread around a few smooth blobs (values in [-1, 1]) so that the
    gradient, the anisotropy and the Walsh term are all exercised; flow and vapour populations are
    positive values with small smooth and random parts (the flow base is a fluid near rest).  Any
    state is a legal input of the step; nothing here evaluates the method.

    ``well_conditioned``: the blobs' tails are cut to exactly -1 and the bulk carries no noise, so
    the phase field is either exactly uniform or has gradients well above rounding level (the
    direction of a tiny gradient is ill-conditioned, which amplifies input differences of one ulp).
    """
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    s = -np.ones((ny, nx))
    for _ in range(n_blobs):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        R = rng.uniform(2.0, max(3.0, min(nx, ny) / 4))
        r = np.hypot(x - cx, y - cy)
        s = np.maximum(s, np.tanh((R - r) / math.sqrt(2.0)))
    bulk = np.zeros_like(s, dtype=bool)
    if well_conditioned:
        bulk = s < -1.0 + 1e-3
        s = np.where(bulk, -1.0, s)
    share9 = rng.uniform(0.5, 1.5, size=9)
    share9 /= share9.sum()
    h = share9[:, None, None] * s[None] + np.where(bulk, 0.0, amp * 0.1 * rng.standard_normal((9, ny, nx)))
    U = 0.3 + 0.2 * np.sin(2 * math.pi * x / nx) * np.cos(2 * math.pi * y / ny)
    share5 = rng.uniform(0.5, 1.5, size=5)
    share5 /= share5.sum()
    g = share5[:, None, None] * U[None] * (1 + amp * rng.standard_normal((5, ny, nx)))
    phip = s + np.where(bulk, 0.0, amp * rng.standard_normal((ny, nx)))
    out = {"g": g, "h": h, "phip": phip}
    if flow:
        base = np.array([16, 4, 4, 4, 4, 1, 1, 1, 1], dtype=np.float64) / 36.0
        f = base[:, None, None] * (1.0 + 0.05 * np.sin(2 * math.pi * (x + 2 * y) / nx)[None]
                                   + amp * rng.standard_normal((9, ny, nx)))
        out["f"] = f
    return out


def random_state3d(nx: int, ny: int, nz: int, seed: int, flow: bool = True, amp: float = 0.02,
                   n_blobs: int = 3) -> dict:
    """A seeded, smooth, arbitrary 3D population state [q, z, y, x] (float64) for one-step parity
    tests of the 3D step: phase populations spread around a few smooth balls (values in [-1, 1]) with
    random shares, the exterior exactly -1 without noise (no gradients at rounding level); vapour and
    flow populations positive with small smooth and random parts (the flow near rest).  Any state is a
    legal input of the step; nothing here evaluates the method."""
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    s = -np.ones((nz, ny, nx))
    for _ in range(n_blobs):
        c = rng.uniform(0, 1, 3) * (nx, ny, nz)
        R = rng.uniform(1.5, max(2.5, min(nx, ny, nz) / 3))
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        s = np.maximum(s, np.tanh((R - r) / math.sqrt(2.0)))
    bulk = s < -1.0 + 1e-3
    s = np.where(bulk, -1.0, s)
    share7 = rng.uniform(0.5, 1.5, size=7)
    share7 /= share7.sum()
    h = share7[:, None, None, None] * s[None] + np.where(bulk, 0.0, amp * 0.1 * rng.standard_normal((7,) + s.shape))
    U = 0.3 + 0.2 * np.sin(2 * math.pi * x / nx) * np.cos(2 * math.pi * y / ny) * np.cos(2 * math.pi * z / nz)
    share7g = rng.uniform(0.5, 1.5, size=7)
    share7g /= share7g.sum()
    g = share7g[:, None, None, None] * U[None] * (1 + amp * rng.standard_normal((7,) + s.shape))
    phip = s + np.where(bulk, 0.0, amp * rng.standard_normal(s.shape))
    out = {"g": g, "h": h, "phip": phip}
    if flow:
        base = np.array([12.0] + [2.0] * 6 + [1.0] * 12) / 36.0
        out["f"] = base[:, None, None, None] * (1.0 + 0.05 * np.sin(2 * math.pi * (x + 2 * y + 3 * z) / nx)[None]
                                                + amp * rng.standard_normal((19,) + s.shape))
    return out


# F4: the three-dimensional extension (Sec. 4 proposes it).  A ventilated crystal on 256 x 128 x 128
# (4.2M cells, as many as the 2048^2 workload): inlet u = 0.01 at x = 0, outlet at x = 255, periodic y
# and z, the 2048^2 workload's physics otherwise, spherical seed R = 8 at (80, 64, 64).
F4_3D = dict(COMMON, name="f4_ventilated_3d_256x128x128", nx=256, ny=128, nz=128, flow=1, inout=1, u_in=0.01,
             U_in=0.6, U0=0.6, seed=(80.0, 64.0, 64.0, 8.0), w_init=1.0, steps=2000)
