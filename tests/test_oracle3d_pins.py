"""Pins of the three-dimensional FP64 oracle (CPU only) against what the mathematics fixes:
lattice identities of D3Q19 and D3Q7, exactness and the isotropic error term of the gradient
stencil, the anisotropy against an independent polynomial form and the 2D oracle in the basal plane,
closed-form decay of a shear wave and a Taylor-Green vortex, Gaussian advection-diffusion, the kinetic
speed of flat fronts along the basal and the c axis, exact invariants and mirror symmetry.  The 3D
method extends the paper's 2D one (Sec. 2.2) as its Sec. 4 proposes; the readings are T1-T5 of
oracle/snow_oracle3d.c."""
import math

import numpy as np
import pytest

import oracle
from oracle import sharp_interface as si

C19, W19, W7 = oracle.lattice3()


def params(**kw):
    p = oracle.Params3D()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def uniform_phase(shape, phi=-1.0):
    return W7[:, None, None, None] * phi * np.ones((7,) + shape)


def test_lattice_identities():
    """D3Q19: sum w = 1, sum w c = 0, sum w c c = I/3, fourth-order isotropy (sum w c_x^4 = 3 sum w
    c_x^2 c_y^2 = 1/3); D3Q7 (its first seven velocities): sum w = 1, sum w c = 0, sum w c c = I/4."""
    c = C19.astype(float)
    assert abs(W19.sum() - 1) < 1e-15 and np.abs(W19 @ c).max() < 1e-15
    assert np.abs(np.einsum("q,qi,qj->ij", W19, c, c) - np.eye(3) / 3).max() < 1e-15
    assert abs((W19 * c[:, 0] ** 4).sum() - 1 / 3) < 1e-15
    assert abs((W19 * c[:, 0] ** 2 * c[:, 1] ** 2).sum() - 1 / 9) < 1e-15
    assert abs((W19 * c[:, 1] ** 2 * c[:, 2] ** 2).sum() - 1 / 9) < 1e-15
    c7 = c[:7]
    assert abs(W7.sum() - 1) < 1e-15 and np.abs(W7 @ c7).max() < 1e-15
    assert np.abs(np.einsum("q,qi,qj->ij", W7, c7, c7) - np.eye(3) / 4).max() < 1e-15
    # the 19 velocities are distinct and closed under c -> -c
    assert len({tuple(v) for v in C19}) == 19 and all(tuple(-v) in {tuple(u) for u in C19} for v in C19)


def test_equilibrium_moments():
    """sum f_eq = rho, sum c f_eq = rho u, sum c c f_eq = rho (I/3 + u u); sum g_eq = U, sum c g_eq = U u."""
    rho, u, U = 1.03, np.array([0.02, -0.013, 0.007]), 0.61
    f = oracle.feq3(rho, *u)
    c = C19.astype(float)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(f @ c - rho * u).max() < 1e-16
    assert np.abs(np.einsum("q,qi,qj->ij", f, c, c) - rho * (np.eye(3) / 3 + np.outer(u, u))).max() < 1e-15
    g = oracle.geq3(U, *u)
    assert abs(g.sum() - U) < 1e-15 and np.abs(g @ c[:7] - U * u).max() < 1e-16


def _poly_field(fn, n=12):
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    return x, y, z, fn(x, y, z)


def test_gradient_exact_on_quadratics_and_isotropic_on_cubics():
    """The 3D stencil (w = 1/6 on the axes, 1/12 on the face diagonals) is exact on linear and
    quadratic fields and, being fourth-order isotropic, errs on cubics by exactly (A/2) grad(lap phi)
    with A = sum w c_x^2 c_y^2 = 1/3 (interior cells; the lattice is periodic)."""
    p = params(nx=12, ny=12, nz=12)
    inner = (slice(2, -2),) * 3
    x, y, z, phi = _poly_field(lambda x, y, z: 0.3 * x - 0.2 * y + 0.1 * z + 0.01 * x * y - 0.02 * y * z
                               + 0.015 * x * x - 0.005 * z * z)
    g = oracle.grad3(p, phi)
    want = (0.3 + 0.01 * y + 0.03 * x, -0.2 + 0.01 * x - 0.02 * z, 0.1 - 0.02 * y - 0.01 * z)
    for a, b in zip(g, want):
        assert np.abs(a[inner] - b[inner]).max() < 1e-13
    x, y, z, phi = _poly_field(lambda x, y, z: 1e-3 * (x ** 3 + 2 * x * y * z - y ** 2 * z + 0.5 * z ** 3))
    g = oracle.grad3(p, phi)
    # exact gradient and grad(lap phi): lap phi = 1e-3 (6x - 2z + 3z) = 1e-3 (6x + z)
    exact = (1e-3 * (3 * x * x + 2 * y * z), 1e-3 * (2 * x * z - 2 * y * z), 1e-3 * (2 * x * y - y * y + 1.5 * z * z))
    glap = (6e-3, 0.0, 1e-3)
    for a, b, l in zip(g, exact, glap):
        assert np.abs(a[inner] - b[inner] - l / 6).max() < 1e-13


def _a_poly(eps, g):
    """The hexagonal anisotropy as a polynomial in the normal (complex-safe), a form independent of the
    oracle's trigonometric one: 1 + eps Re((n_x + i n_y)^6), n = g/|g|."""
    gx, gy, gz = g
    G2 = gx * gx + gy * gy + gz * gz
    re6 = gx ** 6 - 15 * gx ** 4 * gy ** 2 + 15 * gx ** 2 * gy ** 4 - gy ** 6
    return 1 + eps * re6 / G2 ** 3


@pytest.mark.parametrize("kappa_N", [1.0, 2.0])
def test_anisotropy_against_polynomial_form_and_complex_step(kappa_N):
    """a equals 1 + eps Re((n_x + i n_y)^6) (reading T3), and the flux N equals
    kappa_N (W0^2/tau0) |g|^2 a da/dg with da/dg from a complex-step derivative of that polynomial."""
    p = params(eps=0.07, W0=1.3, tau0=8.0, kappa_N=kappa_N)
    rng = np.random.default_rng(4)
    for _ in range(200):
        g = rng.standard_normal(3) * 10 ** rng.uniform(-3, 0)
        a, *N = oracle.aniso3(p, *g)
        assert abs(a - _a_poly(p.eps, g)) < 1e-14
        h = 1e-30 * np.linalg.norm(g)
        dadg = np.array([(_a_poly(p.eps, g + 1j * h * e)).imag / h for e in np.eye(3)])
        want = kappa_N * p.W0 ** 2 / p.tau0 * (g @ g) * a * dadg
        assert np.abs(np.array(N) - want).max() <= 1e-12 * max(1e-12, np.abs(want).max())


def test_anisotropy_reduces_to_the_paper_in_the_basal_plane():
    """For a normal in the basal plane (g_z = 0) the 3D anisotropy and flux are the 2D oracle's
    a = 1 + eps cos 6 theta and N (Sec. 2.1, Eq. (e)), with N_z = 0; along the c axis a = 1 and N = 0;
    a is invariant under 60-degree rotations about z and under the mirrors."""
    p3 = params(eps=0.05, kappa_N=1.0)
    p2 = oracle.Params(eps=0.05, kappa_N=1.0, n_fold=6)
    rng = np.random.default_rng(5)
    for _ in range(100):
        gx, gy = rng.standard_normal(2) * 0.3
        a3, Nx3, Ny3, Nz3 = oracle.aniso3(p3, gx, gy, 0.0)
        a2, Nx2, Ny2 = oracle.aniso(p2, gx, gy)
        assert abs(a3 - a2) < 1e-14 and abs(Nx3 - Nx2) < 1e-14 and abs(Ny3 - Ny2) < 1e-14 and Nz3 == 0.0
        gz = rng.standard_normal() * 0.3
        a, *_ = oracle.aniso3(p3, gx, gy, gz)
        c, s = math.cos(math.pi / 3), math.sin(math.pi / 3)
        assert abs(oracle.aniso3(p3, c * gx - s * gy, s * gx + c * gy, gz)[0] - a) < 1e-14
        for sg in ((-gx, gy, gz), (gx, -gy, gz), (gx, gy, -gz), (-gx, -gy, -gz)):
            assert abs(oracle.aniso3(p3, *sg)[0] - a) < 1e-14
    assert oracle.aniso3(p3, 0.0, 0.0, 0.4) == (1.0, 0.0, 0.0, 0.0)
    assert oracle.aniso3(p3, 1e-6, 0.0, 0.0) == (1.0, 0.0, 0.0, 0.0)  # below the threshold


def _flow_state(ux, uy, uz, rho=None):
    shape = ux.shape
    rho = np.ones(shape) if rho is None else rho
    c = C19.astype(float)
    cu = np.einsum("qk,kzyx->qzyx", c, np.stack([ux, uy, uz]))
    uu = (ux * ux + uy * uy + uz * uz)[None]
    return W19[:, None, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def test_shear_wave_and_taylor_green_decay():
    """Pure fluid (phi = -1): a shear wave u_x = U0 sin(k z) decays as exp(-nu k^2 t) and a z-uniform
    Taylor-Green vortex as exp(-2 nu k^2 t) (energy at twice the rate), nu = (tau_f - 1/2)/3 (D3Q19)."""
    tau = 0.65
    nu = (tau - 0.5) / 3
    n = 64
    z, y, x = np.mgrid[0:n, 0:4, 0:4].astype(float)
    k = 2 * np.pi / n
    p = params(nx=4, ny=4, nz=n, flow=1, tau_f=tau)
    o = oracle.Oracle3D(p)
    f = _flow_state(0.01 * np.sin(k * z), 0 * z, 0 * z)
    o.set_state(f=f, g=np.zeros((7,) + z.shape), h=uniform_phase(z.shape), phip=-np.ones(z.shape))
    amps = []
    for t in (200, 1200):
        o.step(t - o.step_count)
        amps.append(np.abs(o.fields()["ux"]).max())
    rate = -math.log(amps[1] / amps[0]) / 1000
    assert abs(rate / (nu * k * k) - 1) < 2e-3
    n = 32
    k = 2 * np.pi / n
    z, y, x = np.mgrid[0:4, 0:n, 0:n].astype(float)
    p = params(nx=n, ny=n, nz=4, flow=1, tau_f=tau)
    o = oracle.Oracle3D(p)
    f = _flow_state(-0.01 * np.cos(k * x) * np.sin(k * y), 0.01 * np.sin(k * x) * np.cos(k * y), 0 * x)
    o.set_state(f=f, g=np.zeros((7,) + x.shape), h=uniform_phase(x.shape), phip=-np.ones(x.shape))
    E = []
    for t in (100, 500):
        o.step(t - o.step_count)
        F = o.fields()
        E.append(np.sum(F["ux"] ** 2 + F["uy"] ** 2 + F["uz"] ** 2))
        assert np.abs(F["uz"]).max() < 1e-15
    rate = -math.log(E[1] / E[0]) / 400 / 2
    assert abs(rate / (2 * nu * k * k) - 1) < 2e-3


def test_gaussian_advection_diffusion_3d():
    """Vapour in pure fluid with a uniform velocity: a 3D Gaussian pulse spreads with
    D = (tau_vap - 1/2)/4 (D3Q7, cs^2 = 1/4) and is carried with u; its amplitude falls as
    (sigma0^2/(sigma0^2 + 2 D t))^(3/2) (periodic images included).  A diffusivity with cs^2 = 1/3
    misses by far more."""
    n, sigma0, T, tau_g = 40, 4.0, 200, 0.9
    u = (0.02, 0.01, -0.015)
    p = params(nx=n, ny=n, nz=n, flow=1, tau_vap=tau_g, L_sat=0.0)
    o = oracle.Oracle3D(p)
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)
    c0 = n / 2
    U = 0.5 + 0.1 * np.exp(-((x - c0) ** 2 + (y - c0) ** 2 + (z - c0) ** 2) / (2 * sigma0 ** 2))
    f = np.broadcast_to(oracle.feq3(1.0, *u)[:, None, None, None], (19,) + x.shape).copy()
    g = oracle.geq3(1.0, *u)[:, None, None, None] * U[None]
    o.set_state(f=f, g=g, h=uniform_phase(x.shape), phip=-np.ones(x.shape))
    o.step(T)
    Un = o.fields()["U"]

    def analytic(D):  # with the periodic images of the pulse
        s2 = sigma0 ** 2 + 2 * D * T
        out = np.full(x.shape, 0.5)
        for ix in (-1, 0, 1):
            for iy in (-1, 0, 1):
                for iz in (-1, 0, 1):
                    d2 = sum(((v - c0 - uu * T + n / 2) % n - n / 2 + k * n) ** 2
                             for v, uu, k in ((x, u[0], ix), (y, u[1], iy), (z, u[2], iz)))
                    out += 0.1 * (sigma0 ** 2 / s2) ** 1.5 * np.exp(-d2 / (2 * s2))
        return out

    err = lambda Ua: np.sqrt(np.sum((Un - Ua) ** 2) / np.sum((Ua - 0.5) ** 2))
    e_ok = err(analytic((tau_g - 0.5) / 4))
    assert e_ok < 5e-3
    assert err(analytic((tau_g - 0.5) / 3)) > 10 * e_ok


def _slab3(axis, W0, U0, n, eps=0.05, lam=3.0, half=8.0):
    tau0 = W0 * W0 / 0.1
    shape = [2, 2, 2]
    shape[2 - axis] = n  # [z, y, x]
    p = params(nx=shape[2], ny=shape[1], nz=shape[0], eps=eps, W0=W0, tau0=tau0, lam=lam, L_sat=0.0)
    o = oracle.Oracle3D(p)
    coords = np.mgrid[0:shape[0], 0:shape[1], 0:shape[2]].astype(float)
    r = coords[2 - axis]
    phi0 = np.tanh((half * W0 - np.abs(r - n / 2)) / (math.sqrt(2) * W0))
    o.set_state(g=W7[:, None, None, None] * U0 * np.ones((7,) + phi0.shape), h=W7[:, None, None, None] * phi0[None],
                phip=phi0)

    def front():
        pr = np.moveaxis(o.fields()["phi"], 2 - axis, 0)[:, 0, 0]
        for i in range(n // 2, n - 1):
            if pr[i] >= 0 > pr[i + 1]:
                return i + pr[i] / (pr[i] - pr[i + 1])
        return float("nan")
    return o, p, front


@pytest.mark.parametrize("axis,a,tol", [(0, 1.05, 0.03), (1, 0.95, 0.045), (2, 1.0, 0.03)])
def test_kinetic_flat_front_speed_3d(axis, a, tol):
    """Flat fronts with L_sat = 0 in uniform U0 move at V = lambda U0 W0 / (a1 tau0 a) (Sec. 2.1):
    a = 1 + eps for a normal along x (a tip direction, theta = 0), 1 - eps along y (theta = 90 degrees,
    between tips), and a = 1 along the c axis (reading T3), as in the 2D method's basal plane."""
    W0, U0, lam = 1.0, 0.05, 3.0
    o, p, front = _slab3(axis, W0, U0, 192)
    o.step(800)
    x1 = front()
    o.step(1600)
    V = (front() - x1) / 1600
    Vth = lam * U0 * W0 / (si.A1 * p.tau0 * a)
    assert abs(V / Vth - 1) < tol, (axis, V, Vth)


def test_conservation_and_symmetry_with_crystal_and_flow():
    """A periodic 3D box with flow and a growing seed centred on a node: total mass is exact, the
    species invariant sum U + (L_sat/2) sum phi_prev is exact (1e-13), and the crystal keeps the mirror
    symmetries of the set-up in x, y and z (1e-12)."""
    n = 20
    p = params(nx=n, ny=n, nz=n, flow=1, eps=0.05, tau_f=0.7)
    o = oracle.Oracle3D(p).init_seed(10.0, 10.0, 10.0, 4.0, 1.0, 0.6)
    d0 = o.diag()
    o.step(60)
    d1 = o.diag()
    assert abs(d1["rho"] / d0["rho"] - 1) < 1e-13
    assert abs(d1["species"] / d0["species"] - 1) < 1e-13
    assert d1["n_solid"] > d0["n_solid"]
    phi = o.fields()["phi"]
    c = phi[1:, 1:, 1:]  # cells 1..19 are mirror images about the centre node 10
    for ax in range(3):
        assert np.abs(c - np.flip(c, ax)).max() < 1e-12
