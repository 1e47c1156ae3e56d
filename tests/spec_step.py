"""A second evaluator of the coupled step, written from the paper's equations and the same readings
of its silent points as the C oracle, in vectorised numpy (test infrastructure only).

It shares no code with the C oracle and exists to check it: brute force on tiny lattices (the two
must agree to rounding), and, because every operation here is generic over the array dtype, complex
arithmetic -- a complex-step derivative of a loss through this evaluator is exact to rounding and
pins the oracle's discrete adjoint.  Branches (the clamps, the normal threshold) are decided on real
parts, so the function stays analytic where it is smooth.

Populations use the canonical layout [q, y, x].  Parameters are a dict with the oracle's names.
"""
import numpy as np

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W5 = np.array([1 / 3] + [1 / 6] * 4)
CS2 = 1.0 / 3.0
# weights by |c|^2 of the gradient stencils of Sec. 3.1.1 (E2 is the central difference)
STENCILS = {2: {1: 1 / 2}, 4: {1: 1 / 3, 2: 1 / 12}, 6: {1: 4 / 15, 2: 1 / 10, 4: 1 / 120},
            8: {1: 4 / 21, 2: 4 / 45, 4: 1 / 60, 5: 2 / 315, 8: 1 / 5040}}


def _shifted(a, dx, dy, inout, ghost):
    """a(x + dx, y + dy) on the lattice: y periodic; x periodic, or (inlet/outlet) `ghost` left of
    x = 0 and column nx - 1 repeated right of it."""
    ny, nx = a.shape
    b = np.roll(a, -dy, axis=0)
    if not inout:
        return np.roll(b, -dx, axis=1)
    xs = np.arange(nx) + dx
    out = b[:, np.clip(xs, 0, nx - 1)].copy()
    out[:, xs < 0] = ghost
    return out


def gradient(p, phi):
    W = STENCILS[p.get("stencil", 4)]
    gx = np.zeros_like(phi)
    gy = np.zeros_like(phi)
    for cy in range(-2, 3):
        for cx in range(-2, 3):
            w = W.get(cx * cx + cy * cy, 0.0)
            if w:
                v = _shifted(phi, cx, cy, p["inout"], -1.0)
                gx = gx + w * cx * v
                gy = gy + w * cy * v
    return gx, gy


def anisotropy(p, gx, gy):
    """a = 1 + eps cos(n theta) and N = kappa_N (W0^2/tau0) |g|^2 a da/dg, theta the angle of the
    normal (cos and sin of n theta written in the unit normal, which is the same function)."""
    G2 = gx * gx + gy * gy
    on = G2.real > p["grad_eps2"]
    G2s = np.where(on, G2, 1.0)
    X, Y, XY = gx * gx / G2s, gy * gy / G2s, gx * gy / G2s
    n = p["n_fold"]
    if n == 6:
        C = X ** 3 - 15 * X ** 2 * Y + 15 * X * Y ** 2 - Y ** 3
        Sn = XY * (6 * X ** 2 - 20 * X * Y + 6 * Y ** 2)
    else:
        C = X ** 2 - 6 * X * Y + Y ** 2
        Sn = 4 * XY * (X - Y)
    a = np.where(on, 1 + p["eps"] * C, 1.0)
    c = np.where(on, p["kappa_N"] * (p["W0"] ** 2 / p["tau0"]) * a * p["eps"] * n * Sn, 0.0)
    return a, c * gy, -c * gx


def step(p, f, g, h, phip):
    """One coupled step.  Returns (f, g, h, phi_prev) at t + 1 (f is None without flow)."""
    inout = p["inout"]
    phi = h.sum(axis=0)
    U = g.sum(axis=0)
    gx, gy = gradient(p, phi)
    a, Nx, Ny = anisotropy(p, gx, gy)
    a2 = a * a
    eta = a2 * (p["W0"] ** 2 / p["tau0"]) / CS2 + 0.5
    Q = phi - phi ** 3 + p["lam"] * U * (1 - phi ** 2) ** 2
    P = []
    for q in range(9):
        heq = W9[q] * (phi - (CX[q] * Nx + CY[q] * Ny) / CS2)
        hs = h[q] - (h[q] - heq) / eta + W9[q] * Q / p["tau0"]
        P.append(hs / a2)
    B = (1 - a2) / a2
    ux = np.zeros_like(phi)
    uy = np.zeros_like(phi)
    fs = None
    if p["flow"]:
        rho = f.sum(axis=0)
        jx = (CX[:, None, None] * f).sum(axis=0)
        jy = (CY[:, None, None] * f).sum(axis=0)
        pc = np.where(phi.real > 1, 1.0, np.where(phi.real < -1, -1.0, phi))
        nu = CS2 * (p["tau_f"] - 0.5)
        k = p["h_drag"] * nu * (1 + pc) ** 2 * (1 - pc) / (4 * p["W0"] ** 2)
        s = 0.5 * (1 - pc)
        ux = s * jx / (rho + 0.5 * k)
        uy = s * jy / (rho + 0.5 * k)
        Fx, Fy = -k * ux, -k * uy
        fs = []
        for q in range(9):
            cu = CX[q] * ux + CY[q] * uy
            feq = W9[q] * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (ux ** 2 + uy ** 2) / (2 * CS2))
            Sg = (1 - 0.5 / p["tau_f"]) * W9[q] * (((CX[q] - ux) * Fx + (CY[q] - uy) * Fy) / CS2
                                                  + cu * (CX[q] * Fx + CY[q] * Fy) / CS2 ** 2)
            fs.append(f[q] - (f[q] - feq) / p["tau_f"] + Sg)
    if p.get("symmetric", 0):
        qd = np.ones_like(phi)
    else:
        qd = 0.5 * (1 - phi)
        qd = np.where(qd.real < 0, 0.0, np.where(qd.real > 1, 1.0, qd))
    tau_g = 0.5 + (p["tau_vap"] - 0.5) * qd
    gs = []
    for q in range(5):
        geq = W5[q] * U * (1 + (CX[q] * ux + CY[q] * uy) / CS2)
        gs.append(g[q] - (g[q] - geq) / tau_g - W5[q] * 0.5 * p["L_sat"] * (phi - phip))
    # push: population q at x comes from x - c_q; h also takes the destination's own old value
    u_in = p.get("u_in", 0.0)
    h2, g2, f2 = [], [], []
    for q in range(9):
        src = lambda a, ghost: _shifted(a, -CX[q], -CY[q], inout, ghost)
        hq = src(P[q], np.nan) - src(B, np.nan) * h[q]
        if inout and CX[q] > 0:  # the inlet ghost's phase populations are h_q = -w_q
            hq[:, 0] = -W9[q]
        h2.append(hq)
        if p["flow"]:
            cu = CX[q] * u_in
            f_in = W9[q] * p["rho0"] * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - u_in ** 2 / (2 * CS2))
            f2.append(src(fs[q], f_in))
        if q < 5:
            g2.append(src(gs[q], W5[q] * p["U_in"] * (1 + CX[q] * u_in / CS2)))
    return (np.array(f2) if p["flow"] else None), np.array(g2), np.array(h2), phi


def init_seed(p, xs, ys, R, w_init, U_init):
    """Circular tanh seed, equilibrium populations at rest (no flow), U from the field U_init."""
    ny, nx = p["ny"], p["nx"]
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi0 = np.tanh((R - np.sqrt((x - xs) ** 2 + (y - ys) ** 2)) / (np.sqrt(2.0) * w_init))
    h = W9[:, None, None] * phi0[None]
    g = W5[:, None, None] * U_init[None]
    return h, g, phi0
