/*
 * snow_oracle.c -- FP64 CPU oracle of the coupled lattice-Boltzmann step for ice-crystal growth
 * (Tan et al., arXiv:2101.07163).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  Plain loops, plain IEEE double
 * arithmetic (built with -ffp-contract=off), one cell at a time, in the order the method states:
 *
 *   state at t : f[9] (flow), g[5] (vapour), h[9] (phase field) per cell, after streaming, and
 *                phi_prev = phi(t-1) for the time derivative of phi in the vapour source.
 *   1. phi = sum_q h_q everywhere                                   (Sec. 2.2.3, phi = sum h)
 *   2. per cell: moments, E4 gradient of phi, anisotropy a and flux N, the three collisions
 *   3. streaming (written per destination: each destination population has exactly one source)
 *   4. phi_prev <- phi, t <- t + 1
 *
 * Readings of points where the paper is silent or ambiguous are marked [Rk]:
 *   R1  gradient: grad phi = sum_c w(|c|^2) phi(x+c) c with the Table 1 weights and no 1/cs^2
 *       (the Table 1 weights already satisfy sum w c c = I; with 1/cs^2 the gradient of x would be 3).
 *       E2 is the central difference of the same section (w(1) = 1/2); E4 is the default.
 *   R2  anisotropic flux N = kappa_N * (W0^2/tau0) * |grad phi|^2 * a * da/d(grad phi); kappa_N = 1
 *       is the variational form, kappa_N = 2 the literal d(a^2)/d(grad phi) of Eq. (e).
 *   R3  vapour diffusivity switch q = (1 - phi)/2 clamped to [0, 1], tau_g = 1/2 + (tau_vap - 1/2) q;
 *       the symmetric (thermal) variant of the Sec. 3.1.1 study takes q = 1 in both phases.
 *   R4  flow: second-order equilibrium, Guo forcing, eta_f = nu; the projected velocity
 *       u = (1 - phi)/2 * j / (rho + k/2) is used in f_eq, in the drag force and in g_eq; phi is
 *       clamped to [-1, 1] inside the projection and drag factors.
 *   R5  Eq. (d): a^2 is taken at the source node x; h_q(x + c_q, t) is the destination's own
 *       pre-collision value, so the scheme streams by "push".
 *   R6  |grad phi|^2 <= grad_eps2: the normal is undefined; a = 1 and N = 0.
 *   R7  d(phi)/dt in the vapour source = phi(t) - phi(t-1); all three solvers read the state at t.
 *   R8  the vapour and phase-field sources carry no (1 - 1/(2 tau)) factor, as printed.
 *   R9  inlet: equilibrium ghost column at x = -1 (rho0, (u_in, 0); U_in; phi = -1, h_q = -w_q);
 *       outlet: ghost column at x = nx copies column nx-1 after collision; gradient ghosts
 *       phi(-1, y) = -1 and phi(nx, y) = phi(nx-1, y).
 *   R10 initial state: phi0 = tanh((R - r)/(sqrt(2) w_init)), h = w phi0, phi_prev = phi0,
 *       f = f_eq(rho0, u0), g = g_eq(U_init, u0), u0 = (1 - phi0)/2 (u_in, 0) for a ventilated
 *       domain and 0 otherwise.
 */
#include "snow_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities and weights (Sec. 2.2.1): rest, 4 axis, 4 diagonal; cs^2 = 1/3. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* D2Q5 for the vapour (Sec. 2.2.2): the first five velocities above. */
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
static const double CS2 = 1.0 / 3.0;
/* Table 1, E4 row: w(1) for the four |c|^2 = 1 neighbours, w(2) for the four |c|^2 = 2 ones. */
/* Table 1 (Sec. 3.1.1): weight of a stencil vector c by |c|^2 = 0..8, for E4, E6 and E8; E2 is the
 * central difference of the same section. */
static const double E2_W[9] = {0.0, 1.0 / 2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
static const double E4_W[9] = {0.0, 1.0 / 3.0, 1.0 / 12.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
static const double E6_W[9] = {0.0, 4.0 / 15.0, 1.0 / 10.0, 0.0, 1.0 / 120.0, 0.0, 0.0, 0.0, 0.0};
static const double E8_W[9] = {0.0, 4.0 / 21.0, 4.0 / 45.0, 0.0, 1.0 / 60.0, 2.0 / 315.0, 0.0, 0.0, 1.0 / 5040.0};

struct orc {
    orc_params p;
    int64_t ncell;
    double *f, *g, *h, *phip;   /* state at t, [cell][q] */
    double *f2, *g2, *h2;       /* state at t+1 while streaming */
    double *phi;                /* phi(t) */
    double *fs, *gs;            /* post-collision f*, g* */
    double *P, *B;              /* phase field: P_q = h*_q / a^2 and B = (1 - a^2)/a^2 */
    double *ux, *uy;            /* velocity used by the collisions */
    int64_t step;
};

static int64_t cell(const orc_params* p, int x, int y) { return (int64_t)y * p->nx + x; }
static int wrap(int i, int n) { return ((i % n) + n) % n; }
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

int32_t orc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- building blocks */

/* Second-order Hermite equilibrium of the isothermal D2Q9 lattice (Sec. 2.2.1, f_eq). */
void orc_feq(double rho, double ux, double uy, double out[9])
{
    double uu = ux * ux + uy * uy;
    for (int q = 0; q < 9; ++q) {
        double cu = CX[q] * ux + CY[q] * uy;
        out[q] = W9[q] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Vapour equilibrium g_eq = w U (1 + c.u / cs^2) (Sec. 2.2.2). */
void orc_geq(double U, double ux, double uy, double out[5])
{
    for (int q = 0; q < 5; ++q) {
        double cu = CX[q] * ux + CY[q] * uy;
        out[q] = W5[q] * U * (1.0 + cu / CS2);
    }
}

/* Guo forcing term (1 - 1/(2 tau_f)) w [ (c - u)/cs^2 + (c.u) c / cs^4 ] . F   [R4] */
void orc_guo(const orc_params* p, double ux, double uy, double Fx, double Fy, double out[9])
{
    double pref = 1.0 - 1.0 / (2.0 * p->tau_f);
    for (int q = 0; q < 9; ++q) {
        double cu = CX[q] * ux + CY[q] * uy;
        double ex = (CX[q] - ux) / CS2 + cu * CX[q] / (CS2 * CS2);
        double ey = (CY[q] - uy) / CS2 + cu * CY[q] / (CS2 * CS2);
        out[q] = pref * W9[q] * (ex * Fx + ey * Fy);
    }
}

/* Anisotropy a_s(n) = 1 + eps cos(n_fold theta), theta the polar angle of n = -grad phi / |grad phi|
 * (Sec. 2.1), and the anisotropic flux N = kappa_N (W0^2/tau0) |grad phi|^2 a da/d(grad phi)
 * of Eq. (e) [R2, R6].  With theta = atan2(-gy, -gx):  d theta / d(gx, gy) = (-gy, gx)/|g|^2, so
 * da/d(grad phi) = -eps n_fold sin(n_fold theta) (-gy, gx)/|g|^2. */
void orc_aniso(const orc_params* p, double gx, double gy, double* a, double* Nx, double* Ny)
{
    double G2 = gx * gx + gy * gy;
    if (!(G2 > p->grad_eps2)) {
        *a = 1.0;
        *Nx = 0.0;
        *Ny = 0.0;
        return;
    }
    double theta = atan2(-gy, -gx);
    double m = (double)p->n_fold;
    double as = 1.0 + p->eps * cos(m * theta);
    double dadgx = -p->eps * m * sin(m * theta) * (-gy) / G2;
    double dadgy = -p->eps * m * sin(m * theta) * (gx) / G2;
    double k = p->kappa_N * (p->W0 * p->W0 / p->tau0) * G2 * as;
    *a = as;
    *Nx = k * dadgx;
    *Ny = k * dadgy;
}

/* phi at (x, y) with the domain closure: y periodic; x periodic or the inlet/outlet ghosts [R9]. */
static double phi_at(const orc_params* p, const double* phi, int x, int y)
{
    y = wrap(y, p->ny);
    if (p->inout) {
        if (x < 0) return -1.0;
        if (x >= p->nx) x = p->nx - 1;
    } else {
        x = wrap(x, p->nx);
    }
    return phi[cell(p, x, y)];
}

static const double* stencil_weights(const orc_params* p)
{
    switch (p->stencil) {
        case 2: return E2_W;
        case 6: return E6_W;
        case 8: return E8_W;
        default: return E4_W;
    }
}

/* Isotropic gradient (Sec. 3.1.1, Table 1) [R1]: every vector c with |c| <= 2 sqrt 2 whose layer
 * |c|^2 has a weight in the chosen stencil. */
static void grad_at(const orc_params* p, const double* phi, int x, int y, double* gx, double* gy)
{
    const double* W = stencil_weights(p);
    double sx = 0.0, sy = 0.0;
    for (int cy = -2; cy <= 2; ++cy)
        for (int cx = -2; cx <= 2; ++cx) {
            double w = W[cx * cx + cy * cy];
            if (w == 0.0) continue;
            double v = phi_at(p, phi, x + cx, y + cy);
            sx += w * cx * v;
            sy += w * cy * v;
        }
    *gx = sx;
    *gy = sy;
}

void orc_grad(const orc_params* p, const double* phi, double* gx, double* gy)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x)
            grad_at(p, phi, x, y, &gx[cell(p, x, y)], &gy[cell(p, x, y)]);
}

/* ---------------------------------------------------------------- lifecycle */

orc* orc_create(const orc_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1) return NULL;
    if (p->stencil != 0 && p->stencil != 2 && p->stencil != 4 && p->stencil != 6 && p->stencil != 8) return NULL;
    if (p->symmetric != 0 && p->symmetric != 1) return NULL;
    orc* o = (orc*)calloc(1, sizeof(orc));
    if (!o) return NULL;
    o->p = *p;
    o->ncell = (int64_t)p->nx * p->ny;
    size_t n = (size_t)o->ncell;
    o->f = calloc(9 * n, sizeof(double));
    o->g = calloc(5 * n, sizeof(double));
    o->h = calloc(9 * n, sizeof(double));
    o->phip = calloc(n, sizeof(double));
    o->f2 = calloc(9 * n, sizeof(double));
    o->g2 = calloc(5 * n, sizeof(double));
    o->h2 = calloc(9 * n, sizeof(double));
    o->phi = calloc(n, sizeof(double));
    o->fs = calloc(9 * n, sizeof(double));
    o->gs = calloc(5 * n, sizeof(double));
    o->P = calloc(9 * n, sizeof(double));
    o->B = calloc(n, sizeof(double));
    o->ux = calloc(n, sizeof(double));
    o->uy = calloc(n, sizeof(double));
    if (!o->f || !o->g || !o->h || !o->phip || !o->f2 || !o->g2 || !o->h2 || !o->phi || !o->fs ||
        !o->gs || !o->P || !o->B || !o->ux || !o->uy) {
        orc_destroy(o);
        return NULL;
    }
    return o;
}

void orc_destroy(orc* o)
{
    if (!o) return;
    free(o->f); free(o->g); free(o->h); free(o->phip);
    free(o->f2); free(o->g2); free(o->h2); free(o->phi);
    free(o->fs); free(o->gs); free(o->P); free(o->B); free(o->ux); free(o->uy);
    free(o);
}

int64_t orc_step_count(const orc* o) { return o->step; }

/* Initial condition [R10]. */
void orc_init_seed(orc* o, double xs, double ys, double R, double w_init, double U0,
                   const double* U_init)
{
    const orc_params* p = &o->p;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            int64_t i = cell(p, x, y);
            double r = sqrt((x - xs) * (x - xs) + (y - ys) * (y - ys));
            double phi0 = tanh((R - r) / (sqrt(2.0) * w_init));
            double ux0 = 0.0, uy0 = 0.0;
            if (p->flow && p->inout) ux0 = 0.5 * (1.0 - phi0) * p->u_in;
            double U = U_init ? U_init[i] : U0;
            for (int q = 0; q < 9; ++q) o->h[9 * i + q] = W9[q] * phi0;
            o->phip[i] = phi0;
            orc_feq(p->rho0, ux0, uy0, &o->f[9 * i]);
            orc_geq(U, ux0, uy0, &o->g[5 * i]);
        }
    o->step = 0;
}

void orc_set_state(orc* o, const double* f, const double* g, const double* h, const double* phip)
{
    int64_t n = o->ncell;
    for (int64_t i = 0; i < n; ++i) {
        if (f) for (int q = 0; q < 9; ++q) o->f[9 * i + q] = f[q * n + i];
        if (g) for (int q = 0; q < 5; ++q) o->g[5 * i + q] = g[q * n + i];
        if (h) for (int q = 0; q < 9; ++q) o->h[9 * i + q] = h[q * n + i];
        if (phip) o->phip[i] = phip[i];
    }
}

void orc_get_state(const orc* o, double* f, double* g, double* h, double* phip)
{
    int64_t n = o->ncell;
    for (int64_t i = 0; i < n; ++i) {
        if (f) for (int q = 0; q < 9; ++q) f[q * n + i] = o->f[9 * i + q];
        if (g) for (int q = 0; q < 5; ++q) g[q * n + i] = o->g[5 * i + q];
        if (h) for (int q = 0; q < 9; ++q) h[q * n + i] = o->h[9 * i + q];
        if (phip) phip[i] = o->phip[i];
    }
}

/* ---------------------------------------------------------------- one step */

static void collide(orc* o, int x, int y)
{
    const orc_params* p = &o->p;
    int64_t i = cell(p, x, y);
    const double* h = &o->h[9 * i];
    const double* g = &o->g[5 * i];
    double phi = o->phi[i];

    /* supersaturation U = sum g (Sec. 2.2.2) */
    double U = 0.0;
    for (int q = 0; q < 5; ++q) U += g[q];

    /* gradient, anisotropy and anisotropic flux (Sec. 3.1.1; Sec. 2.1; Eq. (e)) */
    double gx, gy, a, Nx, Ny;
    grad_at(p, o->phi, x, y, &gx, &gy);
    orc_aniso(p, gx, gy, &a, &Nx, &Ny);
    double a2 = a * a;

    /* phase field, Eq. (d) with its source Q and relaxation time eta (Sec. 2.2.3) */
    double Dphi = p->W0 * p->W0 / p->tau0;
    double eta = a2 * Dphi / CS2 + 0.5;
    double Q = (phi - phi * phi * phi) + p->lambda * U * (1.0 - phi * phi) * (1.0 - phi * phi);
    for (int q = 0; q < 9; ++q) {
        double heq = W9[q] * (phi - (CX[q] * Nx + CY[q] * Ny) / CS2);
        double hs = h[q] - (h[q] - heq) / eta + W9[q] * Q / p->tau0;
        o->P[9 * i + q] = hs / a2;
    }
    o->B[i] = (1.0 - a2) / a2;

    /* flow with the crystal as a phase-dependent solid (Sec. 2.2.1) [R4] */
    double ux = 0.0, uy = 0.0;
    if (p->flow) {
        const double* f = &o->f[9 * i];
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int q = 0; q < 9; ++q) {
            rho += f[q];
            jx += CX[q] * f[q];
            jy += CY[q] * f[q];
        }
        double pc = clampd(phi, -1.0, 1.0);
        double s = 0.5 * (1.0 - pc);
        double nu = CS2 * (p->tau_f - 0.5);
        double k = p->h_drag * nu * (1.0 + pc) * (1.0 + pc) * (1.0 - pc) / (4.0 * p->W0 * p->W0);
        ux = s * jx / (rho + 0.5 * k);
        uy = s * jy / (rho + 0.5 * k);
        double Fx = -k * ux, Fy = -k * uy;
        double feq[9], S[9];
        orc_feq(rho, ux, uy, feq);
        orc_guo(p, ux, uy, Fx, Fy, S);
        for (int q = 0; q < 9; ++q) o->fs[9 * i + q] = f[q] - (f[q] - feq[q]) / p->tau_f + S[q];
    }
    o->ux[i] = ux;
    o->uy[i] = uy;

    /* vapour advection-diffusion-reaction (Sec. 2.2.2) [R3, R7] */
    double qd = p->symmetric ? 1.0 : clampd(0.5 * (1.0 - phi), 0.0, 1.0);
    double tau_g = 0.5 + (p->tau_vap - 0.5) * qd;
    double geq[5];
    orc_geq(U, ux, uy, geq);
    double dphidt = phi - o->phip[i];
    for (int q = 0; q < 5; ++q)
        o->gs[5 * i + q] = g[q] - (g[q] - geq[q]) / tau_g - W5[q] * 0.5 * p->L_sat * dphidt;
}

/* Streaming into destination (x, y) [R5, R9]. */
static void stream_into(orc* o, int x, int y)
{
    const orc_params* p = &o->p;
    int64_t d = cell(p, x, y);
    double f_in[9], g_in[5];
    orc_feq(p->rho0, p->u_in, 0.0, f_in);
    orc_geq(p->U_in, p->u_in, 0.0, g_in);
    for (int q = 0; q < 9; ++q) {
        int xs = x - CX[q];
        int ys = wrap(y - CY[q], p->ny);
        double hold = o->h[9 * d + q]; /* h_q(x + c_q, t) of Eq. (d): the destination's old value */
        if (!p->inout) xs = wrap(xs, p->nx);
        if (xs < 0) { /* inlet ghost */
            o->h2[9 * d + q] = -W9[q];
            if (p->flow) o->f2[9 * d + q] = f_in[q];
            if (q < 5) o->g2[5 * d + q] = g_in[q];
            continue;
        }
        if (xs >= p->nx) xs = p->nx - 1; /* outlet ghost: copy of column nx-1 */
        int64_t s = cell(p, xs, ys);
        o->h2[9 * d + q] = o->P[9 * s + q] - o->B[s] * hold;
        if (p->flow) o->f2[9 * d + q] = o->fs[9 * s + q];
        if (q < 5) o->g2[5 * d + q] = o->gs[5 * s + q];
    }
}

static void swap_ptr(double** a, double** b)
{
    double* t = *a;
    *a = *b;
    *b = t;
}

static void compute_phi(orc* o)
{
    int64_t n = o->ncell;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = 0; q < 9; ++q) s += o->h[9 * i + q];
        o->phi[i] = s;
    }
}

void orc_step(orc* o, int32_t n)
{
    const orc_params* p = &o->p;
    for (int32_t t = 0; t < n; ++t) {
        compute_phi(o);
#pragma omp parallel for schedule(static)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) collide(o, x, y);
#pragma omp parallel for schedule(static)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) stream_into(o, x, y);
        memcpy(o->phip, o->phi, (size_t)o->ncell * sizeof(double));
        swap_ptr(&o->h, &o->h2);
        swap_ptr(&o->g, &o->g2);
        if (p->flow) swap_ptr(&o->f, &o->f2);
        o->step += 1;
    }
}

/* ---------------------------------------------------------------- read-out */

void orc_fields(const orc* o, double* phi, double* U, double* rho, double* ux, double* uy)
{
    const orc_params* p = &o->p;
    int64_t n = o->ncell;
    for (int64_t i = 0; i < n; ++i) {
        double sp = 0.0, su = 0.0, r = 0.0, jx = 0.0, jy = 0.0;
        for (int q = 0; q < 9; ++q) sp += o->h[9 * i + q];
        for (int q = 0; q < 5; ++q) su += o->g[5 * i + q];
        if (p->flow)
            for (int q = 0; q < 9; ++q) {
                r += o->f[9 * i + q];
                jx += CX[q] * o->f[9 * i + q];
                jy += CY[q] * o->f[9 * i + q];
            }
        double vx = 0.0, vy = 0.0;
        if (p->flow) {
            double pc = clampd(sp, -1.0, 1.0);
            double s = 0.5 * (1.0 - pc);
            double nu = CS2 * (p->tau_f - 0.5);
            double k = p->h_drag * nu * (1.0 + pc) * (1.0 + pc) * (1.0 - pc) / (4.0 * p->W0 * p->W0);
            vx = s * jx / (r + 0.5 * k);
            vy = s * jy / (r + 0.5 * k);
        }
        if (phi) phi[i] = sp;
        if (U) U[i] = su;
        if (rho) rho[i] = r;
        if (ux) ux[i] = vx;
        if (uy) uy[i] = vy;
    }
}

void orc_diag(const orc* o, double out[8])
{
    const orc_params* p = &o->p;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < o->ncell; ++i) {
        double ph = 0.0, U = 0.0, r = 0.0, jx = 0.0, jy = 0.0;
        int bad = 0;
        for (int q = 0; q < 9; ++q) { ph += o->h[9 * i + q]; bad |= !isfinite(o->h[9 * i + q]); }
        for (int q = 0; q < 5; ++q) { U += o->g[5 * i + q]; bad |= !isfinite(o->g[5 * i + q]); }
        if (p->flow)
            for (int q = 0; q < 9; ++q) {
                r += o->f[9 * i + q];
                jx += CX[q] * o->f[9 * i + q];
                jy += CY[q] * o->f[9 * i + q];
                bad |= !isfinite(o->f[9 * i + q]);
            }
        bad |= !isfinite(o->phip[i]);
        s[0] += r; s[1] += jx; s[2] += jy; s[3] += U; s[4] += ph; s[5] += o->phip[i];
        s[6] += (ph > 0.0) ? 1.0 : 0.0;
        s[7] += bad ? 1.0 : 0.0;
    }
    memcpy(out, s, sizeof(s));
}
