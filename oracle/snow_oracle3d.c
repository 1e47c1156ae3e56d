/*
 * snow_oracle3d.c -- FP64 CPU oracle of the coupled lattice-Boltzmann step in three dimensions.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library's 3D step is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  Plain loops, plain
 * IEEE double arithmetic (built with -ffp-contract=off), one cell at a time, in the order of the
 * two-dimensional method (Sec. 2.2), which Sec. 4 names for extension to three dimensions:
 *
 *   state at t : f[19] (flow), g[7] (vapour), h[7] (phase field) per cell, after streaming, and
 *                phi_prev = phi(t-1).
 *   1. phi = sum_q h_q everywhere                                    (Sec. 2.2.3)
 *   2. per cell: moments, the isotropic gradient of phi, anisotropy a and flux N, three collisions
 *   3. streaming, written per destination (each destination population has exactly one source)
 *   4. phi_prev <- phi, t <- t + 1
 *
 * The paper gives the method in two dimensions only.  Its readings there (the 2D oracle's R1-R10) carry
 * over unchanged; the three-dimensional ones are marked [Tk]:
 *   T1  lattices: D3Q19 for the flow (weights 1/3, 1/18 on the 6 axes, 1/36 on the 12 face
 *       diagonals, cs^2 = 1/3), D3Q7 for the vapour g and the phase field h (weights 1/4 at rest and
 *       1/8 on the axes, cs^2 = 1/4), the 3D counterparts of D2Q9 and D2Q5 of Sec. 2.2.1-2.2.3.  The
 *       vapour diffusivity is D = (tau_vap - 1/2)/4 and the phase-field relaxation
 *       eta = a^2 (W0^2/tau0)/cs^2 + 1/2 with cs^2 = 1/4.
 *   T2  gradient: grad phi = sum_c w(|c|^2) phi(x + c) c over the 18 D3Q19 neighbours with
 *       w(1) = 1/6, w(2) = 1/12, the three-dimensional analogue of the E4 row of Table 1
 *       (sum w c c = I, fourth-order isotropic), with no 1/cs^2 in front (as R1).
 *   T3  anisotropy: the hexagonal a_s of Sec. 2.1 taken about the crystal's c axis (z):
 *       a = 1 + eps cos(6 theta) sin^6(psi), theta the azimuth of the normal n in the basal (x, y)
 *       plane and psi its angle to the z axis; in the basal plane (n_z = 0) this is the paper's
 *       1 + eps cos(6 theta), and along the c axis a = 1.  The flux is N = kappa_N (W0^2/tau0)
 *       |grad phi|^2 a da/d(grad phi) as in R2.
 *   T4  boundaries: x periodic or inlet/outlet as R9 (the inlet ghost plane at x = -1 carries
 *       (rho0, (u_in, 0, 0); U_in; phi = -1), the outlet ghost plane at x = nx copies plane nx-1
 *       after collision); y and z periodic.
 *   T5  initial state: the spherical seed phi0 = tanh((R - r)/(sqrt 2 w_init)), h = w phi0,
 *       phi_prev = phi0, f = f_eq(rho0, u0), g = g_eq(U_init, u0), u0 = (1 - phi0)/2 (u_in, 0, 0) for a
 *       ventilated domain and 0 otherwise.
 */
#include "snow_oracle3d.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19: rest, 6 axis, 12 face diagonals [T1]; D3Q7 is the first seven. */
static const int C3[19][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},   {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double CS2_19 = 1.0 / 3.0;
static const double CS2_7 = 1.0 / 4.0;

static double w19(int q) { return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
static double w7(int q) { return q == 0 ? 1.0 / 4.0 : 1.0 / 8.0; }

struct orc3 {
    orc3_params p;
    int64_t ncell;
    double *f, *g, *h, *phip;
    double *f2, *g2, *h2;
    double *phi, *fs, *gs, *P, *B;
    int64_t step;
};

static int wrap(int i, int n) { return ((i % n) + n) % n; }
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int64_t cell3(const orc3_params* p, int x, int y, int z) { return ((int64_t)z * p->ny + y) * p->nx + x; }

void orc3_lattice(int32_t* c19, double* ww19, double* ww7)
{
    for (int q = 0; q < 19; ++q) {
        for (int k = 0; k < 3; ++k) c19[3 * q + k] = C3[q][k];
        ww19[q] = w19(q);
        if (q < 7) ww7[q] = w7(q);
    }
}

/* second-order D3Q19 equilibrium (the 3D form of f_eq of Sec. 2.2.1) */
void orc3_feq(double rho, double ux, double uy, double uz, double out[19])
{
    double uu = ux * ux + uy * uy + uz * uz;
    for (int q = 0; q < 19; ++q) {
        double cu = C3[q][0] * ux + C3[q][1] * uy + C3[q][2] * uz;
        out[q] = w19(q) * rho * (1.0 + cu / CS2_19 + cu * cu / (2.0 * CS2_19 * CS2_19) - uu / (2.0 * CS2_19));
    }
}

/* D3Q7 vapour equilibrium w U (1 + c.u/cs^2) (the 3D form of g_eq of Sec. 2.2.2) */
void orc3_geq(double U, double ux, double uy, double uz, double out[7])
{
    for (int q = 0; q < 7; ++q) {
        double cu = C3[q][0] * ux + C3[q][1] * uy + C3[q][2] * uz;
        out[q] = w7(q) * U * (1.0 + cu / CS2_7);
    }
}

/* Guo forcing on D3Q19: (1 - 1/(2 tau_f)) w [(c - u)/cs^2 + (c.u) c/cs^4] . F */
static void guo3(const orc3_params* p, const double u[3], const double F[3], double out[19])
{
    double pref = 1.0 - 1.0 / (2.0 * p->tau_f);
    for (int q = 0; q < 19; ++q) {
        double cu = C3[q][0] * u[0] + C3[q][1] * u[1] + C3[q][2] * u[2];
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += ((C3[q][k] - u[k]) / CS2_19 + cu * C3[q][k] / (CS2_19 * CS2_19)) * F[k];
        out[q] = pref * w19(q) * s;
    }
}

/* Anisotropy [T3] in its trigonometric form and the flux N = kappa_N Dphi |g|^2 a da/dg.  With
 * r2 = gx^2 + gy^2, G2 = r2 + gz^2, theta = atan2(gy, gx) (cos 6 theta is the same for n = -g/|g|):
 *   a = 1 + eps cos(6 theta) s6,   s6 = (r2/G2)^3 = sin^6(psi),
 *   d theta/dg = (-gy, gx, 0)/r2,  d s6/dg = 3 (r2/G2)^2 * 2 (gx gz^2, gy gz^2, -r2 gz)/G2^2. */
void orc3_aniso(const orc3_params* p, double gx, double gy, double gz, double* a, double* Nx, double* Ny,
                double* Nz)
{
    double r2 = gx * gx + gy * gy;
    double G2 = r2 + gz * gz;
    *a = 1.0;
    *Nx = *Ny = *Nz = 0.0;
    if (!(G2 > p->grad_eps2) || !(r2 > 0.0)) return;
    double theta = atan2(gy, gx);
    double c6 = cos(6.0 * theta), sn6 = sin(6.0 * theta);
    double t = r2 / G2;
    double s6 = t * t * t;
    double as = 1.0 + p->eps * c6 * s6;
    double dth[3] = {-gy / r2, gx / r2, 0.0};
    double ds6[3] = {3.0 * t * t * 2.0 * gx * gz * gz / (G2 * G2), 3.0 * t * t * 2.0 * gy * gz * gz / (G2 * G2),
                     -3.0 * t * t * 2.0 * r2 * gz / (G2 * G2)};
    double k = p->kappa_N * (p->W0 * p->W0 / p->tau0) * G2 * as;
    double N[3];
    for (int c = 0; c < 3; ++c) N[c] = k * p->eps * (-6.0 * sn6 * s6 * dth[c] + c6 * ds6[c]);
    *a = as;
    *Nx = N[0];
    *Ny = N[1];
    *Nz = N[2];
}

/* phi at a lattice position with the closure [T4]. */
static double phi_at3(const orc3_params* p, const double* phi, int x, int y, int z)
{
    y = wrap(y, p->ny);
    z = wrap(z, p->nz);
    if (p->inout) {
        if (x < 0) return -1.0;
        if (x >= p->nx) x = p->nx - 1;
    } else {
        x = wrap(x, p->nx);
    }
    return phi[cell3(p, x, y, z)];
}

/* isotropic gradient [T2] */
static void grad_at3(const orc3_params* p, const double* phi, int x, int y, int z, double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    for (int q = 1; q < 19; ++q) {
        double w = q < 7 ? 1.0 / 6.0 : 1.0 / 12.0;
        double v = phi_at3(p, phi, x + C3[q][0], y + C3[q][1], z + C3[q][2]);
        for (int k = 0; k < 3; ++k) g[k] += w * C3[q][k] * v;
    }
}

void orc3_grad(const orc3_params* p, const double* phi, double* gx, double* gy, double* gz)
{
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double g[3];
                grad_at3(p, phi, x, y, z, g);
                int64_t i = cell3(p, x, y, z);
                gx[i] = g[0];
                gy[i] = g[1];
                gz[i] = g[2];
            }
}

orc3* orc3_create(const orc3_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    orc3* o = (orc3*)calloc(1, sizeof(orc3));
    if (!o) return NULL;
    o->p = *p;
    o->ncell = (int64_t)p->nx * p->ny * p->nz;
    size_t n = (size_t)o->ncell;
    o->f = calloc(19 * n, sizeof(double));
    o->f2 = calloc(19 * n, sizeof(double));
    o->fs = calloc(19 * n, sizeof(double));
    o->g = calloc(7 * n, sizeof(double));
    o->g2 = calloc(7 * n, sizeof(double));
    o->gs = calloc(7 * n, sizeof(double));
    o->h = calloc(7 * n, sizeof(double));
    o->h2 = calloc(7 * n, sizeof(double));
    o->P = calloc(7 * n, sizeof(double));
    o->phip = calloc(n, sizeof(double));
    o->phi = calloc(n, sizeof(double));
    o->B = calloc(n, sizeof(double));
    if (!o->f || !o->f2 || !o->fs || !o->g || !o->g2 || !o->gs || !o->h || !o->h2 || !o->P || !o->phip ||
        !o->phi || !o->B) {
        orc3_destroy(o);
        return NULL;
    }
    return o;
}

void orc3_destroy(orc3* o)
{
    if (!o) return;
    free(o->f); free(o->f2); free(o->fs); free(o->g); free(o->g2); free(o->gs);
    free(o->h); free(o->h2); free(o->P); free(o->phip); free(o->phi); free(o->B);
    free(o);
}

int64_t orc3_step_count(const orc3* o) { return o->step; }

/* initial state [T5] */
void orc3_init_seed(orc3* o, double xs, double ys, double zs, double R, double w_init, double U0,
                    const double* U_init)
{
    const orc3_params* p = &o->p;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = cell3(p, x, y, z);
                double r = sqrt((x - xs) * (x - xs) + (y - ys) * (y - ys) + (z - zs) * (z - zs));
                double phi0 = tanh((R - r) / (sqrt(2.0) * w_init));
                double ux0 = (p->flow && p->inout) ? 0.5 * (1.0 - phi0) * p->u_in : 0.0;
                double U = U_init ? U_init[i] : U0;
                for (int q = 0; q < 7; ++q) o->h[7 * i + q] = w7(q) * phi0;
                o->phip[i] = phi0;
                orc3_feq(p->rho0, ux0, 0.0, 0.0, &o->f[19 * i]);
                orc3_geq(U, ux0, 0.0, 0.0, &o->g[7 * i]);
            }
    o->step = 0;
}

void orc3_set_state(orc3* o, const double* f, const double* g, const double* h, const double* phip)
{
    int64_t n = o->ncell;
    for (int64_t i = 0; i < n; ++i) {
        if (f) for (int q = 0; q < 19; ++q) o->f[19 * i + q] = f[q * n + i];
        if (g) for (int q = 0; q < 7; ++q) o->g[7 * i + q] = g[q * n + i];
        if (h) for (int q = 0; q < 7; ++q) o->h[7 * i + q] = h[q * n + i];
        if (phip) o->phip[i] = phip[i];
    }
}

void orc3_get_state(const orc3* o, double* f, double* g, double* h, double* phip)
{
    int64_t n = o->ncell;
    for (int64_t i = 0; i < n; ++i) {
        if (f) for (int q = 0; q < 19; ++q) f[q * n + i] = o->f[19 * i + q];
        if (g) for (int q = 0; q < 7; ++q) g[q * n + i] = o->g[7 * i + q];
        if (h) for (int q = 0; q < 7; ++q) h[q * n + i] = o->h[7 * i + q];
        if (phip) phip[i] = o->phip[i];
    }
}

/* velocity of the collisions from a cell's flow populations and phase (R4 of the 2D method) */
static void velocity3(const orc3_params* p, const double* f, double phi, double* rho_out, double j[3],
                      double u[3], double* k_out)
{
    double rho = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    for (int q = 0; q < 19; ++q) {
        rho += f[q];
        for (int k = 0; k < 3; ++k) j[k] += C3[q][k] * f[q];
    }
    double pc = clampd(phi, -1.0, 1.0);
    double s = 0.5 * (1.0 - pc);
    double nu = CS2_19 * (p->tau_f - 0.5);
    double kd = p->h_drag * nu * (1.0 + pc) * (1.0 + pc) * (1.0 - pc) / (4.0 * p->W0 * p->W0);
    for (int k = 0; k < 3; ++k) u[k] = s * j[k] / (rho + 0.5 * kd);
    *rho_out = rho;
    *k_out = kd;
}

static void collide3(orc3* o, int x, int y, int z)
{
    const orc3_params* p = &o->p;
    int64_t i = cell3(p, x, y, z);
    const double* h = &o->h[7 * i];
    const double* g = &o->g[7 * i];
    double phi = o->phi[i];

    double U = 0.0;
    for (int q = 0; q < 7; ++q) U += g[q];

    double gr[3], a, N[3];
    grad_at3(p, o->phi, x, y, z, gr);
    orc3_aniso(p, gr[0], gr[1], gr[2], &a, &N[0], &N[1], &N[2]);
    double a2 = a * a;

    /* phase field: Eq. (d)/(e) on D3Q7 [T1] */
    double Dphi = p->W0 * p->W0 / p->tau0;
    double eta = a2 * Dphi / CS2_7 + 0.5;
    double Q = (phi - phi * phi * phi) + p->lambda * U * (1.0 - phi * phi) * (1.0 - phi * phi);
    for (int q = 0; q < 7; ++q) {
        double cN = C3[q][0] * N[0] + C3[q][1] * N[1] + C3[q][2] * N[2];
        double heq = w7(q) * (phi - cN / CS2_7);
        double hs = h[q] - (h[q] - heq) / eta + w7(q) * Q / p->tau0;
        o->P[7 * i + q] = hs / a2;
    }
    o->B[i] = (1.0 - a2) / a2;

    /* flow with the crystal as a phase-dependent solid (Sec. 2.2.1 on D3Q19) */
    double u[3] = {0.0, 0.0, 0.0};
    if (p->flow) {
        const double* f = &o->f[19 * i];
        double rho, j[3], kd;
        velocity3(p, f, phi, &rho, j, u, &kd);
        double F[3] = {-kd * u[0], -kd * u[1], -kd * u[2]};
        double feq[19], S[19];
        orc3_feq(rho, u[0], u[1], u[2], feq);
        guo3(p, u, F, S);
        for (int q = 0; q < 19; ++q) o->fs[19 * i + q] = f[q] - (f[q] - feq[q]) / p->tau_f + S[q];
    }

    /* vapour (Sec. 2.2.2 on D3Q7) */
    double qd = clampd(0.5 * (1.0 - phi), 0.0, 1.0);
    double tau_g = 0.5 + (p->tau_vap - 0.5) * qd;
    double geq[7];
    orc3_geq(U, u[0], u[1], u[2], geq);
    double dphidt = phi - o->phip[i];
    for (int q = 0; q < 7; ++q)
        o->gs[7 * i + q] = g[q] - (g[q] - geq[q]) / tau_g - w7(q) * 0.5 * p->L_sat * dphidt;
}

/* streaming into destination (x, y, z) [T4] */
static void stream_into3(orc3* o, int x, int y, int z)
{
    const orc3_params* p = &o->p;
    int64_t d = cell3(p, x, y, z);
    double f_in[19], g_in[7];
    orc3_feq(p->rho0, p->u_in, 0.0, 0.0, f_in);
    orc3_geq(p->U_in, p->u_in, 0.0, 0.0, g_in);
    for (int q = 0; q < 19; ++q) {
        int xs = x - C3[q][0];
        int ys = wrap(y - C3[q][1], p->ny);
        int zs = wrap(z - C3[q][2], p->nz);
        if (!p->inout) xs = wrap(xs, p->nx);
        if (xs < 0) { /* inlet ghost */
            if (q < 7) {
                o->h2[7 * d + q] = -w7(q);
                o->g2[7 * d + q] = g_in[q];
            }
            if (p->flow) o->f2[19 * d + q] = f_in[q];
            continue;
        }
        if (xs >= p->nx) xs = p->nx - 1; /* outlet ghost: copy of plane nx-1 */
        int64_t s = cell3(p, xs, ys, zs);
        if (q < 7) {
            double hold = o->h[7 * d + q]; /* h_q(x + c_q, t): the destination's old value */
            o->h2[7 * d + q] = o->P[7 * s + q] - o->B[s] * hold;
            o->g2[7 * d + q] = o->gs[7 * s + q];
        }
        if (p->flow) o->f2[19 * d + q] = o->fs[19 * s + q];
    }
}

static void swap_ptr(double** a, double** b)
{
    double* t = *a;
    *a = *b;
    *b = t;
}

void orc3_step(orc3* o, int32_t n)
{
    const orc3_params* p = &o->p;
    for (int32_t t = 0; t < n; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < o->ncell; ++i) {
            double s = 0.0;
            for (int q = 0; q < 7; ++q) s += o->h[7 * i + q];
            o->phi[i] = s;
        }
#pragma omp parallel for schedule(static) collapse(2)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) collide3(o, x, y, z);
#pragma omp parallel for schedule(static) collapse(2)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) stream_into3(o, x, y, z);
        memcpy(o->phip, o->phi, (size_t)o->ncell * sizeof(double));
        swap_ptr(&o->h, &o->h2);
        swap_ptr(&o->g, &o->g2);
        if (p->flow) swap_ptr(&o->f, &o->f2);
        o->step += 1;
    }
}

void orc3_fields(const orc3* o, double* phi, double* U, double* rho, double* ux, double* uy, double* uz)
{
    const orc3_params* p = &o->p;
    for (int64_t i = 0; i < o->ncell; ++i) {
        double sp = 0.0, su = 0.0, r = 0.0, j[3], u[3] = {0.0, 0.0, 0.0}, kd;
        for (int q = 0; q < 7; ++q) sp += o->h[7 * i + q];
        for (int q = 0; q < 7; ++q) su += o->g[7 * i + q];
        if (p->flow) velocity3(p, &o->f[19 * i], sp, &r, j, u, &kd);
        if (phi) phi[i] = sp;
        if (U) U[i] = su;
        if (rho) rho[i] = r;
        if (ux) ux[i] = u[0];
        if (uy) uy[i] = u[1];
        if (uz) uz[i] = u[2];
    }
}

void orc3_diag(const orc3* o, double out[9])
{
    const orc3_params* p = &o->p;
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < o->ncell; ++i) {
        double ph = 0.0, U = 0.0, r = 0.0, j[3] = {0.0, 0.0, 0.0};
        int bad = 0;
        for (int q = 0; q < 7; ++q) {
            ph += o->h[7 * i + q];
            U += o->g[7 * i + q];
            bad |= !isfinite(o->h[7 * i + q]) || !isfinite(o->g[7 * i + q]);
        }
        if (p->flow)
            for (int q = 0; q < 19; ++q) {
                r += o->f[19 * i + q];
                for (int k = 0; k < 3; ++k) j[k] += C3[q][k] * o->f[19 * i + q];
                bad |= !isfinite(o->f[19 * i + q]);
            }
        bad |= !isfinite(o->phip[i]);
        s[0] += r; s[1] += j[0]; s[2] += j[1]; s[3] += j[2]; s[4] += U; s[5] += ph; s[6] += o->phip[i];
        s[7] += (ph > 0.0) ? 1.0 : 0.0;
        s[8] += bad ? 1.0 : 0.0;
    }
    memcpy(out, s, sizeof(s));
}
