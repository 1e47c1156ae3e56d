/*
 * snow_oracle_adj.c -- FP64 discrete adjoint of the oracle's coupled step, without flow
 * (Tan et al., arXiv:2101.07163; the forward step is in snow_oracle.c).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU adjoint is checked against.
 *
 * For the loss L(phi_T) of the phase field after n steps, the adjoint state
 * lambda_t = dL/d(state at t) = (dF/d state)^T lambda_{t+1}, with lambda_T = dL/dphi_T on every h_q
 * (phi = sum h) and 0 on g and phi_prev, is propagated backwards through the exact reverse of each
 * operation of the forward step, in reverse order (one cell at a time, plain loops).  Along the
 * way the explicit dependence of each step on eps is accumulated into dL/deps.  The initial
 * vapour populations are g_q = w_q U_init, so dL/dU_init = sum_q w_q lambda_g,q(t = 0).
 *
 * The states the reverse sweep needs are recomputed from checkpoints taken every `stride` steps
 * (stride 0: ceil(sqrt(n))), so memory holds about 2 sqrt(n) states.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "snow_oracle.h"

static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
static const double CS2 = 1.0 / 3.0;
static const double E4_W[3] = {0.0, 1.0 / 3.0, 1.0 / 12.0};

typedef struct {
    double *h, *g, *p; /* [cell][q], [cell][q], [cell] */
} state;

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static void state_alloc(state* s, size_t n)
{
    s->h = malloc(9 * n * sizeof(double));
    s->g = malloc(5 * n * sizeof(double));
    s->p = malloc(n * sizeof(double));
}
static void state_free(state* s)
{
    free(s->h);
    free(s->g);
    free(s->p);
}
static void state_from_oracle(const orc* o, const orc_params* p, state* s)
{
    int64_t n = (int64_t)p->nx * p->ny;
    double* h = malloc(9 * n * sizeof(double));
    double* g = malloc(5 * n * sizeof(double));
    orc_get_state(o, NULL, g, h, s->p);
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < 9; ++q) s->h[9 * i + q] = h[q * n + i];
        for (int q = 0; q < 5; ++q) s->g[5 * i + q] = g[q * n + i];
    }
    free(h);
    free(g);
}
static void state_to_oracle(orc* o, const orc_params* p, const state* s)
{
    int64_t n = (int64_t)p->nx * p->ny;
    double* h = malloc(9 * n * sizeof(double));
    double* g = malloc(5 * n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < 9; ++q) h[q * n + i] = s->h[9 * i + q];
        for (int q = 0; q < 5; ++q) g[q * n + i] = s->g[5 * i + q];
    }
    orc_set_state(o, NULL, g, h, s->p);
    free(h);
    free(g);
}

/* Anisotropy with the derivatives the reverse sweep needs: with theta the angle of the normal,
 * C = cos(n theta), S = sin(n theta), dC/dG = n S (gy, -gx)/|G|^2 and dS/dG = n C (-gy, gx)/|G|^2. */
typedef struct {
    int on;            /* |G|^2 above the threshold */
    double C, S, a, c; /* a = 1 + eps C; N = c (gy, -gx), c = kappa Dphi n eps a S */
    double Nx, Ny;
} aniso_t;

static aniso_t aniso(const orc_params* p, double gx, double gy)
{
    aniso_t r;
    double G2 = gx * gx + gy * gy;
    r.on = G2 > p->grad_eps2;
    if (!r.on) {
        r.C = r.S = r.c = r.Nx = r.Ny = 0.0;
        r.a = 1.0;
        return r;
    }
    double theta = atan2(-gy, -gx);
    double m = (double)p->n_fold;
    r.C = cos(m * theta);
    r.S = sin(m * theta);
    r.a = 1.0 + p->eps * r.C;
    r.c = p->kappa_N * (p->W0 * p->W0 / p->tau0) * m * p->eps * r.a * r.S;
    r.Nx = r.c * gy;
    r.Ny = -r.c * gx;
    return r;
}

/* One reverse step: state s at t, adjoint lin at t+1 -> lout at t; returns the explicit
 * dL/deps contribution of this step.  Periodic domain, no flow. */
static double adj_step(const orc_params* p, const state* s, const state* lin, state* lout, double* phi,
                       double* Gbx, double* Gby, double* Bv, double* Ah, double* phib)
{
    const int nx = p->nx, ny = p->ny;
    const int64_t n = (int64_t)nx * ny;
    const double Dphi = p->W0 * p->W0 / p->tau0;
    const double cN = p->kappa_N * Dphi * (double)p->n_fold; /* c = cN eps a S */
    double* deps_row = calloc((size_t)ny, sizeof(double));  /* per-row sums, added in row order */

    for (int64_t i = 0; i < n; ++i) {
        double v = 0.0;
        for (int q = 0; q < 9; ++q) v += s->h[9 * i + q];
        phi[i] = v;
    }
    /* pass 1: everything local to a cell, plus the adjoint of its gradient */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t i = (int64_t)y * nx + x;
            const double* h = &s->h[9 * i];
            const double* g = &s->g[5 * i];
            const double ph = phi[i];
            double U = 0.0;
            for (int q = 0; q < 5; ++q) U += g[q];
            /* forward recompute */
            double gx = 0.0, gy = 0.0;
            for (int q = 1; q < 9; ++q) {
                double w = E4_W[CX[q] * CX[q] + CY[q] * CY[q]];
                double v = phi[(int64_t)wrap(y + CY[q], ny) * nx + wrap(x + CX[q], nx)];
                gx += w * CX[q] * v;
                gy += w * CY[q] * v;
            }
            aniso_t A = aniso(p, gx, gy);
            double a2 = A.a * A.a, ia2 = 1.0 / a2, B = (1.0 - a2) / a2;
            double eta = a2 * Dphi / CS2 + 0.5, ie = 1.0 / eta;
            double om = 1.0 - ph * ph;
            double Q = (ph - ph * ph * ph) + p->lambda * U * om * om;
            double heq[9], hs[9];
            for (int q = 0; q < 9; ++q) {
                heq[q] = W9[q] * (ph - (CX[q] * A.Nx + CY[q] * A.Ny) / CS2);
                hs[q] = h[q] - (h[q] - heq[q]) * ie + W9[q] * Q / p->tau0;
            }
            /* reverse of the phase-field collision and push (P_q = hs_q / a^2, B = (1-a^2)/a^2) */
            double ia2b = 0.0, Bb = 0.0, ieb = 0.0, Qb = 0.0, phb = 0.0, Nxb = 0.0, Nyb = 0.0;
            for (int q = 0; q < 9; ++q) {
                int64_t d = (int64_t)wrap(y + CY[q], ny) * nx + wrap(x + CX[q], nx);
                double Pb = lin->h[9 * d + q];     /* dL/dP_q(x) = lambda_h,q(x + c_q) */
                double hold = s->h[9 * d + q];     /* h_q(x + c_q, t) */
                Bb -= Pb * hold;
                ia2b += Pb * hs[q];
                double hsb = Pb * ia2;
                ieb += hsb * (heq[q] - h[q]);
                double heqb = hsb * ie;
                Qb += hsb * W9[q] / p->tau0;
                phb += W9[q] * heqb;
                Nxb -= W9[q] * heqb * CX[q] / CS2;
                Nyb -= W9[q] * heqb * CY[q] / CS2;
            }
            phb += Qb * (1.0 - 3.0 * ph * ph - 4.0 * p->lambda * U * ph * om);
            double Ub = Qb * p->lambda * om * om;
            ia2b += Bb;                          /* B = ia2 - 1 */
            double a2b = -ia2 * ia2 * ia2b;
            double etab = -ie * ie * ieb;
            a2b += etab * Dphi / CS2;
            double ab = 2.0 * A.a * a2b;
            double gxb = 0.0, gyb = 0.0;
            if (A.on) {
                double cb = gy * Nxb - gx * Nyb;  /* N = c (gy, -gx) */
                gxb += -A.c * Nyb;
                gyb += A.c * Nxb;
                ab += cN * p->eps * A.S * cb;
                double Sb = cN * p->eps * A.a * cb;
                deps_row[y] += A.C * ab + cN * A.a * A.S * cb;
                double Cb = p->eps * ab;
                double G2 = gx * gx + gy * gy, m = (double)p->n_fold;
                gxb += Cb * m * A.S * gy / G2 + Sb * m * A.C * (-gy) / G2;
                gyb += Cb * m * A.S * (-gx) / G2 + Sb * m * A.C * gx / G2;
            }
            /* reverse of the vapour collision and push */
            double qd = 0.5 * (1.0 - ph);
            int inside = qd > 0.0 && qd < 1.0;
            qd = qd < 0.0 ? 0.0 : (qd > 1.0 ? 1.0 : qd);
            double tg = 0.5 + (p->tau_vap - 0.5) * qd, itg = 1.0 / tg;
            double itgb = 0.0, srcb = 0.0;
            for (int q = 0; q < 5; ++q) {
                int64_t d = (int64_t)wrap(y + CY[q], ny) * nx + wrap(x + CX[q], nx);
                double gsb = lin->g[5 * d + q];
                double geq = W5[q] * U;
                itgb -= gsb * (g[q] - geq);
                Ub += W5[q] * gsb * itg;          /* through g_eq */
                srcb -= W5[q] * gsb;
                lout->g[5 * i + q] = gsb * (1.0 - itg);
            }
            phb += 0.5 * p->L_sat * srcb;
            lout->p[i] = -0.5 * p->L_sat * srcb;
            double tgb = -itg * itg * itgb;
            if (inside) phb += -0.5 * (p->tau_vap - 0.5) * tgb;
            phb += lin->p[i];                      /* phi_prev(t+1) = phi(t) */
            for (int q = 0; q < 5; ++q) lout->g[5 * i + q] += Ub;  /* U = sum g */
            Gbx[i] = gxb;
            Gby[i] = gyb;
            Bv[i] = B;
            Ah[i] = ia2 * (1.0 - ie);
            phib[i] = phb;
        }
    /* pass 2: the adjoint of h gathers the gradient stencil and the destination term of Eq. (d) */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t i = (int64_t)y * nx + x;
            double phb = phib[i];
            for (int k = 1; k < 9; ++k) {  /* phi(x) entered G(x - c_k) with weight W_k c_k */
                int64_t j = (int64_t)wrap(y - CY[k], ny) * nx + wrap(x - CX[k], nx);
                double w = E4_W[CX[k] * CX[k] + CY[k] * CY[k]];
                phb += w * (CX[k] * Gbx[j] + CY[k] * Gby[j]);
            }
            for (int q = 0; q < 9; ++q) {
                int64_t d = (int64_t)wrap(y + CY[q], ny) * nx + wrap(x + CX[q], nx);
                int64_t u = (int64_t)wrap(y - CY[q], ny) * nx + wrap(x - CX[q], nx);
                double v = lin->h[9 * d + q] * Ah[i];    /* through h*_q(x) into P_q(x)        */
                v -= Bv[u] * lin->h[9 * i + q];          /* as h_q(x) in the push from x - c_q */
                lout->h[9 * i + q] = v + phb;            /* phi = sum h                         */
            }
        }
    double deps = 0.0;
    for (int y = 0; y < ny; ++y) deps += deps_row[y];
    free(deps_row);
    return deps;
}

double orc_adj_run(const orc_params* p, double xs, double ys, double R, double w_init, const double* U_init,
                   const double* phi_target, int32_t nsteps, int32_t stride, double* dL_dUinit, double* dL_deps,
                   double* phiT_out)
{
    if (!p || p->flow || p->inout || nsteps < 0 || (p->stencil != 0 && p->stencil != 4) || p->symmetric)
        return NAN;
    const int64_t n = (int64_t)p->nx * p->ny;
    int s = stride > 0 ? stride : (int)ceil(sqrt((double)(nsteps > 0 ? nsteps : 1)));
    int nck = nsteps > 0 ? (nsteps + s - 1) / s : 1;
    orc* o = orc_create(p);
    if (!o) return NAN;
    orc_init_seed(o, xs, ys, R, w_init, 0.0, U_init);

    /* forward sweep with checkpoints */
    state* ck = calloc((size_t)nck, sizeof(state));
    for (int k = 0; k < nck; ++k) {
        state_alloc(&ck[k], (size_t)n);
        state_from_oracle(o, p, &ck[k]);
        int len = nsteps - k * s < s ? nsteps - k * s : s;
        orc_step(o, len);
    }
    double* phi = malloc(n * sizeof(double));
    orc_fields(o, phi, NULL, NULL, NULL, NULL);
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) L += (phi[i] - phi_target[i]) * (phi[i] - phi_target[i]);
    if (phiT_out) memcpy(phiT_out, phi, n * sizeof(double));

    /* reverse sweep */
    state la, lb;
    state_alloc(&la, (size_t)n);
    state_alloc(&lb, (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        double v = 2.0 * (phi[i] - phi_target[i]);
        for (int q = 0; q < 9; ++q) la.h[9 * i + q] = v;
        for (int q = 0; q < 5; ++q) la.g[5 * i + q] = 0.0;
        la.p[i] = 0.0;
    }
    state* seg = calloc((size_t)s, sizeof(state));
    for (int k = 0; k < s; ++k) state_alloc(&seg[k], (size_t)n);
    double* Gbx = malloc(n * sizeof(double));
    double* Gby = malloc(n * sizeof(double));
    double* Bv = malloc(n * sizeof(double));
    double* Ah = malloc(n * sizeof(double));
    double* phib = malloc(n * sizeof(double));
    double deps = 0.0;
    for (int k = nck - 1; k >= 0; --k) {
        int len = nsteps - k * s < s ? nsteps - k * s : s;
        state_to_oracle(o, p, &ck[k]);
        for (int t = 0; t < len; ++t) {
            state_from_oracle(o, p, &seg[t]);
            if (t + 1 < len) orc_step(o, 1);
        }
        for (int t = len - 1; t >= 0; --t) {
            deps += adj_step(p, &seg[t], &la, &lb, phi, Gbx, Gby, Bv, Ah, phib);
            state tmp = la;
            la = lb;
            lb = tmp;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double v = 0.0;
        for (int q = 0; q < 5; ++q) v += W5[q] * la.g[5 * i + q];
        dL_dUinit[i] = v;
    }
    *dL_deps = deps;

    for (int k = 0; k < nck; ++k) state_free(&ck[k]);
    for (int k = 0; k < s; ++k) state_free(&seg[k]);
    free(ck);
    free(seg);
    state_free(&la);
    state_free(&lb);
    free(Gbx);
    free(Gby);
    free(Bv);
    free(Ah);
    free(phib);
    free(phi);
    orc_destroy(o);
    return L;
}

double orc_loss(const orc_params* p, double xs, double ys, double R, double w_init, const double* U_init,
                const double* phi_target, int32_t nsteps, double* phiT_out)
{
    const int64_t n = (int64_t)p->nx * p->ny;
    orc* o = orc_create(p);
    if (!o) return NAN;
    orc_init_seed(o, xs, ys, R, w_init, 0.0, U_init);
    orc_step(o, nsteps);
    double* phi = malloc(n * sizeof(double));
    orc_fields(o, phi, NULL, NULL, NULL, NULL);
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) L += (phi[i] - phi_target[i]) * (phi[i] - phi_target[i]);
    if (phiT_out) memcpy(phiT_out, phi, n * sizeof(double));
    free(phi);
    orc_destroy(o);
    return L;
}
