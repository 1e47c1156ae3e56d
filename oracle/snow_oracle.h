/*
 * snow_oracle.h -- FP64 CPU oracle of the coupled lattice-Boltzmann step for ice-crystal growth
 * (Tan, Hosseini, Seidel-Morgenstern, Thevenin, Lorenz, "Modeling ice crystal growth using the
 * lattice Boltzmann method", arXiv:2101.07163).
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously-correct reference that the GPU
 * library is checked against. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code, header or table with the GPU library.
 *
 * Units: lattice units, dx = dt = 1.  All host memory.  Population arrays exchanged through this
 * API use the canonical layout [q][y][x] (plane of direction q, rows of length nx).
 */
#ifndef SNOW_ORACLE_H
#define SNOW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;
    int32_t flow;     /* 1: D2Q9 flow solver on (Sec. 2.2.1); 0: u = 0 everywhere            */
    int32_t inout;    /* 0: periodic in x; 1: fixed-velocity inlet at x = 0, zero-gradient outlet
                         at x = nx-1 (Sec. 3.1.3, 3.2.2); y is always periodic                  */
    int32_t n_fold;   /* symmetry of the anisotropy function: 6 (Sec. 2.1) or 4 (Sec. 3.1.2)     */
    int32_t stencil;  /* isotropic gradient of Sec. 3.1.1: 2 (central difference), 4, 6 or 8
                         (the E4, E6, E8 weights of Table 1); 0 means 4                            */
    double eps;       /* anisotropy strength epsilon_xy                                         */
    double W0, tau0;  /* interface width and characteristic time                                */
    double lambda;    /* phase / supersaturation coupling                                        */
    double L_sat;     /* depletion ("absorption") rate                                           */
    double tau_vap;   /* vapour relaxation time in the fluid: D = cs2 (tau_vap - 1/2)            */
    double tau_f;     /* flow relaxation time: nu = cs2 (tau_f - 1/2)                            */
    double h_drag;    /* dimensionless drag constant h of the solid force (2.757)                */
    double kappa_N;   /* factor on the anisotropic flux: 1 = a da/dgrad(phi), 2 = d(a^2)/dgrad   */
    double rho0, u_in, U_in;  /* inlet state (density, x-velocity, supersaturation)             */
    double grad_eps2; /* |grad phi|^2 below which the normal is undefined (a = 1, N = 0)          */
    int32_t symmetric; /* 0: diffusivity switch q(phi) = (1 - phi)/2 of Eq. (b) (vapour, one-sided);
                          1: q = 1 in both phases (the thermal model of the Sec. 3.1.1 study)       */
    int32_t pad_;
} orc_params;

typedef struct orc orc;

/* Lifecycle.  Returns NULL on invalid sizes or allocation failure. */
orc* orc_create(const orc_params* p);
void orc_destroy(orc* o);

/* Circular seed (tanh profile) centred at (xs, ys) of radius R and width w_init, uniform
 * supersaturation U0 (or the per-cell field U_init[y*nx+x] when non-NULL), equilibrium populations. */
void orc_init_seed(orc* o, double xs, double ys, double R, double w_init, double U0,
                   const double* U_init);

/* Raw state exchange in canonical layout.  Any pointer may be NULL (that part is left alone). */
void orc_set_state(orc* o, const double* f, const double* g, const double* h, const double* phip);
void orc_get_state(const orc* o, double* f, double* g, double* h, double* phip);

/* Advance n steps. */
void orc_step(orc* o, int32_t n);
int64_t orc_step_count(const orc* o);

/* Macroscopic fields at the current step, each ny*nx, x fastest.  Any pointer may be NULL.
 * ux, uy are the velocity seen by the collisions (after drag and the solid projection). */
void orc_fields(const orc* o, double* phi, double* U, double* rho, double* ux, double* uy);

/* FP64 diagnostics: sum rho, sum jx, sum jy, sum U, sum phi, sum phi_prev, #(phi > 0), #non-finite */
void orc_diag(const orc* o, double out[8]);

/* Pure building blocks, exposed so that tests can pin them one by one. */
void orc_feq(double rho, double ux, double uy, double out[9]);
void orc_geq(double U, double ux, double uy, double out[5]);
void orc_guo(const orc_params* p, double ux, double uy, double Fx, double Fy, double out[9]);
void orc_aniso(const orc_params* p, double gx, double gy, double* a, double* Nx, double* Ny);
/* Isotropic gradient (the stencil of this parameter set) of phi[y*nx+x] with its boundary ghosts. */
void orc_grad(const orc_params* p, const double* phi, double* gx, double* gy);

/* Discrete adjoint (no flow, periodic, E4 gradient, one-sided diffusivity): runs n steps from the seed with the per-cell initial
 * supersaturation U_init, evaluates L = sum (phi_T - phi_target)^2, and returns L together with
 * dL/dU_init (ny*nx) and dL/deps, propagated backwards from checkpoints every `stride` steps
 * (0: ceil(sqrt(n))).  phiT_out (optional) receives phi_T.  NaN on invalid input. */
double orc_adj_run(const orc_params* p, double xs, double ys, double R, double w_init, const double* U_init,
                   const double* phi_target, int32_t nsteps, int32_t stride, double* dL_dUinit, double* dL_deps,
                   double* phiT_out);
/* The same loss without gradients (for finite differences). */
double orc_loss(const orc_params* p, double xs, double ys, double R, double w_init, const double* U_init,
                const double* phi_target, int32_t nsteps, double* phiT_out);

/* Threads the oracle runs on (OpenMP). */
int32_t orc_threads(void);
/* Number of OpenMP threads of the following calls (n > 0). */
void orc_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
