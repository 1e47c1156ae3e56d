/*
 * snow_oracle3d.h -- FP64 CPU oracle of the three-dimensional coupled lattice-Boltzmann step for
 * ice-crystal growth: the extension of the method of Tan, Hosseini, Seidel-Morgenstern, Thevenin and
 * Lorenz (arXiv:2101.07163) that its Sec. 4 names as future work, built on the readings listed in
 * snow_oracle3d.c.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library's 3D step is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the GPU library.
 *
 * Units: lattice units, dx = dt = 1.  Population arrays exchanged through this API use the canonical
 * layout [q][z][y][x]; fields are [z][y][x], x fastest.
 */
#ifndef SNOW_ORACLE3D_H
#define SNOW_ORACLE3D_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    int32_t flow;     /* 1: D3Q19 flow solver on; 0: u = 0 everywhere                           */
    int32_t inout;    /* 0: periodic in x; 1: fixed-velocity inlet at x = 0, zero-gradient outlet
                         at x = nx-1; y and z are always periodic                                 */
    int32_t pad_;
    double eps;       /* anisotropy strength                                                    */
    double W0, tau0;  /* interface width and characteristic time                                */
    double lambda;    /* phase / supersaturation coupling                                        */
    double L_sat;     /* depletion rate                                                          */
    double tau_vap;   /* vapour relaxation time in the fluid: D = cs2 (tau_vap - 1/2), cs2 = 1/4 */
    double tau_f;     /* flow relaxation time: nu = (tau_f - 1/2)/3                             */
    double h_drag;    /* drag constant h of the solid force (2.757)                              */
    double kappa_N;   /* factor on the anisotropic flux: 1 = a da/dgrad(phi), 2 = d(a^2)/dgrad   */
    double rho0, u_in, U_in;  /* inlet state (density, x-velocity, supersaturation)             */
    double grad_eps2; /* |grad phi|^2 at or below which the normal is undefined (a = 1, N = 0)  */
} orc3_params;

typedef struct orc3 orc3;

orc3* orc3_create(const orc3_params* p);
void orc3_destroy(orc3* o);

/* Spherical seed (tanh profile) centred at (xs, ys, zs) of radius R and width w_init, uniform
 * supersaturation U0 (or the per-cell field U_init[(z ny + y) nx + x] when non-NULL), equilibria. */
void orc3_init_seed(orc3* o, double xs, double ys, double zs, double R, double w_init, double U0,
                    const double* U_init);
void orc3_set_state(orc3* o, const double* f, const double* g, const double* h, const double* phip);
void orc3_get_state(const orc3* o, double* f, double* g, double* h, double* phip);
void orc3_step(orc3* o, int32_t n);
int64_t orc3_step_count(const orc3* o);
/* phi, U, rho and the velocity seen by the collisions (after drag and projection); any may be NULL. */
void orc3_fields(const orc3* o, double* phi, double* U, double* rho, double* ux, double* uy, double* uz);
/* sum rho, sum jx, sum jy, sum jz, sum U, sum phi, sum phi_prev, #(phi > 0), #non-finite */
void orc3_diag(const orc3* o, double out[9]);

/* Building blocks, exposed for the pins. */
void orc3_feq(double rho, double ux, double uy, double uz, double out[19]);
void orc3_geq(double U, double ux, double uy, double uz, double out[7]);
void orc3_aniso(const orc3_params* p, double gx, double gy, double gz, double* a, double* Nx, double* Ny,
                double* Nz);
void orc3_grad(const orc3_params* p, const double* phi, double* gx, double* gy, double* gz);
/* lattice tables: velocities (19 x 3 ints) and weights (19) of D3Q19, weights of D3Q7 (7) */
void orc3_lattice(int32_t* c19, double* w19, double* w7);

#ifdef __cplusplus
}
#endif
#endif
