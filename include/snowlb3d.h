/*
 * snowlb3d.h -- C ABI of the three-dimensional coupled lattice-Boltzmann ice-growth step on MI355X
 * (gfx950): the extension to three dimensions that Sec. 4 of Tan, Hosseini, Seidel-Morgenstern,
 * Thevenin, Lorenz, "Modeling ice crystal growth using the lattice Boltzmann method"
 * (arXiv:2101.07163) names as future work.  The paper gives the method in two dimensions only; the
 * three-dimensional step applies its Sec. 2.2 on
 *   - a D3Q19 flow lattice (BGK, second-order equilibrium, Guo forcing of the solid drag, the velocity
 *     projection u* = (1 - phi)/2 u of Sec. 2.2.1);
 *   - D3Q7 lattices (cs^2 = 1/4) for the supersaturation U (Sec. 2.2.2; D = (tau_vap - 1/2)/4) and the
 *     phase field (Eq. (d), (e) of Sec. 2.2.3; eta = 4 a^2 W0^2/tau0 + 1/2);
 *   - the isotropic gradient over the 18 D3Q19 neighbours (weights 1/6 on the axes, 1/12 on the face
 *     diagonals: the three-dimensional analogue of the E4 row of Table 1);
 *   - the hexagonal anisotropy of Sec. 2.1 about the crystal's c axis (z):
 *     a = 1 + eps Re((n_x + i n_y)^6) = 1 + eps cos(6 theta) sin^6(psi), the paper's 1 + eps cos 6 theta
 *     for normals in the basal plane and 1 along the c axis.
 *
 * Conventions are those of snowlb.h (status codes, *_dev / *_host pointers, `stream` as void*).  Fields
 * are nz x ny x nx, x fastest; population sets exchanged with the caller are FP32 [q][z][y][x].
 * Storage is FP32.  y and z are periodic; x is periodic or has the inlet / outlet of snowlb.h.
 */
#ifndef SNOWLB3D_H
#define SNOWLB3D_H
#include <stdint.h>

#include "snowlb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* fields for snowlb3d_read */
#define SNOWLB3D_FIELD_PHI 0
#define SNOWLB3D_FIELD_U 1
#define SNOWLB3D_FIELD_RHO 2 /* 0 without flow */
#define SNOWLB3D_FIELD_UX 3  /* velocity the collisions use (after drag and projection) */
#define SNOWLB3D_FIELD_UY 4
#define SNOWLB3D_FIELD_UZ 5
/* population sets: SNOWLB_POP_F (19 planes), SNOWLB_POP_G (7), SNOWLB_POP_H (7), SNOWLB_POP_PHIP (1) */
#define SNOWLB3D_DIAG_COUNT 10

typedef struct {
    int32_t nx, ny, nz;  /* lattice size, 2 <= each <= 65535; the populations of one copy padded
                            to whole 64 x 2 x 2 blocks within 4 GiB (about 32M cells with flow)      */
    int32_t flow;        /* 1: D3Q19 flow on; 0: u = 0                                                */
    int32_t bc_x;        /* SNOWLB_BC_PERIODIC or SNOWLB_BC_INOUT (needs flow = 1)                    */
    int32_t diag_every;  /* > 0: snowlb3d_step checks for non-finite values every this many steps     */
    double eps;          /* anisotropy strength, 0 <= eps < 0.5                                       */
    double W0, tau0;     /* interface width and time, > 0                                             */
    double lambda, L_sat;
    double tau_vap;      /* > 1/2: vapour diffusivity D = (tau_vap - 1/2)/4                            */
    double tau_f;        /* > 1/2: nu = (tau_f - 1/2)/3                                               */
    double h_drag, kappa_N, rho0, u_in, U_in, grad_eps2, U0;
    double seed_x, seed_y, seed_z, seed_r, init_width; /* spherical tanh seed                        */
} snowlb3d_params;

typedef struct snowlb3d_ctx snowlb3d_ctx;

/* Defaults: 64^3 periodic, no flow, eps 0.05, W0 1, tau0 10, lambda 3, L_sat 1.6, tau_vap 0.8,
 * tau_f 0.6, h 2.757, kappa_N 1, U0 0.5, seed R 5 at the centre.  Never fails. */
void snowlb3d_params_default(snowlb3d_params* p);
/* EINVAL with a message (static storage) for an out-of-range parameter; no GPU call. */
snowlb_status snowlb3d_validate(const snowlb3d_params* p, const char** msg_out);
/* Create a context on the current HIP device (validates first); *out is NULL on failure. */
snowlb_status snowlb3d_create(const snowlb3d_params* p, snowlb3d_ctx** out);
void snowlb3d_destroy(snowlb3d_ctx* ctx); /* NULL-safe; synchronises the device first */
/* Last error message of a context, or of the last failed snowlb3d_create on this thread (ctx NULL). */
const char* snowlb3d_last_error(const snowlb3d_ctx* ctx);

/* Initial state: the spherical seed phi0 = tanh((R - r)/(sqrt 2 width)) around (seed_x, seed_y,
 * seed_z) in the supersaturation U_init (nz x ny x nx device field, caller-owned) or params.U0 (NULL),
 * h_q = w_q phi0, phi_prev = phi0, equilibrium f and g at the velocity (1 - phi0)/2 (u_in, 0, 0) when
 * ventilated (0 otherwise).  Resets the step count. */
snowlb_status snowlb3d_init(snowlb3d_ctx* ctx, const float* U_init_dev, void* stream);
/* Advance n >= 0 steps (asynchronous, replayed from captured graphs).  ESTATE before init. */
snowlb_status snowlb3d_step(snowlb3d_ctx* ctx, int32_t n, void* stream);
int64_t snowlb3d_step_count(const snowlb3d_ctx* ctx);
/* A macroscopic field (SNOWLB3D_FIELD_*) into dst_dev (dst_elems >= nx*ny*nz floats). */
snowlb_status snowlb3d_read(snowlb3d_ctx* ctx, int32_t field, float* dst_dev, int64_t dst_elems, void* stream);
/* Population sets (SNOWLB_POP_*) to / from caller memory, FP32 [q][z][y][x] (elems >= Q nx ny nz). */
snowlb_status snowlb3d_read_populations(snowlb3d_ctx* ctx, int32_t set, float* dst_dev, int64_t elems,
                                        void* stream);
snowlb_status snowlb3d_write_populations(snowlb3d_ctx* ctx, int32_t set, const float* src_dev, int64_t elems,
                                         void* stream);
/* FP64 sums, synchronous: out[0..9] = sum rho, sum jx, sum jy, sum jz, sum U, sum phi, sum phi_prev,
 * #(phi > 0), #non-finite cells, and the species invariant sum U + (L_sat/2) sum phi_prev (constant in
 * a periodic domain: the depletion source of Sec. 2.2.2 removes (L_sat/2) times the phase gained).
 * Fixed-order reduction.  ENONFINITE if out[8] > 0. */
snowlb_status snowlb3d_diag(snowlb3d_ctx* ctx, double* out_host, void* stream);

#ifdef __cplusplus
}
#endif
#endif
