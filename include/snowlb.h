/*
 * snowlb.h -- C ABI of the MI355X (gfx950) coupled lattice-Boltzmann ice-crystal growth step.
 *
 * Method: Tan, Hosseini, Seidel-Morgenstern, Thevenin, Lorenz, "Modeling ice crystal growth using the
 * lattice Boltzmann method" (arXiv:2101.07163).  One step advances, on a 2D lattice (dx = dt = 1):
 *   - the D2Q9 BGK flow with the crystal as a phase-dependent solid: drag force and the velocity
 *     projection u* = (1 - phi)/2 u (Sec. 2.2.1);
 *   - the D2Q5 advection-diffusion-reaction LB for the supersaturation U, with the depletion source
 *     -w (L_sat/2) d(phi)/dt and diffusivity switched off in the ice (Sec. 2.2.2, Eq. b);
 *   - the phase-field LB of Eq. (d) with the equilibrium of Eq. (e), the 6-fold anisotropy
 *     a_s(n) = 1 + eps cos(6 theta) (Sec. 2.1) and the isotropic E4 gradient of Table 1 (Sec. 3.1.1).
 *
 * Conventions
 *   - Every function returns a snowlb_status (0 = OK) or is documented otherwise; nothing aborts or
 *     throws across this boundary.  On error, snowlb_last_error(ctx) holds a message.
 *   - Pointers named *_dev are device pointers (e.g. a torch tensor's data_ptr()); *_host are host
 *     pointers.  The caller owns every buffer it passes; the library owns its context's buffers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is enqueued
 *     asynchronously on it unless stated otherwise.
 *   - Fields are ny x nx, row-major, x fastest.  Population sets exchanged with the caller are in the
 *     canonical layout [q][y][x] as FP32, whatever the internal storage.
 *   - A context is used from one host thread at a time; distinct contexts may be used concurrently.
 *     The library keeps no global mutable state except the per-thread error string of context-free
 *     calls and the autotuner's cache file (read and appended under file locks).
 *
 * Environment (read once per use, all optional)
 *   SNOWLB_TUNE_CACHE      file of the autotuner's cache (default $HOME/.cache/snowlb_tune.txt)
 *   SNOWLB_TUNE_STEPS      steps per timing sample of the autotuner (default 20, even)
 *   SNOWLB_BUFFER_STAGGER  bytes added after each 64 KiB-padded buffer of a lattice so that the
 *                          buffers a tile touches start on different HBM channels (default 2304)
 *   SNOWLB_GRAPH_STEPS     steps per captured graph of snowlb_step (default 32, even); fewer steps
 *                          than that are replayed from a captured two-step graph
 *   SNOWLB_NO_GRAPH        1: launch every step directly instead of replaying graphs
 *   SNOWLB_ADJ_OVERLAP     0: run the adjoint backward pass in serial order on the caller's stream
 *                          (default 1: recompute the next checkpoint interval on a second stream of
 *                          the context while the current one is reversed; bitwise the same results)
 */
#ifndef SNOWLB_H
#define SNOWLB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t snowlb_status;
#define SNOWLB_OK 0
#define SNOWLB_EINVAL (-1)       /* invalid argument or parameter set (checked before any GPU call) */
#define SNOWLB_ENOMEM (-2)       /* device or host allocation failed                                */
#define SNOWLB_EDEVICE (-3)      /* a HIP call failed; snowlb_last_error has the HIP message        */
#define SNOWLB_EUNSUPPORTED (-4) /* valid request the library does not support                      */
#define SNOWLB_ENONFINITE (-5)   /* a diagnostic found non-finite populations                       */
#define SNOWLB_ESTATE (-6)       /* call out of order (e.g. step before init)                       */

/* internal storage of the populations (the collision arithmetic is FP32 in all cases) */
#define SNOWLB_STORE_FP32 0
#define SNOWLB_STORE_FP16 1 /* FP16 deviations d = p/w - m, round-to-nearest-even, from local
                               references m: for f_q, rho + 3 c_q.j of the cell it streamed from;
                               for g_q, U (1 + 3 c_q.j) of that cell (U alone without flow); for
                               h_q, phi(t-1) of the cell that holds it.  Each cell's U, rho, jx, jy,
                               rounded to the same 16-bit format, are kept in 16-bit reference
                               planes inside the population buffer, so writer and reader use the
                               same rounded values.  phi_prev stays FP32.                        */
#define SNOWLB_STORE_BF16 2 /* BF16 deviations, same encoding                                   */

/* closure in x (y is always periodic) */
#define SNOWLB_BC_PERIODIC 0
#define SNOWLB_BC_INOUT 1 /* fixed-velocity inlet at x = 0, zero-gradient outlet at x = nx-1 (Sec. 3.1.3) */

/* macroscopic fields for snowlb_read */
#define SNOWLB_FIELD_PHI 0 /* phase field phi = sum h                                          */
#define SNOWLB_FIELD_U 1   /* supersaturation U = sum g                                        */
#define SNOWLB_FIELD_RHO 2 /* density sum f (0 without flow)                                  */
#define SNOWLB_FIELD_UX 3  /* x-velocity used by the collisions (after drag and projection)    */
#define SNOWLB_FIELD_UY 4

/* population sets for snowlb_read_populations / snowlb_write_populations */
#define SNOWLB_POP_F 0    /* 9 planes (flow; only when params.flow = 1) */
#define SNOWLB_POP_G 1    /* 5 planes (vapour)                          */
#define SNOWLB_POP_H 2    /* 9 planes (phase field)                     */
#define SNOWLB_POP_PHIP 3 /* 1 plane: phi at the previous step          */

typedef struct {
    int32_t nx, ny;     /* lattice size: 2 <= nx, ny <= 65536, and the populations of one copy
                           (with their 16-bit references) on the lattice padded to whole 64 x 4
                           blocks within 4 GiB (every byte offset inside a buffer fits 32 bits):
                           at most 46.7M cells in FP32 with flow, 76.7M without; 79.5M / 143M in
                           16-bit storage                                                     */
    int32_t flow;       /* 1: D2Q9 flow solver on; 0: u = 0 (no f populations stored)           */
    int32_t bc_x;       /* SNOWLB_BC_PERIODIC or SNOWLB_BC_INOUT (needs flow = 1)               */
    int32_t storage;    /* SNOWLB_STORE_*                                                       */
    int32_t n_fold;     /* 6 (hexagonal ice, Sec. 2.1) or 4 (Sec. 3.1.2)                        */
    double eps;         /* anisotropy strength, 0 <= eps < 0.5 (a_s = 1 + eps cos stays positive)  */
    double W0, tau0;    /* interface width and time, > 0                                         */
    double lambda;      /* coupling constant                                                      */
    double L_sat;       /* depletion rate                                                         */
    double tau_vap;     /* vapour relaxation time in the fluid, > 1/2: D = (tau_vap - 1/2)/3       */
    double tau_f;       /* flow relaxation time, > 1/2: nu = (tau_f - 1/2)/3                       */
    double h_drag;      /* drag constant h of the solid force (2.757)                            */
    double kappa_N;     /* 1: flux |grad phi|^2 a da/d(grad phi); 2: |grad phi|^2 d(a^2)/d(grad phi) */
    double rho0;        /* reference / inlet density                                              */
    double u_in;        /* inlet x-velocity, |u_in| < 0.1                                         */
    double U_in;        /* inlet supersaturation                                                  */
    double grad_eps2;   /* |grad phi|^2 at or below which a = 1 and the flux N = 0 (1e-10)        */
    double U0;          /* initial supersaturation (when no U_init field is given)                */
    double seed_x, seed_y, seed_r; /* circular seed: centre and radius (cells)                   */
    double init_width;  /* width of the tanh seed profile (cells)                                 */
    int32_t diag_every; /* >0: snowlb_step checks for non-finite values every this many steps     */
    int32_t tile;       /* step-kernel tile configuration; -1 = autotune, 0 = default            */
    int32_t stencil;    /* isotropic gradient of phi (Sec. 3.1.1): 4 = E4 (default), 6 = E6, 8 = E8
                           (Table 1 weights), 2 = E2 (the central difference of the same section);
                           E6 and E8 reach two cells and stage a two-cell halo                      */
    int32_t symmetric;  /* 0: diffusivity switch q(phi) = (1 - phi)/2 of Eq. (b) (vapour, no
                           diffusion in the ice); 1: q = 1 in both phases (the symmetric thermal
                           model of the Sec. 3.1.1 stencil study)                                   */
} snowlb_params;

typedef struct snowlb_ctx snowlb_ctx;

/* Defaults: the 128^2 periodic, flow-off workload (eps 0.05, W0 1, tau0 10, lambda 3, L_sat 1.6,
 * tau_vap 0.8, tau_f 0.6, h 2.757, kappa_N 1, seed R 5 at the centre, U0 0.5). Never fails. */
void snowlb_params_default(snowlb_params* p);

/* Validate a parameter set without touching the GPU.  EINVAL with a message in *msg_out (static
 * storage, may be NULL) when a value is out of range. */
snowlb_status snowlb_validate(const snowlb_params* p, const char** msg_out);

/* Human-readable name of a status code (static storage). */
const char* snowlb_status_str(snowlb_status s);
/* Last error message of a context (valid until the next call on it); "" if none; ctx may be NULL,
 * then the message of the last failed context-free call (snowlb_create, snowlb_bw_probe) on this
 * thread is returned. */
const char* snowlb_last_error(const snowlb_ctx* ctx);

/* Create a context on the current HIP device: validates (EINVAL before any GPU call), then
 * allocates two copies of the populations and phi_prev.  *out is NULL on failure. */
snowlb_status snowlb_create(const snowlb_params* p, snowlb_ctx** out);
/* Release a context (NULL-safe).  Synchronises the device first. */
void snowlb_destroy(snowlb_ctx* ctx);

/* Initial state (the circular seed of radius R of Sec. 3.1.2 and Sec. 3.2.2 in uniform
 * supersaturation): phi0 = tanh((R - r)/(sqrt 2 width)) around (seed_x, seed_y), phi_prev = phi0,
 * h_q = w_q phi0, equilibrium populations g = g_eq(U, u0) of Sec. 2.2.2 at U = U_init (ny x nx device
 * field, caller-owned, read before the call's work completes) or at params.U0 when U_init_dev is
 * NULL, f = f_eq(rho0, u0) of Sec. 2.2.1 with the projected velocity u0 = (1 - phi0)/2 (u_in, 0) for a
 * ventilated domain and 0 otherwise.  Resets the step count.  EINVAL for a NULL ctx. */
snowlb_status snowlb_init(snowlb_ctx* ctx, const float* U_init_dev, void* stream);

/* Advance n >= 0 steps (asynchronous).  With diag_every > 0 the host synchronises every diag_every
 * steps and returns ENONFINITE as soon as a non-finite population is found.  ESTATE before init. */
snowlb_status snowlb_step(snowlb_ctx* ctx, int32_t n, void* stream);
int64_t snowlb_step_count(const snowlb_ctx* ctx);

/* Write one macroscopic field (SNOWLB_FIELD_*) of the current state into dst_dev (float,
 * dst_elems >= nx*ny, caller-owned, ny x nx, x fastest): the moments of the populations, phi = sum h
 * (Sec. 2.2.3), U = sum g (Sec. 2.2.2), rho = sum f, and the velocity of Sec. 2.2.1 that the
 * collisions use, u = (1 - phi)/2 j/(rho + k/2) (the momentum after the half-force drag correction,
 * then the projection; 0 without flow).  EINVAL for an unknown field or a short buffer, ESTATE before
 * the state is initialised. */
snowlb_status snowlb_read(snowlb_ctx* ctx, int32_t field, float* dst_dev, int64_t dst_elems,
                          void* stream);

/* Debugging and tests: overwrite one macroscopic field of the current state from src_dev (float,
 * src_elems >= nx*ny, caller-owned, x fastest).  SNOWLB_FIELD_PHI sets h_q = w_q phi and
 * phi_prev = phi (the phase field at rest, without the anisotropic flux); SNOWLB_FIELD_U sets
 * g_q = g_eq(U, u) with the velocity u the collisions currently see (0 without flow).  Other fields:
 * SNOWLB_EINVAL.  Needs an initialised state (SNOWLB_ESTATE otherwise). */
snowlb_status snowlb_write_field(snowlb_ctx* ctx, int32_t field, const float* src_dev, int64_t src_elems,
                                 void* stream);

/* Copy a population set (SNOWLB_POP_*) of the current state to / from caller memory in the canonical
 * FP32 layout [q][y][x] (elems >= Q*nx*ny).  Writing encodes into the context's storage format. */
snowlb_status snowlb_read_populations(snowlb_ctx* ctx, int32_t set, float* dst_dev, int64_t elems,
                                      void* stream);
snowlb_status snowlb_write_populations(snowlb_ctx* ctx, int32_t set, const float* src_dev,
                                       int64_t elems, void* stream);

/* FP64 conservation diagnostics of the current state, synchronous (waits for `stream`); out_host
 * holds SNOWLB_DIAG_COUNT doubles:
 *   out[0..7] = sum rho, sum jx, sum jy, sum U, sum phi, sum phi_prev, #(phi > 0), #non-finite cells;
 *   out[8]    = the species invariant sum U + (L_sat/2) sum phi_prev.
 * Mass and momentum are the moments of the flow populations (Sec. 2.2.1); the invariant follows from
 * the depletion source -w (L_sat/2) d(phi)/dt of Sec. 2.2.2 taken as phi(t) - phi(t-1): the vapour
 * lost by a collision is (L_sat/2) times the phase gained, so out[8] is constant in a periodic
 * domain.  Sums are reduced in FP64 in a fixed order (deterministic).  Returns ENONFINITE if
 * out[7] > 0 (out is filled), EINVAL for NULL arguments, ESTATE before the state is initialised. */
#define SNOWLB_DIAG_COUNT 9
snowlb_status snowlb_diag(snowlb_ctx* ctx, double* out_host, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the diagnostics of snowlb_diag, bitwise the same values, written
 * asynchronously on `stream` to out_dev (SNOWLB_DIAG_COUNT doubles of caller-owned device memory)
 * without waiting for the stream and without allocating anything.  The per-workgroup partial sums
 * go to a static device array of the library (2048 x 8 doubles = 128 KiB, one copy per GPU, held until
 * the process ends); every call on a GPU shares that array, so calls that overlap on one GPU (on
 * concurrent streams) race, and their results are undefined.  Nothing in the array needs to start at
 * zero: each call writes every partial it reads.  The partial count is at most 2048 for any lattice
 * (larger lattices sum more cells per thread); a larger demand would return EINVAL.  Non-finite
 * cells are counted in out_dev[7]; the call itself returns OK.  EINVAL for NULL arguments, ESTATE
 * before the state is initialised. */
snowlb_status snowlb_diag_noalloc(snowlb_ctx* ctx, double* out_dev, void* stream);

/* Checkpoint / resume: the whole state (populations, phi_prev) and the step count, as an opaque
 * device buffer of snowlb_state_bytes() bytes.  load_state requires a buffer saved from a context
 * with identical sizes and storage. */
int64_t snowlb_state_bytes(const snowlb_ctx* ctx);
snowlb_status snowlb_save_state(snowlb_ctx* ctx, void* buf_dev, int64_t bytes, void* stream);
snowlb_status snowlb_load_state(snowlb_ctx* ctx, const void* buf_dev, int64_t bytes, void* stream);

/* Step-kernel tile configurations.  snowlb_tile_count() configurations exist; snowlb_tile_name(i)
 * describes one ("64x4" = 64 cells in x by 4 in y per workgroup).  snowlb_set_tile selects one for
 * a context; results are bitwise identical for every configuration.  Grid modes (0..5): bit 0 selects
 * a persistent grid of resident workgroups looping over the tiles (else one workgroup per tile);
 * grid_mode >> 1 the tile order: 0 row order, 1 vertical strips 512 cells wide, 2 four vertical strips
 * of nearly equal width (each strip walked row by row).  0 is the default; the autotuner (tile = -1)
 * times all six.  Other values are rejected with SNOWLB_EINVAL. */
int32_t snowlb_tile_count(void);
const char* snowlb_tile_name(int32_t i);
snowlb_status snowlb_set_tile(snowlb_ctx* ctx, int32_t tile);
int32_t snowlb_get_tile(const snowlb_ctx* ctx);
snowlb_status snowlb_set_grid_mode(snowlb_ctx* ctx, int32_t grid_mode);
int32_t snowlb_get_grid_mode(const snowlb_ctx* ctx);

/* ---------------------------------------------------------------------------------------------
 * Discrete adjoint (contexts with flow = 0, periodic x, FP32 storage, stencil 4 and symmetric = 0;
 * EUNSUPPORTED otherwise).
 *
 * snowlb_adj_forward runs n >= 1 steps from the current state (normally right after snowlb_init),
 * keeping a checkpoint of the state every ckpt_stride steps (0: ceil(sqrt(n))); afterwards the
 * context holds phi_T (read it with snowlb_read).  snowlb_adj_backward then takes dL/dphi_T
 * (ny x nx device field) for any loss L(phi_T) and returns, by the hand-written reverse of each step
 * with the states recomputed from the checkpoints: dL/dU_init (ny x nx device field, the gradient
 * with respect to the initial supersaturation field), dL/deps and dL/dU0 = sum dL/dU_init (host
 * doubles, reduced in FP64 in a fixed order).  Memory: about (n/stride + 2 stride) state copies.
 * The backward may be called several times after one forward (different dL/dphi_T).  It recomputes
 * checkpoint intervals on a second stream that the context owns (see SNOWLB_ADJ_OVERLAP), ordered
 * after all work queued on `stream` before the call; it returns when the work of both is done. */
snowlb_status snowlb_adj_forward(snowlb_ctx* ctx, int32_t n_steps, int32_t ckpt_stride, void* stream);
snowlb_status snowlb_adj_backward(snowlb_ctx* ctx, const float* dL_dphiT_dev, float* dL_dUinit_dev,
                                  double* dL_deps_host, double* dL_dU0_host, void* stream);
/* Change the anisotropy strength of a context (0 <= eps < 0.5); takes effect at the next step. */
snowlb_status snowlb_set_eps(snowlb_ctx* ctx, double eps);

/* ---------------------------------------------------------------------------------------------
 * Batches: many independent crystals (each its own lattice size and parameters) advanced together,
 * one launch per step over the tiles of all domains, replayed from a captured HIP graph.  All
 * domains must share flow, bc_x, storage, n_fold and the reach of the stencil (E2/E4 or E6/E8;
 * they select the kernel); everything else may differ.  Each domain evolves exactly as a context created from the same parameters would
 * (bitwise: same kernel, same per-domain arithmetic). */
typedef struct snowlb_batch snowlb_batch;

/* Create a batch of n >= 1 domains from params[0..n-1] (validated like snowlb_create; EINVAL if
 * they do not share flow, bc_x, storage, n_fold and the stencil reach).  *out is NULL on failure. */
snowlb_status snowlb_batch_create(const snowlb_params* params, int32_t n, snowlb_batch** out);
void snowlb_batch_destroy(snowlb_batch* b);
int32_t snowlb_batch_size(const snowlb_batch* b);
/* Total lattice cells over all domains (-1 for NULL). */
int64_t snowlb_batch_cells(const snowlb_batch* b);
/* Initial state of every domain from its own parameters (seed, U0). */
snowlb_status snowlb_batch_init(snowlb_batch* b, void* stream);
/* Advance every domain n >= 0 steps (asynchronous).  With tile = -1 in params[0], the first call
 * autotunes the tile shape and grid mode for the whole batch. */
snowlb_status snowlb_batch_step(snowlb_batch* b, int32_t n, void* stream);
int64_t snowlb_batch_step_count(const snowlb_batch* b);
/* Field / diagnostics of domain i, as snowlb_read / snowlb_diag (out_host: SNOWLB_DIAG_COUNT doubles). */
snowlb_status snowlb_batch_read(snowlb_batch* b, int32_t i, int32_t field, float* dst_dev, int64_t dst_elems,
                                void* stream);
snowlb_status snowlb_batch_diag(snowlb_batch* b, int32_t i, double* out_host, void* stream);
snowlb_status snowlb_batch_set_tile(snowlb_batch* b, int32_t tile, int32_t grid_mode);
int32_t snowlb_batch_get_tile(const snowlb_batch* b);
const char* snowlb_batch_last_error(const snowlb_batch* b);

/* Practical HBM ceiling probe: copy `bytes` (a multiple of 16) from src_dev to dst_dev with a plain
 * coalesced 16-byte-per-lane grid-stride kernel on `stream`.  Used to report measured bandwidth next
 * to the published peak, and to calibrate byte counters.  Buffers must not overlap. */
snowlb_status snowlb_bw_probe(void* dst_dev, const void* src_dev, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
