// snowlb_internal.h -- descriptors shared by the HIP kernels and the host runtime of libsnowlb.
//
// Device layout (per domain): one buffer per copy holds the populations (f_0..f_8 with flow, g_0..g_4,
// h_0..h_8: npop planes) followed, for 16-bit storage, by the 16-bit reference planes U, rho, jx, jy
// (U only without flow) that neighbours read to decode the populations a cell emitted -- nqb planes
// in all; phi_prev (one FP32 plane) has a buffer of its own.  Both store the lattice in blocks of
// 64 x 4 cells with the block's planes side by side (cell_index below).  Two copies of each (index
// par) ping-pong between steps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snowlb {

// address space of device global memory (lets the compiler emit global rather than flat accesses)
#define GMEM __attribute__((address_space(1)))

// Cell order of a buffer of nq planes: blocks of 64 x 4 cells, blocks along x (nbx per block row) and
// block rows along y; inside a block its nq planes follow each other as runs of 256 elements, each
// run four rows of 64 cells.  Element (q, x, y) sits at
//     ((y / 4) nbx + x / 64) nq 256  +  256 q  +  64 (y % 4)  +  x % 64,
// so a 64 x 4 workgroup tile reads and writes one contiguous run of nq * 256 elements and the
// workgroups resident at one time sweep a dense address range.  The index is separable (an x part
// plus a y part), so the nine push destinations cost one add each.  The host keeps every byte offset
// inside one buffer below 2^32.
constexpr int kBlockX = 64, kBlockY = 4, kBlockCells = kBlockX * kBlockY;
constexpr int64_t kMaxBufferBytes = int64_t(1) << 32;  // every in-buffer byte offset fits 32 bits
__host__ __device__ __forceinline__ uint32_t cell_xpart(int x, int nq) {
    return (uint32_t)(x >> 6) * ((uint32_t)nq << 8) + (uint32_t)(x & 63);
}
__host__ __device__ __forceinline__ uint32_t cell_ypart(int nbx, int nq, int y) {
    return (uint32_t)(y >> 2) * (((uint32_t)nbx * (uint32_t)nq) << 8) + ((uint32_t)(y & 3) << 6);
}
__host__ __device__ __forceinline__ int64_t cell_index(int nbx, int nq, int x, int y) {
    return (int64_t)cell_ypart(nbx, nq, y) + cell_xpart(x, nq);
}

// Global accesses of the hot kernels: a base that is uniform over the workgroup plus a 32-bit
// per-lane byte offset.  The empty asm pins the base in scalar registers and keeps the compiler from
// folding a plane stride into a 64-bit per-lane address, so each access is one global load or store
// in scalar-base + vector-offset form (every caller passes a workgroup-uniform base).
template <class T>
__device__ __forceinline__ T gld(const GMEM char* base, uint32_t boff) {
    asm("" : "+s"(base));
    return *(const GMEM T*)(base + boff);
}
template <class T>
__device__ __forceinline__ void gst(GMEM char* base, uint32_t boff, T v) {
    asm("" : "+s"(base));
    *(GMEM T*)(base + boff) = v;
}

struct DomDesc {
    int32_t nx, ny, nbx, npop;    // nbx: 64 x 4 blocks per block row; npop: planes per copy (23 with
                                  // flow, 14 without)
    int64_t plane;                // elements between consecutive planes of a block (kBlockCells)
    void* pop[2];                 // the two population copies
    float* phip[2];               // phi(t-1), FP32, one plane (nq = 1)
    void* refs[2];                // 16-bit storage only: the reference planes U, rho, jx, jy, which
                                  // follow the populations in pop[par] (else null)
    int64_t rplane;               // elements between consecutive reference planes (kBlockCells)
    double grad_eps2;             // |grad phi|^2 (FP64) at or below which a = 1 and N = 0
    int32_t off_g, off_h;         // plane index of g_0 and h_0
    int32_t n_fold, storage;
    int32_t inout;                // x closure: 1 = inlet/outlet
    int32_t nqb;                  // planes per block of a population buffer: npop, plus the
                                  // reference planes (4 with flow, 1 without) in 16-bit storage
    // physics in FP32 (lattice units)
    float eps;          // anisotropy strength
    float Dphi;         // W0^2 / tau0
    float aniso_coef;   // kappa_N * Dphi * n_fold * eps  (flux N = coef * a * S_n * (gy, -gx))
    float inv_tau0;
    float lam;
    float half_Lsat;    // L_sat / 2
    float tauv_m_half;  // tau_vap - 1/2
    float omega_f;      // 1 / tau_f
    float guo;          // 1 - 1/(2 tau_f)
    float kdrag;        // h nu / (4 W0^2), nu = (tau_f - 1/2)/3
    float ref_f;        // 16-bit storage reference of f (rho0)
    float U_in;         // inlet supersaturation
    float u_in;         // inlet x-velocity
    float df_in[9];     // inlet ghost populations f_eq(rho0, (u_in, 0)) - w (flow deviations)
    float g_in[5];      // inlet ghost populations g_eq(U_in, (u_in, 0))
    int32_t sym;        // 1: vapour diffusivity switch q = 1 in both phases (thermal variant);
                        // 0: q = (1 - phi)/2 clamped to [0, 1]
    int32_t stencil;    // isotropic gradient: 2, 4 (one-cell reach) or 6, 8 (two-cell reach)
    float tauf_m_half;  // tau_f - 1/2 (= guo / omega_f)
    double gw[5];       // gradient weights of the layers |c|^2 = 1, 2, 4, 5, 8 (Sec. 3.1.1, Table 1)
};

struct TileDesc {
    int32_t dom, x0, y0, pad;
};

// Launchers (defined in snowlb_kernels.hip).  All are asynchronous on `stream` and return the
// hipError_t of the launch.
int tile_config_count();
const char* tile_config_name(int i);
int tile_config_tx(int i);
int tile_config_ty(int i);
// One step of every tile in `tiles` (device array of ntiles entries), reading copy `par` and writing
// copy 1 - par.  `flow`, `inout`, `storage` and the gradient reach `rad` (1 for E2/E4, 2 for E6/E8)
// must be the same for every domain referenced.
hipError_t launch_step(int tile_cfg, int storage, int flow, int inout, int rad, const DomDesc* doms_dev,
                       const TileDesc* tiles_dev, int ntiles, int grid, int par, hipStream_t s);
// Grid size of a step launch over `ntiles` tiles: grid_mode 0 = one workgroup per tile,
// 1 = persistent (one wave of resident workgroups looping over the tiles).
int step_grid(int tile_cfg, int ntiles, int storage, int flow, int inout, int rad, int grid_mode);
// reach of a gradient stencil in cells
inline int stencil_reach(int stencil) { return stencil >= 6 ? 2 : 1; }

hipError_t launch_init(const DomDesc& d, int par, const float* U_init, float U0, float seed_x,
                       float seed_y, float seed_r, float width, float u_in, hipStream_t s);
hipError_t launch_read(const DomDesc& d, int par, int field, float* dst, hipStream_t s);
hipError_t launch_write_field(const DomDesc& d, int par, int field, const float* src, hipStream_t s);
hipError_t launch_pop_io(const DomDesc& d, int par, int set, int to_canonical, float* canon,
                         hipStream_t s);
// FP64 diagnostics: partials (diag_blocks() x 8 doubles, at most kDiagMaxBlocks x 8) then out[9]:
// the eight sums and the species invariant sum U + half_Lsat sum phi_prev.
constexpr int kDiagMaxBlocks = 2048;
int diag_blocks(const DomDesc& d);
hipError_t launch_diag(const DomDesc& d, int par, double* partials, double* out, double half_Lsat, hipStream_t s);
// Device address, on the current device, of the diagnostics' static scratch array (kDiagMaxBlocks x 8
// doubles), looked up on the first call per device.
hipError_t diag_scratch(double** out);

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

// ---- discrete adjoint (snowlb_adjoint.hip): no flow, periodic, FP32 storage
struct AdjDesc {
    int32_t nx, ny, nbx, n_fold;
    const float* st;     // state at t: g_0..4, h_0..8 (14 planes, the populations' cell order)
    const float* lin;    // lambda(t+1) of g_0..4, h_0..8 (same order)
    float* lout;         // lambda(t) of g_0..4, h_0..8
    const float* lppin;  // lambda(t+1) of phi_prev (one plane)
    float* lppout;       // lambda(t) of phi_prev
    double* epart;       // per-workgroup dL/deps partials, accumulated over the reverse sweep
    double grad_eps2;
    float eps, Dphi, coefN, inv_tau0, lam, half_Lsat, tauv_m_half, pad_;
};
constexpr int kAdjPlanes = 14;  // g_0..4, h_0..8 of the no-flow state
int adj_blocks(const AdjDesc& A);
hipError_t launch_adj_seed(const AdjDesc& A, const float* dphi, hipStream_t s);
hipError_t launch_adj_step(const AdjDesc& A, hipStream_t s);
// dU[y*nx + x] = dL/dU_init; rows: ny doubles of scratch; out[0] = dL/deps, out[1] = sum dU
hipError_t launch_adj_finish(const AdjDesc& A, float* dU, double* rows, double* out, hipStream_t s);

}  // namespace snowlb
