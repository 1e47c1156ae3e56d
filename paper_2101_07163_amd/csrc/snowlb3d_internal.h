// snowlb3d_internal.h -- descriptors shared by the 3D kernels and the 3D host runtime of libsnowlb.
//
// Device layout (per lattice): one buffer per copy holds the populations (f_0..f_18 with flow, g_0..g_6,
// h_0..h_6: npop planes) in blocks of cells with the block's planes side by side; phi_prev
// (one FP32 plane) has a buffer of its own in the same cell order (blocks of kBX x kBY x kBZ cells).
// Two copies of each ping-pong.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snowlb3d {

constexpr int kBX = 64, kBY = 2, kBZ = 2, kBlockCells = kBX * kBY * kBZ;
constexpr int kSX = 6, kSY = 1, kSZ = 1;  // log2 of the block sides
static_assert((1 << kSX) == kBX && (1 << kSY) == kBY && (1 << kSZ) == kBZ && kBlockCells == 256, "block shape");

// Element (q, x, y, z) of a buffer of nq planes sits at
//     ((z / BZ) nby nbx + (y / BY) nbx + x / BX) nq 256  +  256 q  +  BX BY (z % BZ) + BX (y % BY) + x % BX,
// the sum of an x, a y and a z part (blocks of BX x BY x BZ = 64 x 2 x 2 cells: 64-cell rows in x keep the
// shifted push stores coalesced; measured 4.61 TB/s against 4.53 for 32 x 4 x 2, 4.27 for 64 x 4 x 1 and
// 4.24 for 16 x 4 x 4 on the 256 x 128 x 128 ventilated step).  The host keeps every
// byte offset inside a buffer below 2^32.
__host__ __device__ __forceinline__ uint32_t xpart(int x, int nq) {
    return (uint32_t)(x >> kSX) * ((uint32_t)nq << 8) + (uint32_t)(x & (kBX - 1));
}
__host__ __device__ __forceinline__ uint32_t ypart(int y, int nbx, int nq) {
    return (uint32_t)(y >> kSY) * (((uint32_t)nbx * (uint32_t)nq) << 8) + ((uint32_t)(y & (kBY - 1)) << kSX);
}
__host__ __device__ __forceinline__ uint32_t zpart(int z, int nbx, int nby, int nq) {
    return (uint32_t)(z >> kSZ) * (((uint32_t)nbx * (uint32_t)nby * (uint32_t)nq) << 8) +
           ((uint32_t)(z & (kBZ - 1)) << (kSX + kSY));
}

struct Dom3 {
    int32_t nx, ny, nz, nbx, nby, nbz, npop, flow, inout, pad0;
    float* pop[2];   // the two population copies
    float* phip[2];  // phi(t-1), one plane each
    double grad_eps2;
    float eps, Dphi, coefN, inv_tau0, lam, half_Lsat, tauv_m_half, omega_f, guo, kdrag, rho0, u_in, U_in;
    float tauf_m_half;  // tau_f - 1/2 (= guo / omega_f)
    float df_in[19];  // inlet ghost f_eq(rho0, (u_in, 0, 0)) - w
    float g_in[7];    // inlet ghost g_eq(U_in, (u_in, 0, 0))
};

// One step of every block of the lattice, reading copy par and writing copy 1 - par.
hipError_t launch_step3(const Dom3& d, const Dom3* d_dev, int par, hipStream_t s);
hipError_t launch_init3(const Dom3& d, int par, const float* U_init, float U0, float sx, float sy, float sz,
                        float R, float width, hipStream_t s);
// field: 0 phi, 1 U, 2 rho, 3 ux, 4 uy, 5 uz -> dst [z][y][x]
hipError_t launch_read3(const Dom3& d, int par, int field, float* dst, hipStream_t s);
// set: 0 f (19), 1 g (7), 2 h (7), 3 phi_prev; canonical [q][z][y][x] FP32
hipError_t launch_pop_io3(const Dom3& d, int par, int set, int to_canonical, float* canon, hipStream_t s);
// FP64 diagnostics: partials (diag_blocks3() x 9 doubles) then out[10] (the 9 sums, then the species
// invariant sum U + half_Lsat sum phi_prev)
int diag_blocks3(const Dom3& d);
hipError_t launch_diag3(const Dom3& d, int par, double* partials, double* out, double half_Lsat, hipStream_t s);

}  // namespace snowlb3d
