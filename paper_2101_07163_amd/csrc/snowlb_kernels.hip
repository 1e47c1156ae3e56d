// snowlb_kernels.hip -- gfx950 kernels of the coupled lattice-Boltzmann ice-growth step
// (Tan et al., arXiv:2101.07163).
//
// k_step fuses, per lattice cell, the three LB updates of one time step:
//   flow   : D2Q9 BGK with the solid drag force and the velocity projection (Sec. 2.2.1),
//   vapour : D2Q5 advection-diffusion-reaction with the depletion source (Sec. 2.2.2),
//   phase  : the capacity-form LB of Eq. (d) with the equilibrium of Eq. (e) (Sec. 2.2.3),
// with the E4 isotropic gradient of Table 1 (Sec. 3.1.1) and the anisotropy of Sec. 2.1.
//
// The step is bound by HBM bandwidth (about 2 flop per byte against a balance of about 20), so the
// kernel is built around memory traffic: every population is read once and written once per step,
// and a 64 x 4 tile's populations are one contiguous run of memory (planes side by side per block,
// see cell_index).  The only neighbour data the step needs -- phi at the eight neighbours
// (gradient) and h_q at x + c_q (the destination term of Eq. (d)) -- is staged in LDS from a
// one-cell halo of the 9 h planes, so halo re-reads hit LDS/L2 instead of HBM.
//
// Streaming is "push": Eq. (d) evaluates a_s^2 at the source node and needs the destination's own
// pre-collision h_q(x + c_q, t), so each cell writes h'_q(x + c_q) = P_q(x) - B(x) h_q(x + c_q, t),
// with P_q = h*_q / a^2 and B = (1 - a^2)/a^2.  Every (destination, q) pair is written by exactly one
// thread, so there is no race.
//
// 16-bit storage keeps each population as a deviation d = p / w - m from a local reference m
// (collision arithmetic stays FP32):
//   h   : m = phi(t-1) of the cell that holds the population (its phi_prev; the writer knows it from
//         the LDS phi of the destination, the reader from its phi_prev plane);
//   g_q : m = U of the cell the population streamed from;
//   f_q : m = rho + 3 c_q . j of the cell the population streamed from (its first-order equilibrium,
//         so the velocity term leaves the deviation).
// The source cell stores its U, rho, jx, jy rounded to the 16-bit format in reference planes; writer
// and reader use exactly those rounded values (the reader stages them with the halo), so any
// rounding of the references cancels.  The deviations are then small (time changes and
// non-equilibrium parts), and so is the 16-bit rounding error in absolute terms.  phi_prev and the
// reference planes come in two copies, because neighbours read them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snowlb_internal.h"

namespace snowlb {

// ---------------------------------------------------------------------------------------------
// lattice constants (D2Q9: rest, 4 axis, 4 diagonal; D2Q5: the first five)
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr float W9[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,  1.f / 9.f, 1.f / 9.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
__device__ constexpr float IW9[9] = {2.25f, 9.f, 9.f, 9.f, 9.f, 36.f, 36.f, 36.f, 36.f};
__device__ constexpr float W5[5] = {1.f / 3.f, 1.f / 6.f, 1.f / 6.f, 1.f / 6.f, 1.f / 6.f};
__device__ constexpr float IW5[5] = {3.f, 6.f, 6.f, 6.f, 6.f};

// ---------------------------------------------------------------------------------------------
// storage policies: FP32 values, or 16-bit deviations d = p / w - m (see the header comment)
struct StoreF32 {
    using T = float;
    static constexpr bool kLocalRef = false;
    static __device__ __forceinline__ float dec(T v, float, float) { return v; }
    static __device__ __forceinline__ T enc(float p, float, float) { return p; }
    static __device__ __forceinline__ T to_ref(float v) { return v; }
    static __device__ __forceinline__ float from_ref(T v) { return v; }
};
struct StoreF16 {
    using T = _Float16;
    static constexpr bool kLocalRef = true;
    static __device__ __forceinline__ float dec(T v, float w, float ref) { return __builtin_fmaf(w, (float)v, w * ref); }
    static __device__ __forceinline__ T enc(float p, float iw, float ref) {
        return (_Float16)(p * iw - ref);  // v_cvt_f16_f32: round to nearest even
    }
    static __device__ __forceinline__ T to_ref(float v) { return (_Float16)v; }
    static __device__ __forceinline__ float from_ref(T v) { return (float)v; }
};
struct StoreBF16 {
    using T = uint16_t;
    static constexpr bool kLocalRef = true;
    static __device__ __forceinline__ float dec(T v, float w, float ref) {
        return __builtin_fmaf(w, __uint_as_float((uint32_t)v << 16), w * ref);
    }
    static __device__ __forceinline__ T enc(float p, float iw, float ref) { return to_ref(p * iw - ref); }
    static __device__ __forceinline__ T to_ref(float v) {
        return __builtin_bit_cast(uint16_t, (__bf16)v);  // v_cvt_pk_bf16_f32: nearest even
    }
    static __device__ __forceinline__ float from_ref(T v) { return __uint_as_float((uint32_t)v << 16); }
};

// Reference of a 16-bit f_q: rho + 3 c_q . j of its source, with one explicit fused rounding so
// that the writer and every reader produce the same bits.
__device__ __forceinline__ float f_ref(float rho, float jx, float jy, int cx, int cy) {
    return __builtin_fmaf(3.f, (float)cx * jx + (float)cy * jy, rho);
}

// Flow populations are carried as deviations from the lattice weights, df_q = f_q - w_q, through the
// step: the density deviation, the momentum and every equilibrium and collision term are then small
// numbers, so FP32 rounding acts on O(u) quantities rather than on O(1) ones.  FP32 storage holds df
// itself; 16-bit storage keeps its deviation from the local reference and converts at the edges.
template <class S>
__device__ __forceinline__ float f_dev_dec(typename S::T v, int q, float m) {
    if constexpr (S::kLocalRef) return S::dec(v, W9[q], m) - W9[q];
    else return v;
}
template <class S>
__device__ __forceinline__ typename S::T f_dev_enc(float df, int q, float m) {
    if constexpr (S::kLocalRef) return S::enc(df + W9[q], IW9[q], m);
    else return df;
}
// the same populations as plain FP32 values f_q (read-out, diagnostics, population exchange)
template <class S>
__device__ __forceinline__ float f_abs_dec(typename S::T v, int q, float m) {
    if constexpr (S::kLocalRef) return S::dec(v, W9[q], m);
    else return W9[q] + v;
}
template <class S>
__device__ __forceinline__ typename S::T f_abs_enc(float f, int q, float m) {
    if constexpr (S::kLocalRef) return S::enc(f, IW9[q], m);
    else return f - W9[q];
}

// reference planes: U, rho, jx, jy (the last three with flow only)
enum { R_U = 0, R_RHO = 1, R_JX = 2, R_JY = 3 };

// Sum of the eight moving populations in a fixed pairwise order.
__device__ __forceinline__ float sum8(const float v[9]) {
    return ((v[1] + v[2]) + (v[3] + v[4])) + ((v[5] + v[6]) + (v[7] + v[8]));
}

__device__ __forceinline__ int wrapi(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) i = ((i % n) + n) % n;
    return i;
}

// Every buffer lives in device global memory.  The plane pointers are read from the descriptor,
// so the compiler cannot infer that and would emit flat (generic) accesses, which wait on both the
// memory and the LDS counters; the casts below make them global accesses.
template <class S>
__device__ __forceinline__ const GMEM typename S::T* plane_ptr(const DomDesc& d, int par, int q) {
    return (const GMEM typename S::T*)(d.pop[par]) + (int64_t)q * d.plane;
}
template <class S>
__device__ __forceinline__ GMEM typename S::T* plane_ptr_w(const DomDesc& d, int par, int q) {
    return (GMEM typename S::T*)(d.pop[par]) + (int64_t)q * d.plane;
}
__device__ __forceinline__ GMEM float* phip_ptr(const DomDesc& d, int par) {
    return (GMEM float*)(d.phip[par]);
}

// The y part of cell_index with a full-rate 24-bit multiply (v_mul_u32_u24): every lattice the host
// accepts has fewer than 2^14 block rows and a block-row stride (64 nbx nq) below 2^24 elements, and its
// offsets below 2^32.
__device__ __forceinline__ uint32_t cell_ypart24(int nbx, int nq, int y) {
    return __umul24((uint32_t)(y >> 2), ((uint32_t)nbx * (uint32_t)nq) << 8) + ((uint32_t)(y & 3) << 6);
}

// Closure of the domain for a lattice position (gx, gy) that may lie outside it: y periodic; x
// periodic, or (inlet/outlet) the inlet ghost left of x = 0 (returns false) and a copy of column
// nx-1 right of it.  (sx, sy) receives the position it maps to.
template <bool INOUT>
__device__ __forceinline__ bool map_pos(const DomDesc& d, int gx, int gy, int& sx, int& sy) {
    sy = wrapi(gy, d.ny);
    if (INOUT) {
        if (gx < 0) {
            sx = 0;
            return false;
        }
        sx = gx < d.nx ? gx : d.nx - 1;
    } else {
        sx = wrapi(gx, d.nx);
    }
    return true;
}

// Reference values (U, rho, jx, jy) of lattice position (gx, gy) with the closure: the inlet ghost
// carries (U_in, rho0, rho0 u_in, 0) rounded to the storage format.
template <class S>
__device__ __forceinline__ void ref_at(const DomDesc& d, int par, int gx, int gy, float r[4]) {
    if (!S::kLocalRef) {
        r[0] = r[1] = r[2] = r[3] = 0.f;
        return;
    }
    const int sy = wrapi(gy, d.ny);
    if (d.inout) {
        if (gx < 0) {
            r[R_U] = S::from_ref(S::to_ref(d.U_in));
            r[R_RHO] = S::from_ref(S::to_ref(d.ref_f));
            r[R_JX] = S::from_ref(S::to_ref(d.ref_f * d.u_in));
            r[R_JY] = 0.f;
            return;
        }
        if (gx >= d.nx) gx = d.nx - 1;
    } else {
        gx = wrapi(gx, d.nx);
    }
    const int64_t i = cell_index(d.nbx, d.nqb, gx, sy);
    const GMEM typename S::T* b = (const GMEM typename S::T*)(d.refs[par]);
    r[R_U] = S::from_ref(b[i]);
    if (d.npop == 23) {
        r[R_RHO] = S::from_ref(b[d.rplane + i]);
        r[R_JX] = S::from_ref(b[2 * d.rplane + i]);
        r[R_JY] = S::from_ref(b[3 * d.rplane + i]);
    } else {
        r[R_RHO] = r[R_JX] = r[R_JY] = 0.f;
    }
}

// Decode every population of an in-domain cell (non-hot kernels).
template <class S>
__device__ __forceinline__ void decode_cell(const DomDesc& d, int par, int x, int y, bool flow, float f[9],
                                            float g[5], float h[9]) {
    const int64_t i = cell_index(d.nbx, d.nqb, x, y);
    const float hr = S::kLocalRef ? phip_ptr(d, par)[cell_index(d.nbx, 1, x, y)] : 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) h[q] = S::dec(plane_ptr<S>(d, par, d.off_h + q)[i], W9[q], hr);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        float r[4];
        ref_at<S>(d, par, x - CX[q], y - CY[q], r);
        if (q < 5) g[q] = S::dec(plane_ptr<S>(d, par, d.off_g + q)[i], W5[q], r[R_U]);
        f[q] = flow ? f_abs_dec<S>(plane_ptr<S>(d, par, q)[i], q, f_ref(r[R_RHO], r[R_JX], r[R_JY], CX[q], CY[q]))
                    : 0.f;
    }
}

// ---------------------------------------------------------------------------------------------
// the fused step
template <int TX, int TY, class S, bool FLOW, bool INOUT>
__global__ void __launch_bounds__(TX * TY)
k_step(const DomDesc* __restrict__ doms, const TileDesc* __restrict__ tiles, int ntiles, int par, int xcd_remap) {
    using T = typename S::T;
    constexpr bool REF = S::kLocalRef;
    constexpr int NR = REF ? (FLOW ? 4 : 1) : 1;  // reference planes staged in LDS
    constexpr int NT = TX * TY;
    constexpr int LX = TX + 2, LY = TY + 2, LN = LX * LY;
    constexpr int RING = 2 * LX + 2 * TY;
    constexpr int PF = 0, PG = FLOW ? 9 : 0, PH = PG + 5;  // first plane of f, g and h in a copy
    constexpr int NP = (FLOW ? 23 : 14) + (REF ? NR : 0);  // planes per block of a copy (d.nqb)
    constexpr uint32_t ES = sizeof(T);
    __shared__ double s_phi[LN];
    __shared__ float s_h[9][LN];
    __shared__ float s_ref[NR][REF ? LN : 1];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int own = (ty + 1) * LX + (tx + 1);
    const int npar = 1 - par;

    // XCD-aware order (optional): consecutive workgroup ids are spread over the 8 XCDs; give each
    // XCD a contiguous run of tiles so neighbouring tiles share halo lines in that XCD's L2.
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int per_xcd = G / 8;
    const int slot = (xcd_remap && G % 8 == 0) ? ((b % 8) * per_xcd + b / 8) : b;

    auto ring_pos = [&](int r, int& lx, int& ly) {
        if (r < LX) { lx = r; ly = 0; }
        else if (r < 2 * LX) { lx = r - LX; ly = LY - 1; }
        else if (r < 2 * LX + TY) { lx = 0; ly = 1 + (r - 2 * LX); }
        else { lx = LX - 1; ly = 1 + (r - 2 * LX - TY); }
    };

    for (int t = slot; t < ntiles; t += G) {
        const TileDesc td = tiles[t];
        const DomDesc& d = doms[td.dom];
        // uniform bases: population copies, phi_prev, reference planes
        const uint64_t pb = (uint64_t)kBlockCells * ES;  // bytes between the planes of a block
        const uint64_t rb = (uint64_t)kBlockCells * ES;
        const GMEM char* pin = (const GMEM char*)d.pop[par];
        GMEM char* pout = (GMEM char*)d.pop[npar];
        const GMEM char* phin = (const GMEM char*)d.phip[par];
        GMEM char* phout = (GMEM char*)d.phip[npar];
        const GMEM char* rin = REF ? (const GMEM char*)d.refs[par] : nullptr;
        GMEM char* rout = REF ? (GMEM char*)d.refs[npar] : nullptr;

        const int x = td.x0 + tx, y = td.y0 + ty;
        const bool active = (x < d.nx) && (y < d.ny);
        // element offsets of a position in the population buffer (p; the 16-bit reference planes share
        // its blocks, r = p) and in the phi_prev plane (f)
        struct Off {
            uint32_t p, f, r;
        };
        auto offs = [&](int sx, int sy) {
            Off o;
            o.p = cell_xpart(sx, NP) + cell_ypart24(d.nbx, NP, sy);
            o.f = cell_xpart(sx, 1) + cell_ypart24(d.nbx, 1, sy);
            o.r = o.p;
            return o;
        };
        const uint32_t xp = cell_xpart(x, NP), yp = cell_ypart24(d.nbx, NP, y);
        const uint32_t co = xp + yp;  // population offset of this lane's cell (active lanes)

        // ---- issue every global load of this tile first (own position and the first pass over the
        // halo ring, with the 16-bit references that decode them), so that they are all in flight
        // together; decode and stage afterwards.  Lanes outside the domain stage the position their
        // LDS slot stands for, which can be the halo of an active neighbour.
        T graw[5], fraw[9], hraw[9], rraw[9];
        T oref[NR], rref[NR];
        float ophi = 0.f, rphi = 0.f;  // phi_prev of the staged positions
        int osx, osy;
        const bool oreal = map_pos<INOUT>(d, x, y, osx, osy);  // (x, y) itself for active lanes
        const Off oo = offs(osx, osy);
        if (oreal) {
#pragma unroll
            for (int q = 0; q < 9; ++q) hraw[q] = gld<T>(pin + (PH + q) * pb, oo.p * ES);
            ophi = gld<float>(phin, oo.f * 4);
            if (REF) {
#pragma unroll
                for (int k = 0; k < NR; ++k) oref[k] = gld<T>(rin + k * rb, oo.r * ES);
            }
        }
        if (active) {
#pragma unroll
            for (int q = 0; q < 5; ++q) graw[q] = gld<T>(pin + (PG + q) * pb, co * ES);
            if (FLOW) {
#pragma unroll
                for (int q = 0; q < 9; ++q) fraw[q] = gld<T>(pin + (PF + q) * pb, co * ES);
            }
        }
        int rlx = 0, rly = 0;
        bool rreal = false;
        const bool has_ring = tid < RING;
        if (has_ring) {
            ring_pos(tid, rlx, rly);
            int sx, sy;
            rreal = map_pos<INOUT>(d, td.x0 + rlx - 1, td.y0 + rly - 1, sx, sy);
            const Off ro = offs(sx, sy);
            if (rreal) {
#pragma unroll
                for (int q = 0; q < 9; ++q) rraw[q] = gld<T>(pin + (PH + q) * pb, ro.p * ES);
                if (REF) {
                    rphi = gld<float>(phin, ro.f * 4);
#pragma unroll
                    for (int k = 0; k < NR; ++k) rref[k] = gld<T>(rin + k * rb, ro.r * ES);
                }
            }
        }
        // Decode h of one staged position and write phi, h and the 16-bit references to LDS.  phi is
        // summed in FP64: it is close to -1 or 1 in the bulk, and an E4 gradient of FP32 sums would
        // carry cancellation error of order 1e-7 / |grad phi| into the direction of the normal, i.e.
        // into a and N where |grad phi| is small.  h is stored against its holder's phi_prev.
        auto stage = [&](bool real, const T raw[9], float href, const T refs[NR], int li, float hh[9]) {
            double p64 = -1.0;  // inlet ghost: phi = -1 (its h are never read)
            if (real) {
                p64 = 0.0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    hh[q] = S::dec(raw[q], W9[q], href);
                    p64 += (double)hh[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) hh[q] = 0.f;
            }
            s_phi[li] = p64;
#pragma unroll
            for (int q = 0; q < 9; ++q) s_h[q][li] = hh[q];
            if (REF) {
                if (real) {
#pragma unroll
                    for (int k = 0; k < NR; ++k) s_ref[k][li] = S::from_ref(refs[k]);
                } else {
                    s_ref[R_U][li] = S::from_ref(S::to_ref(d.U_in));
                    if (FLOW) {
                        s_ref[R_RHO][li] = S::from_ref(S::to_ref(d.ref_f));
                        s_ref[R_JX][li] = S::from_ref(S::to_ref(d.ref_f * d.u_in));
                        s_ref[R_JY][li] = 0.f;
                    }
                }
            }
        };
        float h[9];
        stage(oreal, hraw, ophi, oref, own, h);
        if (has_ring) {
            float hr[9];
            stage(rreal, rraw, rphi, rref, rly * LX + rlx, hr);
        }
        // rings larger than the workgroup (e.g. 128 x 2 tiles) take further passes
        for (int r = tid + NT; r < RING; r += NT) {
            int lx, ly;
            ring_pos(r, lx, ly);
            int sx, sy;
            const bool real = map_pos<INOUT>(d, td.x0 + lx - 1, td.y0 + ly - 1, sx, sy);
            const Off eo = offs(sx, sy);
            T raw[9], refs[NR];
            float pr = 0.f;
            if (real) {
#pragma unroll
                for (int q = 0; q < 9; ++q) raw[q] = gld<T>(pin + (PH + q) * pb, eo.p * ES);
                if (REF) {
                    pr = gld<float>(phin, eo.f * 4);
#pragma unroll
                    for (int k = 0; k < NR; ++k) refs[k] = gld<T>(rin + k * rb, eo.r * ES);
                }
            }
            float hr[9];
            stage(real, raw, pr, refs, ly * LX + lx, hr);
        }
        __syncthreads();

        if (active) {
            const float phip = ophi;  // phi(t-1) of this cell
            // ---- vapour and flow populations (16-bit: references of their source cells)
            float g[5], f[9];
#pragma unroll
            for (int q = 0; q < 5; ++q) g[q] = S::dec(graw[q], W5[q], REF ? s_ref[R_U][own - CY[q] * LX - CX[q]] : 0.f);
            if (FLOW) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    float m = 0.f;
                    if (REF) {
                        const int ls = own - CY[q] * LX - CX[q];
                        m = f_ref(s_ref[R_RHO][ls], s_ref[R_JX][ls], s_ref[R_JY][ls], CX[q], CY[q]);
                    }
                    f[q] = f_dev_dec<S>(fraw[q], q, m);  // f_q - w_q
                }
            }
            const float U = (g[0] + g[1]) + (g[2] + g[3]) + g[4];

            // ---- E4 gradient (Table 1: 1/3 on axis neighbours, 1/12 on diagonals, no 1/cs^2), FP64
            const double phi64 = s_phi[own];
            const float phi = (float)phi64;
            const double* P = s_phi + own;
            const double pE = P[1], pW = P[-1], pN = P[LX], pS = P[-LX];
            const double pNE = P[LX + 1], pNW = P[LX - 1], pSW = P[-LX - 1], pSE = P[-LX + 1];
            const double gx64 = (1.0 / 3.0) * (pE - pW) + (1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
            const double gy64 = (1.0 / 3.0) * (pN - pS) + (1.0 / 12.0) * ((pNE + pNW) - (pSE + pSW));
            const bool has_normal = gx64 * gx64 + gy64 * gy64 > d.grad_eps2;
            const float gx = (float)gx64, gy = (float)gy64;

            // ---- anisotropy a = 1 + eps cos(n theta) and flux N = kappa Dphi |g|^2 a da/dg, as
            // polynomials in the unit normal (theta-free, sign-free): with X = gx^2/|g|^2,
            // Y = gy^2/|g|^2, cos 6t = X^3 - 15 X^2 Y + 15 X Y^2 - Y^3,
            // sin 6t = (gx gy/|g|^2)(6 X^2 - 20 X Y + 6 Y^2), and d cos(nt)/dg = n sin(nt)(gy,-gx)/|g|^2.
            float a = 1.f, Nx = 0.f, Ny = 0.f;
            if (has_normal) {
                const float inv = 1.f / (gx * gx + gy * gy);
                const float X = gx * gx * inv, Y = gy * gy * inv, XY = gx * gy * inv;
                float Cn, Sn;
                if (d.n_fold == 6) {
                    Cn = X * X * X - 15.f * X * X * Y + 15.f * X * Y * Y - Y * Y * Y;
                    Sn = XY * (6.f * X * X - 20.f * X * Y + 6.f * Y * Y);
                } else {
                    Cn = X * X - 6.f * X * Y + Y * Y;
                    Sn = XY * 4.f * (X - Y);
                }
                a = 1.f + d.eps * Cn;
                const float c = d.aniso_coef * a * Sn;
                Nx = c * gy;
                Ny = -c * gx;
            }

            // ---- phase field, Eq. (d)/(e): relaxation eta = a^2 Dphi / cs^2 + 1/2, source Q / tau0
            const float a2 = a * a;
            const float ia2 = 1.f / a2;
            const float B = ia2 - 1.f;
            const float ieta = 1.f / (3.f * d.Dphi * a2 + 0.5f);
            const float om = 1.f - phi * phi;
            const float srcQ = (phi - phi * phi * phi + d.lam * U * om * om) * d.inv_tau0;

            // The FP32 lattice weights do not sum to one (float(1/3) + 4 float(1/6) = 1 + 3e-8), which
            // would make every collision a tiny systematic source of mass, vapour and phase.  Each
            // equilibrium and source therefore takes its rest population as the remainder of the moving
            // ones, so that the zeroth moments close exactly in real arithmetic and only unbiased
            // rounding is left.

            // ---- flow: drag and projection, Guo forcing, 2nd-order equilibrium (Sec. 2.2.1), all in
            // deviations from the weights: f holds f_q - w_q, drho = rho - 1, and
            // f_eq,q - w_q = w_q (drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
            float ux = 0.f, uy = 0.f, rho = 0.f, jx = 0.f, jy = 0.f;
            float fs[9];
            if (FLOW) {
                const float drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
                rho = 1.f + drho;
                jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
                jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
                const float pc = fminf(fmaxf(phi, -1.f), 1.f);
                const float k = d.kdrag * (1.f + pc) * (1.f + pc) * (1.f - pc);
                const float sc = 0.5f * (1.f - pc) / (rho + 0.5f * k);
                ux = jx * sc;
                uy = jy * sc;
                const float Fx = -k * ux, Fy = -k * uy;
                const float uu = ux * ux + uy * uy;
                const float uF = ux * Fx + uy * Fy;
                float feq[9], Sg[9];
#pragma unroll
                for (int q = 1; q < 9; ++q) {
                    const float cu = CX[q] * ux + CY[q] * uy;
                    const float cF = CX[q] * Fx + CY[q] * Fy;
                    feq[q] = W9[q] * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
                    Sg[q] = d.guo * W9[q] * (3.f * (cF - uF) + 9.f * cu * cF);
                }
                feq[0] = drho - sum8(feq);
                Sg[0] = -sum8(Sg);
#pragma unroll
                for (int q = 0; q < 9; ++q) fs[q] = f[q] - (f[q] - feq[q]) * d.omega_f + Sg[q];
            }

            // ---- vapour (Sec. 2.2.2): tau_g = 1/2 + (tau_vap - 1/2) clamp((1 - phi)/2, 0, 1)
            const float sq = fminf(fmaxf(0.5f * (1.f - phi), 0.f), 1.f);
            const float itg = 1.f / (0.5f + d.tauv_m_half * sq);
            const float srcg = d.half_Lsat * (phi - phip);
            float gs[5];
            {
                float geq[5], sgq[5];
#pragma unroll
                for (int q = 1; q < 5; ++q) {
                    geq[q] = W5[q] * U * (1.f + 3.f * (CX[q] * ux + CY[q] * uy));
                    sgq[q] = W5[q] * srcg;
                }
                geq[0] = U - ((geq[1] + geq[2]) + (geq[3] + geq[4]));
                sgq[0] = srcg - ((sgq[1] + sgq[2]) + (sgq[3] + sgq[4]));
#pragma unroll
                for (int q = 0; q < 5; ++q) gs[q] = g[q] - (g[q] - geq[q]) * itg - sgq[q];
            }

            // ---- phase field equilibrium (Eq. e) and source shares, rest population as remainder
            float heq[9], shq[9];
#pragma unroll
            for (int q = 1; q < 9; ++q) {
                heq[q] = W9[q] * (phi - 3.f * (CX[q] * Nx + CY[q] * Ny));
                shq[q] = W9[q] * srcQ;
            }
            heq[0] = phi - sum8(heq);
            shq[0] = srcQ - sum8(shq);

            // ---- references this cell hands to the populations it emits (16-bit storage)
            float rU = 0.f, rR = 0.f, rJx = 0.f, rJy = 0.f;
            if (REF) {
                const T tU = S::to_ref(U);
                gst<T>(rout, oo.r * ES, tU);
                rU = S::from_ref(tU);
                if (FLOW) {
                    const T tR = S::to_ref(rho), tX = S::to_ref(jx), tY = S::to_ref(jy);
                    gst<T>(rout + rb, oo.r * ES, tR);
                    gst<T>(rout + 2 * rb, oo.r * ES, tX);
                    gst<T>(rout + 3 * rb, oo.r * ES, tY);
                    rR = S::from_ref(tR);
                    rJx = S::from_ref(tX);
                    rJy = S::from_ref(tY);
                }
            }

            // ---- push streaming into copy 1 - par (destination offsets: x part + y part)
            const int yN = (y + 1 < d.ny) ? y + 1 : 0;
            const int yS = (y > 0) ? y - 1 : d.ny - 1;
            const int xE = (x + 1 < d.nx) ? x + 1 : (INOUT ? -1 : 0);
            const int xW = (x > 0) ? x - 1 : (INOUT ? -1 : d.nx - 1);
            const uint32_t xpE = cell_xpart(xE < 0 ? 0 : xE, NP), xpW = cell_xpart(xW < 0 ? 0 : xW, NP);
            const uint32_t ypN = cell_ypart24(d.nbx, NP, yN), ypS = cell_ypart24(d.nbx, NP, yS);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int xd = CX[q] > 0 ? xE : (CX[q] < 0 ? xW : x);
                const uint32_t ypd = CY[q] > 0 ? ypN : (CY[q] < 0 ? ypS : yp);
                const float hs = h[q] - (h[q] - heq[q]) * ieta + shq[q];
                const float Pq = hs * ia2;
                const int lq = own + CY[q] * LX + CX[q];
                const float fm = (REF && FLOW) ? f_ref(rR, rJx, rJy, CX[q], CY[q]) : 0.f;
                if (xd >= 0) {
                    const uint32_t dO = ((CX[q] > 0 ? xpE : (CX[q] < 0 ? xpW : xp)) + ypd) * ES;
                    const float href = REF ? (float)s_phi[lq] : 0.f;  // h references its holder's phi(t)
                    gst<T>(pout + (PH + q) * pb, dO, S::enc(Pq - B * s_h[q][lq], IW9[q], href));
                    if (FLOW) gst<T>(pout + (PF + q) * pb, dO, f_dev_enc<S>(fs[q], q, fm));
                    if (q < 5) gst<T>(pout + (PG + q) * pb, dO, S::enc(gs[q], IW5[q], rU));
                }
                if (INOUT) {
                    if (CX[q] < 0 && x == d.nx - 1) {
                        // outlet ghost at x = nx is a copy of this column: it streams into (nx-1, yd)
                        const uint32_t dO = (xp + ypd) * ES;
                        const int ld = own + CY[q] * LX;
                        const float href = REF ? (float)s_phi[ld] : 0.f;
                        gst<T>(pout + (PH + q) * pb, dO, S::enc(Pq - B * s_h[q][ld], IW9[q], href));
                        gst<T>(pout + (PF + q) * pb, dO, f_dev_enc<S>(fs[q], q, fm));
                        if (q < 5) gst<T>(pout + (PG + q) * pb, dO, S::enc(gs[q], IW5[q], rU));
                    }
                    if (CX[q] > 0 && x == 0) {
                        // inlet ghost at x = -1: equilibrium at (rho0, u_in; U_in; phi = -1); its
                        // reference values are the LDS ones of the ghost column
                        const int lg = own - CX[q] - CY[q] * LX;  // the ghost source in the LDS halo
                        float gfm = 0.f, ggm = 0.f;
                        if (REF) {
                            ggm = s_ref[R_U][lg];
                            gfm = f_ref(s_ref[R_RHO][lg], s_ref[R_JX][lg], s_ref[R_JY][lg], CX[q], CY[q]);
                        }
                        gst<T>(pout + (PH + q) * pb, co * ES, S::enc(-W9[q], IW9[q], REF ? phi : 0.f));
                        gst<T>(pout + (PF + q) * pb, co * ES, f_dev_enc<S>(d.df_in[q], q, gfm));
                        if (q < 5) gst<T>(pout + (PG + q) * pb, co * ES, S::enc(d.g_in[q], IW5[q], ggm));
                    }
                }
            }
            gst<float>(phout, oo.f * 4, phi);
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---------------------------------------------------------------------------------------------
// tile configurations
struct TileCfg {
    int tx, ty;
    const char* name;
};
static const TileCfg kTiles[] = {
    {64, 4, "64x4"}, {64, 8, "64x8"}, {128, 2, "128x2"}, {128, 4, "128x4"}, {64, 2, "64x2"}, {32, 8, "32x8"},
};
static constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

int tile_config_count() { return kNumTiles; }
const char* tile_config_name(int i) { return (i >= 0 && i < kNumTiles) ? kTiles[i].name : "?"; }
int tile_config_tx(int i) { return kTiles[i].tx; }
int tile_config_ty(int i) { return kTiles[i].ty; }

template <int TX, int TY, class S, bool FLOW, bool INOUT>
static void* step_fn() {
    return reinterpret_cast<void*>(&k_step<TX, TY, S, FLOW, INOUT>);
}

template <class S, bool FLOW, bool INOUT>
static void* step_fn_tile(int cfg) {
    switch (cfg) {
        case 0: return step_fn<64, 4, S, FLOW, INOUT>();
        case 1: return step_fn<64, 8, S, FLOW, INOUT>();
        case 2: return step_fn<128, 2, S, FLOW, INOUT>();
        case 3: return step_fn<128, 4, S, FLOW, INOUT>();
        case 4: return step_fn<64, 2, S, FLOW, INOUT>();
        case 5: return step_fn<32, 8, S, FLOW, INOUT>();
    }
    return nullptr;
}

template <class S>
static void* step_fn_store(int cfg, int flow, int inout) {
    if (!flow) return step_fn_tile<S, false, false>(cfg);
    if (!inout) return step_fn_tile<S, true, false>(cfg);
    return step_fn_tile<S, true, true>(cfg);
}

static void* step_kernel(int cfg, int storage, int flow, int inout) {
    if (cfg < 0 || cfg >= kNumTiles) return nullptr;
    if (inout && !flow) return nullptr;
    switch (storage) {
        case 0: return step_fn_store<StoreF32>(cfg, flow, inout);
        case 1: return step_fn_store<StoreF16>(cfg, flow, inout);
        case 2: return step_fn_store<StoreBF16>(cfg, flow, inout);
    }
    return nullptr;
}

// Grid of a step launch.  grid_mode 0: one workgroup per tile, dispatched in (XCD-contiguous) tile
// order -- measured best for streaming traffic on MI355X.  grid_mode 1: a persistent grid of one
// wave of resident workgroups that loops over the tiles.
int step_grid(int cfg, int ntiles, int storage, int flow, int inout, int grid_mode) {
    void* fn = step_kernel(cfg, storage, flow, inout);
    if (!fn || ntiles <= 0) return 0;
    if (grid_mode == 0) return ntiles;
    int per_cu = 0;
    const int nt = kTiles[cfg].tx * kTiles[cfg].ty;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), nt, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    long g = (long)per_cu * ncu;
    if (g >= ntiles) return ntiles;
    g -= g % 8;  // a multiple of 8 keeps the XCD-contiguous order a permutation
    return (int)(g > 0 ? g : ntiles);
}

hipError_t launch_step(int cfg, int storage, int flow, int inout, const DomDesc* doms_dev,
                       const TileDesc* tiles_dev, int ntiles, int grid, int par, hipStream_t s) {
    void* fn = step_kernel(cfg, storage, flow, inout);
    if (!fn) return hipErrorInvalidValue;
    if (ntiles <= 0) return hipSuccess;
    const int nt = kTiles[cfg].tx * kTiles[cfg].ty;
    int remap = 1;
    void* args[] = {(void*)&doms_dev, (void*)&tiles_dev, (void*)&ntiles, (void*)&par, (void*)&remap};
    return hipLaunchKernel(fn, dim3(grid), dim3(nt), args, 0, s);
}

// ---------------------------------------------------------------------------------------------
// initial state: circular tanh seed, equilibrium populations (rest population as remainder)
struct InitArgs {
    const float* U_init;  // ny x nx or null
    float U0, sx, sy, R, width, u_in;
};

// Initial phi, x-velocity and U at an in-domain lattice position.
__device__ __forceinline__ void init_at(const DomDesc& d, const InitArgs& a, int x, int y, float& phi0, float& ux,
                                        float& U) {
    const float dx = (float)x - a.sx, dy = (float)y - a.sy;
    const float r = sqrtf(dx * dx + dy * dy);
    phi0 = tanhf((a.R - r) / (1.41421356237309505f * a.width));
    ux = (d.npop == 23 && d.inout) ? 0.5f * (1.f - phi0) * a.u_in : 0.f;
    U = a.U_init ? a.U_init[(int64_t)y * d.nx + x] : a.U0;
}

// Reference values of the initial state at any lattice position, with the closure of ref_at.
template <class S>
__device__ __forceinline__ void init_ref_at(const DomDesc& d, const InitArgs& a, int gx, int gy, float r[4]) {
    const int sy = wrapi(gy, d.ny);
    if (d.inout) {
        if (gx < 0) {
            r[R_U] = S::from_ref(S::to_ref(d.U_in));
            r[R_RHO] = S::from_ref(S::to_ref(d.ref_f));
            r[R_JX] = S::from_ref(S::to_ref(d.ref_f * d.u_in));
            r[R_JY] = 0.f;
            return;
        }
        if (gx >= d.nx) gx = d.nx - 1;
    } else {
        gx = wrapi(gx, d.nx);
    }
    float phi0, ux, U;
    init_at(d, a, gx, sy, phi0, ux, U);
    r[R_U] = S::from_ref(S::to_ref(U));
    r[R_RHO] = S::from_ref(S::to_ref(d.ref_f));
    r[R_JX] = S::from_ref(S::to_ref(d.ref_f * ux));
    r[R_JY] = 0.f;
}

template <class S>
__global__ void k_init(DomDesc d, int par, InitArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const bool flow = d.npop == 23;
    const float rho0 = d.ref_f;
    float phi0, ux, U;
    init_at(d, a, x, y, phi0, ux, U);
    const int64_t i = cell_index(d.nbx, d.nqb, x, y);
    phip_ptr(d, par)[cell_index(d.nbx, 1, x, y)] = phi0;
    if (S::kLocalRef) {
        GMEM typename S::T* wb = (GMEM typename S::T*)(d.refs[par]);
        const int64_t ir = i;  // the reference planes share the populations' blocks
        wb[ir] = S::to_ref(U);
        if (flow) {
            wb[d.rplane + ir] = S::to_ref(rho0);
            wb[2 * d.rplane + ir] = S::to_ref(rho0 * ux);
            wb[3 * d.rplane + ir] = S::to_ref(0.f);
        }
    }
    float hq[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) hq[q] = W9[q] * phi0;
    hq[0] = phi0 - sum8(hq);
#pragma unroll
    for (int q = 0; q < 9; ++q)
        plane_ptr_w<S>(d, par, d.off_h + q)[i] = S::enc(hq[q], IW9[q], S::kLocalRef ? phi0 : 0.f);
    float dfq[9], gq[5];  // f_eq - w in deviation form
    const float uu = ux * ux, drho0 = rho0 - 1.f;
#pragma unroll
    for (int q = 1; q < 9; ++q) {
        const float cu = CX[q] * ux;
        dfq[q] = W9[q] * (drho0 + rho0 * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
    }
    dfq[0] = drho0 - sum8(dfq);
#pragma unroll
    for (int q = 1; q < 5; ++q) gq[q] = W5[q] * U * (1.f + 3.f * CX[q] * ux);
    gq[0] = U - ((gq[1] + gq[2]) + (gq[3] + gq[4]));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        float r[4] = {0.f, 0.f, 0.f, 0.f};
        if (S::kLocalRef) init_ref_at<S>(d, a, x - CX[q], y - CY[q], r);
        if (flow) plane_ptr_w<S>(d, par, q)[i] = f_dev_enc<S>(dfq[q], q, f_ref(r[R_RHO], r[R_JX], r[R_JY], CX[q], CY[q]));
        if (q < 5) plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(gq[q], IW5[q], r[R_U]);
    }
}

template <class S>
static hipError_t init_s(const DomDesc& d, int par, const InitArgs& a, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    hipLaunchKernelGGL(k_init<S>, grid, dim3(256), 0, s, d, par, a);
    return hipGetLastError();
}

hipError_t launch_init(const DomDesc& d, int par, const float* U_init, float U0, float sx, float sy,
                       float R, float w, float u_in, hipStream_t s) {
    const InitArgs a{U_init, U0, sx, sy, R, w, u_in};
    switch (d.storage) {
        case 0: return init_s<StoreF32>(d, par, a, s);
        case 1: return init_s<StoreF16>(d, par, a, s);
        case 2: return init_s<StoreBF16>(d, par, a, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// macroscopic field read-out
template <class S>
__global__ void k_read(DomDesc d, int par, int field, float* __restrict__ dst) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const bool flow = d.npop == 23;
    float f[9], g[5], h[9];
    decode_cell<S>(d, par, x, y, flow, f, g, h);
    double p = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) p += (double)h[q];
    const float phi = (float)p;
    float v = 0.f;
    if (field == 0) {
        v = phi;
    } else if (field == 1) {
        v = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
    } else if (flow) {
        const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        if (field == 2) {
            v = rho;
        } else {
            const float jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
            const float jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
            const float pc = fminf(fmaxf(phi, -1.f), 1.f);
            const float k = d.kdrag * (1.f + pc) * (1.f + pc) * (1.f - pc);
            const float sc = 0.5f * (1.f - pc) / (rho + 0.5f * k);
            v = (field == 3 ? jx : jy) * sc;
        }
    }
    dst[(int64_t)y * d.nx + x] = v;
}

template <class S>
static hipError_t read_s(const DomDesc& d, int par, int field, float* dst, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    hipLaunchKernelGGL(k_read<S>, grid, dim3(256), 0, s, d, par, field, dst);
    return hipGetLastError();
}

hipError_t launch_read(const DomDesc& d, int par, int field, float* dst, hipStream_t s) {
    switch (d.storage) {
        case 0: return read_s<StoreF32>(d, par, field, dst, s);
        case 1: return read_s<StoreF16>(d, par, field, dst, s);
        case 2: return read_s<StoreBF16>(d, par, field, dst, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// overwrite one macroscopic field (debugging and tests): PHI sets h_q = w_q phi with phi_prev = phi (the
// phase field at rest, no anisotropic flux); U sets g_q = g_eq(U, u) with the velocity u the
// collisions currently see (0 without flow).  16-bit storage encodes h against the new phi_prev and g
// against a U reference reset to 0 (inlet-ghost sources keep the ghost constant), as a population
// write does.  The U case reads only f, h and phi_prev, none of which it writes.
template <class S>
__global__ void k_write_field(DomDesc d, int par, int field, const float* __restrict__ src) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const int64_t i = cell_index(d.nbx, d.nqb, x, y), i1 = cell_index(d.nbx, 1, x, y);
    const float v = src[(int64_t)y * d.nx + x];
    if (field == 0) {
        phip_ptr(d, par)[i1] = v;
        float hq[9];
#pragma unroll
        for (int q = 1; q < 9; ++q) hq[q] = W9[q] * v;
        hq[0] = v - sum8(hq);
#pragma unroll
        for (int q = 0; q < 9; ++q)
            plane_ptr_w<S>(d, par, d.off_h + q)[i] = S::enc(hq[q], IW9[q], S::kLocalRef ? v : 0.f);
        return;
    }
    const bool flow = d.npop == 23;
    float ux = 0.f, uy = 0.f;
    if (flow) {
        float f[9], g[5], h[9];
        decode_cell<S>(d, par, x, y, true, f, g, h);
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) p += (double)h[q];
        const float pc = fminf(fmaxf((float)p, -1.f), 1.f);
        const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        const float k = d.kdrag * (1.f + pc) * (1.f + pc) * (1.f - pc);
        const float sc = 0.5f * (1.f - pc) / (rho + 0.5f * k);
        ux = ((f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7])) * sc;
        uy = ((f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8])) * sc;
    }
    float gq[5];
#pragma unroll
    for (int q = 1; q < 5; ++q) gq[q] = W5[q] * v * (1.f + 3.f * (CX[q] * ux + CY[q] * uy));
    gq[0] = v - ((gq[1] + gq[2]) + (gq[3] + gq[4]));
    if (S::kLocalRef) ((GMEM typename S::T*)(d.refs[par]))[i] = S::to_ref(0.f);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        float r[4] = {0.f, 0.f, 0.f, 0.f};
        if (S::kLocalRef && d.inout && x - CX[q] < 0) ref_at<S>(d, par, -1, y - CY[q], r);  // ghost constants
        plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(gq[q], IW5[q], r[R_U]);
    }
}

template <class S>
static hipError_t write_field_s(const DomDesc& d, int par, int field, const float* src, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    hipLaunchKernelGGL(k_write_field<S>, grid, dim3(256), 0, s, d, par, field, src);
    return hipGetLastError();
}

hipError_t launch_write_field(const DomDesc& d, int par, int field, const float* src, hipStream_t s) {
    switch (d.storage) {
        case 0: return write_field_s<StoreF32>(d, par, field, src, s);
        case 1: return write_field_s<StoreF16>(d, par, field, src, s);
        case 2: return write_field_s<StoreBF16>(d, par, field, src, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// population sets <-> canonical FP32 [q][y][x]
template <class S>
__global__ void k_pop_get(DomDesc d, int par, int set, float* __restrict__ canon) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const int64_t n = (int64_t)d.nx * d.ny, c = (int64_t)y * d.nx + x;
    if (set == 3) {
        canon[c] = phip_ptr(d, par)[cell_index(d.nbx, 1, x, y)];
        return;
    }
    float f[9], g[5], h[9];
    decode_cell<S>(d, par, x, y, set == 0, f, g, h);
    const int nq = set == 1 ? 5 : 9;
    const float* v = set == 0 ? f : (set == 1 ? g : h);
    for (int q = 0; q < nq; ++q) canon[q * n + c] = v[q];
}

// Writing a set re-encodes it against the references the step will decode it with.  Writing f
// (resp. g) resets the rho, j (resp. U) reference planes to 0 -- any consistent reference is valid;
// populations streamed from the inlet ghost keep the ghost's references.  Writing phi_prev
// re-encodes h.
template <class S>
__global__ void k_pop_set(DomDesc d, int par, int set, const float* __restrict__ canon) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= d.nx || y >= d.ny) return;
    const int64_t n = (int64_t)d.nx * d.ny, c = (int64_t)y * d.nx + x, i = cell_index(d.nbx, d.nqb, x, y);
    const int64_t i1 = cell_index(d.nbx, 1, x, y), ir = i;
    GMEM typename S::T* wb = S::kLocalRef ? (GMEM typename S::T*)(d.refs[par]) : nullptr;
    if (set == 0 || set == 1) {
        if (S::kLocalRef) {
            if (set == 1) wb[ir] = S::to_ref(0.f);
            else for (int k = 1; k < 4; ++k) wb[k * d.rplane + ir] = S::to_ref(0.f);
        }
        const int nq = set == 0 ? 9 : 5;
        for (int q = 0; q < nq; ++q) {
            float r[4] = {0.f, 0.f, 0.f, 0.f};
            if (S::kLocalRef && d.inout && x - CX[q] < 0) ref_at<S>(d, par, -1, y - CY[q], r);  // ghost constants
            if (set == 0)
                plane_ptr_w<S>(d, par, q)[i] = f_abs_enc<S>(canon[q * n + c], q, f_ref(r[R_RHO], r[R_JX], r[R_JY], CX[q], CY[q]));
            else
                plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(canon[q * n + c], IW5[q], r[R_U]);
        }
    } else if (set == 2) {
        const float ref = S::kLocalRef ? phip_ptr(d, par)[i1] : 0.f;
        for (int q = 0; q < 9; ++q) plane_ptr_w<S>(d, par, d.off_h + q)[i] = S::enc(canon[q * n + c], IW9[q], ref);
    } else {
        const float pnew = canon[c];
        if (S::kLocalRef) {
            const float pold = phip_ptr(d, par)[i1];
            for (int q = 0; q < 9; ++q) {
                GMEM typename S::T* p = plane_ptr_w<S>(d, par, d.off_h + q) + i;
                *p = S::enc(S::dec(*p, W9[q], pold), IW9[q], pnew);
            }
        }
        phip_ptr(d, par)[i1] = pnew;
    }
}

template <class S>
static hipError_t pop_io_s(const DomDesc& d, int par, int set, int to_canon, float* canon, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    if (to_canon) hipLaunchKernelGGL(k_pop_get<S>, grid, dim3(256), 0, s, d, par, set, canon);
    else hipLaunchKernelGGL(k_pop_set<S>, grid, dim3(256), 0, s, d, par, set, (const float*)canon);
    return hipGetLastError();
}

hipError_t launch_pop_io(const DomDesc& d, int par, int set, int to_canon, float* canon, hipStream_t s) {
    switch (d.storage) {
        case 0: return pop_io_s<StoreF32>(d, par, set, to_canon, canon, s);
        case 1: return pop_io_s<StoreF16>(d, par, set, to_canon, canon, s);
        case 2: return pop_io_s<StoreBF16>(d, par, set, to_canon, canon, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// FP64 diagnostics: per-thread sums over a fixed set of cells, wave64 shuffle reduction, LDS
// across waves, one partial per workgroup, then a single-workgroup pass in a fixed order.
static constexpr int kDiagThreads = 256;

int diag_blocks(const DomDesc& d) {
    const long cells = (long)d.nx * d.ny;
    long b = (cells + kDiagThreads * 4 - 1) / (kDiagThreads * 4);
    if (b > 2048) b = 2048;
    return (int)(b < 1 ? 1 : b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <class S>
__global__ void __launch_bounds__(kDiagThreads) k_diag(DomDesc d, int par, double* __restrict__ partials) {
    const bool flow = d.npop == 23;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t cells = (int64_t)d.nx * d.ny;
    for (int64_t c = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; c < cells;
         c += (int64_t)gridDim.x * kDiagThreads) {
        const int y = (int)(c / d.nx), x = (int)(c - (int64_t)y * d.nx);
        float f[9], g[5], h[9];
        decode_cell<S>(d, par, x, y, flow, f, g, h);
        double phi = 0, U = 0, rho = 0, jx = 0, jy = 0;
        bool bad = false;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            bad |= !isfinite(h[q]);
            phi += h[q];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bad |= !isfinite(g[q]);
            U += g[q];
        }
        if (flow) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                bad |= !isfinite(f[q]);
                rho += f[q];
                jx += CX[q] * (double)f[q];
                jy += CY[q] * (double)f[q];
            }
        }
        const float pp = phip_ptr(d, par)[cell_index(d.nbx, 1, x, y)];
        bad |= !isfinite(pp);
        acc[0] += rho; acc[1] += jx; acc[2] += jy; acc[3] += U; acc[4] += phi; acc[5] += pp;
        acc[6] += (phi > 0.0) ? 1.0 : 0.0;
        acc[7] += bad ? 1.0 : 0.0;
    }
    __shared__ double s_part[kDiagThreads / 64][8];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) s_part[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double v = 0;
        for (int w = 0; w < kDiagThreads / 64; ++w) v += s_part[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * 8 + threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ partials, int nblk, double* __restrict__ out) {
    // 32 lanes per quantity: lane l of quantity k sums blocks l, l + 32, ... in order, then lane 0
    // adds the 32 lane sums in order.  Fixed order, hence deterministic.
    __shared__ double s[8][32];
    const int k = threadIdx.x / 32, l = threadIdx.x % 32;
    double v = 0;
    for (int b = l; b < nblk; b += 32) v += partials[(int64_t)b * 8 + k];
    s[k][l] = v;
    __syncthreads();
    if (l == 0) {
        double t = 0;
        for (int i = 0; i < 32; ++i) t += s[k][i];
        out[k] = t;
    }
}

template <class S>
static hipError_t diag_s(const DomDesc& d, int par, double* partials, double* out, hipStream_t s) {
    const int nb = diag_blocks(d);
    hipLaunchKernelGGL(k_diag<S>, dim3(nb), dim3(kDiagThreads), 0, s, d, par, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_diag(const DomDesc& d, int par, double* partials, double* out, hipStream_t s) {
    switch (d.storage) {
        case 0: return diag_s<StoreF32>(d, par, partials, out, s);
        case 1: return diag_s<StoreF16>(d, par, partials, out, s);
        case 2: return diag_s<StoreBF16>(d, par, partials, out, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// plain copy: the practical HBM ceiling (read + write of the same byte count)
__global__ void __launch_bounds__(256) k_copy(float4* __restrict__ dst, const float4* __restrict__ src, int64_t n) {
    // one 16-byte element per lane, one workgroup per 4 KiB chunk, dispatched in address order
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 16;
    if (n <= 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)grid), dim3(256), 0, s, (float4*)dst, (const float4*)src, n);
    return hipGetLastError();
}

}  // namespace snowlb
