// snowlb_kernels.hip -- gfx950 kernels of the coupled lattice-Boltzmann ice-growth step
// (Tan et al., arXiv:2101.07163).
//
// k_step fuses, per lattice cell, the three LB updates of one time step:
//   flow   : D2Q9 BGK with the solid drag force and the velocity projection (Sec. 2.2.1),
//   vapour : D2Q5 advection-diffusion-reaction with the depletion source (Sec. 2.2.2),
//   phase  : the capacity-form LB of Eq. (d) with the equilibrium of Eq. (e) (Sec. 2.2.3),
// with an isotropic gradient of Table 1 (Sec. 3.1.1; E4 by default, or E2, E6, E8) and the anisotropy of
// Sec. 2.1.
//
// The step is bound by HBM bandwidth (about 2 flop per byte against a balance of about 20), so the
// kernel is built around memory traffic: every population is read once and written once per step,
// and a 64 x 4 tile's populations are one contiguous run of memory (planes side by side per block,
// see cell_index).  The only neighbour data the step needs -- phi at the eight neighbours
// (gradient) and h_q at x + c_q (the destination term of Eq. (d)) -- is staged in LDS from a
// halo of the 9 h planes (one cell wide, two for E6/E8), so halo re-reads hit LDS/L2 instead of HBM.
//
// Streaming is "push": Eq. (d) evaluates a_s^2 at the source node and needs the destination's own
// pre-collision h_q(x + c_q, t), so each cell writes h'_q(x + c_q) = P_q(x) - B(x) h_q(x + c_q, t),
// with P_q = h*_q / a^2 and B = (1 - a^2)/a^2.  Every (destination, q) pair is written by exactly one
// thread, so there is no race.
//
// The storage formats (FP32, or 16-bit deviations from local references) are described with their
// policies in snowlb_device.h.  Set-up, read-out, population exchange and diagnostics kernels are in
// snowlb_io.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snowlb_device.h"
#include "snowlb_internal.h"

namespace snowlb {

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


// ---------------------------------------------------------------------------------------------
// the fused step; RAD is the reach of the gradient stencil (1: E2, E4; 2: E6, E8), i.e. the width of
// the halo ring staged in LDS
// Occupancy floor: four waves per SIMD (at most 128 VGPRs) for the one-cell-reach tiles at least
// four rows high, which fit without spilling; the others keep the compiler's own choice.
template <int TY, int RAD>
constexpr int kMinWaves = (RAD == 1 && TY >= 4) ? 4 : 1;

template <int TX, int TY, class S, bool FLOW, bool INOUT, int RAD>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(kMinWaves<TY, RAD>)))
k_step(const DomDesc* __restrict__ doms, const TileDesc* __restrict__ tiles, int ntiles, int par, int xcd_remap) {
    using T = typename S::T;
    constexpr bool REF = S::kLocalRef;
    constexpr int NR = REF ? (FLOW ? 4 : 1) : 1;  // reference planes staged in LDS
    constexpr int NT = TX * TY;
    constexpr int LX = TX + 2 * RAD, LY = TY + 2 * RAD, LN = LX * LY;
    constexpr int RING = LN - NT;
    constexpr int PF = 0, PG = FLOW ? 9 : 0, PH = PG + 5;  // first plane of f, g and h in a copy
    constexpr int NP = (FLOW ? 23 : 14) + (REF ? NR : 0);  // planes per block of a copy (d.nqb)
    constexpr uint32_t ES = sizeof(T);
    __shared__ double s_phi[LN];
    __shared__ float s_phif[REF ? LN : 1];  // phi(t) rounded to FP32: the h references
    __shared__ float s_h[9][LN];
    __shared__ float s_ref[NR][REF ? LN : 1];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int own = (ty + RAD) * LX + (tx + RAD);
    const int npar = 1 - par;

    // XCD-aware order (optional): consecutive workgroup ids are spread over the 8 XCDs; give each
    // XCD a contiguous run of tiles so neighbouring tiles share halo lines in that XCD's L2.  XCD x
    // receives G/8 workgroups, one more for x < G % 8; its runs follow each other in x order, so the
    // mapping is a permutation of the grid for any G.  Every other step (input copy 1) walks each run
    // backwards: a step then starts on the tiles the previous one wrote last, whose populations are
    // still in the last-level cache.
    const int G = gridDim.x;
    const int b = blockIdx.x;
    int slot = b;
    if (xcd_remap) {
        const int x = b % 8, k = b / 8, cnt = G / 8 + (x < G % 8 ? 1 : 0);
        slot = x * (G / 8) + min(x, G % 8) + (par ? cnt - 1 - k : k);
    }

    // halo position r of the ring: the RAD rows above and below the tile, then RAD columns left and
    // right of it
    auto ring_pos = [&](int r, int& lx, int& ly) {
        if constexpr (RAD == 1) {
            if (r < LX) { lx = r; ly = 0; }
            else if (r < 2 * LX) { lx = r - LX; ly = LY - 1; }
            else if (r < 2 * LX + TY) { lx = 0; ly = 1 + (r - 2 * LX); }
            else { lx = LX - 1; ly = 1 + (r - 2 * LX - TY); }
        } else {
            constexpr int BAND = RAD * LX;
            if (r < 2 * BAND) {
                const int k = r < BAND ? r : r - BAND;
                ly = k / LX + (r < BAND ? 0 : LY - RAD);
                lx = k % LX;
            } else {
                const int k = r - 2 * BAND;
                const int side = k / (RAD * TY), m = k % (RAD * TY);
                ly = RAD + m / RAD;
                lx = (side ? LX - RAD : 0) + m % RAD;
            }
        }
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
            rreal = map_pos<INOUT>(d, td.x0 + rlx - RAD, td.y0 + rly - RAD, sx, sy);
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
        // summed in FP64: it is close to -1 or 1 in the bulk, and a gradient of FP32 sums would
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
            if (REF) s_phif[li] = (float)p64;
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
            const bool real = map_pos<INOUT>(d, td.x0 + lx - RAD, td.y0 + ly - RAD, sx, sy);
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
            for (int q = 0; q < 5; ++q) {
                float m = 0.f;
                if (REF) {
                    const int ls = own - CY[q] * LX - CX[q];
                    m = FLOW ? g_ref(s_ref[R_U][ls], s_ref[R_JX][ls], s_ref[R_JY][ls], CX[q], CY[q]) : s_ref[R_U][ls];
                }
                g[q] = S::dec(graw[q], W5[q], m);
            }
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
            // FP32 storage closes the zeroth and first moments of each collision exactly (below): the
            // sums of the incoming populations are then taken in FP64, where a sum of a few FP32 values
            // is exact.  In uniform streams every cell rounds the same numbers the same way, so
            // independent roundings of each population add up coherently into a drift of the
            // pressure level and of the species; with the moments closed, the collision changes them
            // by one rounding of a small population only.  16-bit storage rounds every population to
            // 16 bits afterwards anyway and keeps the cheaper FP32 sums.
            constexpr bool EXACT = !REF;
            const double U64 = EXACT ? (((double)g[0] + (double)g[1]) + ((double)g[2] + (double)g[3])) + (double)g[4] : 0.0;
            const float U = EXACT ? (float)U64 : (g[0] + g[1]) + (g[2] + g[3]) + g[4];

            // ---- isotropic gradient (Sec. 3.1.1): sum over the stencil of w(|c|^2) phi(x + c) c with
            // the Table 1 weights (E4: 1/3 on axis neighbours, 1/12 on diagonals; no 1/cs^2), or the
            // central difference (E2: 1/2, 0), in FP64
            const double phi64 = s_phi[own];
            const float phi = (float)phi64;
            const double* P = s_phi + own;
            const double pE = P[1], pW = P[-1], pN = P[LX], pS = P[-LX];
            const double pNE = P[LX + 1], pNW = P[LX - 1], pSW = P[-LX - 1], pSE = P[-LX + 1];
            double gx64 = d.gw[0] * (pE - pW) + d.gw[1] * ((pNE - pNW) + (pSE - pSW));
            double gy64 = d.gw[0] * (pN - pS) + d.gw[1] * ((pNE + pNW) - (pSE + pSW));
            if constexpr (RAD == 2) {
                // E6 / E8: the layers |c|^2 = 4 (2, 0), 5 (2, 1) and (1, 2), and 8 (2, 2)
                auto Q = [&](int i, int j) { return P[j * LX + i]; };
                const double w4 = d.gw[2], w5 = d.gw[3], w8 = d.gw[4];
                gx64 += 2.0 * w4 * (Q(2, 0) - Q(-2, 0)) +
                        w5 * (2.0 * ((Q(2, 1) - Q(-2, 1)) + (Q(2, -1) - Q(-2, -1))) +
                              ((Q(1, 2) - Q(-1, 2)) + (Q(1, -2) - Q(-1, -2)))) +
                        2.0 * w8 * ((Q(2, 2) - Q(-2, 2)) + (Q(2, -2) - Q(-2, -2)));
                gy64 += 2.0 * w4 * (Q(0, 2) - Q(0, -2)) +
                        w5 * (2.0 * ((Q(1, 2) - Q(1, -2)) + (Q(-1, 2) - Q(-1, -2))) +
                              ((Q(2, 1) - Q(2, -1)) + (Q(-2, 1) - Q(-2, -1)))) +
                        2.0 * w8 * ((Q(2, 2) - Q(2, -2)) + (Q(-2, 2) - Q(-2, -2)));
            }
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
                double m64 = 0.0, jx64 = 0.0, jy64 = 0.0;
                float drho;
                if (EXACT) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) m64 += (double)f[q];
                    jx64 = ((double)f[1] - (double)f[3]) + ((double)f[5] - (double)f[6]) + ((double)f[8] - (double)f[7]);
                    jy64 = ((double)f[2] - (double)f[4]) + ((double)f[5] + (double)f[6]) - ((double)f[7] + (double)f[8]);
                    drho = (float)m64;
                    jx = (float)jx64;
                    jy = (float)jy64;
                } else {
                    drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
                    jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
                    jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
                }
                // drag k = h eta_f (1 + phi)^2 (1 - phi) / (4 W0^2) and the projected velocity
                // u = (1 - phi)/2 j / (rho + k/2).  FP32 storage takes this chain in FP64 from the FP64
                // moments: in FP32, rho u differs from j by a few ulps, by the same amount in every cell
                // of a uniform stream, and the momentum closure below would apply that difference as a
                // force on the whole stream at every step
                float k;
                double rho64 = 0.0, k64 = 0.0, ux64 = 0.0, uy64 = 0.0;
                if (EXACT) {
                    rho64 = 1.0 + m64;
                    const double pc64 = fmin(fmax(phi64, -1.0), 1.0);
                    k64 = (double)d.kdrag * (1.0 + pc64) * (1.0 + pc64) * (1.0 - pc64);
                    const double sc64 = 0.5 * (1.0 - pc64) / (rho64 + 0.5 * k64);
                    ux64 = jx64 * sc64;
                    uy64 = jy64 * sc64;
                    rho = (float)rho64;
                    k = (float)k64;
                    ux = (float)ux64;
                    uy = (float)uy64;
                } else {
                    rho = 1.f + drho;
                    const float pc = fminf(fmaxf(phi, -1.f), 1.f);
                    k = d.kdrag * (1.f + pc) * (1.f + pc) * (1.f - pc);
                    const float sc = 0.5f * (1.f - pc) / (rho + 0.5f * k);
                    ux = jx * sc;
                    uy = jy * sc;
                }
                const float uu = ux * ux + uy * uy;
                // BGK relaxation with the Guo term of F = -k u, written as relaxation toward a shifted
                // target: fs_q = f_q - omega (f_q - T_q) with T_q = f_eq,q - w_q + S_q / omega (exact in
                // real arithmetic; the difference f_q - T_q is small near equilibrium, so the update keeps
                // its accuracy in uniform streams).  T_q = w_q (A + Bc c.u + Cc (c.u)^2) with, for
                // G = (tau_f - 1/2) k = guo k / omega,
                //   A = drho - (1.5 rho - 3 G) u.u,  Bc = 3 (rho - G),  Cc = 4.5 rho - 9 G;
                // opposite velocities share w (A + Cc (c.u)^2) and differ in the sign of w Bc c.u; the
                // rest population takes the remainder of the moving ones
                const float omf = d.omega_f, G = d.tauf_m_half * k;
                const float A = drho - (1.5f * rho - 3.f * G) * uu;
                const float Bc = 3.f * (rho - G), Cc = 4.5f * rho - 9.f * G;
                float Tq[9];
                auto pair = [&](int q, int qb, float cu) {  // q along c, qb along -c
                    const float S0 = W9[q] * __builtin_fmaf(Cc * cu, cu, A), D = W9[q] * Bc * cu;
                    Tq[q] = S0 + D;
                    Tq[qb] = S0 - D;
                };
                pair(1, 3, ux);
                pair(2, 4, uy);
                pair(5, 7, ux + uy);
                pair(6, 8, uy - ux);
                Tq[0] = drho - sum8(Tq);
#pragma unroll
                for (int q = 0; q < 9; ++q) fs[q] = __builtin_fmaf(-omf, f[q] - Tq[q], f[q]);
                if (EXACT) {
                    // after collision the first moments are j - omega (j - rho u) + (1 - omega/2) F and the
                    // zeroth is unchanged (Guo forcing, Sec. 2.2.1): fs_1 and fs_2 take the first moments as
                    // remainders, then fs_0 the zeroth, with every sum in FP64
                    const double omd = d.omega_f, gud = d.guo;
                    const double px = jx64 - omd * (jx64 - rho64 * ux64) - gud * k64 * ux64;
                    const double py = jy64 - omd * (jy64 - rho64 * uy64) - gud * k64 * uy64;
                    fs[1] = (float)(px - ((-(double)fs[3] + (double)fs[5]) + ((double)fs[8] - (double)fs[6] - (double)fs[7])));
                    fs[2] = (float)(py - ((-(double)fs[4] + (double)fs[5]) + ((double)fs[6] - (double)fs[7] - (double)fs[8])));
                    double s64 = 0.0;
#pragma unroll
                    for (int q = 1; q < 9; ++q) s64 += (double)fs[q];
                    fs[0] = (float)(m64 - s64);
                }
            }

            // ---- vapour (Sec. 2.2.2): tau_g = 1/2 + (tau_vap - 1/2) q with q = clamp((1 - phi)/2, 0, 1),
            // or q = 1 in both phases for the symmetric (thermal) variant
            const float sq = d.sym ? 1.f : fminf(fmaxf(0.5f * (1.f - phi), 0.f), 1.f);
            const float itg = 1.f / (0.5f + d.tauv_m_half * sq);
            const float srcg = d.half_Lsat * (phi - phip);
            float gs[5];
            {
                // relaxation toward g_eq = w U (1 + 3 c.u) and the source share w srcg, gathered:
                //   gs_q = (1 - itg) g_q + w (itg U - srcg) + 3 w itg U c.u, rest as the remainder
                const float K = itg * U - srcg, G0 = W5[1] * K, G1 = 0.5f * itg * U;  // 3 w = 1/2
                const float Gx = G1 * ux, Gy = G1 * uy, itc = 1.f - itg;
                const float E1 = G0 + Gx, E3 = G0 - Gx, E2 = G0 + Gy, E4 = G0 - Gy;
                gs[1] = __builtin_fmaf(itc, g[1], E1);
                gs[2] = __builtin_fmaf(itc, g[2], E2);
                gs[3] = __builtin_fmaf(itc, g[3], E3);
                gs[4] = __builtin_fmaf(itc, g[4], E4);
                gs[0] = __builtin_fmaf(itc, g[0], K - ((E1 + E2) + (E3 + E4)));
                if (EXACT)  // the zeroth moment after collision is U - src: gs_0 as its remainder
                    gs[0] = (float)((U64 - (double)srcg) - (((double)gs[1] + (double)gs[2]) + ((double)gs[3] + (double)gs[4])));
            }

            // ---- phase field (Eq. d, e): relaxation toward h_eq = w (phi - 3 c.N) plus the source share
            // w srcQ, divided by a^2, gathered into Pq = ia2 (1 - ieta) h_q + ia2 (w K - 3 ieta w c.N)
            // with K = ieta phi + srcQ; opposite velocities share the first term of the bracket and
            // the rest population takes the remainder of the moving ones
            float HP[9];
            const float hc = ia2 * (1.f - ieta);
            {
                const float K = __builtin_fmaf(ieta, phi, srcQ), Ka = ia2 * K, Na = 3.f * ia2 * ieta;
                auto pair = [&](int q, int qb, float cN) {
                    const float S0 = W9[q] * Ka, D = W9[q] * Na * cN;
                    HP[q] = S0 - D;
                    HP[qb] = S0 + D;
                };
                pair(1, 3, Nx);
                pair(2, 4, Ny);
                pair(5, 7, Nx + Ny);
                pair(6, 8, Ny - Nx);
                HP[0] = Ka - sum8(HP);
            }

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
                const float Pq = __builtin_fmaf(hc, h[q], HP[q]);
                const int lq = own + CY[q] * LX + CX[q];
                const float fm = (REF && FLOW) ? f_ref(rR, rJx, rJy, CX[q], CY[q]) : 0.f;
                const float gm = REF ? (FLOW ? g_ref(rU, rJx, rJy, CX[q], CY[q]) : rU) : 0.f;
                if (xd >= 0) {
                    const uint32_t dO = ((CX[q] > 0 ? xpE : (CX[q] < 0 ? xpW : xp)) + ypd) * ES;
                    const float href = REF ? s_phif[lq] : 0.f;  // h references its holder's phi(t)
                    gst<T>(pout + (PH + q) * pb, dO, S::enc(Pq - B * s_h[q][lq], IW9[q], href));
                    if (FLOW) gst<T>(pout + (PF + q) * pb, dO, f_dev_enc<S>(fs[q], q, fm));
                    if (q < 5) gst<T>(pout + (PG + q) * pb, dO, S::enc(gs[q], IW5[q], gm));
                }
                if (INOUT) {
                    if (CX[q] < 0 && x == d.nx - 1) {
                        // outlet ghost at x = nx is a copy of this column: it streams into (nx-1, yd)
                        const uint32_t dO = (xp + ypd) * ES;
                        const int ld = own + CY[q] * LX;
                        const float href = REF ? s_phif[ld] : 0.f;
                        gst<T>(pout + (PH + q) * pb, dO, S::enc(Pq - B * s_h[q][ld], IW9[q], href));
                        gst<T>(pout + (PF + q) * pb, dO, f_dev_enc<S>(fs[q], q, fm));
                        if (q < 5) gst<T>(pout + (PG + q) * pb, dO, S::enc(gs[q], IW5[q], gm));
                    }
                    if (CX[q] > 0 && x == 0) {
                        // inlet ghost at x = -1: equilibrium at (rho0, u_in; U_in; phi = -1); its
                        // reference values are the LDS ones of the ghost column
                        const int lg = own - CX[q] - CY[q] * LX;  // the ghost source in the LDS halo
                        float gfm = 0.f, ggm = 0.f;
                        if (REF) {
                            ggm = g_ref(s_ref[R_U][lg], s_ref[R_JX][lg], s_ref[R_JY][lg], CX[q], CY[q]);
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

template <int TX, int TY, class S, bool FLOW, bool INOUT, int RAD>
static void* step_fn() {
    return reinterpret_cast<void*>(&k_step<TX, TY, S, FLOW, INOUT, RAD>);
}

template <class S, bool FLOW, bool INOUT, int RAD>
static void* step_fn_tile(int cfg) {
    switch (cfg) {
        case 0: return step_fn<64, 4, S, FLOW, INOUT, RAD>();
        case 1: return step_fn<64, 8, S, FLOW, INOUT, RAD>();
        case 2: return step_fn<128, 2, S, FLOW, INOUT, RAD>();
        case 3: return step_fn<128, 4, S, FLOW, INOUT, RAD>();
        case 4: return step_fn<64, 2, S, FLOW, INOUT, RAD>();
        case 5: return step_fn<32, 8, S, FLOW, INOUT, RAD>();
    }
    return nullptr;
}

template <class S, int RAD>
static void* step_fn_store(int cfg, int flow, int inout) {
    if (!flow) return step_fn_tile<S, false, false, RAD>(cfg);
    if (!inout) return step_fn_tile<S, true, false, RAD>(cfg);
    return step_fn_tile<S, true, true, RAD>(cfg);
}

template <int RAD>
static void* step_kernel_rad(int cfg, int storage, int flow, int inout) {
    switch (storage) {
        case 0: return step_fn_store<StoreF32, RAD>(cfg, flow, inout);
        case 1: return step_fn_store<StoreF16, RAD>(cfg, flow, inout);
        case 2: return step_fn_store<StoreBF16, RAD>(cfg, flow, inout);
    }
    return nullptr;
}

static void* step_kernel(int cfg, int storage, int flow, int inout, int rad) {
    if (cfg < 0 || cfg >= kNumTiles) return nullptr;
    if (inout && !flow) return nullptr;
    if (rad == 1) return step_kernel_rad<1>(cfg, storage, flow, inout);
    if (rad == 2) return step_kernel_rad<2>(cfg, storage, flow, inout);
    return nullptr;
}

// Grid of a step launch.  grid_mode 0: one workgroup per tile, dispatched in (XCD-contiguous) tile
// order -- measured best for streaming traffic on MI355X.  grid_mode 1: a persistent grid of one
// wave of resident workgroups that loops over the tiles.
int step_grid(int cfg, int ntiles, int storage, int flow, int inout, int rad, int grid_mode) {
    void* fn = step_kernel(cfg, storage, flow, inout, rad);
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

hipError_t launch_step(int cfg, int storage, int flow, int inout, int rad, const DomDesc* doms_dev,
                       const TileDesc* tiles_dev, int ntiles, int grid, int par, hipStream_t s) {
    void* fn = step_kernel(cfg, storage, flow, inout, rad);
    if (!fn) return hipErrorInvalidValue;
    if (ntiles <= 0) return hipSuccess;
    const int nt = kTiles[cfg].tx * kTiles[cfg].ty;
    int remap = 1;
    void* args[] = {(void*)&doms_dev, (void*)&tiles_dev, (void*)&ntiles, (void*)&par, (void*)&remap};
    return hipLaunchKernel(fn, dim3(grid), dim3(nt), args, 0, s);
}

}  // namespace snowlb
