// snowlb3d_kernels.hip -- gfx950 kernels of the coupled lattice-Boltzmann ice-growth step in three
// dimensions, the extension of the 2D method (Tan et al., arXiv:2101.07163, Sec. 2.2) that its Sec. 4
// proposes.  Lattices: D3Q19 flow, D3Q7 vapour and phase field (cs^2 = 1/4); gradient over the 18
// D3Q19 neighbours with weights 1/6 (axes) and 1/12 (face diagonals); hexagonal anisotropy about the
// z (c) axis, a = 1 + eps Re((n_x + i n_y)^6), which is the paper's 1 + eps cos 6 theta for normals in
// the basal plane; x periodic or inlet/outlet, y and z periodic.
//
// k_step3 is one fused step per block of 64 x 2 x 2 cells, built like the 2D k_step: the block's h
// and phi (FP64) are staged with a one-cell halo in LDS (the gradient and the destination term
// h_q(x + c_q, t) of Eq. (d)), each cell collides all three populations and pushes them to their
// destinations, and every (destination, q) is written by exactly one thread.  FP32 storage; the
// collisions close their zeroth and first moments through FP64 sums, as in 2D.
#include <hip/hip_runtime.h>

#include "snowlb3d_internal.h"

namespace snowlb3d {

#define GMEM __attribute__((address_space(1)))

// D3Q19: rest, 6 axis, 12 face diagonals; D3Q7 is the first seven
__device__ constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__device__ constexpr float W19[19] = {1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                      1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                      1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                      1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
__device__ constexpr float W7[7] = {0.25f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f};

// s += c v for a velocity component c in {-1, 0, 1} known at compile time (no instruction for c = 0)
__device__ __forceinline__ void acc(double& s, int c, double v) {
    if (c > 0) s += v;
    else if (c < 0) s -= v;
}

__device__ __forceinline__ int wrapi(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) i = ((i % n) + n) % n;
    return i;
}

// Closure of a lattice position: y, z periodic; x periodic or (inlet/outlet) the inlet ghost left of
// x = 0 (returns false) and a copy of plane nx - 1 right of it.
template <bool INOUT>
__device__ __forceinline__ bool map3(const Dom3& d, int gx, int gy, int gz, int& sx, int& sy, int& sz) {
    sy = wrapi(gy, d.ny);
    sz = wrapi(gz, d.nz);
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

template <bool FLOW, bool INOUT>
__global__ void __launch_bounds__(kBlockCells) k_step3(const Dom3* __restrict__ dp, int par, int xcd_remap) {
    constexpr int LX = kBX + 2, LY = kBY + 2, LZ = kBZ + 2, LN = LX * LY * LZ;
    constexpr int NP = FLOW ? 33 : 14;                       // planes per block of a copy
    constexpr int PF = 0, PG = FLOW ? 19 : 0, PH = PG + 7;  // first plane of f, g and h
    constexpr uint32_t PB = kBlockCells * 4;                 // bytes between the planes of a block
    __shared__ double s_phi[LN];
    __shared__ float s_h[7][LN];
    const Dom3& d = *dp;

    const int tid = threadIdx.x;
    const int tx = tid & (kBX - 1), ty = (tid >> kSX) & (kBY - 1), tz = tid >> (kSX + kSY);
    // XCD-aware order: each of the 8 XCDs takes a contiguous run of blocks (a permutation for any grid).
    // Odd and even XCDs walk their runs in opposite directions, so the two XCDs on either side of a
    // shared z-slab boundary reach it at the same time and its halo lines meet in the last-level cache;
    // every XCD turns round every other step (input copy 1), so that a step starts on the blocks the
    // previous one wrote last, which are still in that cache (0.2418 -> 0.2386 ms on the 256 x 128 x 128
    // step against the same direction for all XCDs)
    const int G = gridDim.x, b = blockIdx.x;
    int t = b;
    if (xcd_remap) {
        const int x = b % 8, k = b / 8, cnt = G / 8 + (x < G % 8 ? 1 : 0);
        t = x * (G / 8) + min(x, G % 8) + (((x & 1) ^ par) ? cnt - 1 - k : k);
    }
    const int bx = t % d.nbx, by = (t / d.nbx) % d.nby, bz = t / (d.nbx * d.nby);
    const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool active = x < d.nx && y < d.ny && z < d.nz;
    const int par1 = 1 - par;
    const GMEM char* pin = (const GMEM char*)d.pop[par];
    GMEM char* pout = (GMEM char*)d.pop[par1];
    const GMEM char* phin = (const GMEM char*)d.phip[par];
    GMEM char* phout = (GMEM char*)d.phip[par1];

    const uint32_t xp = xpart(x, NP), yp = ypart(y, d.nbx, NP), zp = zpart(z, d.nbx, d.nby, NP);
    const uint32_t co = xp + yp + zp;
    const uint32_t cf = xpart(x, 1) + ypart(y, d.nbx, 1) + zpart(z, d.nbx, d.nby, 1);

    // the cell's own flow, vapour and phi_prev first, then the halo box of h
    float f[19], g[7], phip = 0.f;
    if (active) {
#pragma unroll
        for (int q = 0; q < 7; ++q) g[q] = gld<float>(pin + (PG + q) * PB, co * 4);
        if (FLOW) {
#pragma unroll
            for (int q = 0; q < 19; ++q) f[q] = gld<float>(pin + (PF + q) * PB, co * 4);
        }
        phip = gld<float>(phin, cf * 4);
    }
    for (int p = tid; p < LN; p += kBlockCells) {
        const int lx = p % LX, ly = (p / LX) % LY, lz = p / (LX * LY);
        int sx, sy, sz;
        const bool real = map3<INOUT>(d, x0 + lx - 1, y0 + ly - 1, z0 + lz - 1, sx, sy, sz);
        double p64 = -1.0;  // inlet ghost: phi = -1 (its h are never read)
        float hh[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (real) {
            const uint32_t o = xpart(sx, NP) + ypart(sy, d.nbx, NP) + zpart(sz, d.nbx, d.nby, NP);
            p64 = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                hh[q] = gld<float>(pin + (PH + q) * PB, o * 4);
                p64 += (double)hh[q];
            }
        }
        s_phi[p] = p64;
#pragma unroll
        for (int q = 0; q < 7; ++q) s_h[q][p] = hh[q];
    }
    __syncthreads();
    if (!active) return;  // no barrier follows

    const int own = ((tz + 1) * LY + (ty + 1)) * LX + (tx + 1);
    float h[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) h[q] = s_h[q][own];
    const double phi64 = s_phi[own];
    const float phi = (float)phi64;

    // isotropic gradient over the 18 D3Q19 neighbours, FP64: differences across each pair of
    // opposite neighbours, weighted 1/6 on the axes and 1/12 on the face diagonals
    auto ph = [&](int q) { return s_phi[own + (CZ[q] * LY + CY[q]) * LX + CX[q]]; };
    const double d1 = ph(1) - ph(2), d3 = ph(3) - ph(4), d5 = ph(5) - ph(6);  // x, y, z
    const double d7 = ph(7) - ph(8), d9 = ph(9) - ph(10);                     // (1, 1, 0), (1, -1, 0)
    const double d11 = ph(11) - ph(12), d13 = ph(13) - ph(14);                // (1, 0, 1), (1, 0, -1)
    const double d15 = ph(15) - ph(16), d17 = ph(17) - ph(18);                // (0, 1, 1), (0, 1, -1)
    const double gx64 = d1 * (1.0 / 6.0) + ((d7 + d9) + (d11 + d13)) * (1.0 / 12.0);
    const double gy64 = d3 * (1.0 / 6.0) + ((d7 - d9) + (d15 + d17)) * (1.0 / 12.0);
    const double gz64 = d5 * (1.0 / 6.0) + ((d11 - d13) + (d15 - d17)) * (1.0 / 12.0);
    // anisotropy a = 1 + eps P, P = Re((n_x + i n_y)^6), and the flux N = kappa Dphi |g|^2 a da/dg:
    // with X = gx^2/|g|^2, Y = gy^2/|g|^2,  P = X^3 - 15 X^2 Y + 15 X Y^2 - Y^3 and
    // |g|^2 dP/dg = 6 (gx (X^2 - 10 X Y + 5 Y^2 - P), -gy (5 X^2 - 10 X Y + Y^2 + P), -gz P)
    float a = 1.f, Nx = 0.f, Ny = 0.f, Nz = 0.f;
    if (gx64 * gx64 + gy64 * gy64 + gz64 * gz64 > d.grad_eps2) {
        const float gx = (float)gx64, gy = (float)gy64, gz = (float)gz64;
        const float inv = 1.f / (gx * gx + gy * gy + gz * gz);
        const float X = gx * gx * inv, Y = gy * gy * inv;
        const float P = X * X * X - 15.f * X * X * Y + 15.f * X * Y * Y - Y * Y * Y;
        a = 1.f + d.eps * P;
        const float c = d.coefN * a;  // coefN = 6 kappa_N eps W0^2/tau0
        Nx = c * gx * (X * X - 10.f * X * Y + 5.f * Y * Y - P);
        Ny = -c * gy * (5.f * X * X - 10.f * X * Y + Y * Y + P);
        Nz = -c * gz * P;
    }
    const float a2 = a * a;
    const float ia2 = 1.f / a2;
    const float B = ia2 - 1.f;
    const float ieta = 1.f / (4.f * d.Dphi * a2 + 0.5f);
    const float om = 1.f - phi * phi;

    // vapour: U as an FP64 sum (exact for a few FP32 values)
    const double U64 = (((double)g[0] + (double)g[1]) + ((double)g[2] + (double)g[3])) +
                       (((double)g[4] + (double)g[5]) + (double)g[6]);
    const float U = (float)U64;
    const float srcQ = (phi - phi * phi * phi + d.lam * U * om * om) * d.inv_tau0;

    // flow: deviations df = f - w, FP64 moments, Guo forcing, moments of the collision closed in FP64
    float ux = 0.f, uy = 0.f, uz = 0.f, fs[19];
    if (FLOW) {
        double m64 = 0.0, jx64 = 0.0, jy64 = 0.0, jz64 = 0.0;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const double v = f[q];
            m64 += v;
            acc(jx64, CX[q], v);
            acc(jy64, CY[q], v);
            acc(jz64, CZ[q], v);
        }
        // drag and projected velocity in FP64 from the FP64 moments (in FP32, rho u would differ from j
        // by a few ulps alike in every cell of a uniform stream, which the momentum closure below would
        // apply as a force at every step)
        const double rho64 = 1.0 + m64, pc64 = fmin(fmax(phi64, -1.0), 1.0);
        const double k64 = (double)d.kdrag * (1.0 + pc64) * (1.0 + pc64) * (1.0 - pc64);
        const double sc64 = 0.5 * (1.0 - pc64) / (rho64 + 0.5 * k64);
        const double ux64 = jx64 * sc64, uy64 = jy64 * sc64, uz64 = jz64 * sc64;
        const float drho = (float)m64, rho = (float)rho64, k = (float)k64;
        ux = (float)ux64;
        uy = (float)uy64;
        uz = (float)uz64;
        const float uu = ux * ux + uy * uy + uz * uz;
        // BGK relaxation with the Guo term of F = -k u, as relaxation toward a shifted target:
        // fs_q = f_q - omega (f_q - T_q), T_q = f_eq,q - w_q + S_q / omega (exact in real arithmetic;
        // f_q - T_q is small near equilibrium) = w_q (A + Bc c.u + Cc (c.u)^2) with G = (tau_f - 1/2) k,
        // A = drho - (1.5 rho - 3 G) u.u, Bc = 3 (rho - G), Cc = 4.5 rho - 9 G; opposite velocities
        // share w (A + Cc (c.u)^2).  fs_0 and the axis populations fs_1, fs_3, fs_5 are replaced by
        // the closure below.
        const float omf = d.omega_f, G = d.tauf_m_half * k;
        const float A = drho - (1.5f * rho - 3.f * G) * uu;
        const float Bc = 3.f * (rho - G), Cc = 4.5f * rho - 9.f * G;
        auto pair = [&](int q, int qb, float cu) {  // q along c, qb along -c
            const float S0 = W19[q] * __builtin_fmaf(Cc * cu, cu, A), D = W19[q] * Bc * cu;
            fs[q] = __builtin_fmaf(-omf, f[q] - (S0 + D), f[q]);
            fs[qb] = __builtin_fmaf(-omf, f[qb] - (S0 - D), f[qb]);
        };
        pair(1, 2, ux);
        pair(3, 4, uy);
        pair(5, 6, uz);
        pair(7, 8, ux + uy);
        pair(9, 10, ux - uy);
        pair(11, 12, ux + uz);
        pair(13, 14, ux - uz);
        pair(15, 16, uy + uz);
        pair(17, 18, uy - uz);
        // after collision the first moments are j - omega (j - rho u) + (1 - omega/2) F and the zeroth
        // is unchanged: fs_1, fs_3, fs_5 (+x, +y, +z) take the first moments as remainders, fs_0 the
        // zeroth, every sum in FP64
        const double omd = d.omega_f, gud = d.guo;
        const double px = jx64 - omd * (jx64 - rho64 * ux64) - gud * k64 * ux64;
        const double py = jy64 - omd * (jy64 - rho64 * uy64) - gud * k64 * uy64;
        const double pz = jz64 - omd * (jz64 - rho64 * uz64) - gud * k64 * uz64;
        // the other populations' shares of each first moment (fs_1, fs_3 and fs_5 carry momentum along
        // their own axis only, so the three remainders are independent)
        double rx = 0.0, ry = 0.0, rz = 0.0;
#pragma unroll
        for (int q = 2; q < 19; ++q) {
            const double v = fs[q];
            acc(rx, CX[q], v);
            if (q != 3) acc(ry, CY[q], v);  // fs_3 is the y remainder
            if (q != 5) acc(rz, CZ[q], v);  // fs_5 is the z remainder
        }
        fs[1] = (float)(px - rx);
        fs[3] = (float)(py - ry);
        fs[5] = (float)(pz - rz);
        double s64 = 0.0;
#pragma unroll
        for (int q = 1; q < 19; ++q) s64 += (double)fs[q];
        fs[0] = (float)(m64 - s64);
    }

    // vapour collision (D3Q7, cs^2 = 1/4): tau_g = 1/2 + (tau_vap - 1/2) clamp((1 - phi)/2, 0, 1)
    const float sq = fminf(fmaxf(0.5f * (1.f - phi), 0.f), 1.f);
    const float itg = 1.f / (0.5f + d.tauv_m_half * sq);
    const float srcg = d.half_Lsat * (phi - phip);
    float gs[7];
    {
        // relaxation toward g_eq = w U (1 + 4 c.u) and the source share w srcg, gathered:
        // gs_q = (1 - itg) g_q + w (itg U - srcg) + 4 w itg U c.u (4 w = 1/2); gs_0 by the closure
        const float G0 = W7[1] * (itg * U - srcg), G1 = 0.5f * itg * U, itc = 1.f - itg;
        const float Gx = G1 * ux, Gy = G1 * uy, Gz = G1 * uz;
        gs[1] = __builtin_fmaf(itc, g[1], G0 + Gx);
        gs[2] = __builtin_fmaf(itc, g[2], G0 - Gx);
        gs[3] = __builtin_fmaf(itc, g[3], G0 + Gy);
        gs[4] = __builtin_fmaf(itc, g[4], G0 - Gy);
        gs[5] = __builtin_fmaf(itc, g[5], G0 + Gz);
        gs[6] = __builtin_fmaf(itc, g[6], G0 - Gz);
        double r64 = 0.0;
#pragma unroll
        for (int q = 1; q < 7; ++q) r64 += (double)gs[q];
        gs[0] = (float)((U64 - (double)srcg) - r64);  // the zeroth moment after collision is U - src
    }

    // phase field (Eq. (d)/(e) on D3Q7): relaxation toward w (phi - c.N/cs^2) plus the source share
    // w Q/tau0, divided by a^2, gathered into P_q = ia2 (1 - ieta) h_q + ia2 (w K - 4 ieta w c.N) with
    // K = ieta phi + srcQ; the rest population takes the remainder of the moving ones
    float P7[7];
    {
        const float hc = ia2 * (1.f - ieta), Ka = ia2 * __builtin_fmaf(ieta, phi, srcQ), Na = 4.f * ia2 * ieta;
        const float S0 = W7[1] * Ka, Dx = W7[1] * Na * Nx, Dy = W7[1] * Na * Ny, Dz = W7[1] * Na * Nz;
        const float H1 = S0 - Dx, H2 = S0 + Dx, H3 = S0 - Dy, H4 = S0 + Dy, H5 = S0 - Dz, H6 = S0 + Dz;
        P7[1] = __builtin_fmaf(hc, h[1], H1);
        P7[2] = __builtin_fmaf(hc, h[2], H2);
        P7[3] = __builtin_fmaf(hc, h[3], H3);
        P7[4] = __builtin_fmaf(hc, h[4], H4);
        P7[5] = __builtin_fmaf(hc, h[5], H5);
        P7[6] = __builtin_fmaf(hc, h[6], H6);
        P7[0] = __builtin_fmaf(hc, h[0], Ka - (((H1 + H2) + (H3 + H4)) + (H5 + H6)));
    }

    // push streaming into copy 1 - par; destinations with the closure
    const int yN = y + 1 < d.ny ? y + 1 : 0, yS = y > 0 ? y - 1 : d.ny - 1;
    const int zU = z + 1 < d.nz ? z + 1 : 0, zD = z > 0 ? z - 1 : d.nz - 1;
    const int xE = x + 1 < d.nx ? x + 1 : (INOUT ? -1 : 0);
    const int xW = x > 0 ? x - 1 : (INOUT ? -1 : d.nx - 1);
    const uint32_t xpE = xpart(xE < 0 ? 0 : xE, NP), xpW = xpart(xW < 0 ? 0 : xW, NP);
    const uint32_t ypN = ypart(yN, d.nbx, NP), ypS = ypart(yS, d.nbx, NP);
    const uint32_t zpU = zpart(zU, d.nbx, d.nby, NP), zpD = zpart(zD, d.nbx, d.nby, NP);
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        if (!FLOW && q >= 7) break;
        const int xd = CX[q] > 0 ? xE : (CX[q] < 0 ? xW : x);
        const uint32_t xo = CX[q] > 0 ? xpE : (CX[q] < 0 ? xpW : xp);
        const uint32_t yo = CY[q] > 0 ? ypN : (CY[q] < 0 ? ypS : yp);
        const uint32_t zo = CZ[q] > 0 ? zpU : (CZ[q] < 0 ? zpD : zp);
        const int lq = own + (CZ[q] * LY + CY[q]) * LX + CX[q];  // destination in the halo box
        if (xd >= 0) {
            const uint32_t dO = (xo + yo + zo) * 4;
            if (q < 7) {
                gst<float>(pout + (PH + q) * PB, dO, P7[q] - B * s_h[q][lq]);
                gst<float>(pout + (PG + q) * PB, dO, gs[q]);
            }
            if (FLOW) gst<float>(pout + (PF + q) * PB, dO, fs[q]);
        }
        if (INOUT) {
            if (CX[q] < 0 && x == d.nx - 1) {
                // the outlet ghost at x = nx copies this plane: it streams into (nx-1, y + cy, z + cz)
                const uint32_t dO = (xp + yo + zo) * 4;
                const int ld = own + (CZ[q] * LY + CY[q]) * LX;
                if (q < 7) {
                    gst<float>(pout + (PH + q) * PB, dO, P7[q] - B * s_h[q][ld]);
                    gst<float>(pout + (PG + q) * PB, dO, gs[q]);
                }
                gst<float>(pout + (PF + q) * PB, dO, fs[q]);
            }
            if (CX[q] > 0 && x == 0) {
                // the inlet ghost at x = -1: equilibrium (rho0, (u_in, 0, 0); U_in; phi = -1)
                if (q < 7) {
                    gst<float>(pout + (PH + q) * PB, co * 4, -W7[q]);
                    gst<float>(pout + (PG + q) * PB, co * 4, d.g_in[q]);
                }
                gst<float>(pout + (PF + q) * PB, co * 4, d.df_in[q]);
            }
        }
    }
    gst<float>(phout, cf * 4, phi);
}

template <bool FLOW, bool INOUT>
static void* step_fn() {
    return reinterpret_cast<void*>(&k_step3<FLOW, INOUT>);
}

hipError_t launch_step3(const Dom3& d, const Dom3* d_dev, int par, hipStream_t s) {
    void* fn = !d.flow ? step_fn<false, false>() : (d.inout ? step_fn<true, true>() : step_fn<true, false>());
    if (!d.flow && d.inout) return hipErrorInvalidValue;
    const int grid = d.nbx * d.nby * d.nbz;
    int remap = 1;
    void* args[] = {(void*)&d_dev, (void*)&par, (void*)&remap};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlockCells), args, 0, s);
}

// ------------------------------------------------------------------------------------------ set-up
// and read-out: plain per-cell kernels (not on the per-step path)

__device__ __forceinline__ int64_t idx(const Dom3& d, int nq, int q, int x, int y, int z) {
    return (int64_t)xpart(x, nq) + ypart(y, d.nbx, nq) + zpart(z, d.nbx, d.nby, nq) + (int64_t)q * kBlockCells;
}

__global__ void k_init3(Dom3 d, int par, const float* U_init, float U0, float sx, float sy, float sz, float R,
                        float width) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= d.nx) return;
    const int NP = d.npop, PG = d.flow ? 19 : 0, PH = PG + 7;
    const float dx = x - sx, dy = y - sy, dz = z - sz;
    const float r = sqrtf(dx * dx + dy * dy + dz * dz);
    const float phi0 = tanhf((R - r) / (1.41421356237309505f * width));
    const float ux = (d.flow && d.inout) ? 0.5f * (1.f - phi0) * d.u_in : 0.f;
    const int64_t c = ((int64_t)z * d.ny + y) * d.nx + x;
    const float U = U_init ? U_init[c] : U0;
    float* pb = d.pop[par];
    d.phip[par][idx(d, 1, 0, x, y, z)] = phi0;
    float s = 0.f;
    for (int q = 1; q < 7; ++q) {
        pb[idx(d, NP, PH + q, x, y, z)] = W7[q] * phi0;
        s += W7[q] * phi0;
    }
    pb[idx(d, NP, PH, x, y, z)] = phi0 - s;
    s = 0.f;
    for (int q = 1; q < 7; ++q) {
        const float v = W7[q] * U * (1.f + 4.f * CX[q] * ux);
        pb[idx(d, NP, PG + q, x, y, z)] = v;
        s += v;
    }
    pb[idx(d, NP, PG, x, y, z)] = U - s;
    if (d.flow) {
        const float drho = d.rho0 - 1.f, uu = ux * ux;
        s = 0.f;
        for (int q = 1; q < 19; ++q) {
            const float cu = CX[q] * ux;
            const float v = W19[q] * (drho + d.rho0 * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
            pb[idx(d, NP, q, x, y, z)] = v;
            s += v;
        }
        pb[idx(d, NP, 0, x, y, z)] = drho - s;
    }
}

hipError_t launch_init3(const Dom3& d, int par, const float* U_init, float U0, float sx, float sy, float sz,
                        float R, float width, hipStream_t s) {
    hipLaunchKernelGGL(k_init3, dim3((d.nx + 127) / 128, d.ny, d.nz), dim3(128), 0, s, d, par, U_init, U0, sx, sy,
                       sz, R, width);
    return hipGetLastError();
}

// moments of one cell: phi, U, rho and the velocity the collisions use
__device__ void cell_fields(const Dom3& d, int par, int x, int y, int z, float out[6]) {
    const int NP = d.npop, PG = d.flow ? 19 : 0, PH = PG + 7;
    const float* pb = d.pop[par];
    double phi = 0.0, U = 0.0;
    for (int q = 0; q < 7; ++q) {
        phi += pb[idx(d, NP, PH + q, x, y, z)];
        U += pb[idx(d, NP, PG + q, x, y, z)];
    }
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    if (d.flow)
        for (int q = 0; q < 19; ++q) {
            const double v = pb[idx(d, NP, q, x, y, z)];
            rho += v;
            j[0] += CX[q] * v;
            j[1] += CY[q] * v;
            j[2] += CZ[q] * v;
        }
    out[0] = (float)phi;
    out[1] = (float)U;
    out[2] = d.flow ? (float)(1.0 + rho) : 0.f;
    out[3] = out[4] = out[5] = 0.f;
    if (d.flow) {
        const float pc = fminf(fmaxf(out[0], -1.f), 1.f);
        const float k = d.kdrag * (1.f + pc) * (1.f + pc) * (1.f - pc);
        const float sc = 0.5f * (1.f - pc) / (out[2] + 0.5f * k);
        for (int c = 0; c < 3; ++c) out[3 + c] = (float)j[c] * sc;
    }
}

__global__ void k_read3(Dom3 d, int par, int field, float* dst) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= d.nx) return;
    float v[6];
    cell_fields(d, par, x, y, z, v);
    dst[((int64_t)z * d.ny + y) * d.nx + x] = v[field];
}

hipError_t launch_read3(const Dom3& d, int par, int field, float* dst, hipStream_t s) {
    if (field < 0 || field > 5) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_read3, dim3((d.nx + 127) / 128, d.ny, d.nz), dim3(128), 0, s, d, par, field, dst);
    return hipGetLastError();
}

// canonical FP32 [q][z][y][x] <-> the blocked layout (f is stored as f - w)
__global__ void k_pop_io3(Dom3 d, int par, int set, int to_canon, float* canon) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= d.nx) return;
    const int64_t n = (int64_t)d.nx * d.ny * d.nz, c = ((int64_t)z * d.ny + y) * d.nx + x;
    if (set == 3) {
        float* p = &d.phip[par][idx(d, 1, 0, x, y, z)];
        if (to_canon) canon[c] = *p;
        else *p = canon[c];
        return;
    }
    const int NP = d.npop, PG = d.flow ? 19 : 0, PH = PG + 7;
    const int nq = set == 0 ? 19 : 7, base = set == 0 ? 0 : (set == 1 ? PG : PH);
    for (int q = 0; q < nq; ++q) {
        float* p = &d.pop[par][idx(d, NP, base + q, x, y, z)];
        const float w = set == 0 ? W19[q] : 0.f;
        if (to_canon) canon[q * n + c] = *p + w;
        else *p = canon[q * n + c] - w;
    }
}

hipError_t launch_pop_io3(const Dom3& d, int par, int set, int to_canon, float* canon, hipStream_t s) {
    hipLaunchKernelGGL(k_pop_io3, dim3((d.nx + 127) / 128, d.ny, d.nz), dim3(128), 0, s, d, par, set, to_canon,
                       canon);
    return hipGetLastError();
}

// FP64 diagnostics: per-thread sums over a fixed set of cells, wave64 shuffle, LDS, one partial per
// workgroup, then one workgroup adds the partials in a fixed order (deterministic)
constexpr int kDiagThreads = 256, kDiagQ = 9;

int diag_blocks3(const Dom3& d) {
    const long cells = (long)d.nx * d.ny * d.nz;
    long b = (cells + kDiagThreads * 4 - 1) / (kDiagThreads * 4);
    if (b > 2048) b = 2048;
    return (int)(b < 1 ? 1 : b);
}

__global__ void __launch_bounds__(kDiagThreads) k_diag3(Dom3 d, int par, double* partials) {
    const int NP = d.npop, PG = d.flow ? 19 : 0, PH = PG + 7;
    double acc[kDiagQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
    for (int64_t c = (int64_t)blockIdx.x * kDiagThreads + threadIdx.x; c < cells; c += (int64_t)gridDim.x * kDiagThreads) {
        const int x = (int)(c % d.nx), y = (int)((c / d.nx) % d.ny), z = (int)(c / ((int64_t)d.nx * d.ny));
        const float* pb = d.pop[par];
        double phi = 0.0, U = 0.0, rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        bool bad = false;
        for (int q = 0; q < 7; ++q) {
            const float hv = pb[idx(d, NP, PH + q, x, y, z)], gv = pb[idx(d, NP, PG + q, x, y, z)];
            bad |= !isfinite(hv) || !isfinite(gv);
            phi += hv;
            U += gv;
        }
        if (d.flow)
            for (int q = 0; q < 19; ++q) {
                const float fv = pb[idx(d, NP, q, x, y, z)];
                bad |= !isfinite(fv);
                const double v = (double)(W19[q] + fv);  // f as the read-out gives it (FP32 w + (f - w))
                rho += v;
                j[0] += CX[q] * v;
                j[1] += CY[q] * v;
                j[2] += CZ[q] * v;
            }
        const float pp = d.phip[par][idx(d, 1, 0, x, y, z)];
        bad |= !isfinite(pp);
        acc[0] += rho; acc[1] += j[0]; acc[2] += j[1]; acc[3] += j[2]; acc[4] += U; acc[5] += phi; acc[6] += pp;
        acc[7] += phi > 0.0 ? 1.0 : 0.0;
        acc[8] += bad ? 1.0 : 0.0;
    }
    __shared__ double s_part[kDiagThreads / 64][kDiagQ];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    for (int k = 0; k < kDiagQ; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) s_part[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDiagQ) {
        double v = 0.0;
        for (int w = 0; w < kDiagThreads / 64; ++w) v += s_part[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * kDiagQ + threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(kDiagQ * 32) k_diag3_final(const double* __restrict__ partials, int nblk,
                                                             double half_Lsat, double* __restrict__ out) {
    // 32 lanes per quantity: lane l of quantity k sums blocks l, l + 32, ... in order, then lane 0 adds
    // the 32 lane sums in order (fixed order, hence deterministic); then the species invariant.
    __shared__ double s[kDiagQ][32];
    __shared__ double tot[kDiagQ];
    const int k = threadIdx.x / 32, l = threadIdx.x % 32;
    double v = 0.0;
    for (int b = l; b < nblk; b += 32) v += partials[(int64_t)b * kDiagQ + k];
    s[k][l] = v;
    __syncthreads();
    if (l == 0) {
        double t = 0.0;
        for (int i = 0; i < 32; ++i) t += s[k][i];
        out[k] = t;
        tot[k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) out[kDiagQ] = __dadd_rn(tot[4], __dmul_rn(half_Lsat, tot[6]));  // species invariant
}

hipError_t launch_diag3(const Dom3& d, int par, double* partials, double* out, double half_Lsat, hipStream_t s) {
    const int nb = diag_blocks3(d);
    hipLaunchKernelGGL(k_diag3, dim3(nb), dim3(kDiagThreads), 0, s, d, par, partials);
    hipLaunchKernelGGL(k_diag3_final, dim3(1), dim3(kDiagQ * 32), 0, s, partials, nb, half_Lsat, out);
    return hipGetLastError();
}

}  // namespace snowlb3d
