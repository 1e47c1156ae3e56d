// snowlb_adjoint.hip -- hand-written discrete adjoint of the fused step (no flow, periodic, FP32).
//
// For a loss L(phi_T), the adjoint lambda_t = dL/d(state at t) obeys lambda_t = (dF/ds)^T lambda_{t+1}
// where F is one step of the phase field (Eq. (d)/(e), anisotropy of Sec. 2.1, E4 gradient of
// Table 1) and the vapour ADR solver (Sec. 2.2.2) with u = 0.  Each reverse step is two gather
// kernels over the lattice:
//   k_adj_a (per cell x): recompute the forward quantities of x from the stored state at t (phi with
//     its halo for the gradient, a, N, eta, Q, h_eq, h*), take lambda_{t+1} of the populations x
//     emitted (at x + c_q), and form every adjoint that is local to x: lambda_g(x, t) and
//     lambda_phiprev(x, t) completely, and for the h adjoint the per-cell factors A_h = (1 - 1/eta)/a^2,
//     B = (1 - a^2)/a^2, the adjoint of the gradient Gbar(x) and the local part of phibar(x); the
//     explicit dependence on eps is reduced into per-workgroup FP64 partials.
//   k_adj_b (per cell x): lambda_h,q(x, t) = lambda_h,q(x + c_q) A_h(x)   [through h*_q(x)]
//                                           - B(x - c_q) lambda_h,q(x)      [destination term of Eq. (d)]
//                                           + phibar(x) + sum_k W_k c_k . Gbar(x - c_k)   [phi = sum h]
// Layout: every field is an FP32 plane in the cell order of the state, with the state's plane stride;
// the state slot holds g_0..4 then h_0..8; an adjoint slot holds g_0..4, h_0..8, phi_prev; the
// intermediate slot holds A_h, B, Gbar_x, Gbar_y, phibar.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snowlb_internal.h"

namespace snowlb {

namespace {
__device__ constexpr int AX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int AY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr float AW9[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,  1.f / 9.f, 1.f / 9.f,
                                     1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
__device__ constexpr float AW5[5] = {1.f / 3.f, 1.f / 6.f, 1.f / 6.f, 1.f / 6.f, 1.f / 6.f};

constexpr int ATX = 64, ATY = 4, ANT = ATX * ATY;
constexpr int ALX = ATX + 2, ALY = ATY + 2, ALN = ALX * ALY;

// i mod n for any i (one add or subtract in the common case: neighbours and halos of wide lattices)
__device__ __forceinline__ int wrapn(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) i = ((i % n) + n) % n;
    return i;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
}  // namespace

// Position of LDS slot r of a tile at (x0, y0): the slots form the tile and its one-cell ring, row
// by row (ALX x ALY); a lattice position outside the (periodic) lattice wraps.  Returns the in-plane
// byte offset of that position.
__device__ __forceinline__ uint32_t slot_off(const AdjDesc& A, int x0, int y0, int r) {
    const int lx = r % ALX, ly = r / ALX;
    const int gx = wrapn(x0 + lx - 1, A.nx), gy = wrapn(y0 + ly - 1, A.ny);
    return (cell_xpart(gx) + cell_ypart(A.nbx, gy)) * 4u;
}
// LDS slots of the one-cell ring around a tile: top row, bottom row, left column, right column.
__device__ __forceinline__ int ring_slot(int r) {
    if (r < ALX) return r;
    if (r < 2 * ALX) return (ALY - 1) * ALX + (r - ALX);
    if (r < 2 * ALX + ATY) return (1 + r - 2 * ALX) * ALX;
    return (1 + r - 2 * ALX - ATY) * ALX + ALX - 1;
}
constexpr int ARING = 2 * ALX + 2 * ATY;
static_assert(ARING <= ANT, "one ring pass per workgroup");

__global__ void __launch_bounds__(ANT) k_adj_a(AdjDesc A) {
    __shared__ double s_phi[ALN];
    __shared__ float s_h[9][ALN];
    __shared__ double s_red[ANT / 64];
    const int tid = threadIdx.x, tx = tid % ATX, ty = tid / ATX;
    const int ntx = (A.nx + ATX - 1) / ATX;
    const int x0 = (blockIdx.x % ntx) * ATX, y0 = (blockIdx.x / ntx) * ATY;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < A.nx && y < A.ny;
    const int own = (ty + 1) * ALX + tx + 1;
    const uint64_t pb = (uint64_t)A.plane * 4;  // bytes between planes
    const GMEM char* st = (const GMEM char*)A.st;
    const GMEM char* lin = (const GMEM char*)A.lin;
    GMEM char* lout = (GMEM char*)A.lout;
    GMEM char* mid = (GMEM char*)A.mid;

    // h(t) and phi(t) of the tile and its ring in LDS, phi summed in FP64 as in the forward step.
    // Lanes outside the lattice stage the position their slot wraps to (an active neighbour's halo).
    const uint32_t oo = slot_off(A, x0, y0, own);
    float h[9];
    {
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            h[q] = gld<float>(st + (5 + q) * pb, oo);
            p += (double)h[q];
            s_h[q][own] = h[q];
        }
        s_phi[own] = p;
    }
    if (tid < ARING) {
        const int r = ring_slot(tid);
        const uint32_t ro = slot_off(A, x0, y0, r);
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float v = gld<float>(st + (5 + q) * pb, ro);
            p += (double)v;
            s_h[q][r] = v;
        }
        s_phi[r] = p;
    }
    // every other global load of this cell is issued before the barrier too: g(t), lambda(t + 1) of
    // the populations it emitted (at x + c_q) and lambda_phiprev(t + 1)
    const uint32_t xp = cell_xpart(x), yp = cell_ypart(A.nbx, y);
    const uint32_t io = (xp + yp) * 4u;  // == oo for active lanes
    const int yN = wrapn(y + 1, A.ny), yS = wrapn(y - 1, A.ny), xE = wrapn(x + 1, A.nx), xW = wrapn(x - 1, A.nx);
    const uint32_t xpE = cell_xpart(xE), xpW = cell_xpart(xW);
    const uint32_t ypN = cell_ypart(A.nbx, yN), ypS = cell_ypart(A.nbx, yS);
    auto dest = [&](int q) -> uint32_t {
        return ((AX[q] > 0 ? xpE : (AX[q] < 0 ? xpW : xp)) + (AY[q] > 0 ? ypN : (AY[q] < 0 ? ypS : yp))) * 4u;
    };
    float g[5], lh[9], lg[5], lpp = 0.f;
    if (active) {
#pragma unroll
        for (int q = 0; q < 5; ++q) g[q] = gld<float>(st + q * pb, io);
#pragma unroll
        for (int q = 0; q < 9; ++q) lh[q] = gld<float>(lin + (5 + q) * pb, dest(q));
#pragma unroll
        for (int q = 0; q < 5; ++q) lg[q] = gld<float>(lin + q * pb, dest(q));
        lpp = gld<float>(lin + 14 * pb, io);
    }
    __syncthreads();

    double deps = 0.0;
    if (active) {
        const float phi = (float)s_phi[own];
        const float U = (g[0] + g[1]) + (g[2] + g[3]) + g[4];

        // ---- forward recompute (as the step kernel)
        const double* S = s_phi + own;
        const double gx64 = (1.0 / 3.0) * (S[1] - S[-1]) + (1.0 / 12.0) * ((S[ALX + 1] - S[ALX - 1]) + (S[-ALX + 1] - S[-ALX - 1]));
        const double gy64 = (1.0 / 3.0) * (S[ALX] - S[-ALX]) + (1.0 / 12.0) * ((S[ALX + 1] + S[ALX - 1]) - (S[-ALX + 1] + S[-ALX - 1]));
        const bool on = gx64 * gx64 + gy64 * gy64 > A.grad_eps2;
        const float gx = (float)gx64, gy = (float)gy64;
        float a = 1.f, Cn = 0.f, Sn = 0.f, c = 0.f, iG2 = 0.f;
        if (on) {
            iG2 = __builtin_amdgcn_rcpf(gx * gx + gy * gy);
            const float X = gx * gx * iG2, Y = gy * gy * iG2, XY = gx * gy * iG2;
            if (A.n_fold == 6) {
                Cn = X * X * X - 15.f * X * X * Y + 15.f * X * Y * Y - Y * Y * Y;
                Sn = XY * (6.f * X * X - 20.f * X * Y + 6.f * Y * Y);
            } else {
                Cn = X * X - 6.f * X * Y + Y * Y;
                Sn = XY * 4.f * (X - Y);
            }
            a = 1.f + A.eps * Cn;
            c = A.coefN * A.eps * a * Sn;
        }
        const float Nx = c * gy, Ny = -c * gx;
        const float a2 = a * a, ia2 = __builtin_amdgcn_rcpf(a2), B = ia2 - 1.f;
        const float ie = __builtin_amdgcn_rcpf(3.f * A.Dphi * a2 + 0.5f);
        const float om = 1.f - phi * phi;
        const float Q = phi - phi * phi * phi + A.lam * U * om * om;

        // ---- reverse of the phase-field collision and push
        float ia2b = 0.f, Bb = 0.f, ieb = 0.f, Qb = 0.f, phb = 0.f, Nxb = 0.f, Nyb = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float Pb = lh[q];                                   // lambda_h,q(x + c_q, t + 1)
            const float hold = s_h[q][own + AY[q] * ALX + AX[q]];     // h_q(x + c_q, t)
            const float heq = AW9[q] * (phi - 3.f * (AX[q] * Nx + AY[q] * Ny));
            const float hs = h[q] - (h[q] - heq) * ie + AW9[q] * Q * A.inv_tau0;
            Bb -= Pb * hold;
            ia2b += Pb * hs;
            const float hsb = Pb * ia2;
            ieb += hsb * (heq - h[q]);
            const float heqb = hsb * ie;
            Qb += hsb * AW9[q] * A.inv_tau0;
            phb += AW9[q] * heqb;
            Nxb -= 3.f * AW9[q] * heqb * AX[q];
            Nyb -= 3.f * AW9[q] * heqb * AY[q];
        }
        phb += Qb * (1.f - 3.f * phi * phi - 4.f * A.lam * U * phi * om);
        float Ub = Qb * A.lam * om * om;
        ia2b += Bb;
        const float a2b = -ia2 * ia2 * ia2b + 3.f * A.Dphi * (-ie * ie * ieb);
        float ab = 2.f * a * a2b;
        float Gxb = 0.f, Gyb = 0.f;
        if (on) {
            const float cb = gy * Nxb - gx * Nyb;  // N = c (gy, -gx)
            Gxb += -c * Nyb;
            Gyb += c * Nxb;
            ab += A.coefN * A.eps * Sn * cb;
            const float Sb = A.coefN * A.eps * a * cb;
            deps = (double)(Cn * ab) + (double)(A.coefN * a * Sn * cb);
            const float Cb = A.eps * ab;
            const float m = (float)A.n_fold;
            Gxb += (Cb * m * Sn * gy - Sb * m * Cn * gy) * iG2;
            Gyb += (-Cb * m * Sn * gx + Sb * m * Cn * gx) * iG2;
        }

        // ---- reverse of the vapour collision and push
        const float qd = 0.5f * (1.f - phi);
        const bool inside = qd > 0.f && qd < 1.f;
        const float itg = __builtin_amdgcn_rcpf(0.5f + A.tauv_m_half * fminf(fmaxf(qd, 0.f), 1.f));
        float itgb = 0.f, srcb = 0.f, gsb[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            gsb[q] = lg[q];
            itgb -= gsb[q] * (g[q] - AW5[q] * U);
            Ub += AW5[q] * gsb[q] * itg;
            srcb -= AW5[q] * gsb[q];
        }
        phb += A.half_Lsat * srcb;
        if (inside) phb += -0.5f * A.tauv_m_half * (-itg * itg * itgb);
        phb += lpp;  // phi_prev(t + 1) = phi(t)
#pragma unroll
        for (int q = 0; q < 5; ++q) gst<float>(lout + q * pb, io, gsb[q] * (1.f - itg) + Ub);
        gst<float>(lout + 14 * pb, io, -A.half_Lsat * srcb);
        gst<float>(mid + 0 * pb, io, ia2 * (1.f - ie));
        gst<float>(mid + 1 * pb, io, B);
        gst<float>(mid + 2 * pb, io, Gxb);
        gst<float>(mid + 3 * pb, io, Gyb);
        gst<float>(mid + 4 * pb, io, phb);
    }
    // fixed-order workgroup reduction of the eps contribution
    const double w = wave_sum_d(deps);
    if (tid % 64 == 0) s_red[tid / 64] = w;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < ANT / 64; ++k) t += s_red[k];
        A.epart[blockIdx.x] += t;
    }
}

__global__ void __launch_bounds__(ANT) k_adj_b(AdjDesc A) {
    // B, Gbar_x, Gbar_y of the tile and its ring in LDS (gathered at x - c_q and x - c_k)
    __shared__ float s_B[ALN], s_Gx[ALN], s_Gy[ALN];
    const int tid = threadIdx.x, tx = tid % ATX, ty = tid / ATX;
    const int ntx = (A.nx + ATX - 1) / ATX;
    const int x0 = (blockIdx.x % ntx) * ATX, y0 = (blockIdx.x / ntx) * ATY;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < A.nx && y < A.ny;
    const int own = (ty + 1) * ALX + tx + 1;
    const uint64_t pb = (uint64_t)A.plane * 4;
    const GMEM char* lin = (const GMEM char*)A.lin;
    GMEM char* lout = (GMEM char*)A.lout;
    const GMEM char* mid = (const GMEM char*)A.mid;
    {
        const uint32_t oo = slot_off(A, x0, y0, own);
        s_B[own] = gld<float>(mid + 1 * pb, oo);
        s_Gx[own] = gld<float>(mid + 2 * pb, oo);
        s_Gy[own] = gld<float>(mid + 3 * pb, oo);
    }
    if (tid < ARING) {
        const int r = ring_slot(tid);
        const uint32_t ro = slot_off(A, x0, y0, r);
        s_B[r] = gld<float>(mid + 1 * pb, ro);
        s_Gx[r] = gld<float>(mid + 2 * pb, ro);
        s_Gy[r] = gld<float>(mid + 3 * pb, ro);
    }
    // the cell's own global loads are issued before the barrier too
    const uint32_t xp = cell_xpart(x), yp = cell_ypart(A.nbx, y);
    const uint32_t io = (xp + yp) * 4u;
    const int yN = wrapn(y + 1, A.ny), yS = wrapn(y - 1, A.ny), xE = wrapn(x + 1, A.nx), xW = wrapn(x - 1, A.nx);
    const uint32_t xpE = cell_xpart(xE), xpW = cell_xpart(xW);
    const uint32_t ypN = cell_ypart(A.nbx, yN), ypS = cell_ypart(A.nbx, yS);
    float phb = 0.f, Ah = 0.f, ld[9], lo[9];
    if (active) {
        phb = gld<float>(mid + 4 * pb, io);
        Ah = gld<float>(mid + 0 * pb, io);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const uint32_t dO = ((AX[q] > 0 ? xpE : (AX[q] < 0 ? xpW : xp)) + (AY[q] > 0 ? ypN : (AY[q] < 0 ? ypS : yp))) * 4u;
            ld[q] = gld<float>(lin + (5 + q) * pb, dO);  // lambda_h,q(x + c_q, t + 1)
            lo[q] = gld<float>(lin + (5 + q) * pb, io);  // lambda_h,q(x, t + 1)
        }
    }
    __syncthreads();
    if (!active) return;
#pragma unroll
    for (int k = 1; k < 9; ++k) {  // phi(x) entered G(x - c_k) with weight W_k c_k
        const int j = own - AY[k] * ALX - AX[k];
        const float w = (k < 5) ? (1.f / 3.f) : (1.f / 12.f);
        phb += w * (AX[k] * s_Gx[j] + AY[k] * s_Gy[j]);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const float Bu = s_B[own - AY[q] * ALX - AX[q]];
        gst<float>(lout + (5 + q) * pb, io, ld[q] * Ah - Bu * lo[q] + phb);
    }
}

// lambda_T: dL/dphi_T on every h_q, zero on g and phi_prev
__global__ void __launch_bounds__(256) k_adj_seed(AdjDesc A, const float* __restrict__ dphi) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= A.nx || y >= A.ny) return;
    const int64_t P = A.plane, i = cell_index(A.nbx, x, y);
    const float v = dphi[(int64_t)y * A.nx + x];
#pragma unroll
    for (int q = 0; q < 9; ++q) A.lout[(5 + q) * P + i] = v;
#pragma unroll
    for (int q = 0; q < 5; ++q) A.lout[q * P + i] = 0.f;
    A.lout[14 * P + i] = 0.f;
}

// dL/dU_init(x) = sum_q w_q lambda_g,q(x, 0) (the initial g_q = w_q U_init); per-row FP64 sums
__global__ void __launch_bounds__(256) k_adj_uinit(AdjDesc A, float* __restrict__ dU, double* __restrict__ rows) {
    __shared__ double s_red[4];
    const int y = blockIdx.x, tid = threadIdx.x;
    double acc = 0.0;
    for (int x = tid; x < A.nx; x += 256) {
        const int64_t i = cell_index(A.nbx, x, y);
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < 5; ++q) v += AW5[q] * A.lin[q * A.plane + i];
        dU[(int64_t)y * A.nx + x] = v;
        acc += v;
    }
    const double w = wave_sum_d(acc);
    if (tid % 64 == 0) s_red[tid / 64] = w;
    __syncthreads();
    if (tid == 0) rows[y] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// out[0] = sum of the eps partials, out[1] = sum of the row sums; fixed order
__global__ void __launch_bounds__(64) k_adj_final(const double* __restrict__ epart, int ne,
                                                  const double* __restrict__ rows, int nr, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int k = 0; k < ne; ++k) e += epart[k];
        out[0] = e;
    } else if (threadIdx.x == 1) {
        double u = 0.0;
        for (int k = 0; k < nr; ++k) u += rows[k];
        out[1] = u;
    }
}

int adj_blocks(const AdjDesc& A) { return ((A.nx + ATX - 1) / ATX) * ((A.ny + ATY - 1) / ATY); }

hipError_t launch_adj_seed(const AdjDesc& A, const float* dphi, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_seed, dim3((A.nx + 255) / 256, A.ny), dim3(256), 0, s, A, dphi);
    return hipGetLastError();
}

hipError_t launch_adj_step(const AdjDesc& A, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_a, dim3(adj_blocks(A)), dim3(ANT), 0, s, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_b, dim3(adj_blocks(A)), dim3(ANT), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_adj_finish(const AdjDesc& A, float* dU, double* rows, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_uinit, dim3(A.ny), dim3(256), 0, s, A, dU, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(64), 0, s, A.epart, adj_blocks(A), rows, A.ny, out);
    return hipGetLastError();
}

}  // namespace snowlb
