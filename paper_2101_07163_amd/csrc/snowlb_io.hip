// snowlb_io.hip -- set-up and read-out kernels of libsnowlb (Tan et al., arXiv:2101.07163): the
// initial state, macroscopic field read-out and overwrite, population exchange with a canonical FP32
// layout, FP64 diagnostics and a plain copy that measures the practical HBM ceiling.  None of them is
// on the per-step path; they favour plain per-cell code over speed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include "snowlb_device.h"
#include "snowlb_internal.h"

namespace snowlb {

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
        if (q < 5) g[q] = S::dec(plane_ptr<S>(d, par, d.off_g + q)[i], W5[q], g_ref(r[R_U], r[R_JX], r[R_JY], CX[q], CY[q]));
        f[q] = flow ? f_abs_dec<S>(plane_ptr<S>(d, par, q)[i], q, f_ref(r[R_RHO], r[R_JX], r[R_JY], CX[q], CY[q]))
                    : 0.f;
    }
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
        if (q < 5) plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(gq[q], IW5[q], g_ref(r[R_U], r[R_JX], r[R_JY], CX[q], CY[q]));
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
        plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(gq[q], IW5[q], g_ref(r[R_U], r[R_JX], r[R_JY], CX[q], CY[q]));
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
                plane_ptr_w<S>(d, par, d.off_g + q)[i] = S::enc(canon[q * n + c], IW5[q], g_ref(r[R_U], r[R_JX], r[R_JY], CX[q], CY[q]));
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
    if (b > kDiagMaxBlocks) b = kDiagMaxBlocks;  // larger lattices loop over more cells per thread
    return (int)(b < 1 ? 1 : b);
}

// Scratch of the allocation-free diagnostics (snowlb_diag_noalloc): the per-workgroup partials, at
// most kDiagMaxBlocks x 8 doubles (128 KiB), in a file-scope device array.  Each GPU the library
// runs on holds its own copy until the process ends; host code never passes the array's name to a
// kernel (on the host it is only a stand-in), but the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device and kept.
static __device__ __align__(256) double scratch[kDiagMaxBlocks * 8];

hipError_t diag_scratch(double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = p;
    }
    *out = static_cast<double*>(ptr[dev]);
    return hipSuccess;
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

__global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ partials, int nblk, double half_Lsat,
                                                    double* __restrict__ out) {
    // 32 lanes per quantity: lane l of quantity k sums blocks l, l + 32, ... in order, then lane 0
    // adds the 32 lane sums in order.  Fixed order, hence deterministic.  Then the species invariant
    // sum U + (L_sat/2) sum phi_prev (the vapour the depletion source of Sec. 2.2.2 removes is
    // (L_sat/2) times the phase gained).
    __shared__ double s[8][32];
    __shared__ double tot[8];
    const int k = threadIdx.x / 32, l = threadIdx.x % 32;
    double v = 0;
    for (int b = l; b < nblk; b += 32) v += partials[(int64_t)b * 8 + k];
    s[k][l] = v;
    __syncthreads();
    if (l == 0) {
        double t = 0;
        for (int i = 0; i < 32; ++i) t += s[k][i];
        out[k] = t;
        tot[k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) out[8] = __dadd_rn(tot[3], __dmul_rn(half_Lsat, tot[5]));
}

template <class S>
static hipError_t diag_s(const DomDesc& d, int par, double* partials, double* out, double half_Lsat, hipStream_t s) {
    const int nb = diag_blocks(d);
    hipLaunchKernelGGL(k_diag<S>, dim3(nb), dim3(kDiagThreads), 0, s, d, par, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, partials, nb, half_Lsat, out);
    return hipGetLastError();
}

hipError_t launch_diag(const DomDesc& d, int par, double* partials, double* out, double half_Lsat, hipStream_t s) {
    switch (d.storage) {
        case 0: return diag_s<StoreF32>(d, par, partials, out, half_Lsat, s);
        case 1: return diag_s<StoreF16>(d, par, partials, out, half_Lsat, s);
        case 2: return diag_s<StoreBF16>(d, par, partials, out, half_Lsat, s);
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
