// snowlb_device.h -- device helpers shared by the step kernel and the set-up / read-out kernels of
// libsnowlb: lattice constants, the storage formats of the populations and small index helpers.
//
// 16-bit storage keeps each population as a deviation d = p / w - m from a local reference m
// (collision arithmetic stays FP32):
//   h   : m = phi(t-1) of the cell that holds the population (its phi_prev; the writer knows it from
//         the LDS phi of the destination, the reader from its phi_prev plane);
//   g_q : m = U (1 + 3 c_q . j) of the cell the population streamed from (U without flow);
//   f_q : m = rho + 3 c_q . j of the cell the population streamed from (its first-order equilibrium,
//         so the velocity term leaves the deviation).
// The source cell stores its U, rho, jx, jy rounded to the 16-bit format in reference planes; writer
// and reader use exactly those rounded values (the reader stages them with the halo), so any
// rounding of the references cancels.  The deviations are then small (time changes and
// non-equilibrium parts), and so is the 16-bit rounding error in absolute terms.  phi_prev and the
// reference planes come in two copies, because neighbours read them.
#pragma once
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
// storage policies: FP32 values, or 16-bit deviations d = p / w - m (see the comment at the top of this file)
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

// c . v for a lattice velocity with components in {-1, 0, 1}, known at compile time once the
// population loop is unrolled: zero components cost no instruction (a product with 0.f would have
// to be kept for IEEE semantics).  The value is that of cx vx + cy vy up to the sign of a zero.
__device__ __forceinline__ float cdot(int cx, int cy, float vx, float vy) {
    if (cx == 0) return cy == 0 ? 0.f : (cy > 0 ? vy : -vy);
    const float a = cx > 0 ? vx : -vx;
    if (cy == 0) return a;
    return cy > 0 ? a + vy : a - vy;
}

// Reference of a 16-bit f_q: rho + 3 c_q . j of its source, with one explicit fused rounding so
// that the writer and every reader produce the same bits.
__device__ __forceinline__ float f_ref(float rho, float jx, float jy, int cx, int cy) {
    if (cx == 0 && cy == 0) return rho;
    return __builtin_fmaf(3.f, cdot(cx, cy, jx, jy), rho);
}

// Reference of a 16-bit g_q: U (1 + 3 c_q . j) of its source (its first-order equilibrium with the
// momentum j standing in for the velocity), with one explicit fused rounding so that the writer and
// every reader produce the same bits.  A U reference of 0 gives 0 whatever j holds.
__device__ __forceinline__ float g_ref(float U, float jx, float jy, int cx, int cy) {
    if (cx == 0 && cy == 0) return U;
    return __builtin_fmaf(3.f * U, cdot(cx, cy, jx, jy), U);
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

}  // namespace snowlb
