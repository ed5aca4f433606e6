// Per-cell arithmetic of the diffusion stages, shared by the unfused and the
// fused (temporally blocked) kernels so that both perform identical
// floating-point operations in the same order.
#pragma once

#include "sft_internal.h"

namespace sft {

// The five-diagonal operator at one cell from its neighbours, summed in the
// table's order k-1, j-1, centre, j+1, k+1 with fused multiply-adds.  Every
// diffusion kernel uses these helpers, so the fused and unfused paths perform
// identical arithmetic (the CPU reference evaluates the same sums without
// fusion: the two differ by rounding only).
template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c);
template <>
__device__ __forceinline__ double fmad<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fmad<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ T L5(const DiffRow<T>& d, T w, T n, T c, T s, T e)
{
    T v = d.ph * w;
    v = fmad<T>(d.up, n, v);
    v = fmad<T>(d.d, c, v);
    v = fmad<T>(d.dn, s, v);
    v = fmad<T>(d.ph, e, v);
    return v;
}

// FP64 stage: Y_j = nu Y_{j-2} + mu Y_{j-1} + cy0 Y0 + cL L + cLY0 L(Y0)
// (the Y_{j-2} term first: its register, dead afterwards, takes the result).
__device__ __forceinline__ double sts_f64(const StageCoef& c, double ym1, double ym2, double y0,
                                          double L, double ly0)
{
    double v = c.nu * ym2;
    v = __builtin_fma(c.mu, ym1, v);
    v = __builtin_fma(c.cy0, y0, v);
    v = __builtin_fma(c.cL, L, v);
    v = __builtin_fma(c.cLY0, ly0, v);
    return v;
}

// FP32 increment stage, carried as the increment d and its last change
// e = d_{j-1} - d_{j-2} (e = d_1 at the first blocked stage, d_0 being 0):
//   e_j = (mu + nu - 1) d_{j-1} - nu e_{j-1} + cL L(d_{j-1}) + (cL + cLY0) L(Y0),
//   d_j = d_{j-1} + e_j,
// the three-term recurrence d_j = mu d_{j-1} + nu d_{j-2} + ... rewritten.
// With mu -> 2 and nu -> -1 over a long call that recurrence has a double
// root at 1: a rounding error of d in its own form grows linearly over the
// remaining stages (s^2 eps in all), while here the rounding of d enters the
// non-growing mode and the rounding of e, a change of size d / s, is the one
// that grows (about s eps in all).  mu + nu - 1 = -cy0.
//
// The stage coefficient cL and the diagonal term -cy0 are folded into the
// operator row once per row and stage, in FP64 and rounded to FP32:
//   A = cL ph, U = cL up, C = cL dd - cy0, S = cL dn,
// so that with t = d(k-1) + d(k+1) (the two phi neighbours share ph)
//   e_j = A t + U d(j-1) + C d + S d(j+1) - nu e_{j-1} + (cL + cLY0) L(Y0).
__device__ __forceinline__ float4 fold_row(const StageCoef& c, const DiffRow<double>& d)
{
    return make_float4((float)(c.cL * d.ph), (float)(c.cL * d.up), (float)(c.cL * d.d - c.cy0),
                       (float)(c.cL * d.dn));
}

// e_j of one cell: f the folded row, nnu = (float)(-nu), g = (float)(cL + cLY0).
__device__ __forceinline__ float sts_fold(const float4& f, float nnu, float g, float t, float n, float c,
                                          float s, float e, float ly)
{
    float v = f.x * t;
    v = __builtin_fmaf(f.y, n, v);
    v = __builtin_fmaf(f.z, c, v);
    v = __builtin_fmaf(f.w, s, v);
    v = __builtin_fmaf(nnu, e, v);
    v = __builtin_fmaf(g, ly, v);
    return v;
}

}  // namespace sft
