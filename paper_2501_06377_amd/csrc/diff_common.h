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

// FP32 increment stage: d_j = mu d_{j-1} [+ nu d_{j-2}] + cL L + (cL + cLY0) L(Y0).
__device__ __forceinline__ float sts_mixed(const StageCoef& c, float dm1, float dm2, bool has_dm2,
                                           float L, float ly0)
{
    float v = (float)c.mu * dm1;
    if (has_dm2) v = __builtin_fmaf((float)c.nu, dm2, v);
    v = __builtin_fmaf((float)c.cL, L, v);
    v = __builtin_fmaf((float)(c.cL + c.cLY0), ly0, v);
    return v;
}

}  // namespace sft
