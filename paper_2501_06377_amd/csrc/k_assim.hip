// Data assimilation (eq. data_assim, eq. data_assim_f, eqs. data_assim_deltab
// and fluxbal) and the FP64 analysis reductions of Sec. "Analysis".
//
// Reductions are deterministic: every block reduces a fixed, strided set of
// cells in a fixed tree order into a partial record, and one block per
// realization then reduces the partials in a fixed order.  No float atomics.
#include <algorithm>

#include "sft_internal.h"

namespace sft {

constexpr int RB = 256;   // threads per reduction block

__device__ __forceinline__ double load_any(const void* p, int dtype, size_t i)
{
    return dtype == 1 ? (double)((const float*)p)[i] : ((const double*)p)[i];
}

// F from the disk-centre cosine m of row j (eq. data_assim_f).
__device__ __forceinline__ double weight_of_mu(const AssimReal& a, double m, int j, const double* lat_row)
{
    double f = 0.0;
    if (m > a.mu_lim && fabs(lat_row[j]) < a.lat_lim_rad) {
        if (a.alpha == 4.0) {
            const double m2 = m * m;
            f = m2 * m2;
        } else {
            f = pow(m, a.alpha);
        }
    }
    return f;
}

// Weight F at cell (j, k) for realization parameters a (eq. data_assim_f).
__device__ __forceinline__ double weight_at(const AssimReal& a, const void* weight, int dtype,
                                            int kind, double sb0, double cb0, double l0, size_t i,
                                            int j, int k, int np, const double* st_row,
                                            const double* ct_row, const double* lat_row)
{
    if (kind == 0) return load_any(weight, dtype, i);
    double m;
    if (kind == 1) {
        m = load_any(weight, dtype, i);
    } else {
        const double dph = 2.0 * M_PI / np;
        const double ph = (k + 0.5) * dph;
        m = sb0 * ct_row[j] + cb0 * st_row[j] * cos(ph - l0);
    }
    return weight_of_mu(a, m, j, lat_row);
}

// Block-wide fixed-order sum of two values into red[0], red[1].
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red)
{
    const int t = threadIdx.x;
    red[t] = a;
    red[RB + t] = b;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[t] += red[t + s];
            red[RB + t] += red[RB + t + s];
        }
        __syncthreads();
    }
    a = red[0];
    b = red[RB];
}

// dB = F (data - B) for every realization of the class (stored when dB is
// not NULL); per-block FP64 sums of dB w over dB > 0 and dB < 0.
__global__ __launch_bounds__(RB) void assim_delta_kernel(
    const AssimReal* __restrict__ ar, const void* data, const void* weight, int dtype, int kind,
    double sb0, double cb0, double l0, const double* __restrict__ B, const double* st_row,
    const double* ct_row, const double* lat_row, const double* w_row, double* __restrict__ dB,
    double* __restrict__ partial, int nt, int np)
{
    __shared__ double red[2 * RB];
    const int r = blockIdx.y;
    const AssimReal a = ar[r];
    const size_t cells = (size_t)nt * np;
    const size_t base = (size_t)r * cells;
    double pp = 0.0, pm = 0.0;
    for (size_t i = (size_t)blockIdx.x * RB + threadIdx.x; i < cells; i += (size_t)gridDim.x * RB) {
        const int j = (int)(i / np), k = (int)(i - (size_t)j * np);
        const double F = weight_at(a, weight, dtype, kind, sb0, cb0, l0, i, j, k, np, st_row, ct_row,
                                   lat_row);
        const double d = F * (load_any(data, dtype, i) - B[base + i]);
        if (dB) dB[base + i] = d;
        if (d > 0.0) pp += d * w_row[j];
        else if (d < 0.0) pm += d * w_row[j];
    }
    block_sum2(pp, pm, red);
    if (threadIdx.x == 0) {
        partial[((size_t)r * gridDim.x + blockIdx.x) * 2 + 0] = pp;
        partial[((size_t)r * gridDim.x + blockIdx.x) * 2 + 1] = pm;
    }
}

// ratio[r] = sqrt|Phi+/Phi-| (0 when either sum is zero: no balancing).
__global__ __launch_bounds__(RB) void assim_reduce_kernel(const double* __restrict__ partial,
                                                          int nblk, double* __restrict__ ratio)
{
    __shared__ double red[2 * RB];
    const int r = blockIdx.x;
    double pp = 0.0, pm = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RB) {
        pp += partial[((size_t)r * nblk + b) * 2 + 0];
        pm += partial[((size_t)r * nblk + b) * 2 + 1];
    }
    block_sum2(pp, pm, red);
    if (threadIdx.x == 0) ratio[r] = (pp != 0.0 && pm != 0.0) ? sqrt(fabs(pp / pm)) : 0.0;
}

// Balanced realizations: B += dB / r (dB > 0) or dB * r (dB <= 0), with dB
// read back or, when dB is NULL, formed again exactly as the delta pass
// formed it.  Others: B = F data + (1 - F) B.  A thread owns one column k
// over a group of rows (block x = column chunk + RB-wide chunk count x row
// group), so the disk weight's cos(phi_k - L0) is formed once per column
// and group; every cell's F is the value weight_at gives.
__global__ __launch_bounds__(RB) void assim_apply_kernel(
    const AssimReal* __restrict__ ar, const void* data, const void* weight, int dtype, int kind,
    double sb0, double cb0, double l0, double* __restrict__ B, const double* __restrict__ dB,
    const double* __restrict__ ratio, const double* st_row, const double* ct_row,
    const double* lat_row, int nt, int np)
{
    const int r = blockIdx.y;
    const AssimReal a = ar[r];
    const size_t base = (size_t)r * nt * np;
    const int ncx = (np + RB - 1) / RB, nry = gridDim.x / ncx;
    const int ry = blockIdx.x / ncx, k = (blockIdx.x - ry * ncx) * RB + threadIdx.x;
    if (k >= np || ry >= nry) return;
    const int j0 = (int)((long)nt * ry / nry), j1 = (int)((long)nt * (ry + 1) / nry);
    double cph = 0.0;
    if (kind == 2) {
        const double dph = 2.0 * M_PI / np;
        const double ph = (k + 0.5) * dph;
        cph = cos(ph - l0);
    }
    const double rr = a.balance ? ratio[r] : 0.0;
    for (int j = j0; j < j1; ++j) {
        const size_t i = (size_t)j * np + k;
        double F;
        if (kind == 0) F = load_any(weight, dtype, i);
        else if (kind == 1) F = weight_of_mu(a, load_any(weight, dtype, i), j, lat_row);
        else F = weight_of_mu(a, sb0 * ct_row[j] + cb0 * st_row[j] * cph, j, lat_row);
        if (a.balance) {
            double d = dB ? dB[base + i] : F * (load_any(data, dtype, i) - B[base + i]);
            if (rr != 0.0) d = d > 0.0 ? d / rr : d * rr;
            B[base + i] = B[base + i] + d;
        } else {
            B[base + i] = F * load_any(data, dtype, i) + (1.0 - F) * B[base + i];
        }
    }
}

void launch_assim_delta(hipStream_t st, int R, const AssimReal* ar, const void* data,
                        const void* weight, int dtype, int kind, double sb0, double cb0, double l0,
                        const double* B, const double* st_row, const double* ct_row,
                        const double* lat_row, const double* w_row, double* dB, double* partial,
                        int nblk, int nt, int np)
{
    hipLaunchKernelGGL(assim_delta_kernel, dim3(nblk, R), dim3(RB), 0, st, ar, data, weight, dtype,
                       kind, sb0, cb0, l0, B, st_row, ct_row, lat_row, w_row, dB, partial, nt, np);
}

void launch_assim_reduce(hipStream_t st, int R, const double* partial, int nblk, double* ratio)
{
    hipLaunchKernelGGL(assim_reduce_kernel, dim3(R), dim3(RB), 0, st, partial, nblk, ratio);
}

void launch_assim_apply(hipStream_t st, int R, const AssimReal* ar, const void* data,
                        const void* weight, int dtype, int kind, double sb0, double cb0, double l0,
                        double* B, const double* dB, const double* ratio, const double* st_row,
                        const double* ct_row, const double* lat_row, int nblk, int nt, int np)
{
    // column chunks x row groups, about 2048 blocks over the class
    (void)nblk;
    const int ncx = (np + RB - 1) / RB;
    int nry = (int)std::min<long>(nt, std::max<long>(1, 2048 / ((long)ncx * R)));
    hipLaunchKernelGGL(assim_apply_kernel, dim3(ncx * nry, R), dim3(RB), 0, st, ar, data, weight, dtype,
                       kind, sb0, cb0, l0, B, dB, ratio, st_row, ct_row, lat_row, nt, np);
}

// ------------------------------------------------------------ diagnostics
__device__ __forceinline__ DiagRec diag_zero()
{
    DiagRec d;
    d.pp = d.pm = d.h1 = d.h2 = d.dax = 0.0;
    d.bmin = INFINITY;
    d.bmax = -INFINITY;
    d.babs = INFINITY;
    d.nonfinite = 0.0;
    d.pad = 0.0;
    return d;
}

__device__ __forceinline__ void diag_merge(DiagRec& a, const DiagRec& b)
{
    a.pp += b.pp;
    a.pm += b.pm;
    a.h1 += b.h1;
    a.h2 += b.h2;
    a.dax += b.dax;
    a.bmin = fmin(a.bmin, b.bmin);
    a.bmax = fmax(a.bmax, b.bmax);
    a.babs = fmin(a.babs, b.babs);
    a.nonfinite += b.nonfinite;
}

__device__ void block_merge(DiagRec& v, DiagRec* red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (t < s) diag_merge(red[t], red[t + s]);
        __syncthreads();
    }
    v = red[0];
}

// Wave-wide fixed-order merge (butterfly over the 64 lanes); every lane ends
// with the wave's record.
__device__ __forceinline__ void wave_merge(DiagRec& v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        DiagRec o;
        o.pp = __shfl_xor(v.pp, m);
        o.pm = __shfl_xor(v.pm, m);
        o.h1 = __shfl_xor(v.h1, m);
        o.h2 = __shfl_xor(v.h2, m);
        o.dax = __shfl_xor(v.dax, m);
        o.bmin = __shfl_xor(v.bmin, m);
        o.bmax = __shfl_xor(v.bmax, m);
        o.babs = __shfl_xor(v.babs, m);
        o.nonfinite = __shfl_xor(v.nonfinite, m);
        diag_merge(v, o);
    }
}

// A block owns the rows j = blockIdx.x, blockIdx.x + gridDim.x, ... of one
// realization, its threads the columns k = threadIdx.x + n RB of each row:
// row factors are block-uniform, no index division per cell, and the block's
// record is merged across lanes, then across its four waves.
__global__ __launch_bounds__(RB) void diag_partial_kernel(
    const double* __restrict__ B, const double* st_row, const double* ct_row, const double* w_row,
    const double* sph, const double* cph, DiagRec* __restrict__ partial, int nt, int np)
{
    __shared__ DiagRec red[RB / 64];
    const int r = blockIdx.y;
    const double* b = B + (size_t)r * nt * np;
    DiagRec v = diag_zero();
    for (int j = blockIdx.x; j < nt; j += gridDim.x) {
        const double w = w_row[j], sw = st_row[j] * w, cw = ct_row[j] * w;
        const double* bj = b + (size_t)j * np;
        // four columns per thread and pass: their loads are issued together
        for (int k0 = threadIdx.x; k0 < np; k0 += 4 * RB) {
            double xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + q * RB;
                xs[q] = k < np ? bj[k] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + q * RB;
                if (k >= np) break;
                const double x = xs[q];
                if (!isfinite(x)) {
                    v.nonfinite += 1.0;
                    continue;
                }
                if (x > 0.0) v.pp += x * w;
                else if (x < 0.0) v.pm += x * w;
                v.h1 += x * sw * cph[k];
                v.h2 += x * sw * sph[k];
                v.dax += x * cw;
                v.bmin = fmin(v.bmin, x);
                v.bmax = fmax(v.bmax, x);
                v.babs = fmin(v.babs, fabs(x));
            }
        }
    }
    wave_merge(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < RB / 64; ++q) diag_merge(v, red[q]);
        partial[(size_t)r * gridDim.x + blockIdx.x] = v;
    }
}

__global__ __launch_bounds__(RB) void diag_final_kernel(const DiagRec* __restrict__ partial, int nblk,
                                                        DiagRec* __restrict__ out)
{
    __shared__ DiagRec red[RB];
    const int r = blockIdx.x;
    DiagRec v = diag_zero();
    for (int b = threadIdx.x; b < nblk; b += RB) diag_merge(v, partial[(size_t)r * nblk + b]);
    block_merge(v, red);
    if (threadIdx.x == 0) {
        const double c = 3.0 / (4.0 * M_PI);
        v.h1 *= c;
        v.h2 *= c;
        v.dax *= c;
        out[r] = v;
    }
}

void launch_diag(hipStream_t st, int R, const double* B, const double* st_row, const double* ct_row,
                 const double* w_row, const double* sph, const double* cph, DiagRec* partial,
                 int nblk, DiagRec* out, int nt, int np)
{
    // row blocks per realization: enough blocks to fill the chip, at most
    // one per row and at most the partial buffer's nblk
    int nb = 1024 / (R > 0 ? R : 1);
    if (nb < 64) nb = 64;
    if (nb > nt) nb = nt;
    if (nb > nblk) nb = nblk;
    hipLaunchKernelGGL(diag_partial_kernel, dim3(nb, R), dim3(RB), 0, st, B, st_row, ct_row, w_row,
                       sph, cph, partial, nt, np);
    hipLaunchKernelGGL(diag_final_kernel, dim3(R), dim3(RB), 0, st, partial, nb, out);
}

// ------------------------------------------------------------ conversions
__global__ void f32_to_f64_kernel(const float* __restrict__ s, double* __restrict__ d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        d[i] = (double)s[i];
}

__global__ void f64_to_f32_kernel(const double* __restrict__ s, float* __restrict__ d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

void launch_f32_to_f64(hipStream_t st, const float* src, double* dst, size_t n)
{
    int b = (int)((n + 255) / 256);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(b), dim3(256), 0, st, src, dst, n);
}

void launch_f64_to_f32(hipStream_t st, const double* src, float* dst, size_t n)
{
    int b = (int)((n + 255) / 256);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(b), dim3(256), 0, st, src, dst, n);
}

}  // namespace sft
