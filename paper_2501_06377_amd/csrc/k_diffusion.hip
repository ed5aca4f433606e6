// Diffusion kernels: the five-diagonal operator of eq. diffusion_matrix
// (scalar diffusivity per realization, per-row coefficients, periodic phi,
// no flux through the pole faces) and the stages of the super-time-stepping
// schemes of Sec. "Diffusion temporal schemes" (RKG2(3/2), RKL2, or forward
// Euler expressed as stages with mu = 1, nu = 0).
//
// FP64 ("paper form"): Y_j = mu Y_{j-1} + nu Y_{j-2} + cy0 Y0 + cL L(Y_{j-1})
//                            + cLY0 L(Y0), evaluated in that order.
// FP32 mixed ("increment form", algebraically identical because L is linear):
//   d_j = Y_j - Y0 = mu d_{j-1} + nu d_{j-2} + cL L(d_{j-1}) + (cL + cLY0) L(Y0),
//   with Y0 and the result kept in FP64 and L(Y0) formed in FP64 arithmetic;
//   carried as (d, e = d_{j-1} - d_{j-2}), the stage coefficients folded into
//   the operator row (fold_row, sts_fold).
//
// Layout: fields [r][j][k] (k = phi contiguous).  Entries of a launch are the
// realizations still active at stage j (blockIdx.z indexes them).
#include "diff_common.h"
#include "sft_internal.h"

namespace sft {

constexpr int DTX = 64;   // unfused kernels: 64 x 4 threads, one cell each
constexpr int DTY = 4;

// L(y) at (j, k) read from global memory.  Pole rows have a zero up/down
// coefficient; their out-of-sphere neighbour index is clamped to a real row
// and multiplied by that zero.
template <typename T, typename Y>
__device__ __forceinline__ T apply_L(const DiffRow<T>& d, const Y* __restrict__ y, int j, int k,
                                     int nt, int np)
{
    const int km = k == 0 ? np - 1 : k - 1;
    const int kp = k == np - 1 ? 0 : k + 1;
    const int ju = j > 0 ? j - 1 : 0;
    const int jd = j < nt - 1 ? j + 1 : nt - 1;
    const size_t row = (size_t)j * np;
    return L5<T>(d, (T)y[row + km], (T)y[(size_t)ju * np + k], (T)y[row + k],
                 (T)y[(size_t)jd * np + k], (T)y[row + kp]);
}

// ------------------------------------------------------------------ FP64
__global__ __launch_bounds__(256) void diff_first_f64_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs,
    const DiffRow<double>* __restrict__ drow, const double* __restrict__ B,
    double* __restrict__ ly0, double* __restrict__ y1, double* __restrict__ y0copy, int nt, int np)
{
    const Entry e = ents[blockIdx.z];
    const int k = blockIdx.x * DTX + threadIdx.x;
    const int j = blockIdx.y * DTY + threadIdx.y;
    if (k >= np || j >= nt) return;
    const size_t base = (size_t)e.r * nt * np;
    const DiffRow<double> d = drow[(size_t)e.r * nt + j];
    const double L = apply_L<double>(d, B + base, j, k, nt, np);
    const size_t i = base + (size_t)j * np + k;
    const double c1 = coefs[e.coef_off + 1].cL;
    ly0[i] = L;
    y1[i] = B[i] + c1 * L;
    if (y0copy) y0copy[i] = B[i];
}

__global__ __launch_bounds__(256) void diff_stage_f64_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs, int jst,
    const DiffRow<double>* __restrict__ drow, double* B, const double* __restrict__ ym1,
    const double* ym2, const double* __restrict__ ly0, double* out, int nt, int np)
{
    const Entry e = ents[blockIdx.z];
    const int k = blockIdx.x * DTX + threadIdx.x;
    const int j = blockIdx.y * DTY + threadIdx.y;
    if (k >= np || j >= nt) return;
    const size_t base = (size_t)e.r * nt * np;
    const DiffRow<double> d = drow[(size_t)e.r * nt + j];
    const StageCoef c = coefs[e.coef_off + jst];
    const double L = apply_L<double>(d, ym1 + base, j, k, nt, np);
    const size_t i = base + (size_t)j * np + k;
    const double v = sts_f64(c, ym1[i], ym2[i], B[i], L, ly0[i]);
    double* o = (jst == e.s) ? B : out;
    o[i] = v;
}

void launch_diff_first_f64(hipStream_t st, const Entry* ents, int n_ent, const StageCoef* coefs,
                           const DiffRow<double>* drow, const double* B, double* ly0, double* y1,
                           double* y0copy, int nt, int np)
{
    dim3 grid((np + DTX - 1) / DTX, (nt + DTY - 1) / DTY, n_ent);
    hipLaunchKernelGGL(diff_first_f64_kernel, grid, dim3(DTX, DTY), 0, st, ents, coefs, drow, B, ly0,
                       y1, y0copy, nt, np);
}

void launch_diff_stage_f64(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs,
                           int j, const DiffRow<double>* drow, double* B, const double* ym1,
                           const double* ym2, const double* ly0, double* out, int nt, int np)
{
    dim3 grid((np + DTX - 1) / DTX, (nt + DTY - 1) / DTY, n_act);
    hipLaunchKernelGGL(diff_stage_f64_kernel, grid, dim3(DTX, DTY), 0, st, ents, coefs, j, drow, B,
                       ym1, ym2, ly0, out, nt, np);
}

// ------------------------------------------------------------ FP32 mixed
// Entry.pad = 1 when the step's advection increment (held in `adv`) must be
// added to the FP64 state to form Y0.
__global__ __launch_bounds__(256) void diff_first_mixed_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs,
    const DiffRow<double>* __restrict__ drow, const double* __restrict__ B,
    const float* __restrict__ adv, float* __restrict__ ly0, float* __restrict__ d1, int nt, int np)
{
    const Entry e = ents[blockIdx.z];
    const int k = blockIdx.x * DTX + threadIdx.x;
    const int j = blockIdx.y * DTY + threadIdx.y;
    if (k >= np || j >= nt) return;
    const size_t base = (size_t)e.r * nt * np;
    const DiffRow<double> d = drow[(size_t)e.r * nt + j];
    double L;
    if (e.pad) {
        const int km = k == 0 ? np - 1 : k - 1;
        const int kp = k == np - 1 ? 0 : k + 1;
        const int ju = j > 0 ? j - 1 : 0;
        const int jd = j < nt - 1 ? j + 1 : nt - 1;
        const double* b = B + base;
        const float* a = adv + base;
        const size_t row = (size_t)j * np;
        L = d.ph * (b[row + km] + (double)a[row + km]);
        L += d.up * (b[(size_t)ju * np + k] + (double)a[(size_t)ju * np + k]);
        L += d.d * (b[row + k] + (double)a[row + k]);
        L += d.dn * (b[(size_t)jd * np + k] + (double)a[(size_t)jd * np + k]);
        L += d.ph * (b[row + kp] + (double)a[row + kp]);
    } else {
        L = apply_L<double>(d, B + base, j, k, nt, np);
    }
    const size_t i = base + (size_t)j * np + k;
    const float lf = (float)L;
    ly0[i] = lf;
    d1[i] = (float)coefs[e.coef_off + 1].cL * lf;
}

// Reads d_{j-1} (with neighbours) and e_{j-1} (absent at j = 2: e_1 = d_1),
// writes d_j to dout (never din) and e_j over e (each cell reads only its own).
// Pole rows have zero up/down coefficients; their out-of-sphere neighbour is
// read from a real row and multiplied by that zero.
__global__ __launch_bounds__(256) void diff_stage_mixed_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs, int jst,
    const DiffRow<double>* __restrict__ drow, double* __restrict__ B, const float* __restrict__ adv,
    const float* __restrict__ din, const float* ein, const float* __restrict__ ly0, float* dout,
    float* eout, int nt, int np)
{
    const Entry en = ents[blockIdx.z];
    const int k = blockIdx.x * DTX + threadIdx.x;
    const int j = blockIdx.y * DTY + threadIdx.y;
    if (k >= np || j >= nt) return;
    const size_t base = (size_t)en.r * nt * np;
    const StageCoef c = coefs[en.coef_off + jst];
    const float4 f = fold_row(c, drow[(size_t)en.r * nt + j]);
    const float* y = din + base;
    const int km = k == 0 ? np - 1 : k - 1;
    const int kp = k == np - 1 ? 0 : k + 1;
    const int ju = j > 0 ? j - 1 : 0;
    const int jd = j < nt - 1 ? j + 1 : nt - 1;
    const size_t row = (size_t)j * np;
    const size_t i = base + row + k;
    const float dv = y[row + k];
    const float ev = sts_fold(f, (float)(-c.nu), (float)(c.cL + c.cLY0), y[row + km] + y[row + kp],
                              y[(size_t)ju * np + k], dv, y[(size_t)jd * np + k], ein ? ein[i] : dv, ly0[i]);
    const float v = dv + ev;
    if (jst == en.s) {
        double y0 = B[i];
        if (en.pad) y0 += (double)adv[i];
        B[i] = y0 + (double)v;
    } else {
        dout[i] = v;
        eout[i] = ev;
    }
}

void launch_diff_first_mixed(hipStream_t st, const Entry* ents, int n_ent, const StageCoef* coefs,
                             const DiffRow<double>* drow64, const double* B, const float* adv,
                             float* ly0, float* d1, int nt, int np)
{
    dim3 grid((np + DTX - 1) / DTX, (nt + DTY - 1) / DTY, n_ent);
    hipLaunchKernelGGL(diff_first_mixed_kernel, grid, dim3(DTX, DTY), 0, st, ents, coefs, drow64, B,
                       adv, ly0, d1, nt, np);
}

void launch_diff_stage_mixed(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs,
                             int j, const DiffRow<double>* drow, double* B, const float* adv,
                             const float* din, const float* ein, const float* ly0, float* dout,
                             float* eout, int nt, int np)
{
    dim3 grid((np + DTX - 1) / DTX, (nt + DTY - 1) / DTY, n_act);
    hipLaunchKernelGGL(diff_stage_mixed_kernel, grid, dim3(DTX, DTY), 0, st, ents, coefs, j, drow, B,
                       adv, din, ein, ly0, dout, eout, nt, np);
}

// Closes a step in the increment form: B = B (+ adv) (+ d).  Used for
// realizations with flow but no diffusion, and for one-stage diffusion calls.
__global__ void mixed_close_kernel(const Entry* __restrict__ ents, double* __restrict__ B,
                                   const float* __restrict__ adv, const float* __restrict__ d,
                                   size_t cells)
{
    const Entry e = ents[blockIdx.y];
    const size_t base = (size_t)e.r * cells;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
         i += (size_t)gridDim.x * blockDim.x) {
        double y = B[base + i];
        if (e.pad) y += (double)adv[base + i];
        if (d) y += (double)d[base + i];
        B[base + i] = y;
    }
}

void launch_mixed_close(hipStream_t st, const Entry* ents, int n_ent, double* B, const float* adv,
                        const float* d, size_t cells)
{
    int bx = (int)((cells + 255) / 256);
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(mixed_close_kernel, dim3(bx, n_ent), dim3(256), 0, st, ents, B, adv, d, cells);
}

}  // namespace sft
