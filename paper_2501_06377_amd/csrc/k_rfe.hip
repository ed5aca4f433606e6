// Random flux emergence (Sec. "Flux emergence"): source maps drawn on the
// device from a counter-based generator, so that map k of a realization is a
// pure function of (seed, realization id, k) and needs no generator state;
// flux balance (eq. fluxbal) with deterministic FP64 sums; and the source
// sub-advance of eq. rfe_s.
//
// Generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  One call gives
// four 32-bit words; two 64-bit words make two uniforms in (0, 1) and the
// Box-Muller transform (Box and Muller 1958) turns them into two standard
// normals, for the two cells of a pair (np is even, so a pair never leaves
// its row).
#include "sft_internal.h"
#include "rfe.h"

namespace sft {

constexpr int GB = 256;      // threads per block
constexpr int GMAXB = 1024;  // generator blocks per realization at most

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ int64_t map_index(const int64_t* kdev, int koff, int64_t kabs)
{
    return kdev ? kdev[0] + koff : kabs;
}

// Fixed-order block sum of two values (result in thread 0).
__device__ __forceinline__ void block_sum2_rfe(double& a, double& b, double* red)
{
    const int t = threadIdx.x;
    red[t] = a;
    red[GB + t] = b;
    __syncthreads();
    for (int s = GB / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[t] += red[t + s];
            red[GB + t] += red[GB + t + s];
        }
        __syncthreads();
    }
    a = red[0];
    b = red[GB];
}

__global__ __launch_bounds__(GB) void rfe_gen_kernel(int nl, int lane, int first_id, uint32_t seed,
                                                     const int64_t* __restrict__ kdev, int koff,
                                                     int64_t kabs, const double* __restrict__ scale_row,
                                                     const double* __restrict__ w_row,
                                                     double* __restrict__ S0, double* __restrict__ S1,
                                                     double* __restrict__ partial, int nt, int np)
{
    __shared__ double red[2 * GB];
    const int r = blockIdx.y;
    if (lane >= 0 && r % nl != lane) return;   // another lane's realization (block-uniform)
    const int64_t k = map_index(kdev, koff, kabs);
    const size_t cells = (size_t)nt * np;
    double* S = ((k & 1) ? S1 : S0) + (size_t)r * cells;
    const uint32_t c1 = (uint32_t)(uint64_t)k, c2 = (uint32_t)((uint64_t)k >> 32);
    const uint32_t key1 = (uint32_t)(first_id + r);
    const size_t npair = cells / 2;
    double pp = 0.0, pm = 0.0;
    for (size_t i = (size_t)blockIdx.x * GB + threadIdx.x; i < npair; i += (size_t)gridDim.x * GB) {
        uint32_t c[4] = {(uint32_t)i, c1, c2, 0u};
        philox4x32_10(c, seed, key1);
        const uint64_t a = ((uint64_t)c[0] << 32) | c[1];
        const uint64_t b = ((uint64_t)c[2] << 32) | c[3];
        const double u1 = ((double)(a >> 11) + 0.5) * 0x1p-53;
        const double u2 = ((double)(b >> 11) + 0.5) * 0x1p-53;
        const double rad = sqrt(-2.0 * log(u1));
        const double t = 2.0 * M_PI * u2;
        const size_t cell = 2 * i;
        const int j = (int)(cell / (size_t)np);
        const double sc = scale_row[j], w = w_row[j];
        double2 v;
        v.x = sc * (rad * cos(t));
        v.y = sc * (rad * sin(t));
        *reinterpret_cast<double2*>(S + cell) = v;
        if (v.x > 0.0) pp += v.x * w;
        else if (v.x < 0.0) pm += v.x * w;
        if (v.y > 0.0) pp += v.y * w;
        else if (v.y < 0.0) pm += v.y * w;
    }
    block_sum2_rfe(pp, pm, red);
    if (threadIdx.x == 0) {
        partial[((size_t)r * gridDim.x + blockIdx.x) * 2 + 0] = pp;
        partial[((size_t)r * gridDim.x + blockIdx.x) * 2 + 1] = pm;
    }
}

__global__ __launch_bounds__(GB) void rfe_reduce_kernel(int nl, int lane, const double* __restrict__ partial,
                                                        int nblk, double* __restrict__ ratio)
{
    __shared__ double red[2 * GB];
    const int r = blockIdx.x;
    if (lane >= 0 && r % nl != lane) return;
    double pp = 0.0, pm = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GB) {
        pp += partial[((size_t)r * nblk + b) * 2 + 0];
        pm += partial[((size_t)r * nblk + b) * 2 + 1];
    }
    block_sum2_rfe(pp, pm, red);
    if (threadIdx.x == 0) ratio[r] = (pp != 0.0 && pm != 0.0) ? sqrt(fabs(pp / pm)) : 0.0;
}

__global__ __launch_bounds__(GB) void rfe_balance_kernel(int nl, int lane, const int64_t* __restrict__ kdev, int koff,
                                                         int64_t kabs, const double* __restrict__ ratio,
                                                         double* __restrict__ S0, double* __restrict__ S1,
                                                         size_t cells)
{
    const int r = blockIdx.y;
    if (lane >= 0 && r % nl != lane) return;
    const double rr = ratio[r];
    if (rr == 0.0) return;
    const int64_t k = map_index(kdev, koff, kabs);
    double* S = ((k & 1) ? S1 : S0) + (size_t)r * cells;
    for (size_t i = (size_t)blockIdx.x * GB + threadIdx.x; i < cells; i += (size_t)gridDim.x * GB) {
        const double s = S[i];
        S[i] = s > 0.0 ? s / rr : s * rr;
    }
}

__global__ void rfe_set_kernel(int64_t* kdev, int64_t k)
{
    if (threadIdx.x == 0) kdev[0] = k;
}

__global__ void rfe_tick_kernel(int64_t* kdev)
{
    if (threadIdx.x == 0) kdev[0] = kdev[0] + 1;
}

__global__ __launch_bounds__(GB) void rfe_apply_kernel(const Entry* __restrict__ ents,
                                                       const double* __restrict__ alpha,
                                                       const int64_t* __restrict__ kdev, int infinite,
                                                       const double* __restrict__ S0,
                                                       const double* __restrict__ S1,
                                                       double* __restrict__ B, size_t cells)
{
    const Entry e = ents[blockIdx.y];
    const size_t base = (size_t)e.r * cells;
    const double h = e.dt;
    double* b = B + base;
    if (infinite) {
        const double* s0 = S0 + base;
        for (size_t i = (size_t)blockIdx.x * GB + threadIdx.x; i < cells; i += (size_t)gridDim.x * GB)
            b[i] = b[i] + h * s0[i];
        return;
    }
    const double a = alpha[e.coef_off];
    const int64_t k = kdev[0];
    const double* sk = ((k & 1) ? S1 : S0) + base;
    const double* sk1 = ((k & 1) ? S0 : S1) + base;
    for (size_t i = (size_t)blockIdx.x * GB + threadIdx.x; i < cells; i += (size_t)gridDim.x * GB)
        b[i] = b[i] + h * ((1.0 - a) * sk[i] + a * sk1[i]);
}

int rfe_gen_blocks(int nt, int np)
{
    const size_t npair = (size_t)nt * np / 2;
    size_t nb = (npair + GB - 1) / GB;
    return (int)(nb < (size_t)GMAXB ? nb : (size_t)GMAXB);
}

void launch_rfe_gen(hipStream_t st, int R, int nl, int lane, int first_id, uint32_t seed,
                    const int64_t* kdev, int koff, int64_t kabs, const double* scale_row,
                    const double* w_row, double* S0, double* S1, double* partial, double* ratio, int nt,
                    int np)
{
    const int nblk = rfe_gen_blocks(nt, np);
    hipLaunchKernelGGL(rfe_gen_kernel, dim3(nblk, R), dim3(GB), 0, st, nl, lane, first_id, seed, kdev, koff,
                       kabs, scale_row, w_row, S0, S1, partial, nt, np);
    hipLaunchKernelGGL(rfe_reduce_kernel, dim3(R), dim3(GB), 0, st, nl, lane, partial, nblk, ratio);
}

static int grid_for(size_t cells)
{
    size_t nb = (cells + GB - 1) / GB;
    return (int)(nb < 2048 ? nb : 2048);
}

void launch_rfe_balance(hipStream_t st, int R, int nl, int lane, const int64_t* kdev, int koff,
                        int64_t kabs, const double* ratio, double* S0, double* S1, int nt, int np)
{
    const size_t cells = (size_t)nt * np;
    hipLaunchKernelGGL(rfe_balance_kernel, dim3(grid_for(cells), R), dim3(GB), 0, st, nl, lane, kdev, koff,
                       kabs, ratio, S0, S1, cells);
}

void launch_rfe_set(hipStream_t st, int64_t* kdev, int64_t k)
{
    hipLaunchKernelGGL(rfe_set_kernel, dim3(1), dim3(64), 0, st, kdev, k);
}

void launch_rfe_tick(hipStream_t st, int64_t* kdev)
{
    hipLaunchKernelGGL(rfe_tick_kernel, dim3(1), dim3(64), 0, st, kdev);
}

void launch_rfe_apply(hipStream_t st, const Entry* ents, int n_ent, const double* alpha,
                      const int64_t* kdev, int infinite, const double* S0, const double* S1, double* B,
                      size_t cells)
{
    hipLaunchKernelGGL(rfe_apply_kernel, dim3(grid_for(cells), n_ent), dim3(GB), 0, st, ents, alpha, kdev,
                       infinite, S0, S1, B, cells);
}

}  // namespace sft
