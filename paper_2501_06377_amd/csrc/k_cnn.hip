// CNN surrogate kernels: a five-layer 3x3 convolutional network on the
// sphere (periodic longitude, across-pole colatitude padding), BF16 operands
// with FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16), FP32 master weights and Adam.
//
// Activations are NHWC bfloat16: act[b][j][k][c], c contiguous.
// MFMA 32x32x16 operand layout (per lane l of a 64-lane wave):
//   A (32 x 16): row l%32, columns 8*(l/32) .. +7   (8 bf16 per lane)
//   B (16 x 32): rows 8*(l/32) .. +7, column l%32
//   C (32 x 32): register r holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
// Convolutions are implicit GEMMs: M = 32 output pixels of a tile row,
// N = 32 output channels, K = 16 input channels of one tap.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sft_internal.h"

namespace sft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ int wrapk(int k, int W)
{
    k %= W;
    return k < 0 ? k + W : k;
}

// Source pixel of padded coordinate (j, k), j in [-1, H]: ghost rows reflect
// across the pole with a half-turn in longitude.  Returns false outside.
__device__ __forceinline__ bool sphere_src(int j, int k, int H, int W, int& sj, int& sk)
{
    k = wrapk(k, W);
    if (j >= 0 && j < H) {
        sj = j;
        sk = k;
        return true;
    }
    if (j == -1) {
        sj = 0;
        sk = (k + W / 2) % W;
        return true;
    }
    if (j == H) {
        sj = H - 1;
        sk = (k + W / 2) % W;
        return true;
    }
    return false;
}

// ------------------------------------------------------------ input features
// X0[b][j][k][0..15]: the field f = B/500 as a pair of bf16 values (hi =
// bf16(f), lo = bf16(f - hi): 16 significant bits, so that a 1-hour increment
// of ~1% of B is resolved), three per-sample features, cos(theta),
// sin(theta), zeros.  The first layer applies the field channel's weight to
// both hi and lo.
template <typename TB>
__global__ void cnn_features_kernel(const TB* __restrict__ Bin, const float* __restrict__ feats,
                                    uint16_t* __restrict__ X0, int H, int W)
{
    const int b = blockIdx.y;
    const size_t n = (size_t)H * W;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(p / W);
        const double th = (j + 0.5) * (M_PI / H);
        const float f = (float)((double)Bin[(size_t)b * n + p] / 500.0);
        const uint16_t hi = f2bf(f);
        float v[16];
        v[0] = bf2f(hi);
        v[1] = f - bf2f(hi);
        v[2] = feats[b * 3 + 0];
        v[3] = feats[b * 3 + 1];
        v[4] = feats[b * 3 + 2];
        v[5] = (float)cos(th);
        v[6] = (float)sin(th);
        for (int c = 7; c < 16; ++c) v[c] = 0.f;
        uint16_t* o = X0 + ((size_t)b * n + p) * 16;
        for (int c = 0; c < 16; ++c) o[c] = f2bf(v[c]);
    }
}

// ------------------------------------------------------ MFMA convolution
// MODE 0 (forward):  out[b][j][k][co] = relu(bias[co] + sum_tap sum_ci
//                    w[tap][co][ci] x[b][pad(j+dy-1, k+dx-1)][ci]), bf16 out.
// MODE 1 (dgrad):    out[b][q+1][k][ci] = sum_tap sum_co w[tap][ci][co]
//                    g[b][q-dy+1][k-dx+1][co] for padded rows q in [-1, H]
//                    (g zero outside [0, H)), FP32 out, H+2 rows.
// Weight layout: w[tap][n][k] with the K index (input of the GEMM) contiguous.
constexpr int CTY = 8, CTX = 32;      // output tile: 8 rows x 32 columns, 2 waves

template <int CIN, int MODE>
__global__ __launch_bounds__(128) void conv_mfma_kernel(const uint16_t* __restrict__ x,
                                                        const uint16_t* __restrict__ w,
                                                        const float* __restrict__ bias,
                                                        void* __restrict__ out, int H, int W)
{
    constexpr int CP = CIN + 8;                 // padded channel stride in LDS
    constexpr int TR = CTY + 2, TC = CTX + 2;   // staged tile with a one-cell halo
    constexpr int NCH = CIN / 16;               // K chunks per tap
    __shared__ __attribute__((aligned(16))) uint16_t tile[TR * TC * CP];

    const int b = blockIdx.z;
    const int k0 = blockIdx.x * CTX;
    const int r0 = (MODE == 0 ? 0 : -1) + blockIdx.y * CTY;   // first output row of the tile
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t plane = (size_t)H * W;
    const uint16_t* xb = x + (size_t)b * plane * CIN;

    // stage rows r0-1 .. r0+CTY, columns k0-1 .. k0+CTX (16-byte chunks)
    constexpr int VPP = CIN / 8;                 // 16-byte vectors per pixel
    for (int v = tid; v < TR * TC * VPP; v += 128) {
        const int pix = v / VPP, cv = v - (v / VPP) * VPP;
        const int tr = pix / TC, tc = pix - (pix / TC) * TC;
        const int j = r0 - 1 + tr, k = k0 - 1 + tc;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (MODE == 0) {
            int sj, sk;
            if (sphere_src(j, k, H, W, sj, sk))
                val = *(const uint4*)(xb + ((size_t)sj * W + sk) * CIN + cv * 8);
        } else {
            if (j >= 0 && j < H) val = *(const uint4*)(xb + ((size_t)j * W + wrapk(k, W)) * CIN + cv * 8);
        }
        *(uint4*)(tile + (tr * TC + tc) * CP + cv * 8) = val;
    }
    __syncthreads();

    f32x16 acc[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.f;

    const int col = lane & 31, kh = lane >> 5;
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap - (tap / 3) * 3;
        const int oy = MODE == 0 ? dy : 2 - dy, ox = MODE == 0 ? dx : 2 - dx;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int kb = ch * 16 + kh * 8;
            bf16x8 bfr[2];
#pragma unroll
            for (int n = 0; n < 2; ++n)
                bfr[n] = *(const bf16x8*)(w + ((size_t)tap * 64 + n * 32 + col) * CIN + kb);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int tr = wv * 4 + m + oy;
                const bf16x8 a = *(const bf16x8*)(tile + (tr * TC + col + ox) * CP + kb);
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bfr[n], acc[m][n], 0, 0, 0);
            }
        }
    }

    // epilogue: C row = pixel column within the tile row, C column = channel
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = r0 + wv * 4 + m;
        const int rlim = MODE == 0 ? H : H + 1;
        if (row > rlim - 1 || row < (MODE == 0 ? 0 : -1)) continue;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int c = n * 32 + col;
            const float bv = MODE == 0 ? bias[c] : 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int px = 8 * (r >> 2) + 4 * kh + (r & 3);
                const int k = k0 + px;
                if (k >= W) continue;
                if (MODE == 0) {
                    float v = acc[m][n][r] + bv;
                    v = v > 0.f ? v : 0.f;
                    ((uint16_t*)out)[((size_t)b * plane + (size_t)row * W + k) * 64 + c] = f2bf(v);
                } else {
                    ((float*)out)[((size_t)b * (H + 2) * W + (size_t)(row + 1) * W + k) * 64 + c] =
                        acc[m][n][r];
                }
            }
        }
    }
}

// dZ[b][j][k][c] = (dXp[j+1] + ghost fold) * (act[b][j][k][c] > 0), bf16.
// The ghost row above row 0 (padded row 0) read row 0 at column k + W/2, so
// its gradient folds back there; likewise the ghost row below the last row.
__global__ void fold_mask_kernel(const float* __restrict__ dxp, const uint16_t* __restrict__ act,
                                 uint16_t* __restrict__ dz, int H, int W)
{
    const int b = blockIdx.y;
    const size_t n = (size_t)H * W * 64;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(e & 63);
        const size_t p = e >> 6;
        const int j = (int)(p / W), k = (int)(p - (size_t)j * W);
        const float* g = dxp + (size_t)b * (H + 2) * W * 64;
        float v = g[((size_t)(j + 1) * W + k) * 64 + c];
        const int ks = (k + W / 2) % W;
        if (j == 0) v += g[((size_t)0 * W + ks) * 64 + c];
        if (j == H - 1) v += g[((size_t)(H + 1) * W + ks) * 64 + c];
        const uint16_t a = act[(size_t)b * n + e];
        dz[(size_t)b * n + e] = (bf2f(a) > 0.f) ? f2bf(v) : (uint16_t)0;
    }
}

// ------------------------------------------------------------ weight grad
// part[blk][tap][co][ci] = sum over the block's pixels p of
//   x[pad(p + tap)][ci] * dz[p][co]   (FP32, MFMA with pixels as K).
// Waves: (ci tile, co tile) in {0,1} x {0,1}; CIN = 16 uses ci tile 0 only,
// zero-extended to 32 rows.
constexpr int WG_PX = 64;    // pixels (one row segment) per staging step

template <int CIN>
__global__ __launch_bounds__(256) void wgrad_mfma_kernel(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ dz,
                                                         float* __restrict__ part, int batch, int H,
                                                         int W)
{
    constexpr int CIP = CIN < 32 ? 32 : CIN;    // ci rows held in LDS
    constexpr int PS = WG_PX + 8;               // pixel stride of a channel row (bf16)
    __shared__ __attribute__((aligned(16))) uint16_t xs[CIP * PS];
    __shared__ __attribute__((aligned(16))) uint16_t gs[64 * PS];

    const int tap = blockIdx.y, dy = tap / 3, dx = tap - (tap / 3) * 3;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ci_t = wv >> 1, co_t = wv & 1;
    const int col = lane & 31, kh = lane >> 5;
    const int segs_per_row = (W + WG_PX - 1) / WG_PX;
    const long nseg = (long)batch * H * segs_per_row;

    if (CIN < 32) {   // zero rows CIN..31 once
        for (int e = tid; e < (CIP - CIN) * PS; e += 256) xs[CIN * PS + e] = 0;
    }
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    for (long sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
        const int b = (int)(sgi / ((long)H * segs_per_row));
        const long rem = sgi - (long)b * H * segs_per_row;
        const int j = (int)(rem / segs_per_row);
        const int k0 = (int)(rem - (long)j * segs_per_row) * WG_PX;
        __syncthreads();
        // stage x (shifted by the tap, sphere padding) and dz, transposed to [c][px]
        for (int v = tid; v < WG_PX * (CIN / 8); v += 256) {
            const int px = v / (CIN / 8), cv = v - (v / (CIN / 8)) * (CIN / 8);
            const int k = k0 + px;
            uint4 val = make_uint4(0, 0, 0, 0);
            int sj, sk;
            if (k < W && sphere_src(j + dy - 1, k + dx - 1, H, W, sj, sk))
                val = *(const uint4*)(x + (((size_t)b * H + sj) * W + sk) * CIN + cv * 8);
            const uint16_t* h = (const uint16_t*)&val;
#pragma unroll
            for (int i = 0; i < 8; ++i) xs[(cv * 8 + i) * PS + px] = h[i];
        }
        for (int v = tid; v < WG_PX * 8; v += 256) {
            const int px = v >> 3, cv = v & 7;
            const int k = k0 + px;
            uint4 val = make_uint4(0, 0, 0, 0);
            if (k < W) val = *(const uint4*)(dz + (((size_t)b * H + j) * W + k) * 64 + cv * 8);
            const uint16_t* h = (const uint16_t*)&val;
#pragma unroll
            for (int i = 0; i < 8; ++i) gs[(cv * 8 + i) * PS + px] = h[i];
        }
        __syncthreads();
        if (CIN < 32 && ci_t == 1) continue;
#pragma unroll
        for (int ks = 0; ks < WG_PX / 16; ++ks) {
            const int pb = ks * 16 + kh * 8;
            const bf16x8 a = *(const bf16x8*)(xs + (ci_t * 32 + col) * PS + pb);
            const bf16x8 bb = *(const bf16x8*)(gs + (co_t * 32 + col) * PS + pb);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
        }
    }
    if (CIN < 32 && ci_t == 1) return;
    // C[ci][co]: row = ci (8*(r/4) + 4*kh + r%4 within the tile), column = co
    float* o = part + ((size_t)blockIdx.x * 9 + tap) * 64 * CIN;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ci = ci_t * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int co = co_t * 32 + col;
        if (ci < CIN) o[co * CIN + ci] = acc[r];
    }
}

// grad[co][mc][dy][dx] (master layout) = sum over blocks, fixed order, of the
// packed slots feeding master channel mc (two slots for the field channel of
// the first layer, whose weight is shared by the hi and lo parts).
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int nblk, int cin, int cin_out,
                                    float* __restrict__ grad)
{
    const int n = 9 * 64 * cin_out;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int tap = e / (64 * cin_out), rem = e - tap * 64 * cin_out;
        const int co = rem / cin_out, mc = rem - co * cin_out;
        float s = 0.f;
        for (int bk = 0; bk < nblk; ++bk) {
            const float* pb = part + ((size_t)bk * 9 + tap) * 64 * cin + (size_t)co * cin;
            if (cin == 16) s += mc == 0 ? pb[0] + pb[1] : pb[mc + 1];
            else s += pb[mc];
        }
        grad[((size_t)co * cin_out + mc) * 9 + tap] = s;
    }
}

// per-block channel sums of dz (bias gradient), then a fixed-order reduce
__global__ __launch_bounds__(256) void bgrad_partial_kernel(const uint16_t* __restrict__ dz, long npix,
                                                            float* __restrict__ part)
{
    __shared__ float red[256];
    const int c = threadIdx.x & 63, sub = threadIdx.x >> 6;
    float s = 0.f;
    for (long p = (long)blockIdx.x * 4 + sub; p < npix; p += (long)gridDim.x * 4)
        s += bf2f(dz[p * 64 + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 64)
        part[(size_t)blockIdx.x * 64 + c] = red[c] + red[64 + c] + red[128 + c] + red[192 + c];
}

__global__ void colsum_reduce_kernel(const float* __restrict__ part, int nblk, int ncol,
                                     float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * ncol + c];
    out[c] = s;
}

// ------------------------------------------------------ last layer (64 -> 1)
// y[b][j][k] = bias + sum_tap sum_c w5[tap][c] x4[pad(j+dy-1, k+dx-1)][c]   (VALU, FP32)
__global__ __launch_bounds__(256) void conv_last_fwd_kernel(const uint16_t* __restrict__ x4,
                                                            const float* __restrict__ w5,
                                                            const float* __restrict__ b5,
                                                            float* __restrict__ y, int H, int W)
{
    __shared__ float ws[9 * 64];
    for (int e = threadIdx.x; e < 9 * 64; e += 256) ws[e] = w5[e];
    __syncthreads();
    const int b = blockIdx.y;
    const size_t n = (size_t)H * W;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256) {
        const int j = (int)(p / W), k = (int)(p - (size_t)j * W);
        float s = b5[0];
        for (int tap = 0; tap < 9; ++tap) {
            int sj, sk;
            sphere_src(j + tap / 3 - 1, k + tap % 3 - 1, H, W, sj, sk);
            const uint4* src = (const uint4*)(x4 + (((size_t)b * H + sj) * W + sk) * 64);
            for (int cv = 0; cv < 8; ++cv) {
                const uint4 v = src[cv];
                const uint16_t* h = (const uint16_t*)&v;
                for (int i = 0; i < 8; ++i) s += ws[tap * 64 + cv * 8 + i] * bf2f(h[i]);
            }
        }
        y[(size_t)b * n + p] = s;
    }
}

// target t = (B_target - B_in)/5 G; dy = 2 (y - t)/count; per-block FP64 loss sums
template <typename TB>
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ y,
                                                        const TB* __restrict__ Bin,
                                                        const TB* __restrict__ Bt, float* __restrict__ dy,
                                                        double* __restrict__ part, size_t n, double count)
{
    __shared__ double red[256];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float t = (float)(((double)Bt[i] - (double)Bin[i]) / 5.0);
        const float d = y[i] - t;
        dy[i] = (float)(2.0 * (double)d / count);
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Gradient of the last layer w.r.t. its input, masked by the layer-4 ReLU:
// dz4[p][c] = (x4[p][c] > 0) * sum over output pixels q that read p through
// tap t (directly, or through a ghost row across a pole) of w5[t][c] dy[q].
__global__ __launch_bounds__(256) void conv_last_dgrad_kernel(const float* __restrict__ dy,
                                                              const float* __restrict__ w5,
                                                              const uint16_t* __restrict__ x4,
                                                              uint16_t* __restrict__ dz4, int H, int W)
{
    __shared__ float ws[9 * 64];
    for (int e = threadIdx.x; e < 9 * 64; e += 256) ws[e] = w5[e];
    __syncthreads();
    const int b = blockIdx.y;
    const size_t n = (size_t)H * W;
    const float* g = dy + (size_t)b * n;
    for (size_t p = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < n; p += (size_t)gridDim.x * 4) {
        const int c = threadIdx.x & 63;
        const int j = (int)(p / W), k = (int)(p - (size_t)j * W);
        float s = 0.f;
        for (int tap = 0; tap < 9; ++tap) {
            const int dyy = tap / 3, dxx = tap % 3;
            const int qj = j - dyy + 1, qk = wrapk(k - dxx + 1, W);
            if (qj >= 0 && qj < H) s += ws[tap * 64 + c] * g[(size_t)qj * W + qk];
        }
        // ghost paths: output row 0 reads row 0 at k + W/2 through tap dy = 0
        if (j == 0)
            for (int dxx = 0; dxx < 3; ++dxx)
                s += ws[dxx * 64 + c] * g[(size_t)0 * W + wrapk(k + W / 2 - dxx + 1, W)];
        if (j == H - 1)
            for (int dxx = 0; dxx < 3; ++dxx)
                s += ws[(6 + dxx) * 64 + c] * g[(size_t)(H - 1) * W + wrapk(k + W / 2 - dxx + 1, W)];
        const size_t e = ((size_t)b * n + p) * 64 + c;
        dz4[e] = bf2f(x4[e]) > 0.f ? f2bf(s) : (uint16_t)0;
    }
}

// per-block partials of dw5[tap][c] = sum_p x4[pad(p+tap)][c] dy[p] and db5
__global__ __launch_bounds__(256) void conv_last_wgrad_kernel(const float* __restrict__ dy,
                                                              const uint16_t* __restrict__ x4,
                                                              float* __restrict__ part, int batch,
                                                              int H, int W)
{
    const size_t n = (size_t)H * W;
    const long tot = (long)batch * n;
    float acc[3];
    int idx[3];
    for (int q = 0; q < 3; ++q) {
        idx[q] = threadIdx.x + q * 256;
        acc[q] = 0.f;
    }
    float db = 0.f;
    for (long pp = blockIdx.x; pp < tot; pp += gridDim.x) {
        const int b = (int)(pp / n);
        const size_t p = pp - (long)b * n;
        const int j = (int)(p / W), k = (int)(p - (size_t)j * W);
        const float g = dy[pp];
        if (threadIdx.x == 0) db += g;
        for (int q = 0; q < 3; ++q) {
            const int e = idx[q];
            if (e >= 9 * 64) continue;
            const int tap = e >> 6, c = e & 63;
            int sj, sk;
            sphere_src(j + tap / 3 - 1, k + tap % 3 - 1, H, W, sj, sk);
            acc[q] += bf2f(x4[(((size_t)b * H + sj) * W + sk) * 64 + c]) * g;
        }
    }
    float* o = part + (size_t)blockIdx.x * (9 * 64 + 1);
    for (int q = 0; q < 3; ++q)
        if (idx[q] < 9 * 64) o[idx[q]] = acc[q];
    if (threadIdx.x == 0) o[9 * 64] = db;
}

// ------------------------------------------------------------ optimizer
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Master input channel feeding packed slot ci: identity, except for the
// first layer (cip = 16), whose slots 0 and 1 (field hi and lo) share master
// channel 0 and slots 2.. take master channels 1.. .
__device__ __forceinline__ int master_channel(int ci, int cin, int cip)
{
    if (cip != 16) return ci < cin ? ci : -1;
    if (ci <= 1) return 0;
    return ci - 1 < cin ? ci - 1 : -1;
}

// master W[co][ci][dy][dx] -> forward layout wf[tap][co][cip] (zero-padded ci)
// and (if wd) data-gradient layout wd[tap][ci][co].
__global__ void pack_weights_kernel(const float* __restrict__ Wm, int cin, int cip,
                                    uint16_t* __restrict__ wf, uint16_t* __restrict__ wd)
{
    const int n = 9 * 64 * cip;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int tap = e / (64 * cip), rem = e - tap * 64 * cip;
        const int co = rem / cip, ci = rem - co * cip;
        const int mc = master_channel(ci, cin, cip);
        const float v = mc >= 0 ? Wm[((size_t)co * cin + mc) * 9 + tap] : 0.f;
        wf[e] = f2bf(v);
        if (wd && ci < cin) wd[((size_t)tap * cin + ci) * 64 + co] = f2bf(v);
    }
}

// last layer master w5[0][c][dy][dx] -> w5t[tap][c] (FP32)
__global__ void pack_last_kernel(const float* __restrict__ Wm, float* __restrict__ w5t)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 9 * 64) {
        const int tap = e >> 6, c = e & 63;
        w5t[e] = Wm[c * 9 + tap];
    }
}

// last-layer weight gradient: grad[c][tap] (master layout) and bias
__global__ void last_reduce_kernel(const float* __restrict__ part, int nblk, float* __restrict__ gw,
                                   float* __restrict__ gb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > 9 * 64) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * (9 * 64 + 1) + e];
    if (e == 9 * 64) {
        gb[0] = s;
    } else {
        const int tap = e >> 6, c = e & 63;
        gw[c * 9 + tap] = s;
    }
}

// ----------------------------------------------- surrogate prediction / check
// pred = B_in + 5 G y (FP64)
__global__ void surrogate_pred_kernel(const double* __restrict__ Bin, const float* __restrict__ y,
                                      double* __restrict__ pred, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        pred[i] = Bin[i] + 5.0 * (double)y[i];
}

// per-block FP64 sums of (a - b)^2 and b^2 per realization
__global__ __launch_bounds__(256) void diff_norm_kernel(const double* __restrict__ a,
                                                        const double* __restrict__ bref,
                                                        double* __restrict__ part, size_t n)
{
    __shared__ double r1[256], r2[256];
    const int r = blockIdx.y;
    double s1 = 0.0, s2 = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double d = a[(size_t)r * n + i] - bref[(size_t)r * n + i];
        s1 += d * d;
        s2 += bref[(size_t)r * n + i] * bref[(size_t)r * n + i];
    }
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((size_t)r * gridDim.x + blockIdx.x) * 2] = r1[0];
        part[((size_t)r * gridDim.x + blockIdx.x) * 2 + 1] = r2[0];
    }
}

// err[r] = sqrt(sum (a-b)^2 / sum b^2); accepted realizations take a.
__global__ void accept_reduce_kernel(const double* __restrict__ part, int nblk, double tol,
                                     double* __restrict__ err, int* __restrict__ accept)
{
    const int r = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s1 += part[((size_t)r * nblk + b) * 2];
        s2 += part[((size_t)r * nblk + b) * 2 + 1];
    }
    const double e = s2 > 0.0 ? sqrt(s1 / s2) : (s1 > 0.0 ? INFINITY : 0.0);
    err[r] = e;
    accept[r] = e <= tol ? 1 : 0;
}

__global__ void accept_copy_kernel(const double* __restrict__ pred, const int* __restrict__ accept,
                                   double* __restrict__ B, size_t n)
{
    const int r = blockIdx.y;
    if (!accept[r]) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        B[(size_t)r * n + i] = pred[(size_t)r * n + i];
}

// ------------------------------------------------------------------ launchers
static int gblocks(size_t n, int per, int cap)
{
    size_t b = (n + per - 1) / per;
    if (b > (size_t)cap) b = cap;
    return b < 1 ? 1 : (int)b;
}

void cnn_features(hipStream_t st, const void* Bin, int dtype, const float* feats, uint16_t* X0, int batch,
                  int H, int W)
{
    dim3 g(gblocks((size_t)H * W, 256, 2048), batch);
    if (dtype == 1)
        hipLaunchKernelGGL(cnn_features_kernel<float>, g, dim3(256), 0, st, (const float*)Bin, feats, X0, H, W);
    else
        hipLaunchKernelGGL(cnn_features_kernel<double>, g, dim3(256), 0, st, (const double*)Bin, feats, X0,
                           H, W);
}

void cnn_conv_fwd(hipStream_t st, int cin, const uint16_t* x, const uint16_t* wf, const float* bias,
                  uint16_t* out, int batch, int H, int W)
{
    dim3 g((W + CTX - 1) / CTX, (H + CTY - 1) / CTY, batch);
    if (cin == 16)
        hipLaunchKernelGGL((conv_mfma_kernel<16, 0>), g, dim3(128), 0, st, x, wf, bias, (void*)out, H, W);
    else
        hipLaunchKernelGGL((conv_mfma_kernel<64, 0>), g, dim3(128), 0, st, x, wf, bias, (void*)out, H, W);
}

void cnn_conv_dgrad(hipStream_t st, const uint16_t* dz, const uint16_t* wd, float* dxp, int batch, int H,
                    int W)
{
    dim3 g((W + CTX - 1) / CTX, (H + 2 + CTY - 1) / CTY, batch);
    hipLaunchKernelGGL((conv_mfma_kernel<64, 1>), g, dim3(128), 0, st, dz, wd, (const float*)nullptr,
                       (void*)dxp, H, W);
}

void cnn_fold_mask(hipStream_t st, const float* dxp, const uint16_t* act, uint16_t* dz, int batch, int H,
                   int W)
{
    dim3 g(gblocks((size_t)H * W * 64, 256, 4096), batch);
    hipLaunchKernelGGL(fold_mask_kernel, g, dim3(256), 0, st, dxp, act, dz, H, W);
}

void cnn_wgrad(hipStream_t st, int cin, int cin_out, const uint16_t* x, const uint16_t* dz, float* part,
               int nblk, float* grad, int batch, int H, int W)
{
    dim3 g(nblk, 9);
    if (cin == 16)
        hipLaunchKernelGGL(wgrad_mfma_kernel<16>, g, dim3(256), 0, st, x, dz, part, batch, H, W);
    else
        hipLaunchKernelGGL(wgrad_mfma_kernel<64>, g, dim3(256), 0, st, x, dz, part, batch, H, W);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(gblocks((size_t)9 * 64 * cin, 256, 1024)), dim3(256), 0,
                       st, part, nblk, cin, cin_out, grad);
}

void cnn_bgrad(hipStream_t st, const uint16_t* dz, long npix, float* part, int nblk, float* gb)
{
    hipLaunchKernelGGL(bgrad_partial_kernel, dim3(nblk), dim3(256), 0, st, dz, npix, part);
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3(1), dim3(64), 0, st, part, nblk, 64, gb);
}

void cnn_last_fwd(hipStream_t st, const uint16_t* x4, const float* w5t, const float* b5, float* y, int batch,
                  int H, int W)
{
    dim3 g(gblocks((size_t)H * W, 256, 2048), batch);
    hipLaunchKernelGGL(conv_last_fwd_kernel, g, dim3(256), 0, st, x4, w5t, b5, y, H, W);
}

void cnn_loss_grad(hipStream_t st, const float* y, const void* Bin, const void* Bt, int dtype, float* dy,
                   double* part, int nblk, size_t n)
{
    if (dtype == 1)
        hipLaunchKernelGGL(loss_grad_kernel<float>, dim3(nblk), dim3(256), 0, st, y, (const float*)Bin,
                           (const float*)Bt, dy, part, n, (double)n);
    else
        hipLaunchKernelGGL(loss_grad_kernel<double>, dim3(nblk), dim3(256), 0, st, y, (const double*)Bin,
                           (const double*)Bt, dy, part, n, (double)n);
}

void cnn_last_bwd(hipStream_t st, const float* dy, const float* w5t, const uint16_t* x4, uint16_t* dz4,
                  float* part, int nblk, float* gw5, float* gb5, int batch, int H, int W)
{
    dim3 g(gblocks((size_t)H * W, 4, 4096), batch);
    hipLaunchKernelGGL(conv_last_dgrad_kernel, g, dim3(256), 0, st, dy, w5t, x4, dz4, H, W);
    hipLaunchKernelGGL(conv_last_wgrad_kernel, dim3(nblk), dim3(256), 0, st, dy, x4, part, batch, H, W);
    hipLaunchKernelGGL(last_reduce_kernel, dim3(3), dim3(256), 0, st, part, nblk, gw5, gb5);
}

void cnn_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr, float b1,
              float b2, float eps, float c1, float c2)
{
    hipLaunchKernelGGL(adam_kernel, dim3(gblocks(n, 256, 1024)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
}

void cnn_pack(hipStream_t st, const float* Wm, int cin, int cip, uint16_t* wf, uint16_t* wd)
{
    hipLaunchKernelGGL(pack_weights_kernel, dim3(gblocks((size_t)9 * 64 * cip, 256, 1024)), dim3(256), 0, st,
                       Wm, cin, cip, wf, wd);
}

void cnn_pack_last(hipStream_t st, const float* Wm, float* w5t)
{
    hipLaunchKernelGGL(pack_last_kernel, dim3(3), dim3(256), 0, st, Wm, w5t);
}

void cnn_pred(hipStream_t st, const double* Bin, const float* y, double* pred, size_t n)
{
    hipLaunchKernelGGL(surrogate_pred_kernel, dim3(gblocks(n, 256, 4096)), dim3(256), 0, st, Bin, y, pred, n);
}

void cnn_check(hipStream_t st, const double* pred, const double* plain, double* part, int nblk, int R,
               size_t n, double tol, double* err, int* accept, double* B)
{
    hipLaunchKernelGGL(diff_norm_kernel, dim3(nblk, R), dim3(256), 0, st, pred, plain, part, n);
    hipLaunchKernelGGL(accept_reduce_kernel, dim3(R), dim3(64), 0, st, part, nblk, tol, err, accept);
    hipLaunchKernelGGL(accept_copy_kernel, dim3(gblocks(n, 256, 2048), R), dim3(256), 0, st, pred, accept, B,
                       n);
}

}  // namespace sft
