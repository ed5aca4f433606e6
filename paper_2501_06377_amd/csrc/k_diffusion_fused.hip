// Temporally blocked diffusion stages, FP64 paper form: one launch advances
// every active realization by up to K super-time-stepping stages (the FP32
// increment form has its own kernel, k_diffusion_mixed.hip).
//
// A block owns a TY x TX tile of output cells and stages the tile plus a
// K-cell halo in LDS (phi wraps periodically; rows beyond the poles are held
// at zero and only ever meet a zero coefficient, so the pole rows stay exact).
// Each stage recomputes the whole staged region from the previous one, in a
// double-buffered LDS array (one barrier per stage); the region that is still
// exact shrinks by one cell per stage, so after k <= K stages the tile
// interior is exact.  Per cell the previous stage, the one before it, L(Y0)
// and (paper form) Y0 live in registers.
//
// The per-cell arithmetic is the same helper the unfused kernels use, so the
// results are bitwise identical to the one-stage-per-launch path for every
// tile shape.
//
// Inputs Y_{j0-1}, Y_{j0-2}, a copy of Y0 and L(Y0) (the strip variant
// computes L(Y0) from the staged Y0 instead of reading it).  An entry whose
// last stage s falls in this launch writes the final field into B, otherwise
// the last two stages go to out1/out2.
#include "diff_common.h"
#include "sft_internal.h"

namespace sft {

template <int TX, int TY, int K, int NT>
__global__ __launch_bounds__(NT) void diff_fused_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs, int j0,
    const DiffRow<double>* __restrict__ drow, const double* __restrict__ in1,
    const double* __restrict__ in2, const double* __restrict__ y0, const double* __restrict__ ly0,
    double* __restrict__ out1, double* __restrict__ out2, double* __restrict__ B, int nt, int np)
{
    using T = double;
    constexpr int LX = TX + 2 * K, LY = TY + 2 * K, NC = LX * LY;
    constexpr int CPT = (NC + NT - 1) / NT;
    static_assert(CPT <= 32, "cell mask holds 32 cells per thread");
    __shared__ T buf[2][NC];
    __shared__ DiffRow<T> rowc[LY];

    const Entry e = ents[blockIdx.z];
    const int kk = min(K, e.s - j0 + 1);
    const bool fin = (j0 + kk - 1 == e.s);
    const size_t base = (size_t)e.r * nt * np;
    const int k0 = blockIdx.x * TX, jt0 = blockIdx.y * TY;
    const int jl0 = jt0 - K, kl0 = k0 - K;
    const int tid = threadIdx.x;
    const bool has_in2 = in2 != nullptr;

    for (int l = tid; l < LY; l += NT) {
        const int j = jl0 + l;
        DiffRow<T> d;
        d.up = d.dn = d.ph = d.d = T(0);
        if (j >= 0 && j < nt) d = drow[(size_t)e.r * nt + j];
        rowc[l] = d;
    }

    T ycur[CPT], ym2[CPT], lyr[CPT], y0r[CPT];
    uint32_t act = 0;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int idx = tid + m * NT;
        T a = T(0), b = T(0), l = T(0);
        double z = 0.0;
        if (idx < NC) {
            const int ly = idx / LX, lx = idx - (idx / LX) * LX;
            const int j = jl0 + ly;
            if (j >= 0 && j < nt) {
                int k = (kl0 + lx) % np;
                if (k < 0) k += np;
                const size_t i = base + (size_t)j * np + k;
                a = in1[i];
                if (has_in2) b = in2[i];
                l = ly0[i];
                z = y0[i];
                if (ly >= 1 && ly <= LY - 2 && lx >= 1 && lx <= LX - 2) act |= 1u << m;
            }
            buf[0][idx] = a;
            buf[1][idx] = a;
        }
        ycur[m] = a;
        ym2[m] = b;
        lyr[m] = l;
        y0r[m] = z;
    }
    __syncthreads();

    int p = 0;
    for (int i = 0; i < kk; ++i) {
        const StageCoef c = coefs[e.coef_off + j0 + i];
        const T* cb = buf[p];
        T* nb = buf[p ^ 1];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (act & (1u << m)) {
                const int idx = tid + m * NT;
                const DiffRow<T> d = rowc[idx / LX];
                const T L = L5<T>(d, cb[idx - 1], cb[idx - LX], ycur[m], cb[idx + LX], cb[idx + 1]);
                const T v = sts_f64(c, ycur[m], ym2[m], y0r[m], L, lyr[m]);
                nb[idx] = v;
                ym2[m] = ycur[m];
                ycur[m] = v;
            }
        }
        p ^= 1;
        __syncthreads();
    }

#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int idx = tid + m * NT;
        if (idx >= NC) continue;
        const int ly = idx / LX, lx = idx - (idx / LX) * LX;
        if (ly < K || ly >= K + TY || lx < K || lx >= K + TX) continue;
        const int j = jt0 + ly - K, k = k0 + lx - K;
        if (j >= nt || k >= np) continue;
        const size_t gi = base + (size_t)j * np + k;
        if (fin) {
            B[gi] = ycur[m];
        } else {
            out1[gi] = ycur[m];
            out2[gi] = ym2[m];
        }
    }
}

// ------------------------------------------------------------ strip variant
// The same K-stage blocking with a different owner map: lane = CPL adjacent
// columns of a 64 * CPL-column staged region (TX = 64 CPL - 2K output
// columns), wave w = a strip of RPT consecutive rows (TY = NW * RPT - 2K
// output rows).  A lane's outer west and east neighbours come from the
// adjacent lanes through whole-wave DPP shifts, the others and north / south
// from the lane's own registers; only the two end rows of each strip are
// exchanged through LDS (double-buffered by stage parity, one barrier per
// stage).  Row coefficients are wave-uniform (scalar loads).  At stage i the
// strips skip their rows among the i outermost of the staged region.
//
// Value of lane l - 1 (west) / l + 1 (east) of the wave, 0 past its ends
// (bound_ctrl: a lane whose source is out of range reads zero).
__device__ __forceinline__ double lane_west(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_east(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int K, int RPT, int NW, int CPL>
__global__ __launch_bounds__(64 * NW) void diff_strip_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs, int j0,
    const DiffRow<double>* __restrict__ drow, const double* __restrict__ in1,
    const double* __restrict__ in2, const double* __restrict__ y0, double* __restrict__ out1,
    double* __restrict__ out2, double* __restrict__ B, int nt, int np)
{
    using T = double;
    constexpr int LX = 64 * CPL, TX = LX - 2 * K, LY = NW * RPT, TY = LY - 2 * K;
    __shared__ T xch[2][2][NW][LX];   // [stage parity][top, bottom row][wave][column]

    // XCD-aware order: the halo a block stages is largely in the L2 its
    // neighbours just filled
    int bx, by, bz;
    xcd_tile((np + TX - 1) / TX, (nt + TY - 1) / TY, bx, by, bz);
    const Entry e = ents[bz];
    const int kk = min(K, e.s - j0 + 1);
    const bool fin = (j0 + kk - 1 == e.s);
    const size_t base = (size_t)e.r * nt * np;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k0 = bx * TX, jt0 = by * TY;
    const int jw = jt0 - K + w * RPT;   // global row of the strip's first cell
    int kc[CPL];                        // global columns of the lane's cells
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        int k = (k0 - K + lane * CPL + c) % np;
        kc[c] = k < 0 ? k + np : k;
    }
    const bool has_in2 = in2 != nullptr;
    const DiffRow<T>* dr = drow + (size_t)e.r * nt;

    // ya / yb alternate as (current, previous); rows beyond the poles start
    // at zero
    T ya[RPT][CPL], yb[RPT][CPL], lyr[RPT][CPL], y0r[RPT][CPL];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int j = jw + m;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            T a = T(0), b = T(0), z = T(0);
            if (j >= 0 && j < nt) {
                const size_t i = base + (size_t)j * np + kc[c];
                a = in1[i];
                if (has_in2) b = in2[i];
                z = y0[i];
            }
            ya[m][c] = a;
            yb[m][c] = b;
            y0r[m][c] = z;
        }
    }

    // L(Y0) of the staged region from the staged Y0 (the first-stage
    // kernel's operator, the same helper and operand order, so the same
    // bits) instead of reading a fourth array.  The outer ring's value is
    // wrong (its outer neighbours read as zero) but, being a pointwise term,
    // it spoils nothing the ring's own wrong stage values do not already.
    {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            xch[1][0][w][lane * CPL + c] = y0r[0][c];
            xch[1][1][w][lane * CPL + c] = y0r[RPT - 1][c];
        }
        __syncthreads();
        T north[CPL], south[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            north[c] = w > 0 ? xch[1][1][w - 1][lane * CPL + c] : T(0);
            south[c] = w < NW - 1 ? xch[1][0][w + 1][lane * CPL + c] : T(0);
        }
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const DiffRow<T> d = dr[min(max(jw + m, 0), nt - 1)];
            const T wl = lane_west(y0r[m][CPL - 1]), el = lane_east(y0r[m][0]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const T wv = c > 0 ? y0r[m][c - 1] : wl;
                const T ev = c < CPL - 1 ? y0r[m][c + 1] : el;
                lyr[m][c] = L5<T>(d, wv, m > 0 ? y0r[m - 1][c] : north[c], y0r[m][c],
                                  m < RPT - 1 ? y0r[m + 1][c] : south[c], ev);
            }
        }
    }

    // One stage: cur holds the stage input, prv the stage before it and
    // receives the result.  Every staged cell in range is updated, the outer
    // ring included (its neighbours outside the region read as zero): the
    // error this starts moves inwards one cell per stage, and the output
    // region lies K cells inside the ring, as in the tiled variant.
    auto stage = [&](int i, T (&cur)[RPT][CPL], T (&prv)[RPT][CPL]) {
        const StageCoef cf = coefs[e.coef_off + j0 + i];
        const int q = i & 1;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            xch[q][0][w][lane * CPL + c] = cur[0][c];
            xch[q][1][w][lane * CPL + c] = cur[RPT - 1][c];
        }
        __syncthreads();
        T north[CPL], south[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            north[c] = w > 0 ? xch[q][1][w - 1][lane * CPL + c] : T(0);
            south[c] = w < NW - 1 ? xch[q][0][w + 1][lane * CPL + c] : T(0);
        }
        // Rows beyond a pole (only in strips that reach it) are updated too,
        // with the pole row's coefficients: they start at zero, stay finite,
        // are never written out, and the pole row meets them only through its
        // zero pole-face coefficient.  No per-row branch, so the row
        // coefficients (wave-uniform scalar loads) can be issued early.
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            // rows i and closer to the top / bottom of the staged region are
            // already wrong after this stage whatever is computed for them
            // (and no row that stays right reads them), so they are skipped
            const int ly = w * RPT + m;
            if (ly < i || ly >= LY - i) continue;
            const DiffRow<T> d = dr[min(max(jw + m, 0), nt - 1)];
            const T wl = lane_west(cur[m][CPL - 1]), el = lane_east(cur[m][0]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const T wv = c > 0 ? cur[m][c - 1] : wl;
                const T ev = c < CPL - 1 ? cur[m][c + 1] : el;
                const T L = L5<T>(d, wv, m > 0 ? cur[m - 1][c] : north[c], cur[m][c],
                                  m < RPT - 1 ? cur[m + 1][c] : south[c], ev);
                prv[m][c] = sts_f64(cf, cur[m][c], prv[m][c], y0r[m][c], L, lyr[m][c]);
            }
        }
    };
    int i = 0;
    for (; i + 1 < kk; i += 2) {
        stage(i, ya, yb);
        stage(i + 1, yb, ya);
    }
    const bool odd = i < kk;
    if (odd) stage(i, ya, yb);

#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int lx = lane * CPL + c, k = k0 + lx - K;
        if (lx < K || lx >= K + TX || k >= np) continue;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w * RPT + m, j = jw + m;
            if (ly < K || ly >= K + TY || j >= nt) continue;
            const T last = odd ? yb[m][c] : ya[m][c], before = odd ? ya[m][c] : yb[m][c];
            const size_t gi = base + (size_t)j * np + k;
            if (fin) {
                B[gi] = last;
            } else {
                out1[gi] = last;
                out2[gi] = before;
            }
        }
    }
}

// ------------------------------------------------------------ configurations
struct FusedCfg {
    int tx, ty, k, nt;
};

// tiled shapes first, then the strip variant (tx = 64 x columns per lane - 2K,
// ty = waves x rows per wave - 2K)
static const FusedCfg kCfg64[] = {
    {64, 16, 4, 256}, {64, 32, 8, 256}, {128, 16, 4, 256}, {32, 32, 4, 256}, {64, 32, 6, 256},
    {48, 48, 8, 256}, {48, 112, 8, 512}, {52, 116, 6, 512}, {48, 48, 8, 512},
    {112, 48, 8, 512}, {116, 52, 6, 512}, {112, 80, 8, 512},
    // short strips: more, lighter blocks for classes with few cells
    {48, 16, 8, 512}, {56, 24, 4, 512}, {48, 32, 8, 512}};

int fused_config_count(bool mixed) { return mixed ? mixed_config_count() : 15; }

int fused_config_k(bool mixed, int cfg) { return mixed ? mixed_config_k(cfg) : kCfg64[cfg].k; }

bool fused_config_reads_ly0(bool mixed, int cfg) { return mixed || cfg < 5; }

void fused_config_desc(bool mixed, int cfg, int* tx, int* ty, int* k, int* nthr)
{
    if (mixed) {
        mixed_config_desc(cfg, tx, ty, k, nthr);
        return;
    }
    const FusedCfg& c = kCfg64[cfg];
    *tx = c.tx;
    *ty = c.ty;
    *k = c.k;
    *nthr = c.nt;
}

template <int TX, int TY, int K, int NT>
static void launch_one(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs, int j0,
                       const void* drow, const void* in1, const void* in2, const double* y0,
                       const void* ly0, void* out1, void* out2, double* B, int nt, int np)
{
    dim3 grid((np + TX - 1) / TX, (nt + TY - 1) / TY, n_act);
    hipLaunchKernelGGL((diff_fused_kernel<TX, TY, K, NT>), grid, dim3(NT), 0, st, ents, coefs, j0,
                       (const DiffRow<double>*)drow, (const double*)in1, (const double*)in2, y0,
                       (const double*)ly0, (double*)out1, (double*)out2, B, nt, np);
}

template <int K, int RPT, int NW, int CPL>
static void launch_strip(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs, int j0,
                         const void* drow, const void* in1, const void* in2, const double* y0,
                         void* out1, void* out2, double* B, int nt, int np)
{
    constexpr int TX = 64 * CPL - 2 * K, TY = NW * RPT - 2 * K;
    const int nblk = ((np + TX - 1) / TX) * ((nt + TY - 1) / TY) * n_act;
    hipLaunchKernelGGL((diff_strip_kernel<K, RPT, NW, CPL>), dim3(nblk), dim3(64 * NW), 0, st, ents, coefs, j0,
                       (const DiffRow<double>*)drow, (const double*)in1, (const double*)in2, y0,
                       (double*)out1, (double*)out2, B, nt, np);
}

void launch_diff_fused(hipStream_t st, bool mixed, int cfg, const Entry* ents, int n_act,
                       const StageCoef* coefs, int j0, const void* drow, const void* in1,
                       const void* in2, const double* y0, const void* ly0, void* out1, void* out2,
                       double* B, const float* adv, int nt, int np)
{
    if (mixed) {
        launch_diff_mixed_blocked(st, cfg, ents, n_act, coefs, j0, (const DiffRow<double>*)drow,
                                  (const float*)in1, (const float*)in2, (const float*)ly0, (float*)out1,
                                  (float*)out2, B, adv, nt, np);
        return;
    }
#define L1(a, b, c, d) launch_one<a, b, c, d>(st, ents, n_act, coefs, j0, drow, in1, in2, y0, ly0, out1, out2, B, nt, np)
#define S1(k, r, w, c) launch_strip<k, r, w, c>(st, ents, n_act, coefs, j0, drow, in1, in2, y0, out1, out2, B, nt, np)
    switch (cfg) {
    case 0: L1(64, 16, 4, 256); break;
    case 1: L1(64, 32, 8, 256); break;
    case 2: L1(128, 16, 4, 256); break;
    case 3: L1(32, 32, 4, 256); break;
    case 4: L1(64, 32, 6, 256); break;
    case 5: S1(8, 16, 4, 1); break;
    case 6: S1(8, 16, 8, 1); break;
    case 7: S1(6, 16, 8, 1); break;
    case 8: S1(8, 8, 8, 1); break;
    case 9: S1(8, 8, 8, 2); break;
    case 10: S1(6, 8, 8, 2); break;
    case 11: S1(8, 12, 8, 2); break;
    case 12: S1(8, 4, 8, 1); break;
    case 13: S1(4, 4, 8, 1); break;
    default: S1(8, 6, 8, 1); break;
    }
#undef L1
#undef S1
}

}  // namespace sft
