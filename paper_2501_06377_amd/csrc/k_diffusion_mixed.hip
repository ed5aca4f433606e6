// Temporally blocked diffusion stages in the FP32 increment form: one launch
// advances every active realization by up to K super-time-stepping stages
// (Sec. "Diffusion temporal schemes"; the increment form and its (d, e)
// recurrence are described with fold_row in diff_common.h).
//
// Owner map.  A block of NW waves stages a 128-column x LY-row region
// (LY = NW x RPT): lane l holds columns 2l and 2l + 1, wave w the RPT rows
// w RPT .. w RPT + RPT - 1.  Per cell the increment d, its last change e and
// L(Y0) live in registers (3 x 2 x RPT values per lane).  A stage first
// forms every row's new change e in place (each reads the old d of its
// neighbours), then adds the changes to the increments, so no row's old
// value has to be kept aside while its neighbour reads it.  The west
// neighbour of column 0 and the east neighbour of column 1 come from the
// adjacent lanes through whole-wave DPP shifts, folded into the add that
// forms their sum; north / south inside a strip are the lane's own
// registers, and only each strip's two end rows go through LDS (double
// buffered by stage parity, one barrier per stage; two zero rows stand for
// the neighbours beyond the first and last strip, so every wave reads both
// rows without a branch).
//
// Tiles.  Columns: 128 - 2K owned per block, phi wrapping periodically.
// Rows: aligned to the poles.  A staged region that ends at a pole needs no
// halo there (the pole face carries no flux), so the first row tile stages
// [0, LY) and owns [0, LY - K), the last stages [nt - LY, nt) and owns from
// its start + K to nt, and the ones between stage [o - K, o + TY + K) and own
// [o, o + TY), TY = LY - 2K.  The staged values next to a non-pole edge go
// stale one row per stage (the rows beyond read as zero), so after k <= K
// stages the owned rows are exact.  Stage i forms no change for the rows it
// leaves stale (a scalar row mask per strip and stage; a skipped row adds
// its previous change, a value no exact row reads again): the stale band
// of a K-stage launch is about K rows at each non-pole edge.  The stale
// columns cannot be skipped (they are lanes of the same wave).  With
// nt <= LY one tile holds the whole sphere plus rows beyond the south pole,
// which start at zero, take the pole row's coefficients and meet the pole
// row only through its zero pole-face coefficient.
//
// Coefficients.  The block folds the stage coefficients into its rows once
// (fold_row, FP64 rounded to FP32; one thread per staged row, so all other
// waves issue their field loads at once) into an LDS table of K x LY quads,
// read back as wave-wide broadcasts.  The unfused stage kernel uses the same
// fold_row and sts_fold, so every configuration gives the same bits.
//
// Memory.  Fields are addressed through buffer resources based at the
// realization: the row offset is wave-uniform (a scalar offset), the lane's
// column offset one VGPR shared by every row.  The library requires an even
// nphi, so a lane's two columns are adjacent and 8-byte aligned (the region
// starts at an even column) and every field moves in 64-bit accesses
// (128-bit for the FP64 state).  Inputs d_{j0-1}, e = d_{j0-1} - d_{j0-2} (d_1 itself when j0 = 2:
// in2 = NULL) and L(Y0); an entry whose last stage s falls in this launch
// writes B = Y0 + d_s (Y0 = B, plus the advection increment adv when the
// entry is padded), the others the last d and e to out1 / out2.
#include "diff_common.h"
#include "sft_internal.h"

namespace sft {

namespace {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Raw buffer resource over [p, p + bytes): stride 0, 32-bit data format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

__device__ __forceinline__ void st2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float a, float b)
{
    u32x2 v;
    v.x = __float_as_uint(a);
    v.y = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, 0);
}

// A wave-uniform value held in a scalar register (buffer scalar offsets must
// be scalar; otherwise the compiler loops over the distinct lane values).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Value of lane l - 1 (west) / l + 1 (east) of the wave, 0 past its ends.
__device__ __forceinline__ float lane_west(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_east(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}

}  // namespace

// Row tiles of a class with nt rows for a staged height LY and K stages.
__host__ __device__ inline int tall_tiles_y(int nt, int LY, int K)
{
    if (nt <= LY) return 1;
    const int own2 = 2 * (LY - K), TY = LY - 2 * K;
    return nt <= own2 ? 2 : 2 + (nt - own2 + TY - 1) / TY;
}

// Staged-region start jl0 and owned rows [lo, hi) of row tile t of n.
__device__ __forceinline__ void tall_rows(int t, int n, int nt, int LY, int K, int& jl0, int& lo, int& hi)
{
    const int TY = LY - 2 * K;
    if (n == 1) {
        jl0 = 0;
        lo = 0;
        hi = nt;
    } else if (t == 0) {
        jl0 = 0;
        lo = 0;
        hi = LY - K;
    } else {
        lo = (LY - K) + (t - 1) * TY;
        if (t == n - 1) {
            jl0 = nt - LY;
            hi = nt;
        } else {
            jl0 = lo - K;
            hi = lo + TY;
        }
    }
}

// ONE: the class has a single row tile (nt <= LY), whose staged rows beyond
// the south pole read the pole row and are set to zero; with more tiles
// every staged row exists.
template <int K, int RPT, int NW, bool ONE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 16 ? 8 : NW == 12 ? 6 : 4))) void diff_mixed_blocked_kernel(
    const Entry* __restrict__ ents, const StageCoef* __restrict__ coefs, int j0,
    const DiffRow<double>* __restrict__ drow, const float* __restrict__ in1, const float* __restrict__ in2,
    const float* __restrict__ ly0, float* __restrict__ out1, float* __restrict__ out2,
    double* __restrict__ B, const float* __restrict__ adv, int nt, int np)
{
    constexpr int LX = 128, TX = LX - 2 * K, LY = NW * RPT;
    // [stage parity][top, bottom row][wave + 1][column]; [.][1][0] and
    // [.][0][NW + 1] stay zero
    __shared__ float xch[2][2][NW + 2][LX];   // [stage parity][top, bottom row][wave][column]
    __shared__ float4 cft[K][LY];         // folded row coefficients [stage][staged row]

    const int nty = tall_tiles_y(nt, LY, K);
    int bx, by, bz;
    xcd_tile((np + TX - 1) / TX, nty, bx, by, bz);
    // block-uniform tile indices in scalar registers (scalar loads, scalar
    // buffer bases and offsets follow)
    bx = (int)uniform((uint32_t)bx);
    by = (int)uniform((uint32_t)by);
    bz = (int)uniform((uint32_t)bz);
    const Entry e = ents[bz];
    const int kk = min(K, e.s - j0 + 1);
    const bool fin = (j0 + kk - 1 == e.s);
    const size_t base = (size_t)e.r * nt * np;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int jl0, lo, hi;
    tall_rows(by, nty, nt, LY, K, jl0, lo, hi);
    const int k0 = bx * TX;
    const int jw = jl0 + w * RPT;   // global row of the strip's first cell

    // folded coefficients of the kk stages for every staged row (rows beyond
    // the south pole take the pole row's): a thread per row, the stage's
    // coefficients scalar loads
    const DiffRow<double>* dr = drow + (size_t)e.r * nt;
    for (int row = threadIdx.x; row < LY; row += 64 * NW) {
        const DiffRow<double> rr = dr[min(jl0 + row, nt - 1)];
        for (int i = 0; i < kk; ++i) cft[i][row] = fold_row(coefs[e.coef_off + j0 + i], rr);
    }
    for (int idx = threadIdx.x; idx < 4 * LX; idx += 64 * NW) {
        const int q = idx / (2 * LX), h = (idx / LX) & 1, c = idx % LX;
        xch[q][h][h ? 0 : NW + 1][c] = 0.f;
    }

    const uint32_t fbytes = (uint32_t)((size_t)nt * np * 4);
    const auto r_in1 = rsrc(in1 + base, fbytes);
    const auto r_e = rsrc((in2 ? in2 : in1) + base, fbytes);
    const auto r_ly = rsrc(ly0 + base, fbytes);
    int kc0 = (k0 - K + 2 * lane) % np;   // even, and kc0 + 1 < np
    if (kc0 < 0) kc0 += np;

    // d: the last stage's increment; ez: its last change; ly: L(Y0)
    float d[RPT][2], ez[RPT][2], ly[RPT][2];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int j = jw + m;
        const uint32_t so = uniform((uint32_t)(ONE ? min(j, nt - 1) : j) * (uint32_t)np * 4u);
        const float2 a = ld2(r_in1, 4u * kc0, so), b = ld2(r_e, 4u * kc0, so), l = ld2(r_ly, 4u * kc0, so);
        const bool in = !ONE || j < nt;
        d[m][0] = in ? a.x : 0.f;
        d[m][1] = in ? a.y : 0.f;
        ez[m][0] = in ? b.x : 0.f;
        ez[m][1] = in ? b.y : 0.f;
        ly[m][0] = in ? l.x : 0.f;
        ly[m][1] = in ? l.y : 0.f;
    }

    // a staged edge that is not a pole loses one exact row per stage: stage
    // i leaves rows [0, i] (top) and [LY - 1 - i, LY) (bottom) stale
    const bool top = nty > 1 && by > 0, bot = nty > 1 && by < nty - 1;
    for (int i = 0; i < kk; ++i) {
        const StageCoef cf = coefs[e.coef_off + j0 + i];
        const float nnu = (float)(-cf.nu), g = (float)(cf.cL + cf.cLY0);
        const int q = i & 1;
        const int rlo = top ? i + 1 : 0, rhi = bot ? LY - 1 - i : LY;
        *(float2*)&xch[q][0][w + 1][2 * lane] = make_float2(d[0][0], d[0][1]);
        *(float2*)&xch[q][1][w + 1][2 * lane] = make_float2(d[RPT - 1][0], d[RPT - 1][1]);
        __syncthreads();
        const float2 nn = *(const float2*)&xch[q][1][w][2 * lane];
        const float2 ss = *(const float2*)&xch[q][0][w + 2][2 * lane];
        // rows m of this strip with rlo <= w RPT + m < rhi, as a scalar mask
        const int mlo = max(rlo - w * RPT, 0), mhi = min(rhi - w * RPT, RPT);
        const uint32_t vm = mlo < mhi ? ((1u << mhi) - 1u) & ~((1u << mlo) - 1u) : 0u;
        // the changes first (each reads the old d of its neighbours and
        // replaces its own e), then the increments of every row: a skipped
        // row adds its previous change, a value no exact row reads again
        // the strip's coefficient rows through one vector address (a scalar
        // one is copied to a vector register again in every branch)
        const float4* cr = &cft[i][0] + (threadIdx.x >> 6) * RPT;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            if (!(vm & (1u << m))) continue;
            const float4 f = cr[m];
            const float c0 = d[m][0], c1 = d[m][1];
            const float n0 = m > 0 ? d[m - 1][0] : nn.x, n1 = m > 0 ? d[m - 1][1] : nn.y;
            const float s0 = m < RPT - 1 ? d[m + 1][0] : ss.x, s1 = m < RPT - 1 ? d[m + 1][1] : ss.y;
            // column 0: west = column 1 of the lane before; column 1: east =
            // column 0 of the lane after (zero past the wave)
            ez[m][0] = sts_fold(f, nnu, g, lane_west(c1) + c1, n0, c0, s0, ez[m][0], ly[m][0]);
            ez[m][1] = sts_fold(f, nnu, g, c0 + lane_east(c0), n1, c1, s1, ez[m][1], ly[m][1]);
        }
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            d[m][0] += ez[m][0];
            d[m][1] += ez[m][1];
        }
    }

    // outputs: the owned rows and the TX owned columns (both columns of a
    // lane are owned or not together: K, TX and nphi are even)
    const int lx = 2 * lane, kout = k0 + lx - K;
    if (lx < K || lx >= K + TX || kout >= np) return;
    const auto r_o1 = rsrc(out1 + base, fbytes);
    const auto r_o2 = rsrc(out2 + base, fbytes);
    const auto r_adv = rsrc(adv + base, fbytes);
    const auto r_B = rsrc(B + base, 2u * fbytes);
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int j = jw + m;
        if (j < lo || j >= hi) continue;
        const uint32_t so = uniform((uint32_t)j * (uint32_t)np * 4u);
        if (fin) {
            const u32x4 y = __builtin_amdgcn_raw_buffer_load_b128(r_B, 8u * kout, 2u * so, 0);
            double y0 = __hiloint2double((int)y.y, (int)y.x), y1 = __hiloint2double((int)y.w, (int)y.z);
            if (e.pad) {
                const float2 a = ld2(r_adv, 4u * kout, so);
                y0 += (double)a.x;
                y1 += (double)a.y;
            }
            y0 += (double)d[m][0];
            y1 += (double)d[m][1];
            u32x4 o;
            o.x = (unsigned)__double2loint(y0);
            o.y = (unsigned)__double2hiint(y0);
            o.z = (unsigned)__double2loint(y1);
            o.w = (unsigned)__double2hiint(y1);
            __builtin_amdgcn_raw_buffer_store_b128(o, r_B, 8u * kout, 2u * so, 0);
        } else {
            st2(r_o1, 4u * kout, so, d[m][0], d[m][1]);
            st2(r_o2, 4u * kout, so, ez[m][0], ez[m][1]);
        }
    }
}

// ------------------------------------------------------------ configurations
// (K, rows per wave, waves); tx = 128 - 2K owned columns, ty = NW RPT - 2K
// rows owned by an interior row tile.  Sixteen-wave blocks of 6-row strips
// (52 registers) hold 128 x 96 cells, of 8-row strips (63) 128 x 128, two
// blocks per compute unit at eight waves per SIMD.  A launch's loads and
// stores take a fixed share of its time that more stages per launch spread
// over more work, while the halo grows with K: 14 to 18 stages on the
// 128 x 128 region balance the two on 1024 x 2048 grids.
struct MixedCfg {
    int k, rpt, nw;
};
static const MixedCfg kCfgMixed[] = {{8, 16, 8}, {12, 16, 8}, {6, 16, 8}, {8, 12, 8}, {12, 12, 8},
                                     {10, 12, 8}, {8, 8, 8},  {4, 8, 8},  {8, 4, 8},  {4, 4, 8},
                                     {12, 8, 12}, {10, 8, 12}, {12, 6, 16}, {14, 6, 16}, {16, 6, 16},
                                     {18, 6, 16}, {16, 8, 12}, {12, 8, 16}, {16, 8, 16}, {18, 8, 16},
                                     {20, 8, 16}, {14, 8, 16}};

int mixed_config_count() { return (int)(sizeof kCfgMixed / sizeof kCfgMixed[0]); }

int mixed_config_k(int cfg) { return kCfgMixed[cfg].k; }

void mixed_config_desc(int cfg, int* tx, int* ty, int* k, int* nthr)
{
    const MixedCfg& c = kCfgMixed[cfg];
    *tx = 128 - 2 * c.k;
    *ty = c.nw * c.rpt - 2 * c.k;
    *k = c.k;
    *nthr = 64 * c.nw;
}

template <int K, int RPT, int NW>
static void launch_cfg(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs, int j0,
                       const DiffRow<double>* drow, const float* in1, const float* in2, const float* ly0,
                       float* out1, float* out2, double* B, const float* adv, int nt, int np)
{
    constexpr int TX = 128 - 2 * K, LY = NW * RPT;
    const int nblk = ((np + TX - 1) / TX) * tall_tiles_y(nt, LY, K) * n_act;
    if (nt <= LY)
        hipLaunchKernelGGL((diff_mixed_blocked_kernel<K, RPT, NW, true>), dim3(nblk), dim3(64 * NW), 0, st, ents,
                           coefs, j0, drow, in1, in2, ly0, out1, out2, B, adv, nt, np);
    else
        hipLaunchKernelGGL((diff_mixed_blocked_kernel<K, RPT, NW, false>), dim3(nblk), dim3(64 * NW), 0, st, ents,
                           coefs, j0, drow, in1, in2, ly0, out1, out2, B, adv, nt, np);
}

void launch_diff_mixed_blocked(hipStream_t st, int cfg, const Entry* ents, int n_act, const StageCoef* coefs,
                               int j0, const DiffRow<double>* drow, const float* in1, const float* in2,
                               const float* ly0, float* out1, float* out2, double* B, const float* adv, int nt,
                               int np)
{
#define M1(k, r, w) launch_cfg<k, r, w>(st, ents, n_act, coefs, j0, drow, in1, in2, ly0, out1, out2, B, adv, nt, np)
    switch (cfg) {
    case 0: M1(8, 16, 8); break;
    case 1: M1(12, 16, 8); break;
    case 2: M1(6, 16, 8); break;
    case 3: M1(8, 12, 8); break;
    case 4: M1(12, 12, 8); break;
    case 5: M1(10, 12, 8); break;
    case 6: M1(8, 8, 8); break;
    case 7: M1(4, 8, 8); break;
    case 8: M1(8, 4, 8); break;
    case 9: M1(4, 4, 8); break;
    case 10: M1(12, 8, 12); break;
    case 11: M1(10, 8, 12); break;
    case 12: M1(12, 6, 16); break;
    case 13: M1(14, 6, 16); break;
    case 14: M1(16, 6, 16); break;
    case 15: M1(18, 6, 16); break;
    case 16: M1(16, 8, 12); break;
    case 17: M1(12, 8, 16); break;
    case 18: M1(16, 8, 16); break;
    case 19: M1(18, 8, 16); break;
    case 20: M1(20, 8, 16); break;
    default: M1(14, 8, 16); break;
    }
#undef M1
}

}  // namespace sft
