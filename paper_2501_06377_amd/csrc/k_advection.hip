// Advection stage kernels: WENO3-CS(h) face fluxes in theta and phi (App. B),
// upwind pole-adjacent theta faces and zero-flux pole faces (App. A and the
// advection boundary conditions), the spherical divergence of the flux
// (Sec. "Advection spatial schemes") and one SSPRK(4,3) / forward-Euler stage
// combination (Sec. "Advection temporal schemes"), fused in one LDS-tiled
// kernel per stage.
//
// Tile: TY rows x ATX columns of output cells per 256-thread block (TY =
// PLAIN_TY for the static flow, ATT_TY for the attenuated one), staged
// in LDS with a 2-cell halo (WENO3 needs cells i-2..i+1 for face i-1/2); phi
// wraps periodically, rows outside the sphere are never used by a face flux
// (pole faces carry no flux, pole-adjacent faces are upwind).
//
// The kernels evaluate the paper's formulas with no FMA contraction (the
// library is built with -ffp-contract=off) except that each one-sided WENO
// value is formed with one division (the nonlinear weights' common factor
// cancelled), which changes results only at the rounding level.  The FP32
// increment path (MIXED) divides with the hardware reciprocal (about one
// ulp) and lets the compiler fuse its multiply-adds in the WENO values: its
// rounding is FP32's anyway, and the divisions were most of its vector-ALU
// work.
//
// Flow attenuation (eq. flow_attenuation): the face velocities of one
// advection advance are scaled by 1 - tanh(m/B0), m the mean of |B| over the
// face's two cells of the field at the start of the advance.  att_faces_kernel
// writes them once per advance (one phi-face and one theta-face value per
// cell); the ATT variant of the stage kernel stages them with a 4-face halo
// and builds the per-cell LLF split factors in LDS (alpha = max |v| over the
// faces i-2 .. i+3 of each cell, as for the static flow).
#include "sft_internal.h"
#include "adv_att.h"

namespace sft {

constexpr int ATX = 64;
constexpr int AH = 2;
constexpr int AW = ATX + 2 * AH;
// tile rows: the static-flow kernels stage 1.25x their output rows; the
// attenuated kernels keep four face and factor arrays in LDS as well
constexpr int PLAIN_TY = 16;
constexpr int ATT_TY = 8;

__device__ __forceinline__ int wrap_col(int k, int np)
{
    k %= np;
    return k < 0 ? k + np : k;
}

// App. B on a uniform grid: u^- from LM_{i-2}, LM_{i-1}, LM_i and u^+ from
// LP_{i-1}, LP_i, LP_{i+1}; F_{i-1/2} = u^+ + u^-.
template <typename T>
__device__ __forceinline__ T weno_face(T lm2, T lm1, T lm0, T lpm1, T lp0, T lpp1,
                                       const WenoConst<T>& c)
{
    const T one = T(1), four = T(4);
    T p0m = (one + c.half) * lm1 - c.half * lm2;
    T p1m = c.half * lm1 + c.half * lm0;
    T t0m = c.half * (lm1 - lm2);
    T t1m = c.half * (lm0 - lm1);
    T b0m = four * t0m * t0m;
    T b1m = four * t1m * t1m;
    // w0 = third / A^2, w1 = twothird / B^2 (A = eps + b0, B = eps + b1), and
    // u = (w0 p0 + w1 p1) / (w0 + w1) = (third B^2 p0 + twothird A^2 p1) /
    // (third B^2 + twothird A^2): one division instead of four
    T a2m = (c.eps + b0m) * (c.eps + b0m), bb2m = (c.eps + b1m) * (c.eps + b1m);
    T v0m = c.third * bb2m, v1m = c.twothird * a2m;
    T um = (v0m * p0m + v1m * p1m) / (v0m + v1m);

    T p0p = (one + c.half) * lp0 - c.half * lpp1;
    T p1p = c.half * lp0 + c.half * lpm1;
    T t0p = c.half * (lpp1 - lp0);
    T t1p = c.half * (lp0 - lpm1);
    T b0p = four * t0p * t0p;
    T b1p = four * t1p * t1p;
    T a2p = (c.eps + b0p) * (c.eps + b0p), bb2p = (c.eps + b1p) * (c.eps + b1p);
    T v0p = c.third * bb2p, v1p = c.twothird * a2p;
    T up = (v0p * p0p + v1p * p1p) / (v0p + v1p);
    return up + um;
}

// FP32: the same formulas, the division by the hardware reciprocal and the
// multiply-adds fused.
template <>
__device__ __forceinline__ float weno_face<float>(float lm2, float lm1, float lm0, float lpm1, float lp0,
                                                  float lpp1, const WenoConst<float>& c)
{
#pragma clang fp contract(fast)
    const float one = 1.f, four = 4.f;
    const float p0m = (one + c.half) * lm1 - c.half * lm2;
    const float p1m = c.half * lm1 + c.half * lm0;
    const float t0m = c.half * (lm1 - lm2), t1m = c.half * (lm0 - lm1);
    const float b0m = four * t0m * t0m, b1m = four * t1m * t1m;
    const float a2m = (c.eps + b0m) * (c.eps + b0m), bb2m = (c.eps + b1m) * (c.eps + b1m);
    const float v0m = c.third * bb2m, v1m = c.twothird * a2m;
    const float um = (v0m * p0m + v1m * p1m) * __builtin_amdgcn_rcpf(v0m + v1m);

    const float p0p = (one + c.half) * lp0 - c.half * lpp1;
    const float p1p = c.half * lp0 + c.half * lpm1;
    const float t0p = c.half * (lpp1 - lp0), t1p = c.half * (lp0 - lpm1);
    const float b0p = four * t0p * t0p, b1p = four * t1p * t1p;
    const float a2p = (c.eps + b0p) * (c.eps + b0p), bb2p = (c.eps + b1p) * (c.eps + b1p);
    const float v0p = c.third * bb2p, v1p = c.twothird * a2p;
    const float up = (v0p * p0p + v1p * p1p) * __builtin_amdgcn_rcpf(v0p + v1p);
    return up + um;
}

// a / b: exact division in FP64, the hardware reciprocal in FP32 (b > 0)
__device__ __forceinline__ double adv_div(double a, double b) { return a / b; }
__device__ __forceinline__ float adv_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Upwind face flux: F = v (1/2)[(1-uw) B_right + (1+uw) B_left], uw = sign(v).
template <typename T>
__device__ __forceinline__ T upwind_face(T v, T bl, T br)
{
    const T one = T(1);
    T sg = v > T(0) ? one : (v < T(0) ? -one : T(0));
    T uw = one * sg;
    return v * T(0.5) * ((one - uw) * br + (one + uw) * bl);
}

// LDS of the attenuated-flow variant: phi faces k0-4 .. k0+ATX+4 of the tile
// rows, theta faces j0-4 .. j0+TY+4 of the tile columns, and per-cell LLF
// split factors of the staged cells.
constexpr int AVW = ATX + 9;
template <typename T, bool ATT, int TY>
struct AttLds {
};
template <typename T, int TY>
struct AttLds<T, true, TY> {
    T vp[TY][AVW];
    T vt[TY + 9][ATX];
    T cpM[TY][AW], cpP[TY][AW];
    T ctM[TY + 2 * AH][ATX], ctP[TY + 2 * AH][ATX];
};

// MIXED = false: T = double, stage values read from fin (FP64 fields).
// MIXED = true : T = float, stage value = (float)(fn + din) (din absent at
//                stage 0), increments written to dout.
// ATT = true   : face velocities from vphf / vthf ([R][nt][np] each: phi face
//                k of row j lies between cells k-1 and k; theta face j lies
//                between rows j-1 and j) instead of the per-row constants.
template <typename T, bool MIXED, bool ATT, int TY>
__global__ __launch_bounds__(256) void adv_stage_kernel(
    const Entry* __restrict__ ents, int stage, int time_scheme, int upwind,
    const AdvRow<T>* __restrict__ rows, Geom<T> g, WenoConst<T> wth, WenoConst<T> wph,
    const double* __restrict__ fn, const T* __restrict__ fin, T* __restrict__ fout,
    const T* __restrict__ vphf, const T* __restrict__ vthf, int nt, int np)
{
    constexpr int ATY = TY, AHT = TY + 2 * AH, AVH = TY + 9;
    __shared__ T tile[AHT][AW];
    __shared__ T fph[ATY][ATX + 1];
    __shared__ T fth[ATY + 1][ATX];
    __shared__ T cthM[AHT], cthP[AHT];
    // per tile row: phi split factors, v_phi, sin(theta) dphi; per theta
    // face j0 .. j0 + TY: v_theta, sin at the face, and the row's
    // sin(theta) dtheta
    __shared__ T rph[ATY][4];
    __shared__ T rth[ATY + 1][3];
    __shared__ AttLds<T, ATT, TY> al;

    const Entry e = ents[blockIdx.z];
    const size_t base = (size_t)e.r * nt * np;
    const int k0 = blockIdx.x * ATX, j0 = blockIdx.y * ATY;
    const AdvRow<T>* rw = rows + (size_t)e.r * (nt + 1);
    const int tid = threadIdx.x;

    // per-row constants into registers first (their loads overlap the tile's)
    T q0 = T(0), q1 = T(0), q2 = T(0), q3 = T(0), q4 = T(0), q5 = T(0), q6 = T(0);
    if (tid < ATY + 1) {
        const int j = j0 + tid;
        if (j < nt) {
            q0 = rw[j].cphM;
            q1 = rw[j].cphP;
            q2 = rw[j].vph;
            q3 = g.den_ph[j];
            q6 = g.den_th[j];
        }
        if (j <= nt) {
            q4 = rw[j].vth;
            q5 = g.sf[j];
        }
    } else if (!ATT && tid >= 64 && tid < 64 + AHT) {
        const int j = j0 + tid - 64 - AH;
        if (j >= 0 && j < nt) {
            q0 = rw[j].cthM;
            q1 = rw[j].cthP;
        }
    }

    // the staged cells: every load issued before any is waited for (rows
    // beyond the poles read a pole row and are set to zero)
    constexpr int NL = (AHT * AW + 255) / 256;
    size_t si[NL];
    bool sin[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int idx = min(tid + 256 * u, AHT * AW - 1);
        const int tj = idx / AW, tk = idx - (idx / AW) * AW;
        const int j = j0 + tj - AH;
        si[u] = base + (size_t)min(max(j, 0), nt - 1) * np + wrap_col(k0 + tk - AH, np);
        sin[u] = j >= 0 && j < nt;
    }
    T sv[NL];
    if constexpr (MIXED) {
        double x[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) x[u] = fn[si[u]];
        if (stage > 0) {
            float f[NL];
#pragma unroll
            for (int u = 0; u < NL; ++u) f[u] = fin[si[u]];
#pragma unroll
            for (int u = 0; u < NL; ++u) x[u] += (double)f[u];
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) sv[u] = sin[u] ? (T)x[u] : T(0);
    } else {
#pragma unroll
        for (int u = 0; u < NL; ++u) sv[u] = fin[si[u]];
#pragma unroll
        for (int u = 0; u < NL; ++u) sv[u] = sin[u] ? sv[u] : T(0);
    }
    // attenuated flow: the tile's face velocities, loaded with its cells
    // (faces outside 0..nt take no part in any window; the pole faces keep
    // the static flow's value)
    constexpr int NVP = ATT ? (ATY * AVW + 255) / 256 : 1, NVT = ATT ? (AVH * ATX + 255) / 256 : 1;
    T vpv[NVP], vtv[NVT];
    if constexpr (ATT) {
#pragma unroll
        for (int u = 0; u < NVP; ++u) {
            const int idx = min(tid + 256 * u, ATY * AVW - 1);
            const int tj = idx / AVW, q = idx - (idx / AVW) * AVW;
            const int j = j0 + tj;
            const T v = vphf[base + (size_t)min(j, nt - 1) * np + wrap_col(k0 - 4 + q, np)];
            vpv[u] = j < nt ? v : T(0);
        }
#pragma unroll
        for (int u = 0; u < NVT; ++u) {
            const int idx = min(tid + 256 * u, AVH * ATX - 1);
            const int q = idx / ATX, c = idx - (idx / ATX) * ATX;
            const int f = j0 - 4 + q;
            const T vf = vthf[base + (size_t)min(max(f, 1), nt - 1) * np + wrap_col(k0 + c, np)];
            const T vs = rw[min(max(f, 0), nt)].vth;
            vtv[u] = (f == 0 || f == nt) ? vs : ((f > 0 && f < nt) ? vf : T(0));
        }
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int idx = tid + 256 * u;
        if (idx < AHT * AW) tile[idx / AW][idx - (idx / AW) * AW] = sv[u];
    }
    if (tid < ATY + 1) {
        if (tid < ATY) {
            rph[tid][0] = q0;
            rph[tid][1] = q1;
            rph[tid][2] = q2;
            rph[tid][3] = q3;
        }
        rth[tid][0] = q4;
        rth[tid][1] = q5;
        rth[tid][2] = q6;
    } else if (!ATT && tid >= 64 && tid < 64 + AHT) {
        cthM[tid - 64] = q0;
        cthP[tid - 64] = q1;
    }
    // what the stage combination reads besides the fluxes (MIXED: the
    // increment of the stage input; FP64: the state fn), loaded now so the
    // flux work hides its latency
    constexpr int NO = ATY * ATX / 256;
    static_assert(NO * 256 == ATY * ATX, "whole rows of output cells per thread pass");
    T pre[NO];
    const bool need = MIXED ? (stage > 0 && time_scheme != 1)
                            : ((time_scheme == 2 && stage > 0) || (time_scheme == 0 && stage == 2));
    if (need) {
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int idx = tid + 256 * u, tj = idx / ATX, c = idx - (idx / ATX) * ATX;
            const size_t i = base + (size_t)min(j0 + tj, nt - 1) * np + min(k0 + c, np - 1);
            if constexpr (MIXED) pre[u] = fin[i];
            else pre[u] = (T)fn[i];
        }
    }
    if constexpr (ATT) {
#pragma unroll
        for (int u = 0; u < NVP; ++u) {
            const int idx = tid + 256 * u;
            if (idx < ATY * AVW) al.vp[idx / AVW][idx - (idx / AVW) * AVW] = vpv[u];
        }
#pragma unroll
        for (int u = 0; u < NVT; ++u) {
            const int idx = tid + 256 * u;
            if (idx < AVH * ATX) al.vt[idx / ATX][idx - (idx / ATX) * ATX] = vtv[u];
        }
    }
    __syncthreads();
    if constexpr (ATT) {
        // staged cell k0+tk-2 of tile row tj: faces (cell-2) .. (cell+3) are
        // vp[tj][tk .. tk+5]; its own left and right faces are tk+2, tk+3
        for (int idx = tid; idx < ATY * AW; idx += 256) {
            const int tj = idx / AW, tk = idx - (idx / AW) * AW;
            const T* v = &al.vp[tj][tk];
            T a = T(0);
            for (int m = 0; m < 6; ++m) a = fmax(a, fabs(v[m]));
            al.cpM[tj][tk] = T(0.5) * (v[2] + a);
            al.cpP[tj][tk] = T(0.5) * (v[3] - a);
        }
        // staged row j0+tr-2: faces (row-2) .. (row+3) are vt[tr .. tr+5]
        for (int idx = tid; idx < AHT * ATX; idx += 256) {
            const int tr = idx / ATX, c = idx - (idx / ATX) * ATX;
            T a = T(0);
            for (int m = 0; m < 6; ++m) a = fmax(a, fabs(al.vt[tr + m][c]));
            al.ctM[tr][c] = T(0.5) * (al.vt[tr + 2][c] + a);
            al.ctP[tr][c] = T(0.5) * (al.vt[tr + 3][c] - a);
        }
        __syncthreads();
    }

    // phi faces: face fk of tile row tj lies between cells k0+fk-1 and k0+fk
    for (int idx = tid; idx < ATY * (ATX + 1); idx += 256) {
        const int tj = idx / (ATX + 1), fk = idx - (idx / (ATX + 1)) * (ATX + 1);
        const int j = j0 + tj;
        T F = T(0);
        if (j < nt) {
            const T* t = &tile[tj + AH][fk];   // t[0..3] = cells fk-2 .. fk+1
            if constexpr (ATT) {
                const T* m = &al.cpM[tj][fk];
                const T* p = &al.cpP[tj][fk];
                if (upwind) {
                    F = upwind_face(al.vp[tj][fk + 4], t[1], t[2]);
                } else {
                    F = weno_face(t[0] * m[0], t[1] * m[1], t[2] * m[2], t[1] * p[1], t[2] * p[2],
                                  t[3] * p[3], wph);
                }
            } else {
                const T cm = rph[tj][0], cp = rph[tj][1];
                if (upwind) {
                    F = upwind_face(rph[tj][2], t[1], t[2]);
                } else {
                    F = weno_face(t[0] * cm, t[1] * cm, t[2] * cm, t[1] * cp, t[2] * cp, t[3] * cp, wph);
                }
            }
        }
        fph[tj][fk] = F;
    }
    // theta faces: face f = j0+fj lies between rows f-1 and f
    for (int idx = tid; idx < (ATY + 1) * ATX; idx += 256) {
        const int fj = idx / ATX, c = idx - (idx / ATX) * ATX;
        const int f = j0 + fj;
        T F = T(0);
        if (f > 0 && f < nt) {
            const int tc = c + AH;
            const T bm1 = tile[fj + 1][tc], b0 = tile[fj + 2][tc];   // rows f-1, f
            if (upwind || f == 1 || f == nt - 1) {
                if constexpr (ATT) F = upwind_face(al.vt[fj + 4][c], bm1, b0);
                else F = upwind_face(rth[fj][0], bm1, b0);
            } else {
                const T bm2 = tile[fj][tc], bp1 = tile[fj + 3][tc];  // rows f-2, f+1
                if constexpr (ATT) {
                    F = weno_face(bm2 * al.ctM[fj][c], bm1 * al.ctM[fj + 1][c], b0 * al.ctM[fj + 2][c],
                                  bm1 * al.ctP[fj + 1][c], b0 * al.ctP[fj + 2][c],
                                  bp1 * al.ctP[fj + 3][c], wth);
                } else {
                    F = weno_face(bm2 * cthM[fj], bm1 * cthM[fj + 1], b0 * cthM[fj + 2],
                                  bm1 * cthP[fj + 1], b0 * cthP[fj + 2], bp1 * cthP[fj + 3], wth);
                }
            }
        }
        fth[fj][c] = F;
    }
    __syncthreads();

    const T hdt = T(0.5) * (T)e.dt;
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        const int idx = tid + 256 * u, tj = idx / ATX, c = idx - (idx / ATX) * ATX;
        const int j = j0 + tj, k = k0 + c;
        if (j >= nt || k >= np) continue;
        const T dthf = adv_div(rth[tj + 1][1] * fth[tj + 1][c] - rth[tj][1] * fth[tj][c], rth[tj][2]);
        const T dphf = adv_div(fph[tj][c + 1] - fph[tj][c], rph[tj][3]);
        const T op = dthf + dphf;
        const size_t i = base + (size_t)j * np + k;
        if constexpr (MIXED) {
            const T dt = (T)e.dt;
            T d;
            if (time_scheme == 1) {
                d = -(dt * op);
            } else if (time_scheme == 2) {
                // SSPRK(3,3) in increments of fn: d1 = -dt A, d2 = d1/4 - (dt/4) A,
                // d3 = 2 d2/3 - (2 dt/3) A
                if (stage == 0) d = -(dt * op);
                else if (stage == 1) d = T(0.25) * pre[u] - (T(0.25) * dt) * op;
                else d = (T(2) / T(3)) * pre[u] - ((T(2) / T(3)) * dt) * op;
            } else if (stage == 0) {
                d = -(hdt * op);
            } else if (stage == 1) {
                d = pre[u] - hdt * op;
            } else if (stage == 2) {
                d = (T(1) / T(3)) * pre[u] - ((T(1) / T(6)) * dt) * op;
            } else {
                d = pre[u] - hdt * op;
            }
            fout[i] = d;
        } else {
            const T dt = (T)e.dt;
            const T cur = tile[tj + AH][c + AH];
            T v;
            if (time_scheme == 1) {
                v = cur - dt * op;
            } else if (time_scheme == 2) {
                // SSPRK(3,3): f1 = fn - dt A(fn), f2 = 3/4 fn + 1/4 f1 - 1/4 dt A(f1),
                // fn+1 = 1/3 fn + 2/3 f2 - 2/3 dt A(f2)
                if (stage == 0) v = cur - dt * op;
                else if (stage == 1) v = 0.75 * pre[u] + 0.25 * cur - 0.25 * dt * op;
                else v = (T(1) / T(3)) * pre[u] + (T(2) / T(3)) * cur - (T(2) / T(3)) * dt * op;
            } else if (stage == 2) {
                v = (T(2) / T(3)) * pre[u] + (T(1) / T(3)) * cur - ((T(1) / T(6)) * dt) * op;
            } else {
                v = cur - hdt * op;
            }
            fout[i] = v;
        }
    }
}

__global__ void copy_entries_kernel(const Entry* __restrict__ ents, const double* __restrict__ src,
                                    double* __restrict__ dst, size_t cells)
{
    const size_t base = (size_t)ents[blockIdx.y].r * cells;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
         i += (size_t)gridDim.x * blockDim.x)
        dst[base + i] = src[base + i];
}

// Attenuated face velocities of one advance for every entry: one thread per
// cell writes the phi face on its left and the theta face above it (row 0:
// the pole face, unattenuated).  Realizations with B0 <= 0 get factor 1.
template <typename T>
__global__ __launch_bounds__(256) void att_faces_kernel(const Entry* __restrict__ ents,
                                                        const AdvRow<double>* __restrict__ rows,
                                                        const double* __restrict__ b0s,
                                                        const double* __restrict__ fn,
                                                        T* __restrict__ vphf, T* __restrict__ vthf,
                                                        int nt, int np)
{
    const Entry e = ents[blockIdx.z];
    const int j = blockIdx.y;
    const double b0 = b0s[e.r];
    const AdvRow<double> a = rows[(size_t)e.r * (nt + 1) + j];
    const size_t row = ((size_t)e.r * nt + j) * np;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < np; k += gridDim.x * 256) {
        const double b = fabs(fn[row + k]);
        double fp = 1.0, ft = 1.0;
        if (b0 > 0.0) {
            const double bl = fabs(fn[row + (k == 0 ? np - 1 : k - 1)]);
            fp = 1.0 - tanh(0.5 * (bl + b) / b0);
            if (j > 0) ft = 1.0 - tanh(0.5 * (fabs(fn[row - np + k]) + b) / b0);
        }
        vphf[row + k] = (T)(a.vph * fp);
        vthf[row + k] = (T)(a.vth * ft);
    }
}

// CFL rate of every cell under the attenuated flow (eq. ssprk43_dt with the
// face velocities of eq. flow_attenuation for the field fn, the same factors
// att_faces_kernel forms): the larger of the cell's two theta-face speeds over
// dth plus the larger of its two phi-face speeds over sin(theta_j) dph.  Each
// block reduces the largest rate of its cells (a wavefront max, then across
// the block's waves) into partial[entry][row][block column].
__global__ __launch_bounds__(256) void att_cfl_partial_kernel(const Entry* __restrict__ ents,
                                                              const AdvRow<double>* __restrict__ rows,
                                                              const double* __restrict__ b0s,
                                                              const double* __restrict__ fn,
                                                              const double* __restrict__ den_ph, double dth,
                                                              double* __restrict__ partial, int nt, int np)
{
    __shared__ double wmax[4];
    const Entry e = ents[blockIdx.z];
    const int j = blockIdx.y;
    const double b0 = b0s[e.r];
    const double vph = rows[(size_t)e.r * (nt + 1) + j].vph;
    const double vn0 = rows[(size_t)e.r * (nt + 1) + j].vth;       // face j (above the row)
    const double vs0 = rows[(size_t)e.r * (nt + 1) + j + 1].vth;   // face j + 1 (below)
    const double den = den_ph[j];
    const size_t row = ((size_t)e.r * nt + j) * np;
    double m = 0.0;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < np; k += gridDim.x * 256) {
        const double b = fabs(fn[row + k]);
        double fw = 1.0, fe = 1.0, fnn = 1.0, fs = 1.0;
        if (b0 > 0.0) {
            const double bw = fabs(fn[row + (k == 0 ? np - 1 : k - 1)]);
            const double be = fabs(fn[row + (k == np - 1 ? 0 : k + 1)]);
            fw = 1.0 - tanh(0.5 * (bw + b) / b0);
            fe = 1.0 - tanh(0.5 * (b + be) / b0);
            if (j > 0) fnn = 1.0 - tanh(0.5 * (fabs(fn[row - np + k]) + b) / b0);
            if (j < nt - 1) fs = 1.0 - tanh(0.5 * (b + fabs(fn[row + np + k])) / b0);
        }
        const double vw = fabs(vph * fw), ve = fabs(vph * fe);
        const double vn = fabs(vn0 * fnn), vs = fabs(vs0 * fs);
        const double vt = vn > vs ? vn : vs, vp = vw > ve ? vw : ve;
        const double r = vt / dth + vp / den;
        m = r > m ? r : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double q = __shfl_xor(m, o);
        m = q > m ? q : m;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = wmax[0];
        for (int w = 1; w < 4; ++w) x = wmax[w] > x ? wmax[w] : x;
        partial[((size_t)blockIdx.z * nt + j) * gridDim.x + blockIdx.x] = x;
    }
}

// Largest CFL rate of each entry's realization from the partials: rmax[r].
__global__ __launch_bounds__(256) void att_cfl_final_kernel(const Entry* __restrict__ ents,
                                                            const double* __restrict__ partial, int nper,
                                                            double* __restrict__ rmax)
{
    __shared__ double wmax[4];
    const Entry e = ents[blockIdx.x];
    const double* p = partial + (size_t)blockIdx.x * nper;
    double m = 0.0;
    for (int i = threadIdx.x; i < nper; i += 256) m = p[i] > m ? p[i] : m;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double q = __shfl_xor(m, o);
        m = q > m ? q : m;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = wmax[0];
        for (int w = 1; w < 4; ++w) x = wmax[w] > x ? wmax[w] : x;
        rmax[e.r] = x;
    }
}

int att_cfl_blocks_per_row(int np) { return np > 1024 ? 4 : (np + 255) / 256; }

void launch_att_cfl(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                    const double* b0s, const double* fn, const double* den_ph, double dth, double* partial,
                    double* rmax, int nt, int np)
{
    const int gx = att_cfl_blocks_per_row(np);
    hipLaunchKernelGGL(att_cfl_partial_kernel, dim3(gx, nt, n_ent), dim3(256), 0, st, ents, rows, b0s, fn,
                       den_ph, dth, partial, nt, np);
    hipLaunchKernelGGL(att_cfl_final_kernel, dim3(n_ent), dim3(256), 0, st, ents, partial, gx * nt, rmax);
}

void launch_adv_stage_f64(hipStream_t st, const Entry* ents, int n_ent, int stage, int time_scheme,
                          int upwind, const AdvRow<double>* rows, Geom<double> g,
                          WenoConst<double> wth, WenoConst<double> wph, const double* fn,
                          const double* fin, double* fout, int nt, int np)
{
    dim3 grid((np + ATX - 1) / ATX, (nt + PLAIN_TY - 1) / PLAIN_TY, n_ent);
    hipLaunchKernelGGL((adv_stage_kernel<double, false, false, PLAIN_TY>), grid, dim3(256), 0, st, ents, stage,
                       time_scheme, upwind, rows, g, wth, wph, fn, fin, fout, nullptr, nullptr, nt,
                       np);
}

void launch_adv_stage_mixed(hipStream_t st, const Entry* ents, int n_ent, int stage, int time_scheme,
                            int upwind, const AdvRow<float>* rows, Geom<float> g,
                            WenoConst<float> wth, WenoConst<float> wph, double* fn,
                            const float* din, float* dout, int nt, int np)
{
    dim3 grid((np + ATX - 1) / ATX, (nt + PLAIN_TY - 1) / PLAIN_TY, n_ent);
    hipLaunchKernelGGL((adv_stage_kernel<float, true, false, PLAIN_TY>), grid, dim3(256), 0, st, ents, stage,
                       time_scheme, upwind, rows, g, wth, wph, fn, din, dout, nullptr, nullptr, nt, np);
}

void launch_att_faces_f64(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                          const double* b0s, const double* fn, double* vphf, double* vthf, int nt,
                          int np)
{
    dim3 grid((np + 255) / 256, nt, n_ent);
    hipLaunchKernelGGL((att_faces_kernel<double>), grid, dim3(256), 0, st, ents, rows, b0s, fn, vphf,
                       vthf, nt, np);
}

void launch_att_faces_f32(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                          const double* b0s, const double* fn, float* vphf, float* vthf, int nt,
                          int np)
{
    dim3 grid((np + 255) / 256, nt, n_ent);
    hipLaunchKernelGGL((att_faces_kernel<float>), grid, dim3(256), 0, st, ents, rows, b0s, fn, vphf,
                       vthf, nt, np);
}

void launch_adv_stage_att_f64(hipStream_t st, const Entry* ents, int n_ent, int stage,
                              int time_scheme, int upwind, const AdvRow<double>* rows,
                              Geom<double> g, WenoConst<double> wth, WenoConst<double> wph,
                              const double* fn, const double* fin, double* fout, const double* vphf,
                              const double* vthf, int nt, int np)
{
    dim3 grid((np + ATX - 1) / ATX, (nt + ATT_TY - 1) / ATT_TY, n_ent);
    hipLaunchKernelGGL((adv_stage_kernel<double, false, true, ATT_TY>), grid, dim3(256), 0, st, ents, stage,
                       time_scheme, upwind, rows, g, wth, wph, fn, fin, fout, vphf, vthf, nt, np);
}

void launch_adv_stage_att_mixed(hipStream_t st, const Entry* ents, int n_ent, int stage,
                                int time_scheme, int upwind, const AdvRow<float>* rows,
                                Geom<float> g, WenoConst<float> wth, WenoConst<float> wph,
                                double* fn, const float* din, float* dout, const float* vphf,
                                const float* vthf, int nt, int np)
{
    dim3 grid((np + ATX - 1) / ATX, (nt + ATT_TY - 1) / ATT_TY, n_ent);
    hipLaunchKernelGGL((adv_stage_kernel<float, true, true, ATT_TY>), grid, dim3(256), 0, st, ents, stage,
                       time_scheme, upwind, rows, g, wth, wph, fn, din, dout, vphf, vthf, nt, np);
}

void launch_copy_f64(hipStream_t st, const Entry* ents, int n_ent, const double* src, double* dst,
                     size_t cells)
{
    int bx = (int)((cells + 255) / 256);
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(copy_entries_kernel, dim3(bx, n_ent), dim3(256), 0, st, ents, src, dst, cells);
}

}  // namespace sft
