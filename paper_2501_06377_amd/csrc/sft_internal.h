// Internal declarations shared by the host scheduler and the HIP kernels of
// the surface-flux-transport library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sft {

// One realization taking part in one phase (advection step or diffusion
// call) of an advance plan.  Entries of a diffusion phase are sorted by
// descending stage count, so the realizations still active at stage j are a
// prefix of the list.
struct Entry {
    int32_t r;         // realization index inside its grid class
    int32_t s;         // diffusion stages of this call (0 for advection phases)
    int32_t coef_off;  // offset of stage j's coefficients: coefs[coef_off + j]
    int32_t pad;
    double dt;         // step (advection) or call length (diffusion), hours
};

// XCD-aware tile order of a 1-D launch over gx * gy * (number of entries)
// tiles.  The hardware deals consecutive workgroups to the 8 XCDs in turn;
// renumbering gives each XCD a contiguous run of tiles (x fastest, then y,
// then the entry), so the halos that neighbouring tiles share are fetched
// into that XCD's L2 once.  A bijection on [0, gridDim.x): correct under any
// dispatch order, only the locality depends on it.
__device__ __forceinline__ void xcd_tile(int gx, int gy, int& bx, int& by, int& bz)
{
    const int nb = gridDim.x, id = blockIdx.x;
    const int xcd = id & 7, pos = id >> 3, q = nb >> 3, rm = nb & 7;
    const int nid = (xcd < rm ? xcd * (q + 1) : rm * (q + 1) + (xcd - rm) * q) + pos;
    bx = nid % gx;
    by = (nid / gx) % gy;
    bz = nid / (gx * gy);
}

// Coefficients of diffusion stage j of one call:
//   Y_j = mu Y_{j-1} + nu Y_{j-2} + cy0 Y0 + cL L(Y_{j-1}) + cLY0 L(Y0)
// (stage 1: Y_1 = Y0 + cL L(Y0)).  cL = mut_j tau, cLY0 = gamt_j tau.
struct StageCoef {
    double mu, nu, cy0, cL, cLY0;
};

// Per-row advection constants of one realization (row j of nt, plus the
// theta face j): LLF split factors LP = B*cP, LM = B*cM for the theta and phi
// sweeps, and the face velocity used by the upwind faces.
template <typename T>
struct AdvRow {
    T cthP, cthM;   // theta sweep: 0.5 (v_{j+1/2} - alpha_j), 0.5 (v_{j-1/2} + alpha_j)
    T cphP, cphM;   // phi sweep (v_phi constant along the row)
    T vth;          // v_theta on the face j (top face of row j)
    T vph;          // v_phi of row j
    T pad0, pad1;
};

// Per-row diffusion coefficients of one realization (eq. diffusion_matrix).
template <typename T>
struct DiffRow {
    T up, dn, ph, d;
};

// Uniform-grid WENO factors of one sweep direction (App. B D factors with
// equal widths x: x/(x+x), x/(x+x+x), (x+x)/(x+x+x)) and eps_w = x.
template <typename T>
struct WenoConst {
    T half, third, twothird, eps;
};

// Geometry of a grid class.
template <typename T>
struct Geom {
    const T* sf;      // sin at theta faces [nt+1], 0 at the poles
    const T* den_th;  // sin(theta_j) dth [nt]
    const T* den_ph;  // sin(theta_j) dph [nt]
};

struct DiagRec {     // device-side analysis partial / record (FP64)
    double pp, pm, h1, h2, dax, bmin, bmax, babs, nonfinite, pad;
};

// ---------------------------------------------------------------- launchers
// Advection: one SSPRK(4,3) (or forward Euler) stage for every entry.
//   FP64:   fin -> fout, stage 2 also reads fn (the state)
//   mixed:  FP32 increments d: value = (float)(fn + din); dout written; the
//           last stage writes the FP64 state.
void launch_adv_stage_f64(hipStream_t st, const Entry* ents, int n_ent, int stage, int time_scheme,
                          int upwind, const AdvRow<double>* rows, Geom<double> g,
                          WenoConst<double> wth, WenoConst<double> wph, const double* fn,
                          const double* fin, double* fout, int nt, int np);
void launch_adv_stage_mixed(hipStream_t st, const Entry* ents, int n_ent, int stage, int time_scheme,
                            int upwind, const AdvRow<float>* rows, Geom<float> g,
                            WenoConst<float> wth, WenoConst<float> wph, double* fn,
                            const float* din, float* dout, int nt, int np);
void launch_copy_f64(hipStream_t st, const Entry* ents, int n_ent, const double* src, double* dst,
                     size_t cells);

// Diffusion.
//   FP64 paper form: ly0 = L(B); y1 = B + cL1 ly0 (stage 1); stage j >= 2
//   writes `out`, or B for an entry whose last stage it is.
void launch_diff_first_f64(hipStream_t st, const Entry* ents, int n_ent, const StageCoef* coefs,
                           const DiffRow<double>* drow, const double* B, double* ly0, double* y1,
                           double* y0copy, int nt, int np);
void launch_diff_stage_f64(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs,
                           int j, const DiffRow<double>* drow, double* B, const double* ym1,
                           const double* ym2, const double* ly0, double* out, int nt, int np);
//   FP32 increment form: Y0 = B (+ adv when Entry.pad), ly0 = (float)L(Y0) in
//   FP64 arithmetic, d1 = cL1 ly0; stage j writes d_j, or B = Y0 + d_s.
void launch_diff_first_mixed(hipStream_t st, const Entry* ents, int n_ent, const StageCoef* coefs,
                             const DiffRow<double>* drow64, const double* B, const float* adv,
                             float* ly0, float* d1, int nt, int np);
void launch_diff_stage_mixed(hipStream_t st, const Entry* ents, int n_act, const StageCoef* coefs,
                             int j, const DiffRow<double>* drow, double* B, const float* adv,
                             const float* din, const float* ein, const float* ly0, float* dout,
                             float* eout, int nt, int np);
//   Temporally blocked stages j0 .. j0+K-1 (K of tile configuration cfg).
//   in1/in2/ly0/out1/out2 are double (FP64) or float (mixed) arrays; y0 is the
//   FP64 copy of Y0 (paper form only).
int fused_config_count(bool mixed);
int fused_config_k(bool mixed, int cfg);
// Whether the shape reads L(Y0) from memory (FP64 strip shapes compute it
// from the staged Y0).
bool fused_config_reads_ly0(bool mixed, int cfg);
void fused_config_desc(bool mixed, int cfg, int* tx, int* ty, int* k, int* nthr);
void launch_diff_fused(hipStream_t st, bool mixed, int cfg, const Entry* ents, int n_act,
                       const StageCoef* coefs, int j0, const void* drow, const void* in1,
                       const void* in2, const double* y0, const void* ly0, void* out1, void* out2,
                       double* B, const float* adv, int nt, int np);
//   FP32 increment form, blocked (k_diffusion_mixed.hip): configurations
//   0 .. mixed_config_count() - 1 of launch_diff_fused(mixed = true).
int mixed_config_count();
int mixed_config_k(int cfg);
void mixed_config_desc(int cfg, int* tx, int* ty, int* k, int* nthr);
void launch_diff_mixed_blocked(hipStream_t st, int cfg, const Entry* ents, int n_act, const StageCoef* coefs,
                               int j0, const DiffRow<double>* drow, const float* in1, const float* in2,
                               const float* ly0, float* out1, float* out2, double* B, const float* adv, int nt,
                               int np);
//   B = B (+ adv when Entry.pad) (+ d when d != NULL), per entry.
void launch_mixed_close(hipStream_t st, const Entry* ents, int n_ent, double* B, const float* adv,
                        const float* d, size_t cells);

// Assimilation (grid class with R realizations).
struct AssimReal {        // per realization
    double alpha, mu_lim, lat_lim_rad;
    int32_t balance;
    int32_t pad;
};
void launch_assim_delta(hipStream_t st, int R, const AssimReal* ar, const void* data,
                        const void* weight, int dtype, int kind, double sb0, double cb0, double l0,
                        const double* B, const double* st_row, const double* ct_row,
                        const double* lat_row, const double* w_row, double* dB, double* partial,
                        int nblk, int nt, int np);
void launch_assim_reduce(hipStream_t st, int R, const double* partial, int nblk, double* ratio);
void launch_assim_apply(hipStream_t st, int R, const AssimReal* ar, const void* data,
                        const void* weight, int dtype, int kind, double sb0, double cb0, double l0,
                        double* B, const double* dB, const double* ratio, const double* st_row,
                        const double* ct_row, const double* lat_row, int nblk, int nt, int np);

// Diagnostics: per-block partials then one fixed-order reduction per realization.
void launch_diag(hipStream_t st, int R, const double* B, const double* st_row, const double* ct_row,
                 const double* w_row, const double* sph, const double* cph, DiagRec* partial,
                 int nblk, DiagRec* out, int nt, int np);

// Conversions.
void launch_f32_to_f64(hipStream_t st, const float* src, double* dst, size_t n);
void launch_f64_to_f32(hipStream_t st, const double* src, float* dst, size_t n);

}  // namespace sft
