// Internal launchers of the attenuated-flow advection path (eq.
// flow_attenuation).  Not part of the public ABI.
#pragma once

#include "sft_internal.h"

namespace sft {

// Face velocities of one advection advance for every entry, from the state fn
// at the start of the advance: vphf[r][j][k] = v_phi(row j) * att on the phi
// face between cells k-1 and k, vthf[r][j][k] = v_theta(face j) * att on the
// theta face between rows j-1 and j (row 0: the pole face, unattenuated);
// att = 1 - tanh(0.5 (|B_a| + |B_b|) / B0) over the face's cells a, b, and 1
// where b0s[r] <= 0.
void launch_att_faces_f64(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                          const double* b0s, const double* fn, double* vphf, double* vthf, int nt,
                          int np);
void launch_att_faces_f32(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                          const double* b0s, const double* fn, float* vphf, float* vthf, int nt,
                          int np);

// Per-step CFL of the attenuated flow (eq. ssprk43_dt on the face speeds of
// eq. flow_attenuation for the field fn): rmax[r] receives, for each entry's
// realization r, the largest over its cells of max(theta-face speeds)/dth +
// max(phi-face speeds)/(sin(theta) dph); the limit is 1/rmax.  partial holds
// n_ent * nt * att_cfl_blocks_per_row(np) doubles of scratch.
int att_cfl_blocks_per_row(int np);
void launch_att_cfl(hipStream_t st, const Entry* ents, int n_ent, const AdvRow<double>* rows,
                    const double* b0s, const double* fn, const double* den_ph, double dth, double* partial,
                    double* rmax, int nt, int np);

// Advection stages as launch_adv_stage_f64 / launch_adv_stage_mixed, with the
// face velocities (and the LLF split factors built from them) taken from
// vphf / vthf.
void launch_adv_stage_att_f64(hipStream_t st, const Entry* ents, int n_ent, int stage,
                              int time_scheme, int upwind, const AdvRow<double>* rows,
                              Geom<double> g, WenoConst<double> wth, WenoConst<double> wph,
                              const double* fn, const double* fin, double* fout, const double* vphf,
                              const double* vthf, int nt, int np);
void launch_adv_stage_att_mixed(hipStream_t st, const Entry* ents, int n_ent, int stage,
                                int time_scheme, int upwind, const AdvRow<float>* rows,
                                Geom<float> g, WenoConst<float> wth, WenoConst<float> wph,
                                double* fn, const float* din, float* dout, const float* vphf,
                                const float* vthf, int nt, int np);

}  // namespace sft
