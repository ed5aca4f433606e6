// Internal launchers of random flux emergence (Sec. "Flux emergence").  Not
// part of the public ABI.
#pragma once

#include "sft_internal.h"

namespace sft {

// Map k of every realization r of a class goes to slot k & 1 (S0 or S1,
// [R][nt][np] FP64 each).  The map index is kdev[0] + koff when kdev is
// non-null (the device's interval counter), else kabs.
//
// Only realizations r with r % nl == lane take part (lane < 0: all).
//
// Draw (not balanced) map k: standard normals from Philox4x32-10 at counter
// (cell pair, k low, k high, 0) and key (seed, first_id + r), Box-Muller,
// times scale_row[j]; per-block FP64 sums of S w_j over S > 0 and S < 0 into
// partial[r][nblk][2], then ratio[r] = sqrt|Phi+ / Phi-| in a fixed order (0
// when either sum is zero).
int rfe_gen_blocks(int nt, int np);
void launch_rfe_gen(hipStream_t st, int R, int nl, int lane, int first_id, uint32_t seed,
                    const int64_t* kdev, int koff, int64_t kabs, const double* scale_row,
                    const double* w_row, double* S0, double* S1, double* partial, double* ratio, int nt,
                    int np);
// Eq. fluxbal on map k: S / ratio[r] where S > 0, S * ratio[r] where S < 0
// (unchanged where ratio[r] = 0).
void launch_rfe_balance(hipStream_t st, int R, int nl, int lane, const int64_t* kdev, int koff,
                        int64_t kabs, const double* ratio, double* S0, double* S1, int nt, int np);
// kdev[0] = k (set) or kdev[0] += 1 (tick); one thread.
void launch_rfe_set(hipStream_t st, int64_t* kdev, int64_t k);
void launch_rfe_tick(hipStream_t st, int64_t* kdev);
// Source sub-advance for every entry e: B_r += e.dt ((1 - a) S_k + a S_k+1),
// a = alpha[e.coef_off], k = kdev[0]; infinite lifetime: B_r += e.dt S_0.
void launch_rfe_apply(hipStream_t st, const Entry* ents, int n_ent, const double* alpha,
                      const int64_t* kdev, int infinite, const double* S0, const double* S1, double* B,
                      size_t cells);

}  // namespace sft
