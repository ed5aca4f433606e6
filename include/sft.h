/*
 * sft.h -- C ABI of the MI355X (gfx950) surface-flux-transport library.
 *
 * The library steps the radial photospheric field B_r(theta, phi) of many
 * ensemble realizations at once through the split operators of the HipFT
 * paper (Caplan et al., "Open-source Flux Transport I: HipFT"):
 *   - advection by differential rotation and meridional flow
 *     (eq. advection, eq. dr, eq. mf; WENO3-CS(h) fluxes of App. B with the
 *     upwind pole rows and finite-volume pole closure of App. A;
 *     SSPRK(4,3), SSPRK(3,3) or forward-Euler time stepping, Sec.
 *     "Advection temporal schemes"),
 *   - surface diffusion (eq. diffusion, eq. diffusion_matrix) advanced by
 *     super time stepping (RKG2(3/2) default, RKL2, or forward Euler,
 *     Sec. "Diffusion temporal schemes"),
 *   - data assimilation (eq. data_assim, eq. data_assim_f, with the optional
 *     flux balance of eqs. data_assim_deltab / fluxbal),
 *   - FP64 analysis reductions (Sec. "Analysis").
 * Steps are operator split without (eq. num_opsplit_nostrang, the default)
 * or with Strang splitting (eq. num_opsplit_strang); assimilation happens at
 * the end of an advance.
 *
 * Grid: uniform cell-centred finite-volume grid of the unit sphere, nt rows
 * in colatitude (theta_j = (j+1/2) pi/nt) and np periodic columns in
 * longitude (phi_k = (k+1/2) 2 pi/np).  A field of one realization is nt*np
 * values, row-major, phi contiguous: B[j*np + k].  A grid class holds R
 * realizations stored back to back: B[(r*nt + j)*np + k].
 *
 * Units at the boundary are the paper's input units (Sec. "Units"):
 * diffusivity km^2/s, flow coefficients m/s, field gauss, time hours,
 * angles degrees.  Internally lengths are solar radii (6.96e8 m).
 *
 * Conventions for every call:
 *  - Status codes only; nothing throws across the ABI.  sft_last_error()
 *    returns a text description of the last failure on a context.
 *  - The caller owns every pointer it passes; pointers are borrowed for the
 *    duration of the call.  Device pointers (on_device = 1) must live on the
 *    context's device; the library reads/writes them in stream order on the
 *    context's stream, so the caller must keep them alive until that stream
 *    has passed the call.  Host pointers are read/written before the call
 *    returns.
 *  - A context is single-threaded: calls on one context must not overlap.
 *    Several contexts may coexist.
 *  - All work is enqueued on the context's HIP stream; only calls that
 *    return host data (sft_get_state to host memory, sft_diagnostics,
 *    sft_sync) wait for it.
 */
#ifndef SFT_H
#define SFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sft_status;
#define SFT_OK 0
#define SFT_ERR_ARG (-1)          /* invalid argument value or null pointer      */
#define SFT_ERR_SHAPE (-2)        /* array shape does not match the grid         */
#define SFT_ERR_OOM (-3)          /* device or host allocation failed            */
#define SFT_ERR_HIP (-4)          /* a HIP runtime call failed                   */
#define SFT_ERR_NOT_FINITE (-5)   /* the field holds NaN or Inf                  */
#define SFT_ERR_STATE (-6)        /* call not valid in the context's state       */
#define SFT_ERR_UNSUPPORTED (-7)  /* option combination not implemented          */

/* precision */
#define SFT_FP64 0          /* every stencil and reduction in FP64                */
#define SFT_FP32_MIXED 1    /* FP32 stencil arithmetic, FP64 state and reductions */
/* advection spatial scheme */
#define SFT_WENO3CSH 0
#define SFT_UPWIND 1
/* advection time scheme */
#define SFT_SSPRK43 0
#define SFT_FE 1
#define SFT_SSPRK33 2
/* diffusion time scheme */
#define SFT_RKG2 0
#define SFT_RKL2 1
#define SFT_DIFF_FE 2
/* element types of state / observation arrays */
#define SFT_DTYPE_F64 0
#define SFT_DTYPE_F32 1
/* meaning of the weight array passed to sft_assimilate */
#define SFT_WEIGHT_F 0      /* the assimilation weight F itself (eq. data_assim)              */
#define SFT_WEIGHT_MU 1     /* mu = cos(disk-centre angle); F from eq. data_assim_f            */
#define SFT_WEIGHT_DISK 2   /* no array: mu from the observer's (b0, l0), then eq. data_assim_f */

typedef struct {
    int32_t precision;    /* SFT_FP64 (default) or SFT_FP32_MIXED                          */
    int32_t adv_scheme;   /* SFT_WENO3CSH (default) or SFT_UPWIND                          */
    int32_t adv_time;     /* SFT_SSPRK43 (default), SFT_FE or SFT_SSPRK33                  */
    int32_t diff_time;    /* SFT_RKG2 (default), SFT_RKL2 or SFT_DIFF_FE                   */
    double cfl_safety;    /* safety factor on the flow CFL limit (default 0.9)             */
    double dt_max;        /* upper bound on a step, hours; 0 = none (default)              */
    double ptl_dt;        /* > 0 splits each diffusion advance into ceil(dt/ptl_dt) calls  */
    int32_t use_graphs;   /* 1 = capture each distinct advance plan in a HIP graph         */
    int32_t sts_fuse;     /* 0 (default) = temporally blocked STS stages, tile shape
                             picked per grid class by the built-in autotuner;
                             1 = one stage per kernel launch                          */
    int32_t diag_every_call; /* 1 (default) = refresh diagnostics after advance/assimilate */
    int32_t sts_tile;     /* -1 (default) = autotune; >= 0 forces a blocked tile shape
                             (index into the library's table; see sft_tile_info)      */
    int32_t strang;       /* 0 (default) = eq. num_opsplit_nostrang; 1 = Strang splitting
                             (eq. num_opsplit_strang): advection over dt/2, diffusion
                             over dt, advection over dt/2, with the CFL limit of the
                             step doubled                                               */
    int32_t rfe_model;    /* random flux emergence (Sec. "Flux emergence"): 0 (default) = none,
                             1 = eq. rfe_m1 maps (unsigned flux per cell), 2 = eq. rfe_m2
                             maps (unsigned flux per unit area)                         */
    uint32_t rfe_seed;    /* key word 0 of every source map's generator; key word 1 is
                             the realization id                                         */
    int32_t lanes;        /* concurrent sub-batches per grid class, 0..16: realizations
                             r with r mod lanes = l advance on stream l (the context's
                             stream for l = 0, library streams for the others, joined
                             before the call returns), so one sub-batch's launches fill
                             the GPU while another's drain; 0 (default) = min(2, R),
                             1 = all on the context's stream; results do not depend on it */
    double rfe_phi_hr;    /* total unsigned flux per hour of a source map, Mx (> 0 when
                             rfe_model != 0)                                            */
    double rfe_lifetime_h;/* time between source maps tau, hours; 0 = infinite (one map) */
    double dt_min;        /* minimum step, hours (Sec. "Time steps" lists a minimum and a
                             maximum step among the user's controls): the step limit
                             min(cfl_safety * CFL, dt_max) is raised to dt_min, which
                             overrides the flow's stability limit; a step still ends on
                             t_end.  0 (default) = none                                 */
    int32_t att_cfl;      /* 0 (default): with flow attenuation the step keeps the
                             unattenuated flow's CFL limit (an upper bound of the
                             attenuated speeds, so one plan per interval length);
                             1: each step of an attenuated realization takes eq.
                             ssprk43_dt of the attenuated flow of the field at the start
                             of the step (a device max-reduction read back per step;
                             no graphs for such advances; not with rfe_model != 0)   */
    int32_t reserved0;
} sft_options;

/* Per-realization parameters (Sec. "Multiple Realizations"). */
typedef struct {
    double nu_km2_s;      /* diffusivity (eq. diffusion), scalar per realization, >= 0   */
    double d0, d2, d4;    /* differential rotation, eq. dr, m/s                          */
    double m1, m3, m5;    /* meridional flow, eq. mf, m/s                                */
    double alpha_mu;      /* weight exponent alpha_mu of eq. data_assim_f                */
    double mu_lim;        /* mu limit of eq. data_assim_f                                */
    double lat_lim_deg;   /* latitude limit of eq. data_assim_f, degrees                 */
    int32_t flux_balance; /* 1 = balance the assimilation increment (eq. fluxbal)        */
    int32_t reserved;
    double att_b0;        /* flow attenuation (eq. flow_attenuation): saturation field B0
                             in gauss, 0 = no attenuation, else > 0.  Each advection
                             advance scales every face velocity by 1 - tanh(m / B0), m
                             the mean of |B| over the face's two cells of the field at
                             the start of the advance; the step length keeps the
                             unattenuated flow's CFL limit (the factor is <= 1)        */
    double nu_grid_alpha; /* flux-preserving smoother (eq. diffgrid): > 0 replaces nu_km2_s
                             by the grid diffusivity alpha [dth^2 + (dph sin theta)^2] at
                             the cell corners, alpha in 1/h (R_sun^2/h on the unit
                             sphere); 0 = scalar nu_km2_s                             */
} sft_params;

/* Analysis record of one realization (Sec. "Analysis"); FP64 reductions. */
typedef struct {
    double t;             /* context time of the record, hours                     */
    double dt_last;       /* last step length used, hours                          */
    int64_t steps;        /* split steps taken since creation                      */
    int64_t stages;       /* stencil stage applications since creation             */
    double phi_pos, phi_neg, phi_net; /* flux integrals of B dOmega (G sr)         */
    double h1, h2, dax;   /* equatorial (h1, h2) and axial (D) dipole strengths    */
    double bmin, bmax, babs_min;
    int32_t nonfinite;    /* number of cells holding NaN or Inf                    */
    int32_t pad;
    int64_t surr_accept, surr_reject;  /* surrogate intervals accepted / rejected  */
} sft_diag;

typedef struct sft_ctx sft_ctx;   /* opaque; owns every internal device buffer */

/* Fills *opt with the defaults listed above.  Errors: SFT_ERR_ARG if opt is NULL. */
sft_status sft_options_default(sft_options* opt);

/* Creates a context on the current HIP device (Sec. "Inputs": the run's
 * parameters; the options are the user choices of Sec. "Time steps",
 * "Operator splitting", "Advection temporal schemes", "Diffusion temporal
 * schemes" and "Flux emergence").  hip_stream is a hipStream_t
 * the context enqueues all work on; the context does not own it.  With NULL
 * the context creates (and later destroys) its own blocking stream, which is
 * ordered with the null stream.  opt may be NULL for the defaults.  On success *ctx receives the
 * handle and the context time is 0 h.  Errors: SFT_ERR_ARG (bad option value),
 * SFT_ERR_HIP, SFT_ERR_OOM. */
sft_status sft_create(sft_ctx** ctx, const sft_options* opt, void* hip_stream);

/* Adds a grid class of nt x np cells (Sec. "Grid": resolution is fixed per
 * map and every input map must match it).  nt >= 8, np >= 8, np even.
 * *grid_id receives the class index.  Allowed only before the first advance.
 * Errors: SFT_ERR_ARG, SFT_ERR_STATE. */
sft_status sft_add_grid(sft_ctx* ctx, int32_t ntheta, int32_t nphi, int32_t* grid_id);

/* Adds n realizations with parameters prm[0..n-1] to a grid class (Sec.
 * "Multiple Realizations").  Their fields start at zero.  *first_id receives
 * the global id of the first one; ids are consecutive.  Allocates the class's
 * device memory.  Allowed only before the first advance.
 * Errors: SFT_ERR_ARG (negative diffusivity, bad limits), SFT_ERR_STATE,
 * SFT_ERR_OOM. */
sft_status sft_add_realizations(sft_ctx* ctx, int32_t grid_id, int32_t n, const sft_params* prm,
                                int32_t* first_id);

/* Copies one realization's field in (set) or out (get): the radial field B_r
 * of eq. main_model in gauss on the grid of Sec. "Grid" (Sec. "Inputs": the
 * initial map; Sec. "Outputs": the maps written during and after a run; a
 * map must match the run's resolution).  br points to nt*np
 * values of dtype SFT_DTYPE_F64 or SFT_DTYPE_F32, on the device when
 * on_device = 1, else in host memory.  Errors: SFT_ERR_ARG (bad id/dtype,
 * NULL), SFT_ERR_HIP. */
sft_status sft_set_state(sft_ctx* ctx, int32_t real_id, const void* br, int32_t dtype,
                         int32_t on_device);
sft_status sft_get_state(sft_ctx* ctx, int32_t real_id, void* br_out, int32_t dtype,
                         int32_t on_device);

/* The same for all R realizations of a grid class at once: br holds R*nt*np
 * values in the class layout [r][j][k]. */
sft_status sft_set_states(sft_ctx* ctx, int32_t grid_id, const void* br, int32_t dtype,
                          int32_t on_device);
sft_status sft_get_states(sft_ctx* ctx, int32_t grid_id, void* br_out, int32_t dtype,
                          int32_t on_device);

/* Advances every realization from the context time t to t_end (hours),
 * landing exactly on t_end (Sec. "Time steps": each realization takes steps
 * dt = min(t_end - t, max(min(cfl_safety * flow CFL limit, dt_max), dt_min));
 * a step that would leave less than 1e-10 h is stretched to t_end).  Each step applies
 * advection then diffusion (eq. num_opsplit_nostrang), or with opt.strang
 * half an advection, the diffusion and the other half (eq.
 * num_opsplit_strang, CFL limit doubled).
 * With opt.rfe_model != 0 (random flux emergence, Sec. "Flux emergence"):
 * source map k of realization id belongs to time k tau (tau =
 * opt.rfe_lifetime_h; with tau = 0 only map 0 exists); its standard normal
 * draws come from the Philox4x32-10 generator (Salmon et al. 2011) at counter
 * (cell pair index, k low word, k high word, 0) and key (opt.rfe_seed, id) by
 * the Box-Muller transform, scaled by eq. rfe_m1 or rfe_m2 and flux balanced
 * (eq. fluxbal), so a map is a pure function of (seed, id, k).  Steps also
 * land on the map times k tau (the interval is cut there and each piece takes
 * the rule above); the source S(t) of eq. rfe_s closes every step (B += dt
 * S(t_mid), the exact integral of the linear interpolant), or opens and
 * closes it over dt/2 each under Strang splitting.  The maps are FP64 in both
 * precisions and are regenerated on the device whenever a step ends on a map
 * time.  Stream-ordered; does
 * not wait for the GPU.  Errors: SFT_ERR_ARG (t_end < t), SFT_ERR_STATE (no
 * realizations), SFT_ERR_HIP. */
sft_status sft_advance(sft_ctx* ctx, double t_end_hours);

/* Assimilates an observed map into every realization of a grid class at the
 * current time (eq. data_assim, eq. data_assim_f, eqs. data_assim_deltab and
 * fluxbal when a realization's flux_balance is set).
 *   data     nt*np observed field values (gauss), dtype SFT_DTYPE_F64/F32;
 *   weight   nt*np values of the same dtype: F itself (SFT_WEIGHT_F) or mu
 *            (SFT_WEIGHT_MU); ignored (may be NULL) for SFT_WEIGHT_DISK, where
 *            mu is the cosine of the angle between a cell and the disk centre
 *            of an observer at latitude b0_deg and longitude l0_deg;
 *   F from mu: F = mu^alpha_mu where mu > mu_lim and |latitude| < lat_lim,
 *            else 0, with each realization's own parameters.
 * Flux sums of the balance are FP64 and deterministic.  Stream-ordered.
 * Errors: SFT_ERR_ARG, SFT_ERR_HIP. */
sft_status sft_assimilate(sft_ctx* ctx, int32_t grid_id, const void* data, const void* weight,
                          int32_t dtype, int32_t weight_kind, double b0_deg, double l0_deg,
                          int32_t on_device);

/* The same assimilation as sft_assimilate (the same bits), for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It allocates nothing: data and
 * weight must be device arrays on the context's device (no host staging),
 * the flux-balance partial sums and ratios live in a 2 MiB device scratch
 * array that the library holds per GPU (no stored increment: the apply pass
 * forms it again), and the analysis record is left to sft_diagnostics.  A
 * grid class needs R x (2 nblk + 1) <= 262144 scratch doubles (nblk =
 * min(512, ceil(cells / 256)): about 255 realizations at 512 x 1024 and
 * above), else SFT_ERR_ARG.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (other streams or threads) race.
 * Stream-ordered.  Errors: SFT_ERR_ARG, SFT_ERR_STATE, SFT_ERR_HIP. */
sft_status sft_assimilate_noalloc(sft_ctx* ctx, int32_t grid_id, const void* data, const void* weight,
                                  int32_t dtype, int32_t weight_kind, double b0_deg, double l0_deg);

/* Returns the latest analysis record of one realization (computed in FP64 on
 * the device after the last advance/assimilate, or now if none is pending).
 * Waits for the stream.  Returns SFT_ERR_NOT_FINITE (with *out filled) when
 * the field holds NaN or Inf.  Errors: SFT_ERR_ARG, SFT_ERR_HIP. */
sft_status sft_diagnostics(sft_ctx* ctx, int32_t real_id, sft_diag* out);

/* Context time in hours (Sec. "Units": time in hours; Sec. "Time steps":
 * every advance ends exactly on its t_end).  Errors: SFT_ERR_ARG. */
sft_status sft_time(sft_ctx* ctx, double* t_hours);

/* Sets the context time (hours) without touching the fields: with
 * sft_set_state(s) this restores a checkpoint taken with sft_get_state(s) and
 * sft_time. */
sft_status sft_set_time(sft_ctx* ctx, double t_hours);

/* Waits for all work enqueued by the context. */
sft_status sft_sync(sft_ctx* ctx);

/* Work counters of one realization since the context was created: split
 * steps, diffusion stages (operator applications of the STS or Euler
 * stages), advection stages (flux-divergence evaluations) and assimilation
 * passes.  Any output pointer may be NULL.  Errors: SFT_ERR_ARG. */
sft_status sft_counts(sft_ctx* ctx, int32_t real_id, int64_t* steps, int64_t* stages,
                      int64_t* adv_stages, int64_t* assim);

/* ------------------------------------------------------------------------
 * Learned surrogate of one 1-hour transport interval (no counterpart in the
 * paper; its plain solver above is both the fallback and the arbiter of its error).
 * Network: five 3x3 convolutions 6 -> 64 -> 64 -> 64 -> 64 -> 1 on the
 * sphere (longitude wraps; the ghost row beyond a pole is the pole row
 * shifted by half a turn), ReLU after the first four, input channels
 * (B/500 G, three per-sample parameter features, cos theta, sin theta),
 * output y with B_next = B + 5 G * y.  BF16 operands on the matrix cores
 * with FP32 accumulation, FP32 master weights, MSE loss on
 * (B_target - B)/5 G, Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Parameter vector (FP32): for each layer W[c_out][c_in][3][3] then b[c_out].
 * ------------------------------------------------------------------------ */
typedef struct sft_net sft_net;

/* Creates a network for nt x np fields and batches of up to max_batch
 * samples (device memory ~0.6 GB per sample at 512 x 1024).  Parameters
 * start at zero (load them with sft_net_set_params).  hip_stream as in
 * sft_create.  Errors: SFT_ERR_ARG, SFT_ERR_OOM, SFT_ERR_HIP. */
sft_status sft_net_create(sft_net** net, int32_t ntheta, int32_t nphi, int32_t max_batch,
                          void* hip_stream);
sft_status sft_net_param_count(const sft_net* net, int64_t* n);
/* Copies the FP32 parameter vector in / out (host or device memory); setting
 * parameters resets the Adam moments. */
sft_status sft_net_set_params(sft_net* net, const float* params, int32_t on_device);
sft_status sft_net_get_params(sft_net* net, float* params, int32_t on_device);
/* Gradient vector of the last training step (same layout as the parameters). */
sft_status sft_net_get_grads(sft_net* net, float* grads, int32_t on_device);
/* Forward pass on device arrays: b_in [batch][nt][np] (dtype F64 or F32),
 * feats [batch][3] FP32, y [batch][nt][np] FP32 (may be NULL). */
sft_status sft_net_forward(sft_net* net, int32_t batch, const void* b_in, int32_t dtype,
                           const float* feats, float* y);
/* Inference only, same arguments and the same y (bitwise) as sft_net_forward:
 * the first layer forms its input channels from b_in while staging its
 * tiles, and the last hidden layer and the output layer's nine tap products
 * run as one pass, so neither the 16-channel input nor the layer-4
 * activations are written.  Afterwards sft_net_get_activation(0) and (4)
 * return SFT_ERR_STATE until the next sft_net_forward or sft_net_train_step.
 * The context's surrogate advance uses this path. */
sft_status sft_net_predict(sft_net* net, int32_t batch, const void* b_in, int32_t dtype,
                           const float* feats, float* y);
/* Copies the bf16 activations (NHWC, uint16 storage) of the last forward pass:
 * layer 0 = the 16-channel input, 1..4 = hidden layer outputs (64 channels);
 * SFT_ERR_STATE for layers 0 and 4 after sft_net_predict. */
sft_status sft_net_get_activation(sft_net* net, int32_t layer, void* out);
/* One training step on device arrays b_in, b_target [batch][nt][np] (dtype F64
 * or F32) and feats [batch][3]: forward, loss, backward; with apply = 1 also
 * the Adam update at learning rate lr.  *loss (may be NULL; waits for the
 * stream) receives the mean squared error of y against (b_target - b_in)/5 G. */
sft_status sft_net_train_step(sft_net* net, int32_t batch, const void* b_in, const void* b_target,
                              int32_t dtype, const float* feats, float lr, int32_t apply,
                              double* loss);
/* Limits the number of blocks of the network's persistent convolution and
 * weight-gradient launches to max_blocks (0, the default: one wave over the
 * compute units).  Each block walks tiles (or weight-gradient work items) at
 * a stride of the grid size, so a small limit runs many per block even on
 * small fields; the convolution outputs do not depend on it, and the weight
 * gradients change only by the regrouping of their FP32 partial sums.  For
 * testing the persistent loops at sizes a CPU reference can follow.
 * Errors: SFT_ERR_ARG. */
sft_status sft_net_set_grid_limit(sft_net* net, int32_t max_blocks);
sft_status sft_net_sync(sft_net* net);
sft_status sft_net_destroy(sft_net* net);

/* Advances the context by one 1-hour interval (t_end - t must be 1 h within
 * 1e-9 h, else SFT_ERR_ARG: the network stands in for one such interval)
 * with the surrogate for grid class grid_id (the network must have the
 * class's resolution); other classes take the plain path.  feats: host
 * [R][3] features of the class's realizations.
 * A checked realization also runs the plain solver (the arbiter) and keeps
 * the surrogate field only if its relative L2 distance (FP64, unweighted
 * over cells) to the plain field is <= tol, else the plain field (the
 * fallback); an unchecked one takes the surrogate field.  Which are checked:
 *   check = 0: none (unverified);
 *   check = 1: all, every interval (validation);
 *   check = K >= 2: throughput mode: a realization is checked on every K-th
 *     surrogate interval it takes (its 1st, (K+1)-th, ...; counted per
 *     realization since the context was created), and after a rejection on
 *     every interval until a check passes again.
 * err_out (host [R], may be NULL) receives the distances (-1 where not
 * checked).  Counts accepted, rejected and unchecked intervals (sft_diag,
 * sft_surrogate_counts).  Errors: SFT_ERR_ARG, SFT_ERR_SHAPE, SFT_ERR_STATE,
 * SFT_ERR_HIP. */
sft_status sft_surrogate_advance(sft_ctx* ctx, int32_t grid_id, sft_net* net, const float* feats,
                                 double t_end, double tol, int32_t check, double* err_out);

/* Surrogate counters of one realization: intervals accepted and rejected by
 * the check, intervals taken unchecked, and whether its last check failed
 * (1: every interval is checked until one passes).  Any output pointer may
 * be NULL.  Errors: SFT_ERR_ARG. */
sft_status sft_surrogate_counts(sft_ctx* ctx, int32_t real_id, int64_t* accepted, int64_t* rejected,
                                int64_t* unchecked, int32_t* escalated);

/* Kernel families for sft_get_timing. */
#define SFT_KFAM_STS_STAGE 0   /* diffusion stages j >= 2 (the hot loop)            */
#define SFT_KFAM_STS_FIRST 1   /* L(Y0) and the first diffusion stage               */
#define SFT_KFAM_ADV_STAGE 2   /* advection stages (fluxes, divergence, combination) */
#define SFT_KFAM_ASSIM 3       /* assimilation passes                               */
#define SFT_KFAM_DIAG 4        /* analysis reductions                               */
#define SFT_KFAM_OTHER 5       /* copies and increment closes                       */
#define SFT_KFAM_SOURCE 6      /* flux-emergence maps and source sub-advances       */
#define SFT_KFAM_COUNT 7

/* Turns per-launch event timing on (1) or off (0).  While on, every kernel
 * launch is bracketed by HIP events on the context's stream and HIP graphs are
 * not used.  Turning it on clears the accumulated totals. */
sft_status sft_set_timing(sft_ctx* ctx, int32_t on);

/* Totals for one kernel family since timing was turned on: summed event time
 * of its launches (ms), number of launches, the algorithmic bytes of the work
 * they did counted per unit of the method (e.g. 40 B per cell and FP64
 * diffusion stage, whether or not stages were fused), and the smallest
 * traffic the launches themselves need (a launch that fuses k stages reads
 * its inputs once and writes its outputs once).  Waits for the stream.
 * Errors: SFT_ERR_ARG (bad family). */
sft_status sft_get_timing(sft_ctx* ctx, int32_t family, double* total_ms, int64_t* launches,
                          double* alg_bytes, double* min_bytes);

/* Describes blocked tile shape `index` of the given precision: output tile
 * tx x ty cells, k fused stages, nthreads per block.  Returns SFT_ERR_ARG past
 * the end of the table (use it to count the shapes). */
sft_status sft_tile_info(int32_t precision, int32_t index, int32_t* tx, int32_t* ty, int32_t* k,
                         int32_t* nthreads);

/* Tile shape chosen for a grid class (-1 = one stage per launch), after the
 * first advance. */
sft_status sft_tile_choice(sft_ctx* ctx, int32_t grid_id, int32_t* index);

/* Fixes the diffusion-stage kernel of one grid class: blocked tile shape
 * `index` of the context's precision (see sft_tile_info), or -1 for one
 * stage per launch, in place of the autotuner's choice (and of the sts_tile
 * and sts_fuse options) for that class from the next advance on.  Cached
 * plans and captured graphs are dropped.  Every shape computes bitwise the
 * same fields; only speed changes (a caller that needs reproducible launch
 * shapes per class, for instance under a profiler, fixes them here).
 * Errors: SFT_ERR_ARG (bad grid or index), SFT_ERR_UNSUPPORTED (a blocked
 * FP32 shape on a class whose FP64 state needs 32-bit byte offsets beyond
 * 2^32). */
sft_status sft_set_class_tile(sft_ctx* ctx, int32_t grid_id, int32_t index);

/* Releases the context and its device memory (after waiting for its work). */
sft_status sft_destroy(sft_ctx* ctx);

/* Static text for a status code; never NULL. */
const char* sft_status_string(sft_status st);

/* Text of the last error on ctx (empty if none); valid until the next call. */
const char* sft_last_error(const sft_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SFT_H */
