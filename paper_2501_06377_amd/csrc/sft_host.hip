// Host side of the surface-flux-transport library: context and grid-class
// management, the per-realization time-step schedule (Sec. "Time steps"),
// advance plans batched over realizations and captured in HIP graphs, data
// assimilation and analysis calls, and the C ABI declared in include/sft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sft.h"
#include "sft_internal.h"
#include "adv_att.h"
#include "rfe.h"

namespace sft {
sft_status net_predict(sft_net* net, hipStream_t st, int batch, const double* Bin, const float* feats,
                       float** y_out);
void net_dims(const sft_net* net, int* H, int* W, int* maxb);
void cnn_pred(hipStream_t st, const double* Bin, const float* y, double* pred, size_t n);
void cnn_check(hipStream_t st, const double* pred, const double* plain, double* part, int nblk, int R,
               size_t n, double tol, double* err, int* accept, double* B, const int* want);
}  // namespace sft

using namespace sft;

namespace {

// Sec. "Units": solar radius 6.96e8 m, time in hours.
const double RSUN_M = 6.96e8;
const double M_S_TO_RS_HR = 3600.0 / RSUN_M;
const double KM2_S_TO_RS2_HR = 3600.0 * 1.0e6 / (RSUN_M * RSUN_M);
// the interval one surrogate evaluation stands in for, hours
const double SURROGATE_INTERVAL_H = 1.0;

struct Phase {
    int kind;        // 0 advection step, 1 diffusion call, 2 copy W1->B (FP64 FE advection),
                     // 3 one-stage diffusion close (mixed), 4 copy W1->B for one-stage
                     // diffusion (FP64), 5 advection-only close (mixed), 6 source
                     // sub-advance, 7 next source map
    int ent_off;     // first entry in the plan's entry table
    int n_ent;
    int max_s;
    std::vector<int> n_act;   // n_act[j] = entries with s >= j
};

struct Plan {
    std::vector<Phase> phases;
    std::vector<Entry> h_ents;
    Entry* d_ents = nullptr;
    StageCoef* d_coefs = nullptr;
    double* d_alpha = nullptr;   // interpolation weight of each source entry (by coef_off)
    int ticks = 0;               // source-map times the plan steps onto
    // per realization of the class
    std::vector<int64_t> steps, stages, adv_stages;
    std::vector<double> dt_last;
};

struct GridClass {
    int nt = 0, np = 0, R = 0, first_id = 0;
    std::vector<sft_params> prm;
    std::vector<double> cfl, dtE;
    std::vector<int> has_flow;
    // device memory
    double* B = nullptr;
    // FP64: W0 Y1 / ping, W1 pong, W2 L(Y0), W3 copy of Y0, W4/W5 second pair
    double* W[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // mixed: A0 advection increment, A1 d1 / ping, A2 pong, A3 L(Y0), A4/A5 second pair
    float* A[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double* dB = nullptr;   // FP64 assimilation increment (mixed precision only)
    AdvRow<double>* adv64 = nullptr;
    AdvRow<float>* adv32 = nullptr;
    // flow attenuation (allocated when some realization has B0 > 0): B0 per
    // realization and the face velocities of the advance in progress
    bool att = false;
    double* att_b0 = nullptr;
    double* vf64[2] = {nullptr, nullptr};
    float* vf32[2] = {nullptr, nullptr};
    // per-step attenuated CFL (att_cfl): entries of the realizations still
    // stepping, per-block partial maxima and the per-realization largest rate
    Entry* cfl_ents = nullptr;
    double *cfl_partial = nullptr, *cfl_rmax = nullptr;
    std::vector<Entry> h_cfl_ents;
    // random flux emergence: map k of the class in slot k & 1, per-row scale
    // of eq. rfe_m1 / rfe_m2, the device's interval index k (the map of the
    // current interval's start) and its host mirror (-1: no maps yet)
    double* rfe_S[2] = {nullptr, nullptr};
    double* rfe_scale = nullptr;
    int64_t* rfe_kdev = nullptr;
    int64_t rfe_k = -1;
    double *rfe_partial = nullptr, *rfe_ratio = nullptr;
    int rfe_nblk = 0;
    DiffRow<double>* dr64 = nullptr;
    double *sf64 = nullptr, *denth64 = nullptr, *denph64 = nullptr;
    float *sf32 = nullptr, *denth32 = nullptr, *denph32 = nullptr;
    double *st_row = nullptr, *ct_row = nullptr, *lat_row = nullptr, *w_row = nullptr;
    double *sph = nullptr, *cph = nullptr;
    AssimReal* ar = nullptr;
    double *assim_partial = nullptr, *assim_ratio = nullptr;
    int red_nblk = 0;
    DiagRec *diag_partial = nullptr, *diag_out = nullptr;
    void* stage_in = nullptr;    // host-upload staging for assimilation inputs (2 maps)
    bool diag_valid = false;
    int tile = -2;               // blocked tile shape (-1 = unfused, -2 = not chosen yet)
    std::map<uint64_t, std::vector<Plan*>> plans;   // one plan per lane
    int nl = 1;                                     // lanes (concurrent sub-batches)
    std::vector<hipEvent_t> lane_ev;                // fork + one join per extra lane
    // surrogate buffers (allocated on first use)
    double* pred = nullptr;
    float* sfeat = nullptr;
    double *spart = nullptr, *serr = nullptr;
    int *sacc = nullptr, *swant = nullptr;
    std::vector<int> h_swant;   // realizations checked in the current surrogate interval
    // counters since creation
    std::vector<int64_t> steps, stages, adv_stages, assim, s_acc, s_rej, s_unchk;
    // surrogate intervals taken per realization, and whether its last check
    // failed (then every interval is checked until one passes)
    std::vector<int64_t> s_count;
    std::vector<int> s_esc;
    std::vector<double> dt_last;
    size_t cells() const { return (size_t)nt * np; }
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

}  // namespace

struct sft_ctx {
    sft_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    double t = 0.0;
    bool started = false;
    std::vector<GridClass*> grids;
    std::map<uint64_t, GraphEntry> graphs;
    std::string err;
    std::vector<void*> allocs;
    std::vector<hipStream_t> lane_st;   // library streams of lanes 1, 2, ...
    // per-kernel-family event timing (sft_set_timing)
    struct Pending {
        hipEvent_t a, b;
        int fam;
        double bytes, min_bytes;
    };
    bool timing = false;
    hipEvent_t cur_a = nullptr;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_ev;
    double fam_ms[SFT_KFAM_COUNT] = {};
    int64_t fam_n[SFT_KFAM_COUNT] = {};
    double fam_bytes[SFT_KFAM_COUNT] = {};
    double fam_min[SFT_KFAM_COUNT] = {};
};

namespace {

sft_status fail(sft_ctx* c, sft_status st, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), SFT_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

// ------------------------------------------------------ event timing
hipEvent_t take_event(sft_ctx* c)
{
    if (!c->free_ev.empty()) {
        hipEvent_t e = c->free_ev.back();
        c->free_ev.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Folds finished launches [0, upto) into the per-family totals.
void harvest(sft_ctx* c, size_t upto)
{
    if (upto > c->pending.size()) upto = c->pending.size();
    if (!upto) return;
    (void)hipEventSynchronize(c->pending[upto - 1].b);
    for (size_t i = 0; i < upto; ++i) {
        auto& q = c->pending[i];
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, q.a, q.b);
        c->fam_ms[q.fam] += ms;
        c->fam_n[q.fam] += 1;
        c->fam_bytes[q.fam] += q.bytes;
        c->fam_min[q.fam] += q.min_bytes;
        c->free_ev.push_back(q.a);
        c->free_ev.push_back(q.b);
    }
    c->pending.erase(c->pending.begin(), c->pending.begin() + upto);
}

inline void tbeg(sft_ctx* c)
{
    if (!c->timing) return;
    c->cur_a = take_event(c);
    (void)hipEventRecord(c->cur_a, c->stream);
}

inline void tend(sft_ctx* c, int fam, double bytes, double min_bytes = -1.0)
{
    if (!c->timing) return;
    hipEvent_t b = take_event(c);
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back(sft_ctx::Pending{c->cur_a, b, fam, bytes, min_bytes < 0 ? bytes : min_bytes});
    if (c->pending.size() > 16384) harvest(c, 8192);
}

template <typename T>
sft_status dalloc(sft_ctx* c, T** p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SFT_ERR_OOM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T),
                    hipGetErrorString(e));
    }
    c->allocs.push_back((void*)*p);
    return SFT_OK;
}

template <typename T>
sft_status upload(sft_ctx* c, T* dst, const std::vector<T>& src)
{
    HIPCHK(c, hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return SFT_OK;
}

#define TRY(x)                              \
    do {                                    \
        sft_status s_ = (x);                \
        if (s_ != SFT_OK) return s_;        \
    } while (0)

uint64_t dbits(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

// ----------------------------------------------------------- host numerics
// Flow profiles eq. dr (at row centres) and eq. mf (at theta faces), R_sun/h.
void flows(int nt, const sft_params& p, std::vector<double>& vph, std::vector<double>& vth)
{
    const double dth = M_PI / nt;
    vph.assign(nt, 0.0);
    vth.assign(nt + 1, 0.0);
    for (int j = 0; j < nt; ++j) {
        const double th = (j + 0.5) * dth;
        const double c = cos(th), s = sin(th);
        const double c2 = c * c;
        const double v = (p.d0 + p.d2 * c2 + p.d4 * c2 * c2) * s;
        vph[j] = v * M_S_TO_RS_HR;
    }
    for (int f = 0; f <= nt; ++f) {
        const double th = f * dth;
        const double c = cos(th), s = sin(th);
        const double c2 = c * c;
        const double v = -(p.m1 * c + p.m3 * c2 * c + p.m5 * c2 * c2 * c) * s;
        vth[f] = v * M_S_TO_RS_HR;
    }
    vth[0] = 0.0;
    vth[nt] = 0.0;
}

// Eq. ssprk43_dt (SSPRK(4,3)) or eq. advection_timestep (forward Euler): the
// limit without safety factor, from the larger flanking face velocity.
double cfl_limit(int nt, int np, const std::vector<double>& vph, const std::vector<double>& vth,
                 int adv_time)
{
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    double rmax = 0.0;
    for (int j = 0; j < nt; ++j) {
        const double s = sin((j + 0.5) * dth);
        const double a = fabs(vth[j]), b = fabs(vth[j + 1]);
        const double vt = a > b ? a : b;
        const double vp = fabs(vph[j]);
        const double r = vt / dth + vp / (s * dph);
        if (r > rmax) rmax = r;
    }
    if (rmax == 0.0) return INFINITY;
    double lim = 1.0 / rmax;
    if (adv_time != SFT_SSPRK43) lim *= 0.5;
    return lim;
}

// Eq. diffusion_matrix rows for a scalar diffusivity nu (R_sun^2/h).
// Eq. diffusion_matrix with the diffusivity at the cell corners given per
// theta face (nuf[f], f = 0..nt; it depends on colatitude only): phi
// neighbours take the mean of the row's two faces, theta neighbours the
// shared face's value.  A scalar nu (all faces equal) gives the constant-
// coefficient rows.
void diff_rows(int nt, int np, const std::vector<double>& nuf, std::vector<DiffRow<double>>& out)
{
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    out.resize(nt);
    for (int j = 0; j < nt; ++j) {
        const double s = sin((j + 0.5) * dth);
        const double sfu = j == 0 ? 0.0 : sin(j * dth);
        const double sfd = j == nt - 1 ? 0.0 : sin((j + 1) * dth);
        DiffRow<double> d;
        d.ph = (nuf[j + 1] + nuf[j]) / (2.0 * dph * dph * s * s);
        d.up = (nuf[j] + nuf[j]) * sfu / (2.0 * dth * dth * s);
        d.dn = (nuf[j + 1] + nuf[j + 1]) * sfd / (2.0 * dth * dth * s);
        d.d = -(d.up + d.dn + d.ph + d.ph);
        out[j] = d;
    }
}

// Corner diffusivities of one realization: the scalar nu everywhere, or the
// grid diffusivity of eq. diffgrid, alpha [dth^2 + (dph sin theta_f)^2]
// (sin = 0 at the pole faces).
void corner_nu(int nt, int np, const sft_params& p, std::vector<double>& nuf)
{
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    nuf.assign(nt + 1, p.nu_km2_s * KM2_S_TO_RS2_HR);
    if (p.nu_grid_alpha > 0.0) {
        for (int f = 0; f <= nt; ++f) {
            const double sf = (f == 0 || f == nt) ? 0.0 : sin(f * dth);
            const double x = dph * sf;
            nuf[f] = p.nu_grid_alpha * (dth * dth + x * x);
        }
    }
}

// Super-time-stepping stage counts and coefficients (RKG2(3/2), RKL2) from
// their Gegenbauer / Legendre stability polynomials; forward Euler sub-steps.
int sts_stages(double tau, double dtE, int scheme)
{
    const double r = tau / dtE;
    double s;
    if (scheme == SFT_RKL2)
        s = ceil((sqrt(9.0 + 16.0 * r) - 1.0) / 2.0);
    else
        s = ceil((sqrt(25.0 + 24.0 * r) - 3.0) / 2.0);
    if (s < 2.0) s = 2.0;
    return (int)s;
}

double sts_b(int j, int scheme)
{
    if (scheme == SFT_RKL2) {
        if (j < 2) return 1.0 / 3.0;
        return ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
    }
    if (j == 0) return 1.0;
    if (j == 1) return 1.0 / 3.0;
    return 4.0 * (j - 1.0) * (j + 4.0) / (3.0 * j * (j + 1.0) * (j + 2.0) * (j + 3.0));
}

double sts_p1(int j, int scheme) { return scheme == SFT_RKL2 ? 1.0 : (j + 1.0) * (j + 2.0) / 2.0; }

void sts_coefs(int s, int scheme, double tau, std::vector<StageCoef>& out)
{
    out.assign(s + 1, StageCoef{0, 0, 0, 0, 0});
    const double w1 =
        scheme == SFT_RKL2 ? 4.0 / ((double)s * s + s - 2.0) : 6.0 / ((s + 4.0) * (s - 1.0));
    const double mut1 = (scheme == SFT_RKL2 ? sts_b(1, scheme) : 3.0 * sts_b(1, scheme)) * w1;
    out[1].cL = mut1 * tau;
    for (int j = 2; j <= s; ++j) {
        const double bj = sts_b(j, scheme), bj1 = sts_b(j - 1, scheme), bj2 = sts_b(j - 2, scheme);
        const double cj = scheme == SFT_RKL2 ? (2.0 * j - 1.0) / j : (2.0 * j + 1.0) / j;
        const double ej = scheme == SFT_RKL2 ? (j - 1.0) / j : (j + 1.0) / j;
        const double aj1 = 1.0 - bj1 * sts_p1(j - 1, scheme);
        const double mu = cj * bj / bj1;
        const double nu = -ej * bj / bj2;
        const double mut = mu * w1;
        const double gamt = -aj1 * mut;
        out[j].mu = mu;
        out[j].nu = nu;
        out[j].cy0 = 1.0 - mu - nu;
        out[j].cL = mut * tau;
        out[j].cLY0 = gamt * tau;
    }
}

void fe_coefs(int n, double h, std::vector<StageCoef>& out)
{
    out.assign(n + 1, StageCoef{0, 0, 0, 0, 0});
    out[1].cL = h;
    for (int j = 2; j <= n; ++j) {
        out[j].mu = 1.0;
        out[j].cL = h;
    }
}

// Length of the next step with time rem left (Sec. "Time steps"): the
// remaining time, cut to the flow limit lim (safety included) and dt_max,
// that cap raised to dt_min, and stretched to the end when it would leave
// less than 1e-10 h.  *fin tells whether the step ends the interval.
double next_step(double rem, double lim, double dt_max, double dt_min, bool* fin)
{
    double cap = lim;
    if (dt_max > 0.0 && dt_max < cap) cap = dt_max;
    if (dt_min > 0.0 && cap < dt_min) cap = dt_min;
    double dt = rem;
    if (cap < dt) dt = cap;
    *fin = false;
    if (rem - dt < 1e-10) {
        dt = rem;
        *fin = true;
    }
    return dt;
}

// Greedy step sequence over an interval of length len (Sec. "Time steps").
void step_sequence(double len, double lim, double dt_max, double dt_min, std::vector<double>& dts)
{
    dts.clear();
    double el = 0.0;
    while (el < len) {
        const double rem = len - el;
        bool fin = false;
        const double dt = next_step(rem, lim, dt_max, dt_min, &fin);
        dts.push_back(dt);
        el = fin ? len : el + dt;
    }
}

// --------------------------------------------------------------- planning
// Index k of the source-map interval [k tau, (k+1) tau) holding time t; a
// time within 1e-10 h below a boundary counts as on it.
int64_t rfe_interval(double t, double tau)
{
    int64_t k = (int64_t)floor(t / tau);
    if ((double)(k + 1) * tau - t < 1e-10) k += 1;
    if (t < (double)k * tau - 1e-10) k -= 1;
    return k;
}

struct Segment {
    double a, b;       // absolute start and end, hours
    int64_t k;         // source-map interval of the segment
    bool tick_after;   // a step ends on map time (k+1) tau at b
};

// Pieces of [t0, t_end] cut at the source-map times k tau (Sec. "Time
// steps": steps land on the times a new source map is generated).  Without
// finite-lifetime flux emergence: one piece.
void segments(double t0, double t_end, bool cut, double tau, std::vector<Segment>& out)
{
    out.clear();
    double a = t0;
    for (;;) {
        double b = t_end;
        int64_t k = 0;
        if (cut) {
            k = rfe_interval(a, tau);
            const double nb = (double)(k + 1) * tau;
            if (nb < t_end - 1e-10) b = nb;
        }
        out.push_back(Segment{a, b, k, false});
        if (b == t_end) break;
        out.back().tick_after = true;
        a = b;
    }
    if (cut && rfe_interval(t_end, tau) == out.back().k + 1) out.back().tick_after = true;
}

// Plan of one lane's share of an advance from t0 to t_end.  With fixed_dt
// the plan is a single step of fixed_dt[r] hours for each realization r
// (none where it is 0), the step rule having been applied by the caller.
// With mask, only the realizations r with mask[r] != 0 take part.
sft_status build_plan(sft_ctx* c, GridClass* g, int lane, double t0, double t_end, double len, Plan** out,
                      const std::vector<double>* fixed_dt = nullptr, const std::vector<char>* mask = nullptr)
{
    // the lane's realizations: r % nl == lane
    auto off = [&](int r) { return r % g->nl != lane || (mask && !(*mask)[r]); };
    const sft_options& o = c->opt;
    const bool mixed = o.precision == SFT_FP32_MIXED;
    const bool rfe = o.rfe_model != 0;
    const double tau = o.rfe_lifetime_h;
    Plan* p = new Plan();
    p->steps.assign(g->R, 0);
    p->stages.assign(g->R, 0);
    p->adv_stages.assign(g->R, 0);
    p->dt_last.assign(g->R, 0.0);
    std::vector<Segment> segs;
    if (rfe && tau > 0.0) segments(t0, t_end, true, tau, segs);
    else segs.push_back(Segment{t0, t_end, 0, false});
    std::vector<std::vector<double>> seq(g->R);
    std::vector<Entry> ents;
    std::vector<StageCoef> coefs;
    std::vector<StageCoef> tmp;
    std::vector<double> alphas;
    // Strang splitting: each advection advance is half a step, so the CFL
    // limit of the step doubles
    const bool strang = o.strang != 0;
    const int adv_nst = o.adv_time == SFT_SSPRK43 ? 4 : (o.adv_time == SFT_SSPRK33 ? 3 : 1);
    const double adv_frac = strang ? 0.5 : 1.0;
    // start of each realization's current step (absolute hours)
    std::vector<double> el(g->R, 0.0);
    for (const Segment& sg : segs) {
        // the first piece has the plan's own length (t_end - t0, as the
        // caller computed it); later pieces their end minus their start
        const double slen = segs.size() == 1 ? len : sg.b - sg.a;
        size_t max_steps = 0;
        for (int r = 0; r < g->R; ++r) {
            if (off(r)) {
                seq[r].clear();
                continue;
            }
            if (fixed_dt) {
                seq[r].clear();
                if ((*fixed_dt)[r] > 0.0) seq[r].push_back((*fixed_dt)[r]);
            } else {
                step_sequence(slen, (strang ? 2.0 : 1.0) * o.cfl_safety * g->cfl[r], o.dt_max, o.dt_min,
                              seq[r]);
            }
            max_steps = std::max(max_steps, seq[r].size());
            el[r] = 0.0;
        }
        // one advection advance of adv_frac * dt for every realization with flow
        // that takes step i (FP64 forward Euler: copy the result back to B)
        auto advection_phase = [&](size_t i) {
            Phase pa{0, (int)ents.size(), 0, 0, {}};
            for (int r = 0; r < g->R; ++r) {
                if (i >= seq[r].size() || !g->has_flow[r]) continue;
                Entry e{r, 0, 0, 0, adv_frac * seq[r][i]};
                ents.push_back(e);
                p->adv_stages[r] += adv_nst;
            }
            pa.n_ent = (int)ents.size() - pa.ent_off;
            if (pa.n_ent) {
                p->phases.push_back(pa);
                if (!mixed && o.adv_time == SFT_FE) {
                    Phase pc{2, pa.ent_off, pa.n_ent, 0, {}};
                    p->phases.push_back(pc);
                }
            }
        };
        // source sub-advance of length frac * dt starting at frac0 * dt into
        // step i (eq. rfe_s integrated exactly: length times the source at the
        // sub-advance's midpoint)
        auto source_phase = [&](size_t i, double frac0, double frac) {
            Phase ps{6, (int)ents.size(), 0, 0, {}};
            for (int r = 0; r < g->R; ++r) {
                if (i >= seq[r].size()) continue;
                const double dt = seq[r][i];
                const double ta = frac0 > 0.0 ? sg.a + el[r] + frac0 * dt : sg.a + el[r];
                const double h = frac * dt;
                double a = 0.0;
                if (tau > 0.0) a = ((ta + 0.5 * h) - (double)sg.k * tau) / tau;
                ents.push_back(Entry{r, 0, (int)alphas.size(), 0, h});
                alphas.push_back(a);
            }
            ps.n_ent = (int)ents.size() - ps.ent_off;
            if (ps.n_ent) p->phases.push_back(ps);
        };
        for (size_t i = 0; i < max_steps; ++i) {
            // Strang: the source's first half opens the step (eq. num_opsplit_strang)
            if (rfe && strang) source_phase(i, 0.0, 0.5);
            // advection (eq. num_opsplit_nostrang), or its first half (eq. num_opsplit_strang)
            advection_phase(i);
            // diffusion calls (several when the PTL hook splits the step)
            int ncall_max = 0;
            std::vector<int> ncall(g->R, 0);
            for (int r = 0; r < g->R; ++r) {
                if (i >= seq[r].size() || !std::isfinite(g->dtE[r])) continue;
                const double dt = seq[r][i];
                int nc = 1;
                if (o.ptl_dt > 0.0 && dt > o.ptl_dt) nc = (int)ceil(dt / o.ptl_dt);
                ncall[r] = nc;
                ncall_max = std::max(ncall_max, nc);
            }
            for (int call = 0; call < ncall_max; ++call) {
                std::vector<Entry> de;
                for (int r = 0; r < g->R; ++r) {
                    if (call >= ncall[r]) continue;
                    const double tc = seq[r][i] / ncall[r];
                    int s;
                    if (o.diff_time == SFT_DIFF_FE) {
                        s = (int)ceil(tc / g->dtE[r]);
                        fe_coefs(s, tc / s, tmp);
                    } else {
                        s = sts_stages(tc, g->dtE[r], o.diff_time);
                        sts_coefs(s, o.diff_time, tc, tmp);
                    }
                    Entry e{r, s, (int)coefs.size(), (mixed && call == 0 && g->has_flow[r]) ? 1 : 0, tc};
                    coefs.insert(coefs.end(), tmp.begin(), tmp.end());
                    de.push_back(e);
                    p->stages[r] += s;
                }
                std::stable_sort(de.begin(), de.end(), [](const Entry& a, const Entry& b) { return a.s > b.s; });
                Phase pd{1, (int)ents.size(), (int)de.size(), de.empty() ? 0 : de[0].s, {}};
                pd.n_act.assign(pd.max_s + 1, 0);
                for (int j = 0; j <= pd.max_s; ++j)
                    for (auto& e : de) pd.n_act[j] += e.s >= j ? 1 : 0;
                ents.insert(ents.end(), de.begin(), de.end());
                p->phases.push_back(pd);
                // one-stage calls (forward Euler only) finish outside the stage loop
                std::vector<Entry> one;
                for (auto& e : de)
                    if (e.s == 1) one.push_back(e);
                if (!one.empty()) {
                    Phase po{mixed ? 3 : 4, (int)ents.size(), (int)one.size(), 0, {}};
                    ents.insert(ents.end(), one.begin(), one.end());
                    p->phases.push_back(po);
                }
            }
            // mixed: realizations with flow but no diffusion fold the increment in
            if (mixed) {
                Phase pcl{5, (int)ents.size(), 0, 0, {}};
                for (int r = 0; r < g->R; ++r) {
                    if (i >= seq[r].size() || !g->has_flow[r] || ncall[r] > 0) continue;
                    ents.push_back(Entry{r, 0, 0, 1, seq[r][i]});
                }
                pcl.n_ent = (int)ents.size() - pcl.ent_off;
                if (pcl.n_ent) p->phases.push_back(pcl);
            }
            if (strang) {
                // second half advection after the diffusion; in the mixed path its
                // increment is folded into B by a close phase
                advection_phase(i);
                if (mixed) {
                    Phase pcl{5, (int)ents.size(), 0, 0, {}};
                    for (int r = 0; r < g->R; ++r) {
                        if (i >= seq[r].size() || !g->has_flow[r]) continue;
                        ents.push_back(Entry{r, 0, 0, 1, adv_frac * seq[r][i]});
                    }
                    pcl.n_ent = (int)ents.size() - pcl.ent_off;
                    if (pcl.n_ent) p->phases.push_back(pcl);
                }
            }
            // the source closes the step (its second half under Strang splitting)
            if (rfe) {
                if (strang) source_phase(i, 0.5, 0.5);
                else source_phase(i, 0.0, 1.0);
            }
            for (int r = 0; r < g->R; ++r)
                if (i < seq[r].size()) {
                    p->steps[r] += 1;
                    p->dt_last[r] = seq[r][i];
                    el[r] = el[r] + seq[r][i];
                }
        }
        if (sg.tick_after) {
            p->phases.push_back(Phase{7, (int)ents.size(), 0, 0, {}});
            p->ticks += 1;
        }
    }
    p->h_ents = ents;
    if (!ents.empty()) {
        sft_status st = dalloc(c, &p->d_ents, ents.size());
        if (st == SFT_OK) st = upload(c, p->d_ents, ents);
        if (st != SFT_OK) {
            delete p;
            return st;
        }
    }
    if (!coefs.empty()) {
        sft_status st = dalloc(c, &p->d_coefs, coefs.size());
        if (st == SFT_OK) st = upload(c, p->d_coefs, coefs);
        if (st != SFT_OK) {
            delete p;
            return st;
        }
    }
    if (!alphas.empty()) {
        sft_status st = dalloc(c, &p->d_alpha, alphas.size());
        if (st == SFT_OK) st = upload(c, p->d_alpha, alphas);
        if (st != SFT_OK) {
            delete p;
            return st;
        }
    }
    *out = p;
    return SFT_OK;
}

WenoConst<double> weno_const(double x)
{
    WenoConst<double> w;
    w.half = x / (x + x);
    w.third = x / (x + x + x);
    w.twothird = (x + x) / (x + x + x);
    w.eps = x;
    return w;
}

WenoConst<float> weno_const_f(double x)
{
    WenoConst<double> d = weno_const(x);
    WenoConst<float> w;
    w.half = (float)d.half;
    w.third = (float)d.third;
    w.twothird = (float)d.twothird;
    w.eps = (float)d.eps;
    return w;
}

void launch_diag_class(sft_ctx* c, GridClass* g)
{
    tbeg(c);
    launch_diag(c->stream, g->R, g->B, g->st_row, g->ct_row, g->w_row, g->sph, g->cph, g->diag_partial,
                g->red_nblk, g->diag_out, g->nt, g->np);
    tend(c, SFT_KFAM_DIAG, 8.0 * (double)g->cells() * g->R);
    g->diag_valid = true;
}

// Algorithmic bytes per cell of one diffusion stage launch: the reads of
// Y_{j-1}, Y_{j-2}, Y0, L(Y0) and the write of Y_j (FP64), or of d_{j-1},
// d_{j-2}, L(Y0) and d_j (FP32); an entry's last FP32 stage also reads the
// FP64 state (and the advection increment) and writes the FP64 state.
double stage_bytes(const Plan* p, const Phase& ph, int j, bool mixed, size_t cells)
{
    double b = 0.0;
    for (int i = 0; i < ph.n_act[j]; ++i) {
        const Entry& e = p->h_ents[ph.ent_off + i];
        if (!mixed) b += 40.0;
        else b += (j == 2 ? 12.0 : 16.0) + (e.s == j ? 12.0 + (e.pad ? 4.0 : 0.0) : 0.0);
    }
    return b * (double)cells;
}

// Temporally blocked stages 2..s of one diffusion phase: launch g covers
// stages j0 = 2 + gK .. j0 + K - 1 for the entries with s >= j0 (a prefix of
// the list); an entry whose last stage falls in a launch writes the state.
// Buffers rotate between two pairs so no launch writes what it reads.
void run_fused_groups(sft_ctx* c, GridClass* g, Plan* p, const Phase& ph)
{
    const bool mixed = c->opt.precision == SFT_FP32_MIXED;
    const int K = fused_config_k(mixed, g->tile);
    const Entry* E = p->d_ents + ph.ent_off;
    const double cells = (double)g->cells();
    for (int j0 = 2, grp = 0; j0 <= ph.max_s; j0 += K, ++grp) {
        const int n_act = ph.n_act[j0];
        const void *in1, *in2, *ly0, *drow;
        void *out1, *out2;
        const double* y0 = nullptr;
        if (!mixed) {
            in1 = grp == 0 ? g->W[0] : (grp & 1) ? g->W[4] : g->W[0];
            in2 = grp == 0 ? g->W[3] : (grp & 1) ? g->W[5] : g->W[1];
            out1 = (grp & 1) ? g->W[0] : g->W[4];
            out2 = (grp & 1) ? g->W[1] : g->W[5];
            ly0 = g->W[2];
            y0 = g->W[3];
            drow = g->dr64;
        } else {
            in1 = grp == 0 ? g->A[1] : (grp & 1) ? g->A[4] : g->A[1];
            in2 = grp == 0 ? nullptr : (grp & 1) ? g->A[5] : g->A[2];
            out1 = (grp & 1) ? g->A[1] : g->A[4];
            out2 = (grp & 1) ? g->A[2] : g->A[5];
            ly0 = g->A[3];
            drow = g->dr64;
        }
        // algorithmic bytes (per cell and stage of the method) and the
        // launch's own minimum traffic (inputs read once, outputs written once)
        double alg = 0.0, mn = 0.0;
        for (int i = 0; i < n_act; ++i) {
            const Entry& e = p->h_ents[ph.ent_off + i];
            const int kk = std::min(K, e.s - j0 + 1);
            const bool fin = j0 + kk - 1 == e.s;
            for (int jj = j0; jj < j0 + kk; ++jj) {
                if (!mixed) alg += 40.0;
                else alg += (jj == 2 ? 12.0 : 16.0) + (jj == e.s ? 12.0 + (e.pad ? 4.0 : 0.0) : 0.0);
            }
            if (!mixed) mn += (fin ? 40.0 : 48.0) - (fused_config_reads_ly0(false, g->tile) ? 0.0 : 8.0);
            else mn += (in2 ? 12.0 : 8.0) + (fin ? 16.0 + (e.pad ? 4.0 : 0.0) : 8.0);
        }
        tbeg(c);
        launch_diff_fused(c->stream, mixed, g->tile, E, n_act, p->d_coefs, j0, drow, in1, in2, y0, ly0,
                          out1, out2, g->B, g->A[0], g->nt, g->np);
        tend(c, SFT_KFAM_STS_STAGE, alg * cells, mn * cells);
    }
}

// Picks the diffusion-stage kernel for a grid class: one stage per launch or
// a blocked tile shape, by timing every candidate on the class's own buffers
// (zeroed first) over all its realizations.  The candidates compute
// identical results, so the choice changes speed only.
sft_status choose_tile(sft_ctx* c, GridClass* g)
{
    const sft_options& o = c->opt;
    const bool mixed = o.precision == SFT_FP32_MIXED;
    if (o.sts_fuse == 1) {
        g->tile = -1;
        return SFT_OK;
    }
    // the blocked FP32 kernel addresses one realization's FP64 state with
    // 32-bit byte offsets
    const bool fits32 = g->cells() * sizeof(double) <= 0xFFFFFFFFull;
    if (o.sts_tile >= 0) {
        if (mixed && !fits32)
            return fail(c, SFT_ERR_UNSUPPORTED, "blocked FP32 stages need nt*np*8 < 2^32 bytes (grid %dx%d)",
                        g->nt, g->np);
        g->tile = o.sts_tile;
        return SFT_OK;
    }
    if (mixed && !fits32) {
        g->tile = -1;
        return SFT_OK;
    }
    const int S = 1000;
    std::vector<Entry> ents(g->R);
    for (int r = 0; r < g->R; ++r) ents[r] = Entry{r, S, 0, 0, 1.0};
    std::vector<StageCoef> coefs(S + 1, StageCoef{0, 0, 0, 0, 0});
    Entry* d_ents = nullptr;
    StageCoef* d_coefs = nullptr;
    HIPCHK(c, hipMalloc((void**)&d_ents, ents.size() * sizeof(Entry)));
    HIPCHK(c, hipMalloc((void**)&d_coefs, coefs.size() * sizeof(StageCoef)));
    HIPCHK(c, hipMemcpy(d_ents, ents.data(), ents.size() * sizeof(Entry), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(d_coefs, coefs.data(), coefs.size() * sizeof(StageCoef), hipMemcpyHostToDevice));
    const size_t n = (size_t)g->R * g->cells();
    for (int i = 0; i < 6; ++i) {
        if (!mixed) HIPCHK(c, hipMemsetAsync(g->W[i], 0, n * sizeof(double), c->stream));
        else if (i != 0) HIPCHK(c, hipMemsetAsync(g->A[i], 0, n * sizeof(float), c->stream));
    }
    hipEvent_t ea, eb;
    HIPCHK(c, hipEventCreate(&ea));
    HIPCHK(c, hipEventCreate(&eb));
    // average launch time of the best of three rounds of reps launches
    auto time_it = [&](auto&& fn, int reps) -> float {
        fn();  // warm-up
        float best_ms = 1e30f;
        for (int round = 0; round < 3; ++round) {
            (void)hipEventRecord(ea, c->stream);
            for (int i = 0; i < reps; ++i) fn();
            (void)hipEventRecord(eb, c->stream);
            (void)hipEventSynchronize(eb);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ea, eb);
            best_ms = std::min(best_ms, ms / reps);
        }
        return best_ms;
    };
    const int nt = g->nt, np = g->np, R = g->R;
    float best;
    int best_cfg = -1;
    // one stage per launch
    if (!mixed)
        best = time_it([&] {
            launch_diff_stage_f64(c->stream, d_ents, R, d_coefs, 10, g->dr64, g->B, g->W[0], g->W[1],
                                  g->W[2], g->W[4], nt, np);
        }, 4);
    else
        best = time_it([&] {
            launch_diff_stage_mixed(c->stream, d_ents, R, d_coefs, 10, g->dr64, g->B, g->A[0], g->A[1],
                                    g->A[2], g->A[3], g->A[4], g->A[2], nt, np);
        }, 4);
    // SFT_TUNE_LOG set: the candidates' times per stage go to stderr
    const bool log = std::getenv("SFT_TUNE_LOG") != nullptr;
    if (log) std::fprintf(stderr, "sft tile tuning %dx%d x%d: one stage per launch %.2f us\n", nt, np, R, 1e3f * best);
    for (int cfg = 0; cfg < fused_config_count(mixed); ++cfg) {
        const int K = fused_config_k(mixed, cfg);
        float t;
        if (!mixed)
            t = time_it([&] {
                launch_diff_fused(c->stream, false, cfg, d_ents, R, d_coefs, 10, g->dr64, g->W[0],
                                  g->W[1], g->W[3], g->W[2], g->W[4], g->W[5], g->B, nullptr, nt, np);
            }, 3);
        else
            t = time_it([&] {
                launch_diff_fused(c->stream, true, cfg, d_ents, R, d_coefs, 10, g->dr64, g->A[1],
                                  g->A[2], nullptr, g->A[3], g->A[4], g->A[5], g->B, g->A[0], nt, np);
            }, 3);
        if (log) std::fprintf(stderr, "  tile %2d (K %2d): %.2f us per stage\n", cfg, K, 1e3f * t / K);
        if (t / K < best) {
            best = t / K;
            best_cfg = cfg;
        }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    HIPCHK(c, hipGetLastError());
    (void)hipFree(d_ents);
    (void)hipFree(d_coefs);
    g->tile = best_cfg;
    return SFT_OK;
}

// Source map (kdev[0] + koff, or kabs without kdev) of the realizations of
// one lane of a class (lane < 0: all): draw, FP64 flux sums, eq. fluxbal
// balance.
void rfe_make_map(sft_ctx* c, GridClass* g, const int64_t* kdev, int koff, int64_t kabs, int lane)
{
    const double nr = lane < 0 ? g->R : (g->R - lane + g->nl - 1) / g->nl;
    tbeg(c);
    launch_rfe_gen(c->stream, g->R, g->nl, lane, g->first_id, c->opt.rfe_seed, kdev, koff, kabs, g->rfe_scale,
                   g->w_row, g->rfe_S[0], g->rfe_S[1], g->rfe_partial, g->rfe_ratio, g->nt, g->np);
    launch_rfe_balance(c->stream, g->R, g->nl, lane, kdev, koff, kabs, g->rfe_ratio, g->rfe_S[0], g->rfe_S[1],
                       g->nt, g->np);
    tend(c, SFT_KFAM_SOURCE, 24.0 * (double)g->cells() * nr);
}

// Enqueue every phase of a lane's plan on the context's current stream.
void run_plan(sft_ctx* c, GridClass* g, Plan* p, int lane)
{
    const sft_options& o = c->opt;
    const bool mixed = o.precision == SFT_FP32_MIXED;
    hipStream_t st = c->stream;
    const int nt = g->nt, np = g->np;
    const double cells = (double)g->cells();
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    const int upwind = o.adv_scheme == SFT_UPWIND;
    const int ts = o.adv_time == SFT_SSPRK43 ? 0 : (o.adv_time == SFT_SSPRK33 ? 2 : 1);
    for (const Phase& ph : p->phases) {
        const Entry* E = p->d_ents + ph.ent_off;
        const double ne = (double)ph.n_ent;
        if (ph.kind == 0) {
            if (!mixed) {
                Geom<double> geo{g->sf64, g->denth64, g->denph64};
                WenoConst<double> wt = weno_const(dth), wp = weno_const(dph);
                double *B = g->B, *W1 = g->W[0], *W2 = g->W[1];
                // SSPRK(4,3): B -> W1 -> W2 -> W1 -> B; SSPRK(3,3): B -> W1 -> W2 -> B
                const double* fin[4] = {B, W1, W2, W1};
                double* fout[4] = {W1, W2, ts == 2 ? B : W1, B};
                const int nst = ts == 1 ? 1 : (ts == 2 ? 3 : 4);
                if (g->att) {
                    // attenuated face velocities from the state at the start of the advance
                    tbeg(c);
                    launch_att_faces_f64(st, E, ph.n_ent, g->adv64, g->att_b0, B, g->vf64[0], g->vf64[1],
                                         nt, np);
                    tend(c, SFT_KFAM_OTHER, 24.0 * cells * ne);
                }
                for (int k = 0; k < nst; ++k) {
                    tbeg(c);
                    if (g->att)
                        launch_adv_stage_att_f64(st, E, ph.n_ent, k, ts, upwind, g->adv64, geo, wt, wp, B,
                                                 fin[k], fout[k], g->vf64[0], g->vf64[1], nt, np);
                    else
                        launch_adv_stage_f64(st, E, ph.n_ent, k, ts, upwind, g->adv64, geo, wt, wp, B,
                                             fin[k], fout[k], nt, np);
                    tend(c, SFT_KFAM_ADV_STAGE,
                         ((k == 2 || (ts == 2 && k == 1) ? 24.0 : 16.0) + (g->att ? 16.0 : 0.0)) * cells * ne);
                }
            } else {
                Geom<float> geo{g->sf32, g->denth32, g->denph32};
                WenoConst<float> wt = weno_const_f(dth), wp = weno_const_f(dph);
                float *A0 = g->A[0], *A1 = g->A[1], *A2 = g->A[2];
                const float* din[4] = {nullptr, A1, A2, A1};
                float* dout[4] = {ts == 1 ? A0 : A1, A2, ts == 2 ? A0 : A1, A0};
                const int nst = ts == 1 ? 1 : (ts == 2 ? 3 : 4);
                if (g->att) {
                    tbeg(c);
                    launch_att_faces_f32(st, E, ph.n_ent, g->adv64, g->att_b0, g->B, g->vf32[0], g->vf32[1],
                                         nt, np);
                    tend(c, SFT_KFAM_OTHER, 16.0 * cells * ne);
                }
                for (int k = 0; k < nst; ++k) {
                    tbeg(c);
                    if (g->att)
                        launch_adv_stage_att_mixed(st, E, ph.n_ent, k, ts, upwind, g->adv32, geo, wt, wp, g->B,
                                                   din[k], dout[k], g->vf32[0], g->vf32[1], nt, np);
                    else
                        launch_adv_stage_mixed(st, E, ph.n_ent, k, ts, upwind, g->adv32, geo, wt, wp, g->B,
                                               din[k], dout[k], nt, np);
                    tend(c, SFT_KFAM_ADV_STAGE, ((k == 0 ? 12.0 : 16.0) + (g->att ? 8.0 : 0.0)) * cells * ne);
                }
            }
        } else if (ph.kind == 1) {
            const bool fused = g->tile >= 0;
            if (!mixed) {
                double *B = g->B, *W1 = g->W[0], *W2 = g->W[1], *LY = g->W[2];
                tbeg(c);
                launch_diff_first_f64(st, E, ph.n_ent, p->d_coefs, g->dr64, B, LY, W1,
                                      fused ? g->W[3] : nullptr, nt, np);
                tend(c, SFT_KFAM_STS_FIRST, (fused ? 32.0 : 24.0) * cells * ne);
                if (fused) {
                    run_fused_groups(c, g, p, ph);
                } else {
                    for (int j = 2; j <= ph.max_s; ++j) {
                        const double *ym1, *ym2;
                        double* out;
                        if (j == 2) {
                            ym1 = W1;
                            ym2 = B;
                            out = W2;
                        } else if (j & 1) {
                            ym1 = W2;
                            ym2 = W1;
                            out = W1;
                        } else {
                            ym1 = W1;
                            ym2 = W2;
                            out = W2;
                        }
                        tbeg(c);
                        launch_diff_stage_f64(st, E, ph.n_act[j], p->d_coefs, j, g->dr64, B, ym1, ym2,
                                              LY, out, nt, np);
                        tend(c, SFT_KFAM_STS_STAGE, stage_bytes(p, ph, j, false, g->cells()));
                    }
                }
            } else {
                float *A0 = g->A[0], *P1 = g->A[1], *P2 = g->A[2], *LY = g->A[3];
                double npad = 0.0;
                for (int i = 0; i < ph.n_ent; ++i) npad += p->h_ents[ph.ent_off + i].pad ? 1.0 : 0.0;
                tbeg(c);
                launch_diff_first_mixed(st, E, ph.n_ent, p->d_coefs, g->dr64, g->B, A0, LY, P1, nt, np);
                tend(c, SFT_KFAM_STS_FIRST, (16.0 * ne + 4.0 * npad) * cells);
                if (fused) {
                    run_fused_groups(c, g, p, ph);
                } else {
                    // d alternates between P1 and P2 (a stage reads its
                    // neighbours); e = d_{j-1} - d_{j-2} is updated in place in A[4]
                    float* EA = g->A[4];
                    for (int j = 2; j <= ph.max_s; ++j) {
                        const float* din = (j & 1) ? P2 : P1;
                        float* dout = (j & 1) ? P1 : P2;
                        tbeg(c);
                        launch_diff_stage_mixed(st, E, ph.n_act[j], p->d_coefs, j, g->dr64, g->B, A0, din,
                                                j == 2 ? nullptr : EA, LY, dout, EA, nt, np);
                        tend(c, SFT_KFAM_STS_STAGE, stage_bytes(p, ph, j, true, g->cells()));
                    }
                }
            }
        } else if (ph.kind == 2 || ph.kind == 4) {
            tbeg(c);
            launch_copy_f64(st, E, ph.n_ent, g->W[0], g->B, g->cells());
            tend(c, SFT_KFAM_OTHER, 16.0 * cells * ne);
        } else if (ph.kind == 3) {
            // one-stage diffusion calls: B = Y0 + d1 (d1 in A[1])
            tbeg(c);
            launch_mixed_close(st, E, ph.n_ent, g->B, g->A[0], g->A[1], g->cells());
            tend(c, SFT_KFAM_OTHER, 24.0 * cells * ne);
        } else if (ph.kind == 5) {
            // flow but no diffusion: B = B + advection increment
            tbeg(c);
            launch_mixed_close(st, E, ph.n_ent, g->B, g->A[0], nullptr, g->cells());
            tend(c, SFT_KFAM_OTHER, 20.0 * cells * ne);
        } else if (ph.kind == 6) {
            // source sub-advance on the FP64 state (both precisions)
            const int inf = o.rfe_lifetime_h > 0.0 ? 0 : 1;
            tbeg(c);
            launch_rfe_apply(st, E, ph.n_ent, p->d_alpha, g->rfe_kdev + lane, inf, g->rfe_S[0], g->rfe_S[1],
                             g->B, g->cells());
            tend(c, SFT_KFAM_SOURCE, (inf ? 24.0 : 32.0) * cells * ne);
        } else if (ph.kind == 7) {
            // a step ended on map time (k+1) tau: k += 1, draw map k + 2 into
            // the slot map k held
            tbeg(c);
            launch_rfe_tick(st, g->rfe_kdev + lane);
            tend(c, SFT_KFAM_SOURCE, 0.0);
            rfe_make_map(c, g, g->rfe_kdev + lane, 1, 0, lane);
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

const char* sft_status_string(sft_status st)
{
    switch (st) {
    case SFT_OK: return "ok";
    case SFT_ERR_ARG: return "invalid argument";
    case SFT_ERR_SHAPE: return "shape mismatch";
    case SFT_ERR_OOM: return "out of memory";
    case SFT_ERR_HIP: return "HIP runtime error";
    case SFT_ERR_NOT_FINITE: return "field holds NaN or Inf";
    case SFT_ERR_STATE: return "call not valid in this state";
    case SFT_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

const char* sft_last_error(const sft_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

sft_status sft_options_default(sft_options* opt)
{
    if (!opt) return SFT_ERR_ARG;
    memset(opt, 0, sizeof *opt);
    opt->precision = SFT_FP64;
    opt->adv_scheme = SFT_WENO3CSH;
    opt->adv_time = SFT_SSPRK43;
    opt->diff_time = SFT_RKG2;
    opt->cfl_safety = 0.9;
    opt->dt_max = 0.0;
    opt->ptl_dt = 0.0;
    opt->use_graphs = 0;
    opt->sts_fuse = 0;
    opt->diag_every_call = 1;
    opt->sts_tile = -1;
    return SFT_OK;
}

// ---------------------------------------------------------------- allocation-free scratch
// Device scratch of sft_assimilate_noalloc: the flux-balance partial sums and
// ratios of one call, R x (2 nblk + 1) doubles, in a file-scope device array
// that every GPU the library runs on holds until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device, with that device current (scratch_setup, from
// sft_create), and kept per device.
constexpr size_t kNoAllocDoubles = 262144;   // 2 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Looks up this device's address of `scratch` (first context on a device).
static sft_status scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return SFT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return SFT_ERR_HIP;
        g_scratch_ptr[device] = (double*)ptr;
        g_scratch_done[device] = true;
    }
    return SFT_OK;
}

static double* scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

sft_status sft_create(sft_ctx** ctx, const sft_options* opt, void* hip_stream)
{
    if (!ctx) return SFT_ERR_ARG;
    *ctx = nullptr;
    sft_options o;
    if (opt) o = *opt;
    else sft_options_default(&o);
    if (o.precision != SFT_FP64 && o.precision != SFT_FP32_MIXED) return SFT_ERR_ARG;
    if (o.adv_scheme != SFT_WENO3CSH && o.adv_scheme != SFT_UPWIND) return SFT_ERR_ARG;
    if (o.adv_time != SFT_SSPRK43 && o.adv_time != SFT_FE && o.adv_time != SFT_SSPRK33) return SFT_ERR_ARG;
    if (o.strang != 0 && o.strang != 1) return SFT_ERR_ARG;
    if (o.rfe_model < 0 || o.rfe_model > 2) return SFT_ERR_ARG;
    if (o.lanes < 0 || o.lanes > 16) return SFT_ERR_ARG;
    if (o.rfe_model && (!(o.rfe_phi_hr > 0.0) || !std::isfinite(o.rfe_phi_hr) ||
                        !(o.rfe_lifetime_h >= 0.0) || !std::isfinite(o.rfe_lifetime_h)))
        return SFT_ERR_ARG;
    if (o.diff_time != SFT_RKG2 && o.diff_time != SFT_RKL2 && o.diff_time != SFT_DIFF_FE)
        return SFT_ERR_ARG;
    if (!(o.cfl_safety > 0.0 && o.cfl_safety <= 1.0) || o.dt_max < 0.0 || o.ptl_dt < 0.0)
        return SFT_ERR_ARG;
    if (!(o.dt_min >= 0.0) || !std::isfinite(o.dt_min) || (o.att_cfl != 0 && o.att_cfl != 1))
        return SFT_ERR_ARG;
    if (o.att_cfl && o.rfe_model) return SFT_ERR_UNSUPPORTED;
    if (o.sts_fuse < 0 || o.sts_fuse > 1 || o.sts_tile < -1 ||
        o.sts_tile >= fused_config_count(o.precision == SFT_FP32_MIXED))
        return SFT_ERR_ARG;
    sft_ctx* c = new sft_ctx();
    c->opt = o;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return SFT_ERR_HIP;
    }
    if (const sft_status sst = scratch_setup(c->device); sst != SFT_OK) {
        delete c;
        return sst;
    }
    if (!c->stream) {
        // an own blocking stream (default priority): it orders with the null
        // stream and can be captured into graphs, which the null stream cannot
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return SFT_ERR_HIP;
        }
        c->own_stream = true;
    }
    *ctx = c;
    return SFT_OK;
}

sft_status sft_add_grid(sft_ctx* c, int32_t nt, int32_t np, int32_t* grid_id)
{
    if (!c || !grid_id) return SFT_ERR_ARG;
    if (c->started) return fail(c, SFT_ERR_STATE, "grids must be added before the first advance");
    if (nt < 8 || np < 8 || (np & 1)) return fail(c, SFT_ERR_ARG, "grid %d x %d not allowed", nt, np);
    GridClass* g = new GridClass();
    g->nt = nt;
    g->np = np;
    int first = 0;
    for (auto* h : c->grids) first += h->R;
    g->first_id = first;
    c->grids.push_back(g);
    *grid_id = (int32_t)c->grids.size() - 1;
    return SFT_OK;
}

static sft_status class_alloc(sft_ctx* c, GridClass* g)
{
    const int nt = g->nt, np = g->np, R = g->R;
    const size_t n = (size_t)R * g->cells();
    const bool mixed = c->opt.precision == SFT_FP32_MIXED;
    // lanes: concurrent sub-batches r % nl, each on its own stream
    g->nl = std::max(1, std::min(c->opt.lanes > 0 ? c->opt.lanes : 2, R));
    while ((int)c->lane_st.size() < g->nl - 1) {
        hipStream_t s;
        HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        c->lane_st.push_back(s);
    }
    g->lane_ev.assign(g->nl, nullptr);
    for (int l = 0; l < g->nl && g->nl > 1; ++l)
        HIPCHK(c, hipEventCreateWithFlags(&g->lane_ev[l], hipEventDisableTiming));
    TRY(dalloc(c, &g->B, n));
    HIPCHK(c, hipMemset(g->B, 0, n * sizeof(double)));
    if (!mixed) {
        for (int i = 0; i < 6; ++i) TRY(dalloc(c, &g->W[i], n));
    } else {
        for (int i = 0; i < 6; ++i) TRY(dalloc(c, &g->A[i], n));
        HIPCHK(c, hipMemset(g->A[0], 0, n * sizeof(float)));
    }
    // per-realization tables
    std::vector<AdvRow<double>> a64((size_t)R * (nt + 1));
    std::vector<AdvRow<float>> a32((size_t)R * (nt + 1));
    std::vector<DiffRow<double>> d64((size_t)R * nt);
    std::vector<AssimReal> ar(R);
    g->cfl.assign(R, INFINITY);
    g->dtE.assign(R, INFINITY);
    g->has_flow.assign(R, 0);
    std::vector<double> vph, vth, nuf;
    std::vector<DiffRow<double>> drow;
    for (int r = 0; r < R; ++r) {
        const sft_params& p = g->prm[r];
        flows(nt, p, vph, vth);
        int hf = 0;
        for (double v : vph) hf |= v != 0.0;
        for (double v : vth) hf |= v != 0.0;
        g->has_flow[r] = hf;
        g->cfl[r] = cfl_limit(nt, np, vph, vth, c->opt.adv_time);
        for (int j = 0; j <= nt; ++j) {
            AdvRow<double> a{};
            a.vth = vth[j];
            if (j < nt) {
                double al = 0.0;
                for (int f = j - 2; f <= j + 3; ++f) {
                    if (f < 0 || f > nt) continue;
                    al = std::max(al, fabs(vth[f]));
                }
                a.cthP = 0.5 * (vth[j + 1] - al);
                a.cthM = 0.5 * (vth[j] + al);
                const double ap = fabs(vph[j]);
                a.cphP = 0.5 * (vph[j] - ap);
                a.cphM = 0.5 * (vph[j] + ap);
                a.vph = vph[j];
            }
            a64[(size_t)r * (nt + 1) + j] = a;
            AdvRow<float> b{};
            b.cthP = (float)a.cthP;
            b.cthM = (float)a.cthM;
            b.cphP = (float)a.cphP;
            b.cphM = (float)a.cphM;
            b.vth = (float)a.vth;
            b.vph = (float)a.vph;
            a32[(size_t)r * (nt + 1) + j] = b;
        }
        corner_nu(nt, np, p, nuf);
        diff_rows(nt, np, nuf, drow);
        double m = 0.0;
        for (int j = 0; j < nt; ++j) {
            d64[(size_t)r * nt + j] = drow[j];
            m = std::max(m, fabs(drow[j].d));
        }
        g->dtE[r] = m > 0.0 ? 1.0 / m : INFINITY;
        ar[r].alpha = p.alpha_mu;
        ar[r].mu_lim = p.mu_lim;
        ar[r].lat_lim_rad = p.lat_lim_deg * (M_PI / 180.0);
        ar[r].balance = p.flux_balance ? 1 : 0;
    }
    TRY(dalloc(c, &g->adv64, a64.size()));
    TRY(upload(c, g->adv64, a64));
    TRY(dalloc(c, &g->adv32, a32.size()));
    TRY(upload(c, g->adv32, a32));
    TRY(dalloc(c, &g->dr64, d64.size()));
    TRY(upload(c, g->dr64, d64));
    TRY(dalloc(c, &g->ar, ar.size()));
    TRY(upload(c, g->ar, ar));
    std::vector<double> b0(R);
    for (int r = 0; r < R; ++r) {
        b0[r] = g->prm[r].att_b0;
        g->att |= b0[r] > 0.0;
    }
    if (c->opt.rfe_model) {
        for (int i = 0; i < 2; ++i) TRY(dalloc(c, &g->rfe_S[i], n));
        // eq. rfe_m1: phi / (dA_j N_cells) sqrt(pi/2), dA_j = R^2 sin(theta_j) dth dph;
        // eq. rfe_m2: phi / (4 pi R^2) sqrt(pi/2); R in cm
        const double Rcm = RSUN_M * 100.0, phi = c->opt.rfe_phi_hr;
        const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
        std::vector<double> sc(nt);
        for (int j = 0; j < nt; ++j) {
            if (c->opt.rfe_model == 1) {
                const double dA = Rcm * Rcm * sin((j + 0.5) * dth) * dth * dph;
                sc[j] = phi / (dA * (double)g->cells()) * sqrt(M_PI / 2.0);
            } else {
                sc[j] = phi / (4.0 * M_PI * Rcm * Rcm) * sqrt(M_PI / 2.0);
            }
        }
        TRY(dalloc(c, &g->rfe_scale, nt));
        TRY(upload(c, g->rfe_scale, sc));
        TRY(dalloc(c, &g->rfe_kdev, g->nl));
        g->rfe_nblk = rfe_gen_blocks(nt, np);
        TRY(dalloc(c, &g->rfe_partial, (size_t)R * g->rfe_nblk * 2));
        TRY(dalloc(c, &g->rfe_ratio, R));
    }
    if (g->att) {
        TRY(dalloc(c, &g->att_b0, b0.size()));
        TRY(upload(c, g->att_b0, b0));
        for (int i = 0; i < 2; ++i) {
            if (!mixed) TRY(dalloc(c, &g->vf64[i], n));
            else TRY(dalloc(c, &g->vf32[i], n));
        }
        if (c->opt.att_cfl) {
            TRY(dalloc(c, &g->cfl_ents, (size_t)R));
            TRY(dalloc(c, &g->cfl_partial, (size_t)R * nt * att_cfl_blocks_per_row(np)));
            TRY(dalloc(c, &g->cfl_rmax, (size_t)R));
        }
    }
    // geometry
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    std::vector<double> sf(nt + 1), dthv(nt), dphv(nt), st(nt), ct(nt), lat(nt), w(nt), sp(np), cp(np);
    for (int f = 0; f <= nt; ++f) sf[f] = sin(f * dth);
    sf[0] = 0.0;
    sf[nt] = 0.0;
    for (int j = 0; j < nt; ++j) {
        const double th = (j + 0.5) * dth;
        st[j] = sin(th);
        ct[j] = cos(th);
        dthv[j] = st[j] * dth;
        dphv[j] = st[j] * dph;
        lat[j] = M_PI / 2.0 - th;
        w[j] = sin(th) * dth * dph;
    }
    for (int k = 0; k < np; ++k) {
        const double ph = (k + 0.5) * dph;
        sp[k] = sin(ph);
        cp[k] = cos(ph);
    }
    auto f32 = [](const std::vector<double>& v) {
        std::vector<float> o(v.size());
        for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
        return o;
    };
    TRY(dalloc(c, &g->sf64, nt + 1));
    TRY(upload(c, g->sf64, sf));
    TRY(dalloc(c, &g->denth64, nt));
    TRY(upload(c, g->denth64, dthv));
    TRY(dalloc(c, &g->denph64, nt));
    TRY(upload(c, g->denph64, dphv));
    TRY(dalloc(c, &g->sf32, nt + 1));
    TRY(upload(c, g->sf32, f32(sf)));
    TRY(dalloc(c, &g->denth32, nt));
    TRY(upload(c, g->denth32, f32(dthv)));
    TRY(dalloc(c, &g->denph32, nt));
    TRY(upload(c, g->denph32, f32(dphv)));
    TRY(dalloc(c, &g->st_row, nt));
    TRY(upload(c, g->st_row, st));
    TRY(dalloc(c, &g->ct_row, nt));
    TRY(upload(c, g->ct_row, ct));
    TRY(dalloc(c, &g->lat_row, nt));
    TRY(upload(c, g->lat_row, lat));
    TRY(dalloc(c, &g->w_row, nt));
    TRY(upload(c, g->w_row, w));
    TRY(dalloc(c, &g->sph, np));
    TRY(upload(c, g->sph, sp));
    TRY(dalloc(c, &g->cph, np));
    TRY(upload(c, g->cph, cp));
    // reductions: a fixed number of blocks per realization
    int nblk = (int)((g->cells() + 255) / 256);
    if (nblk > 512) nblk = 512;
    g->red_nblk = nblk;
    TRY(dalloc(c, &g->assim_partial, (size_t)R * nblk * 2));
    TRY(dalloc(c, &g->assim_ratio, R));
    TRY(dalloc(c, &g->diag_partial, (size_t)R * nblk));
    TRY(dalloc(c, &g->diag_out, R));
    g->steps.assign(R, 0);
    g->stages.assign(R, 0);
    g->adv_stages.assign(R, 0);
    g->assim.assign(R, 0);
    g->s_acc.assign(R, 0);
    g->s_rej.assign(R, 0);
    g->s_unchk.assign(R, 0);
    g->s_count.assign(R, 0);
    g->s_esc.assign(R, 0);
    g->dt_last.assign(R, 0.0);
    return SFT_OK;
}

sft_status sft_add_realizations(sft_ctx* c, int32_t grid_id, int32_t n, const sft_params* prm,
                                int32_t* first_id)
{
    if (!c || !prm || !first_id || n <= 0) return SFT_ERR_ARG;
    if (grid_id < 0 || grid_id >= (int)c->grids.size()) return fail(c, SFT_ERR_ARG, "bad grid id");
    if (c->started) return fail(c, SFT_ERR_STATE, "realizations must be added before the first advance");
    GridClass* g = c->grids[grid_id];
    if (g->R) return fail(c, SFT_ERR_STATE, "grid %d already has realizations", grid_id);
    for (int i = 0; i < n; ++i) {
        const sft_params& p = prm[i];
        if (!(p.nu_km2_s >= 0.0) || !std::isfinite(p.nu_km2_s) || !(p.alpha_mu > 0.0) ||
            !(p.lat_lim_deg >= 0.0) || !(p.att_b0 >= 0.0) || !std::isfinite(p.att_b0) ||
            !(p.nu_grid_alpha >= 0.0) || !std::isfinite(p.nu_grid_alpha))
            return fail(c, SFT_ERR_ARG, "realization %d: invalid parameters", i);
    }
    // ids are consecutive over grid classes in creation order
    int first = 0;
    for (int i = 0; i < grid_id; ++i) first += c->grids[i]->R;
    for (size_t i = grid_id + 1; i < c->grids.size(); ++i)
        if (c->grids[i]->R) return fail(c, SFT_ERR_STATE, "add realizations in grid order");
    g->first_id = first;
    g->R = n;
    g->prm.assign(prm, prm + n);
    sft_status st = class_alloc(c, g);
    if (st != SFT_OK) g->R = 0;
    *first_id = first;
    return st;
}

static bool find_real(sft_ctx* c, int32_t id, GridClass** g, int* r)
{
    for (auto* h : c->grids) {
        if (id >= h->first_id && id < h->first_id + h->R) {
            *g = h;
            *r = id - h->first_id;
            return true;
        }
    }
    return false;
}

static sft_status copy_in(sft_ctx* c, double* dst, const void* src, size_t n, int dtype, int on_device)
{
    if (dtype == SFT_DTYPE_F64) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
        if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
        return SFT_OK;
    }
    if (dtype != SFT_DTYPE_F32) return fail(c, SFT_ERR_ARG, "bad dtype %d", dtype);
    if (on_device) {
        launch_f32_to_f64(c->stream, (const float*)src, dst, n);
        return SFT_OK;
    }
    std::vector<double> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (double)((const float*)src)[i];
    HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SFT_OK;
}

static sft_status copy_out(sft_ctx* c, void* dst, const double* src, size_t n, int dtype, int on_device)
{
    if (dtype == SFT_DTYPE_F64) {
        HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
        if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
        return SFT_OK;
    }
    if (dtype != SFT_DTYPE_F32) return fail(c, SFT_ERR_ARG, "bad dtype %d", dtype);
    if (on_device) {
        launch_f64_to_f32(c->stream, src, (float*)dst, n);
        return SFT_OK;
    }
    std::vector<double> tmp(n);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < n; ++i) ((float*)dst)[i] = (float)tmp[i];
    return SFT_OK;
}

sft_status sft_set_state(sft_ctx* c, int32_t id, const void* br, int32_t dtype, int32_t on_device)
{
    if (!c || !br) return SFT_ERR_ARG;
    GridClass* g;
    int r;
    if (!find_real(c, id, &g, &r)) return fail(c, SFT_ERR_ARG, "bad realization id %d", id);
    g->diag_valid = false;
    return copy_in(c, g->B + (size_t)r * g->cells(), br, g->cells(), dtype, on_device);
}

sft_status sft_get_state(sft_ctx* c, int32_t id, void* br, int32_t dtype, int32_t on_device)
{
    if (!c || !br) return SFT_ERR_ARG;
    GridClass* g;
    int r;
    if (!find_real(c, id, &g, &r)) return fail(c, SFT_ERR_ARG, "bad realization id %d", id);
    return copy_out(c, br, g->B + (size_t)r * g->cells(), g->cells(), dtype, on_device);
}

sft_status sft_set_states(sft_ctx* c, int32_t gid, const void* br, int32_t dtype, int32_t on_device)
{
    if (!c || !br || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    GridClass* g = c->grids[gid];
    if (!g->R) return fail(c, SFT_ERR_STATE, "grid %d has no realizations", gid);
    g->diag_valid = false;
    return copy_in(c, g->B, br, (size_t)g->R * g->cells(), dtype, on_device);
}

sft_status sft_get_states(sft_ctx* c, int32_t gid, void* br, int32_t dtype, int32_t on_device)
{
    if (!c || !br || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    GridClass* g = c->grids[gid];
    if (!g->R) return fail(c, SFT_ERR_STATE, "grid %d has no realizations", gid);
    return copy_out(c, br, g->B, (size_t)g->R * g->cells(), dtype, on_device);
}

static sft_status advance_impl(sft_ctx* c, double t_end, int sub_gid = -1,
                               const std::vector<char>* sub_mask = nullptr);

static void dfree(sft_ctx* c, void* ptr)
{
    if (!ptr) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), ptr);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(ptr);
}

// Frees every cached plan and graph (after the stream has drained).
static void drop_plans(sft_ctx* c)
{
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    c->graphs.clear();
    for (auto* g : c->grids) {
        for (auto& kv : g->plans) {
            for (Plan* p : kv.second) {
                dfree(c, p->d_ents);
                dfree(c, p->d_coefs);
                dfree(c, p->d_alpha);
                delete p;
            }
        }
        g->plans.clear();
    }
}

sft_status sft_advance(sft_ctx* c, double t_end)
{
    if (!c) return SFT_ERR_ARG;
    return advance_impl(c, t_end, -1);
}

// Runs one plan per lane of a class: lanes other than 0 on the library's
// streams, forked from and joined back into the context's stream.
static void run_class_lanes(sft_ctx* c, GridClass* g, const std::vector<Plan*>& lp)
{
    const hipStream_t main = c->stream;
    if (g->nl > 1) {
        (void)hipEventRecord(g->lane_ev[0], main);
        for (int l = 1; l < g->nl; ++l) (void)hipStreamWaitEvent(c->lane_st[l - 1], g->lane_ev[0], 0);
    }
    for (int l = 0; l < g->nl; ++l) {
        c->stream = l == 0 ? main : c->lane_st[l - 1];
        run_plan(c, g, lp[l], l);
    }
    c->stream = main;
    if (g->nl > 1) {
        for (int l = 1; l < g->nl; ++l) {
            (void)hipEventRecord(g->lane_ev[l], c->lane_st[l - 1]);
            (void)hipStreamWaitEvent(main, g->lane_ev[l], 0);
        }
    }
}

static void free_plans(sft_ctx* c, std::vector<Plan*>& lp)
{
    for (Plan* p : lp) {
        if (!p) continue;
        dfree(c, p->d_ents);
        dfree(c, p->d_coefs);
        dfree(c, p->d_alpha);
        delete p;
    }
    lp.clear();
}

static bool att_cfl_class(const sft_ctx* c, const GridClass* g) { return c->opt.att_cfl && g->att && g->R; }

// Advance of a class with attenuated flow under the per-step CFL limit
// (opt.att_cfl; Sec. "Time steps" with eq. ssprk43_dt of the flow of eq.
// flow_attenuation): each step starts with a device max-reduction of the
// attenuated flow's CFL rate over the current field of every realization
// with time left, read back to the host; each realization's step then
// follows the step rule, and the step runs as a one-step plan per lane.
static sft_status advance_att_cfl(sft_ctx* c, GridClass* g, double t0, double t_end, double len,
                                  const std::vector<char>* mask)
{
    const sft_options& o = c->opt;
    const double fac = (o.adv_time == SFT_SSPRK43 ? 1.0 : 0.5) * (o.strang ? 2.0 : 1.0);
    const double dth = M_PI / g->nt;
    std::vector<double> el(g->R, 0.0), rmax(g->R, 0.0), fixed(g->R, 0.0);
    std::vector<char> done(g->R, 0);
    if (mask)
        for (int r = 0; r < g->R; ++r) done[r] = !(*mask)[r];
    std::vector<Plan*> prev;
    for (;;) {
        g->h_cfl_ents.clear();
        for (int r = 0; r < g->R; ++r)
            if (!done[r]) g->h_cfl_ents.push_back(Entry{r, 0, 0, 0, 0.0});
        if (g->h_cfl_ents.empty()) break;
        const int ne = (int)g->h_cfl_ents.size();
        HIPCHK(c, hipMemcpyAsync(g->cfl_ents, g->h_cfl_ents.data(), ne * sizeof(Entry), hipMemcpyHostToDevice,
                                 c->stream));
        tbeg(c);
        launch_att_cfl(c->stream, g->cfl_ents, ne, g->adv64, g->att_b0, g->B, g->denph64, dth, g->cfl_partial,
                       g->cfl_rmax, g->nt, g->np);
        tend(c, SFT_KFAM_OTHER, 8.0 * (double)g->cells() * ne);
        HIPCHK(c, hipMemcpyAsync(rmax.data(), g->cfl_rmax, g->R * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_plans(c, prev);   // the previous step has drained
        for (int r = 0; r < g->R; ++r) {
            fixed[r] = 0.0;
            if (done[r]) continue;
            const double lim = rmax[r] > 0.0 ? fac / rmax[r] : INFINITY;
            bool fin = false;
            fixed[r] = next_step(len - el[r], o.cfl_safety * lim, o.dt_max, o.dt_min, &fin);
            el[r] = fin ? len : el[r] + fixed[r];
            if (fin) done[r] = 1;
        }
        prev.assign(g->nl, nullptr);
        for (int l = 0; l < g->nl; ++l) {
            sft_status st = build_plan(c, g, l, t0, t_end, len, &prev[l], &fixed);
            if (st != SFT_OK) {
                free_plans(c, prev);
                return st;
            }
        }
        run_class_lanes(c, g, prev);
        HIPCHK(c, hipGetLastError());
        for (Plan* p : prev)
            for (int r = 0; r < g->R; ++r) {
                g->steps[r] += p->steps[r];
                g->stages[r] += p->stages[r];
                g->adv_stages[r] += p->adv_stages[r];
                if (p->steps[r]) g->dt_last[r] = p->dt_last[r];
            }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_plans(c, prev);
    return SFT_OK;
}

// 64-bit hash of a realization mask (0 for none), for plan and graph keys.
static uint64_t mask_hash(const std::vector<char>* m)
{
    if (!m) return 0;
    uint64_t h = 0xcbf29ce484222325ull;
    for (char x : *m) h = (h ^ (uint64_t)(x != 0)) * 0x100000001b3ull;
    return h | 1;
}

// Advances every class to t_end.  Class sub_gid (if >= 0) advances only the
// realizations r with (*sub_mask)[r] != 0, none when sub_mask is NULL.
static sft_status advance_impl(sft_ctx* c, double t_end, int sub_gid, const std::vector<char>* sub_mask)
{
    const uint64_t mh = mask_hash(sub_mask);
    bool sub_none = sub_gid >= 0 && !sub_mask;
    if (sub_mask) {
        sub_none = true;
        for (char x : *sub_mask) sub_none &= x == 0;
    }
    if (!(t_end >= c->t) || !std::isfinite(t_end))
        return fail(c, SFT_ERR_ARG, "t_end %.17g before context time %.17g", t_end, c->t);
    bool any = false;
    for (auto* g : c->grids) any |= g->R > 0;
    if (!any) return fail(c, SFT_ERR_STATE, "no realizations");
    c->started = true;
    for (auto* g : c->grids)
        if (g->R && g->tile == -2) TRY(choose_tile(c, g));
    const double len = t_end - c->t;
    if (len == 0.0) return SFT_OK;
    // random flux emergence: a plan also depends on where the advance starts
    // in its source-map interval; k0 is the interval holding the start
    const bool rfe = c->opt.rfe_model != 0;
    const double tau = c->opt.rfe_lifetime_h;
    int64_t k0 = 0;
    uint64_t rkey = 0;
    if (rfe && tau > 0.0) {
        k0 = rfe_interval(c->t, tau);
        rkey = dbits(c->t - (double)k0 * tau) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
        // start phases need not repeat (tau incommensurate with the advances):
        // keep the caches bounded
        size_t np_max = 0;
        for (auto* g : c->grids) np_max = std::max(np_max, g->plans.size());
        if (np_max >= 64) drop_plans(c);
    }
    std::vector<std::vector<Plan*>*> plans;   // per class: one plan per lane
    for (size_t gi = 0; gi < c->grids.size(); ++gi) {
        GridClass* g = c->grids[gi];
        const bool sub = (int)gi == sub_gid;
        if (!g->R || (sub && sub_none) || att_cfl_class(c, g)) {
            plans.push_back(nullptr);
            continue;
        }
        const uint64_t key = dbits(len) ^ rkey ^ (sub ? mh : 0);
        auto it = g->plans.find(key);
        if (it == g->plans.end()) {
            std::vector<Plan*> lp(g->nl, nullptr);
            for (int l = 0; l < g->nl; ++l) {
                sft_status st = build_plan(c, g, l, c->t, t_end, len, &lp[l], nullptr, sub ? sub_mask : nullptr);
                if (st != SFT_OK) {
                    for (Plan* q : lp) delete q;
                    return st;
                }
            }
            it = g->plans.emplace(key, lp).first;
        }
        plans.push_back(&it->second);
    }
    // lanes of a class run on their own streams between a fork and a join
    // on the context's stream (captured as parallel branches in graphs)
    auto enqueue = [&]() {
        const hipStream_t main = c->stream;
        for (size_t i = 0; i < c->grids.size(); ++i) {
            GridClass* g = c->grids[i];
            if (!plans[i]) continue;
            c->stream = main;
            run_class_lanes(c, g, *plans[i]);
            if (c->opt.diag_every_call) launch_diag_class(c, g);
        }
    };
    bool work = false, dyn = false;
    for (auto* p : plans) work |= p != nullptr;
    for (size_t gi = 0; gi < c->grids.size(); ++gi)
        dyn |= !((int)gi == sub_gid && sub_none) && att_cfl_class(c, c->grids[gi]);
    if (!work && !dyn) {
        c->t = t_end;
        return SFT_OK;
    }
    // source maps of interval k0 (and k0 + 1) unless the device holds them
    // already (first advance, or a time set by the caller)
    if (rfe) {
        for (size_t i = 0; i < c->grids.size(); ++i) {
            GridClass* g = c->grids[i];
            if (!plans[i] || g->rfe_k == k0) continue;
            tbeg(c);
            for (int l = 0; l < g->nl; ++l) launch_rfe_set(c->stream, g->rfe_kdev + l, k0);
            tend(c, SFT_KFAM_SOURCE, 0.0);
            rfe_make_map(c, g, nullptr, 0, k0, -1);
            if (tau > 0.0) rfe_make_map(c, g, nullptr, 0, k0 + 1, -1);
            g->rfe_k = k0;
        }
    }
    if (!work) {
        // only classes stepped under the per-step attenuated CFL limit
    } else if (c->opt.use_graphs && !c->timing) {
        const uint64_t key = (dbits(len) ^ rkey) ^ (c->opt.diag_every_call ? 0x5bd1e995ull : 0) ^
                             ((uint64_t)(sub_gid + 1) << 52) ^ mh;
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            GraphEntry ge;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
            enqueue();
            HIPCHK(c, hipStreamEndCapture(c->stream, &ge.graph));
            HIPCHK(c, hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
            it = c->graphs.emplace(key, ge).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second.exec, c->stream));
    } else {
        enqueue();
        HIPCHK(c, hipGetLastError());
    }
    for (size_t i = 0; i < c->grids.size(); ++i) {
        GridClass* g = c->grids[i];
        if (!plans[i]) continue;
        g->rfe_k += (*plans[i])[0]->ticks;   // every lane steps onto the same map times
        for (Plan* p : *plans[i]) {
            for (int r = 0; r < g->R; ++r) {
                g->steps[r] += p->steps[r];
                g->stages[r] += p->stages[r];
                g->adv_stages[r] += p->adv_stages[r];
                if (p->steps[r]) g->dt_last[r] = p->dt_last[r];
            }
        }
        if (c->opt.diag_every_call) g->diag_valid = true;
        else g->diag_valid = false;
    }
    for (size_t gi = 0; gi < c->grids.size(); ++gi) {
        GridClass* g = c->grids[gi];
        const bool sub = (int)gi == sub_gid;
        if ((sub && sub_none) || !att_cfl_class(c, g)) continue;
        TRY(advance_att_cfl(c, g, c->t, t_end, len, sub ? sub_mask : nullptr));
        if (c->opt.diag_every_call) launch_diag_class(c, g);
        g->diag_valid = c->opt.diag_every_call != 0;
    }
    c->t = t_end;
    return SFT_OK;
}

sft_status sft_assimilate(sft_ctx* c, int32_t gid, const void* data, const void* weight, int32_t dtype,
                          int32_t kind, double b0_deg, double l0_deg, int32_t on_device)
{
    if (!c || !data || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    if (kind != SFT_WEIGHT_F && kind != SFT_WEIGHT_MU && kind != SFT_WEIGHT_DISK)
        return fail(c, SFT_ERR_ARG, "bad weight kind %d", kind);
    if (kind != SFT_WEIGHT_DISK && !weight) return fail(c, SFT_ERR_ARG, "weight array missing");
    if (dtype != SFT_DTYPE_F64 && dtype != SFT_DTYPE_F32) return fail(c, SFT_ERR_ARG, "bad dtype");
    GridClass* g = c->grids[gid];
    if (!g->R) return fail(c, SFT_ERR_STATE, "grid %d has no realizations", gid);
    const size_t n = g->cells();
    const size_t esz = dtype == SFT_DTYPE_F64 ? 8 : 4;
    const void* d_data = data;
    const void* d_w = weight;
    if (!on_device) {
        if (!g->stage_in) {
            hipError_t e = hipMalloc(&g->stage_in, 2 * n * sizeof(double));
            if (e != hipSuccess) return fail(c, SFT_ERR_OOM, "staging allocation failed");
            c->allocs.push_back(g->stage_in);
        }
        char* s = (char*)g->stage_in;
        HIPCHK(c, hipMemcpyAsync(s, data, n * esz, hipMemcpyHostToDevice, c->stream));
        d_data = s;
        if (kind != SFT_WEIGHT_DISK) {
            HIPCHK(c, hipMemcpyAsync(s + n * sizeof(double), weight, n * esz, hipMemcpyHostToDevice,
                                     c->stream));
            d_w = s + n * sizeof(double);
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    bool any_bal = false;
    for (auto& p : g->prm) any_bal |= p.flux_balance != 0;
    const double b0 = b0_deg * (M_PI / 180.0), l0 = l0_deg * (M_PI / 180.0);
    const double sb0 = sin(b0), cb0 = cos(b0);
    double* dB = nullptr;
    if (any_bal) {
        if (c->opt.precision == SFT_FP64) {
            dB = g->W[0];
        } else {
            if (!g->dB) TRY(dalloc(c, &g->dB, (size_t)g->R * n));
            dB = g->dB;
        }
        tbeg(c);
        launch_assim_delta(c->stream, g->R, g->ar, d_data, d_w, dtype, kind, sb0, cb0, l0, g->B, g->st_row,
                           g->ct_row, g->lat_row, g->w_row, dB, g->assim_partial, g->red_nblk, g->nt,
                           g->np);
        launch_assim_reduce(c->stream, g->R, g->assim_partial, g->red_nblk, g->assim_ratio);
        tend(c, SFT_KFAM_ASSIM, (double)n * g->R * (24.0 + (kind != SFT_WEIGHT_DISK ? 8.0 : 0.0)));
    }
    tbeg(c);
    launch_assim_apply(c->stream, g->R, g->ar, d_data, d_w, dtype, kind, sb0, cb0, l0, g->B, dB,
                       g->assim_ratio, g->st_row, g->ct_row, g->lat_row, g->red_nblk, g->nt, g->np);
    {
        double per = 0.0;
        for (auto& p : g->prm)
            per += p.flux_balance ? 24.0 : 24.0 + (kind != SFT_WEIGHT_DISK ? 8.0 : 0.0);
        tend(c, SFT_KFAM_ASSIM, per * (double)n);
    }
    for (int r = 0; r < g->R; ++r) g->assim[r] += 1;
    if (c->opt.diag_every_call) launch_diag_class(c, g);
    else g->diag_valid = false;
    HIPCHK(c, hipGetLastError());
    return SFT_OK;
}

sft_status sft_assimilate_noalloc(sft_ctx* c, int32_t gid, const void* data, const void* weight,
                                  int32_t dtype, int32_t kind, double b0_deg, double l0_deg)
{
    if (!c || !data || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    if (kind != SFT_WEIGHT_F && kind != SFT_WEIGHT_MU && kind != SFT_WEIGHT_DISK)
        return fail(c, SFT_ERR_ARG, "bad weight kind %d", kind);
    if (kind != SFT_WEIGHT_DISK && !weight) return fail(c, SFT_ERR_ARG, "weight array missing");
    if (dtype != SFT_DTYPE_F64 && dtype != SFT_DTYPE_F32) return fail(c, SFT_ERR_ARG, "bad dtype");
    GridClass* g = c->grids[gid];
    if (!g->R) return fail(c, SFT_ERR_STATE, "grid %d has no realizations", gid);
    const size_t need = (size_t)g->R * (2 * (size_t)g->red_nblk + 1);
    if (need > kNoAllocDoubles)
        return fail(c, SFT_ERR_ARG, "grid %d needs %zu scratch doubles, the limit is %zu", gid, need,
                    kNoAllocDoubles);
    double* sp = scratch_ptr(c->device);
    if (!sp) return fail(c, SFT_ERR_HIP, "no scratch address for device %d", c->device);
    double* partial = sp;
    double* ratio = sp + (size_t)g->R * 2 * g->red_nblk;
    bool any_bal = false;
    for (auto& p : g->prm) any_bal |= p.flux_balance != 0;
    const double b0 = b0_deg * (M_PI / 180.0), l0 = l0_deg * (M_PI / 180.0);
    const double sb0 = sin(b0), cb0 = cos(b0);
    // no stored increment: the apply pass forms dB again, with the same bits
    if (any_bal) {
        launch_assim_delta(c->stream, g->R, g->ar, data, weight, dtype, kind, sb0, cb0, l0, g->B, g->st_row,
                           g->ct_row, g->lat_row, g->w_row, nullptr, partial, g->red_nblk, g->nt, g->np);
        launch_assim_reduce(c->stream, g->R, partial, g->red_nblk, ratio);
    }
    launch_assim_apply(c->stream, g->R, g->ar, data, weight, dtype, kind, sb0, cb0, l0, g->B, nullptr, ratio,
                       g->st_row, g->ct_row, g->lat_row, g->red_nblk, g->nt, g->np);
    for (int r = 0; r < g->R; ++r) g->assim[r] += 1;
    g->diag_valid = false;
    HIPCHK(c, hipGetLastError());
    return SFT_OK;
}

sft_status sft_diagnostics(sft_ctx* c, int32_t id, sft_diag* out)
{
    if (!c || !out) return SFT_ERR_ARG;
    GridClass* g;
    int r;
    if (!find_real(c, id, &g, &r)) return fail(c, SFT_ERR_ARG, "bad realization id %d", id);
    if (!g->diag_valid) launch_diag_class(c, g);
    DiagRec d;
    HIPCHK(c, hipMemcpyAsync(&d, g->diag_out + r, sizeof d, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    memset(out, 0, sizeof *out);
    out->t = c->t;
    out->dt_last = g->dt_last[r];
    out->steps = g->steps[r];
    out->stages = g->stages[r];
    out->phi_pos = d.pp;
    out->phi_neg = d.pm;
    out->phi_net = d.pp + d.pm;
    out->h1 = d.h1;
    out->h2 = d.h2;
    out->dax = d.dax;
    out->bmin = d.bmin;
    out->bmax = d.bmax;
    out->babs_min = d.babs;
    out->nonfinite = (int32_t)d.nonfinite;
    out->surr_accept = g->s_acc[r];
    out->surr_reject = g->s_rej[r];
    if (out->nonfinite) return fail(c, SFT_ERR_NOT_FINITE, "realization %d holds %d non-finite cells", id,
                                    out->nonfinite);
    return SFT_OK;
}

sft_status sft_surrogate_advance(sft_ctx* c, int32_t gid, sft_net* net, const float* feats, double t_end,
                                 double tol, int32_t check, double* err_out)
{
    if (!c || !net || !feats || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    GridClass* g = c->grids[gid];
    if (!g->R) return fail(c, SFT_ERR_STATE, "grid %d has no realizations", gid);
    int H, W, maxb;
    net_dims(net, &H, &W, &maxb);
    if (H != g->nt || W != g->np) return fail(c, SFT_ERR_SHAPE, "network grid %dx%d != class %dx%d", H, W,
                                              g->nt, g->np);
    if (!(fabs(t_end - c->t - SURROGATE_INTERVAL_H) <= 1e-9))
        return fail(c, SFT_ERR_ARG, "the surrogate advances one %g h interval (t_end - t = %.17g)",
                    SURROGATE_INTERVAL_H, t_end - c->t);
    if (check < 0) return fail(c, SFT_ERR_ARG, "check must be >= 0 (got %d)", check);
    if (!(tol >= 0.0)) return fail(c, SFT_ERR_ARG, "tol must be >= 0");
    const size_t n = g->cells();
    if (!g->pred) {
        TRY(dalloc(c, &g->pred, (size_t)g->R * n));
        TRY(dalloc(c, &g->sfeat, (size_t)g->R * 3));
        TRY(dalloc(c, &g->spart, (size_t)g->R * g->red_nblk * 2));
        TRY(dalloc(c, &g->serr, (size_t)g->R));
        TRY(dalloc(c, &g->sacc, (size_t)g->R));
        TRY(dalloc(c, &g->swant, (size_t)g->R));
    }
    // which realizations the plain solver checks this interval: all (check
    // = 1), none (0), or every check-th surrogate interval of each
    // realization and every interval of one whose last check failed
    g->h_swant.assign(g->R, 0);
    int nwant = 0;
    for (int r = 0; r < g->R; ++r) {
        const bool w = check == 1 || (check > 1 && (g->s_esc[r] || g->s_count[r] % check == 0));
        g->h_swant[r] = w ? 1 : 0;
        nwant += w ? 1 : 0;
    }
    HIPCHK(c, hipMemcpyAsync(g->sfeat, feats, (size_t)g->R * 3 * sizeof(float), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(g->swant, g->h_swant.data(), (size_t)g->R * sizeof(int), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->started = true;
    // surrogate prediction for every realization of the class, before the
    // plain solver touches the state
    for (int r0 = 0; r0 < g->R; r0 += maxb) {
        const int nb = std::min(maxb, g->R - r0);
        float* y = nullptr;
        TRY(net_predict(net, c->stream, nb, g->B + (size_t)r0 * n, g->sfeat + (size_t)r0 * 3, &y));
        cnn_pred(c->stream, g->B + (size_t)r0 * n, y, g->pred + (size_t)r0 * n, (size_t)nb * n);
    }
    if (nwant) {
        // plain advance of the checked realizations (and of every other
        // class), then each checked realization keeps the surrogate field
        // only within tol (relative L2) of the plain one; the unchecked ones
        // take the surrogate field
        std::vector<char> mask(g->R);
        for (int r = 0; r < g->R; ++r) mask[r] = (char)g->h_swant[r];
        TRY(advance_impl(c, t_end, nwant == g->R ? -1 : gid, nwant == g->R ? nullptr : &mask));
        cnn_check(c->stream, g->pred, g->B, g->spart, g->red_nblk, g->R, n, tol, g->serr, g->sacc, g->B,
                  nwant == g->R ? nullptr : g->swant);
        std::vector<int> acc(g->R);
        std::vector<double> err(g->R);
        HIPCHK(c, hipMemcpyAsync(acc.data(), g->sacc, g->R * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(err.data(), g->serr, g->R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int r = 0; r < g->R; ++r) {
            if (g->h_swant[r]) {
                if (acc[r]) g->s_acc[r] += 1;
                else g->s_rej[r] += 1;
                g->s_esc[r] = acc[r] ? 0 : 1;
            } else {
                g->s_unchk[r] += 1;
            }
            if (err_out) err_out[r] = g->h_swant[r] ? err[r] : -1.0;
        }
    } else {
        TRY(advance_impl(c, t_end, gid, nullptr));
        HIPCHK(c, hipMemcpyAsync(g->B, g->pred, (size_t)g->R * n * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
        for (int r = 0; r < g->R; ++r) {
            g->s_unchk[r] += 1;
            if (err_out) err_out[r] = -1.0;
        }
        c->t = t_end;
    }
    for (int r = 0; r < g->R; ++r) g->s_count[r] += 1;
    if (c->opt.diag_every_call) launch_diag_class(c, g);
    else g->diag_valid = false;
    HIPCHK(c, hipGetLastError());
    return SFT_OK;
}

sft_status sft_surrogate_counts(sft_ctx* c, int32_t id, int64_t* accepted, int64_t* rejected,
                                int64_t* unchecked, int32_t* escalated)
{
    if (!c) return SFT_ERR_ARG;
    GridClass* g;
    int r;
    if (!find_real(c, id, &g, &r)) return fail(c, SFT_ERR_ARG, "bad realization id %d", id);
    if (accepted) *accepted = g->s_acc[r];
    if (rejected) *rejected = g->s_rej[r];
    if (unchecked) *unchecked = g->s_unchk[r];
    if (escalated) *escalated = g->s_esc[r];
    return SFT_OK;
}

sft_status sft_time(sft_ctx* c, double* t)
{
    if (!c || !t) return SFT_ERR_ARG;
    *t = c->t;
    return SFT_OK;
}

sft_status sft_set_time(sft_ctx* c, double t)
{
    if (!c || !std::isfinite(t)) return SFT_ERR_ARG;
    c->t = t;
    return SFT_OK;
}

sft_status sft_sync(sft_ctx* c)
{
    if (!c) return SFT_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SFT_OK;
}

sft_status sft_counts(sft_ctx* c, int32_t id, int64_t* steps, int64_t* stages, int64_t* adv_stages,
                      int64_t* assim)
{
    if (!c) return SFT_ERR_ARG;
    GridClass* g;
    int r;
    if (!find_real(c, id, &g, &r)) return fail(c, SFT_ERR_ARG, "bad realization id %d", id);
    if (steps) *steps = g->steps[r];
    if (stages) *stages = g->stages[r];
    if (adv_stages) *adv_stages = g->adv_stages[r];
    if (assim) *assim = g->assim[r];
    return SFT_OK;
}

sft_status sft_set_timing(sft_ctx* c, int32_t on)
{
    if (!c) return SFT_ERR_ARG;
    harvest(c, c->pending.size());
    for (int f = 0; f < SFT_KFAM_COUNT; ++f) {
        c->fam_ms[f] = 0.0;
        c->fam_n[f] = 0;
        c->fam_bytes[f] = 0.0;
        c->fam_min[f] = 0.0;
    }
    c->timing = on != 0;
    return SFT_OK;
}

sft_status sft_get_timing(sft_ctx* c, int32_t fam, double* total_ms, int64_t* launches, double* bytes,
                          double* min_bytes)
{
    if (!c || fam < 0 || fam >= SFT_KFAM_COUNT) return SFT_ERR_ARG;
    harvest(c, c->pending.size());
    if (total_ms) *total_ms = c->fam_ms[fam];
    if (launches) *launches = c->fam_n[fam];
    if (bytes) *bytes = c->fam_bytes[fam];
    if (min_bytes) *min_bytes = c->fam_min[fam];
    return SFT_OK;
}

sft_status sft_tile_info(int32_t precision, int32_t index, int32_t* tx, int32_t* ty, int32_t* k,
                         int32_t* nthreads)
{
    const bool mixed = precision == SFT_FP32_MIXED;
    if ((precision != SFT_FP64 && !mixed) || index < 0 || index >= fused_config_count(mixed))
        return SFT_ERR_ARG;
    int a, b, cc, d;
    fused_config_desc(mixed, index, &a, &b, &cc, &d);
    if (tx) *tx = a;
    if (ty) *ty = b;
    if (k) *k = cc;
    if (nthreads) *nthreads = d;
    return SFT_OK;
}

sft_status sft_tile_choice(sft_ctx* c, int32_t gid, int32_t* index)
{
    if (!c || !index || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    *index = c->grids[gid]->tile;
    return SFT_OK;
}

sft_status sft_set_class_tile(sft_ctx* c, int32_t gid, int32_t index)
{
    if (!c || gid < 0 || gid >= (int)c->grids.size()) return SFT_ERR_ARG;
    const bool mixed = c->opt.precision == SFT_FP32_MIXED;
    if (index < -1 || index >= fused_config_count(mixed)) return fail(c, SFT_ERR_ARG, "bad tile index %d", index);
    GridClass* g = c->grids[gid];
    if (mixed && index >= 0 && g->cells() * sizeof(double) > 0xFFFFFFFFull)
        return fail(c, SFT_ERR_UNSUPPORTED, "blocked FP32 stages need nt*np*8 < 2^32 bytes (grid %dx%d)", g->nt,
                    g->np);
    drop_plans(c);
    g->tile = index;
    return SFT_OK;
}

sft_status sft_destroy(sft_ctx* c)
{
    if (!c) return SFT_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    for (hipStream_t s : c->lane_st) (void)hipStreamSynchronize(s);
    for (auto& kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    harvest(c, c->pending.size());
    for (hipEvent_t e : c->free_ev) (void)hipEventDestroy(e);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    for (hipStream_t s : c->lane_st) (void)hipStreamDestroy(s);
    for (auto* g : c->grids) {
        for (auto& kv : g->plans)
            for (Plan* p : kv.second) delete p;
        for (hipEvent_t e : g->lane_ev)
            if (e) (void)hipEventDestroy(e);
        delete g;
    }
    delete c;
    return SFT_OK;
}

}  // extern "C"
