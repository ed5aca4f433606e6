/*
 * Plain FP64 CPU oracle of the surface-flux-transport hot path
 * (Caplan et al., "Open-source Flux Transport I: HipFT").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against an
 * independent, slow, obviously-correct implementation written straight from
 * the paper.  It shares no code, header or table with the GPU library.
 *
 * Every routine follows one passage of the paper, cited by section and
 * equation label.  The arithmetic is kept in the paper's order; the only
 * parallelism is an OpenMP loop over grid rows, which changes no result.
 *
 * Grid reading (paper Sec. "Grid" and App. A): uniform cell-centred finite
 * volume grid, nt rows in colatitude of width dth = pi/nt with centres
 * theta_j = (j+1/2) dth, np periodic columns of width dph = 2 pi/np with
 * centres phi_k = (k+1/2) dph.  Theta faces f = 0..nt sit at theta = f dth;
 * the two pole faces have zero length (sin = 0) and carry no flux, which is
 * App. A's divergence-theorem closure applied to each pole-row wedge cell.
 * Fields are stored row-major B[j*np + k] (phi contiguous).
 *
 * Units (paper Sec. "Units"): length in solar radii, time in hours,
 * B in gauss.
 *
 * Parity notes: every function here is pinned by a test in tests/ against
 * closed forms, library routines or brute force.  The one rule the paper
 * only cites, the practical time step limit of the diffusion advance, enters
 * as an input (ptl_dt); what is pinned there is the split it drives.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ units */
/* Paper Sec. "Units": R_sun = 6.96e8 m; m/s -> R_sun/h and km^2/s -> R_sun^2/h. */
static const double OR_RSUN_M = 6.96e8;

void or_units(double *m_s_to_rs_hr, double *km2_s_to_rs2_hr)
{
    *m_s_to_rs_hr = 3600.0 / OR_RSUN_M;
    *km2_s_to_rs2_hr = 3600.0 * 1.0e6 / (OR_RSUN_M * OR_RSUN_M);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* --------------------------------------------------------------- geometry */
typedef struct {
    int nt, np;
    double dth, dph;
    double *st;   /* sin(theta_j), cell centres            [nt]   */
    double *ct;   /* cos(theta_j)                          [nt]   */
    double *sf;   /* sin at theta faces, exactly 0 at poles [nt+1] */
} or_geom;

static void geom_init(or_geom *g, int nt, int np)
{
    g->nt = nt;
    g->np = np;
    g->dth = M_PI / nt;
    g->dph = 2.0 * M_PI / np;
    g->st = (double *)malloc(sizeof(double) * nt);
    g->ct = (double *)malloc(sizeof(double) * nt);
    g->sf = (double *)malloc(sizeof(double) * (nt + 1));
    for (int j = 0; j < nt; ++j) {
        double th = (j + 0.5) * g->dth;
        g->st[j] = sin(th);
        g->ct[j] = cos(th);
    }
    for (int f = 0; f <= nt; ++f) g->sf[f] = sin(f * g->dth);
    g->sf[0] = 0.0;
    g->sf[nt] = 0.0;
}

static void geom_free(or_geom *g)
{
    free(g->st);
    free(g->ct);
    free(g->sf);
}

/* Cell weights w_j = sin(theta_j) dth dph: the quadrature of the paper's
 * solid-angle element dOmega = sin(theta) dtheta dphi (Sec. "Analysis"). */
void or_cell_weights(int nt, int np, double *w)
{
    double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    for (int j = 0; j < nt; ++j) w[j] = sin((j + 0.5) * dth) * dth * dph;
}

/* ------------------------------------------------------------------ flows */
/* Eq. dr (differential rotation) evaluated at the cell centres of each row
 * (v_phi is needed on phi faces, which share the row's theta), and eq. mf
 * (meridional flow) evaluated on the theta faces; poles get exactly 0.
 * prm = {d0, d2, d4, m1, m3, m5} in m/s; outputs in R_sun/h. */
void or_flows(int nt, const double *prm, double *vph_row, double *vth_face)
{
    double ms, k2;
    or_units(&ms, &k2);
    double dth = M_PI / nt;
    for (int j = 0; j < nt; ++j) {
        double th = (j + 0.5) * dth;
        double c = cos(th), s = sin(th);
        double c2 = c * c;
        double v = (prm[0] + prm[1] * c2 + prm[2] * c2 * c2) * s;
        vph_row[j] = v * ms;
    }
    for (int f = 0; f <= nt; ++f) {
        double th = f * dth;
        double c = cos(th), s = sin(th);
        double c2 = c * c;
        double v = -(prm[3] * c + prm[4] * c2 * c + prm[5] * c2 * c2 * c) * s;
        vth_face[f] = v * ms;
    }
    vth_face[0] = 0.0;
    vth_face[nt] = 0.0;
}

/* ---------------------------------------------------------------- CFL (dt) */
/* Eq. advection_timestep (forward Euler, factor 1/2) and eq. ssprk43_dt
 * (SSPRK(4,3), twice as large).  Velocities per cell are the larger of the
 * two flanking staggered values in each direction.  Returns the limit
 * without safety factor; +inf when there is no flow.
 * time_scheme: 0 = SSPRK(4,3), 1 = forward Euler, 2 = SSPRK(3,3). */
double or_cfl_dt(int nt, int np, const double *vph_row, const double *vth_face, int time_scheme)
{
    double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    double rmax = 0.0;
    for (int j = 0; j < nt; ++j) {
        double s = sin((j + 0.5) * dth);
        double a = fabs(vth_face[j]), b = fabs(vth_face[j + 1]);
        double vt = a > b ? a : b;
        double vp = fabs(vph_row[j]);
        double r = vt / dth + vp / (s * dph);
        if (r > rmax) rmax = r;
    }
    if (rmax == 0.0) return INFINITY;
    double lim = 1.0 / rmax;
    if (time_scheme != 0) lim *= 0.5;
    return lim;
}

/* Eq. ssprk43_dt (or eq. advection_timestep) for the attenuated flow of
 * eq. flow_attenuation: each face velocity is scaled by 1 - tanh(m/b0), m
 * the mean of |Batt| over the face's two cells (as in the advection
 * operator), and each cell takes the larger of its two flanking face speeds
 * in theta and in phi.  Batt is the field at the start of the step.  Returns
 * the limit without safety factor; +inf when nothing moves. */
double or_cfl_dt_att(int nt, int np, const double *vph_row, const double *vth_face, const double *Batt,
                     double b0, int time_scheme)
{
    double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    double rmax = 0.0;
    for (int j = 0; j < nt; ++j) {
        double s = sin((j + 0.5) * dth);
        for (int k = 0; k < np; ++k) {
            size_t c = (size_t)j * np + k;
            size_t w = (size_t)j * np + (k + np - 1) % np, e = (size_t)j * np + (k + 1) % np;
            double vw = fabs(vph_row[j] * (1.0 - tanh(0.5 * (fabs(Batt[w]) + fabs(Batt[c])) / b0)));
            double ve = fabs(vph_row[j] * (1.0 - tanh(0.5 * (fabs(Batt[c]) + fabs(Batt[e])) / b0)));
            double vn = j == 0 ? fabs(vth_face[0])
                               : fabs(vth_face[j] *
                                      (1.0 - tanh(0.5 * (fabs(Batt[c - np]) + fabs(Batt[c])) / b0)));
            double vs = j == nt - 1 ? fabs(vth_face[nt])
                                    : fabs(vth_face[j + 1] *
                                           (1.0 - tanh(0.5 * (fabs(Batt[c]) + fabs(Batt[c + np])) / b0)));
            double vt = vn > vs ? vn : vs;
            double vp = vw > ve ? vw : ve;
            double r = vt / dth + vp / (s * dph);
            if (r > rmax) rmax = r;
        }
    }
    if (rmax == 0.0) return INFINITY;
    double lim = 1.0 / rmax;
    if (time_scheme != 0) lim *= 0.5;
    return lim;
}

/* ------------------------------------------------------- advection fluxes */
/* Upwind / central face flux (Sec. "Advection spatial schemes"):
 * F_{i-1/2} = v_{i-1/2} (1/2)[(1-uw) B_i + (1+uw) B_{i-1}],
 * uw = alpha_uw sign(v_{i-1/2}), alpha_uw = 1 for upwinding. */
static double flux_upwind(double v, double bl, double br)
{
    double sg = v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0);
    double uw = 1.0 * sg;
    return v * 0.5 * ((1.0 - uw) * br + (1.0 + uw) * bl);
}

/* One line of cells (one row in phi or one column in theta) for WENO3-CS(h)
 * (App. B).  Cells i = 0..n-1 of widths dx[i]; face f (f = 0..n) lies
 * between cells f-1 and f, velocity v[f].  Periodic lines wrap all indices;
 * open (theta) lines use WENO on faces 2..n-2, upwind on faces 1 and n-1
 * and zero flux on faces 0 and n (Sec. "Advection spatial schemes",
 * boundary conditions, and App. A).
 *
 * Readings (the appendix is garbled or silent here):
 *  - the factors printed as "D_i" are the ones at face i-1/2;
 *  - alpha_i is the largest |v| on faces i-5/2 .. i+5/2, clipped to the
 *    existing faces on an open line;
 *  - the LLF split uses the one-sided face velocity exactly as printed;
 *  - eps_w = h is the width of cell i (the cell right of the face) in
 *    radians of the sweep direction; eps_mode > 0 replaces it by eps_mode
 *    (the "WENO3 with constant eps" comparison of App. B).
 * scheme: 0 = WENO3-CS(h) (or constant eps), 1 = upwind everywhere. */
static int wrapi(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

void or_line_flux(int n, int periodic, const double *B, const double *dx, const double *v,
                  int scheme, double eps_mode, double *F)
{
    /* per-cell alpha and the LLF split */
    double *LP = (double *)malloc(sizeof(double) * n);
    double *LM = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int f = i - 2; f <= i + 3; ++f) {
            int ff;
            if (periodic) {
                ff = wrapi(f, n);
            } else {
                if (f < 0 || f > n) continue;
                ff = f;
            }
            double av = fabs(v[ff]);
            if (av > a) a = av;
        }
        int fr = periodic ? wrapi(i + 1, n) : i + 1;
        LP[i] = 0.5 * B[i] * (v[fr] - a);
        LM[i] = 0.5 * B[i] * (v[i] + a);
    }

#define CELL(i) (periodic ? wrapi((i), n) : (i))
    for (int f = 0; f <= n; ++f) {
        if (periodic && f == n) {
            F[n] = F[0];
            continue;
        }
        if (!periodic && (f == 0 || f == n)) {
            F[f] = 0.0;
            continue;
        }
        int use_upwind = (scheme == 1) || (!periodic && (f == 1 || f == n - 1));
        if (use_upwind) {
            F[f] = flux_upwind(v[f], B[CELL(f - 1)], B[CELL(f)]);
            continue;
        }
        int im2 = CELL(f - 2), im1 = CELL(f - 1), i0 = CELL(f), ip1 = CELL(f + 1);
        /* D factors at face f (i-1/2) use dx[i-1], dx[i], dx[i+1];
         * at face f-1 (i-3/2) they use dx[i-2], dx[i-1], dx[i]. */
        double xm2 = dx[im2], xm1 = dx[im1], x0 = dx[i0], xp1 = dx[ip1];
        double Dcp_h = x0 / (x0 + xp1);            /* D^{c/cp}_{i-1/2} */
        double Dcm_h = x0 / (x0 + xm1);            /* D^{c/cm}_{i-1/2} */
        double S_h = xm1 + x0 + xp1;
        double Dmt_h = xm1 / S_h;                  /* D^{m/t}_{i-1/2}  */
        double Dcpt_h = (x0 + xp1) / S_h;          /* D^{cp/t}_{i-1/2} */
        double Dcp_l = xm1 / (xm1 + x0);           /* D^{c/cp}_{i-3/2} */
        double Dcm_l = xm1 / (xm1 + xm2);          /* D^{c/cm}_{i-3/2} */
        double S_l = xm2 + xm1 + x0;
        double Dpt_l = x0 / S_l;                   /* D^{p/t}_{i-3/2}  */
        double Dcmt_l = (xm1 + xm2) / S_l;         /* D^{cm/t}_{i-3/2} */
        double eps = eps_mode > 0.0 ? eps_mode : x0;

        /* right-moving part u^- from LM at i-2, i-1, i */
        double p0m = (1.0 + Dcm_l) * LM[im1] - Dcm_l * LM[im2];
        double p1m = Dcm_h * LM[im1] + Dcp_l * LM[i0];
        double t0m = Dcm_l * (LM[im1] - LM[im2]);
        double t1m = Dcp_l * (LM[i0] - LM[im1]);
        double b0m = 4.0 * t0m * t0m;
        double b1m = 4.0 * t1m * t1m;
        double w0m = Dpt_l / ((eps + b0m) * (eps + b0m));
        double w1m = Dcmt_l / ((eps + b1m) * (eps + b1m));
        double um = (w0m / (w0m + w1m)) * p0m + (w1m / (w0m + w1m)) * p1m;

        /* left-moving part u^+ from LP at i-1, i, i+1 */
        double p0p = (1.0 + Dcp_h) * LP[i0] - Dcp_h * LP[ip1];
        double p1p = Dcp_l * LP[i0] + Dcm_h * LP[im1];
        double t0p = Dcp_h * (LP[ip1] - LP[i0]);
        double t1p = Dcm_h * (LP[i0] - LP[im1]);
        double b0p = 4.0 * t0p * t0p;
        double b1p = 4.0 * t1p * t1p;
        double w0p = Dmt_h / ((eps + b0p) * (eps + b0p));
        double w1p = Dcpt_h / ((eps + b1p) * (eps + b1p));
        double up = (w0p / (w0p + w1p)) * p0p + (w1p / (w0p + w1p)) * p1p;

        F[f] = up + um;
    }
#undef CELL
    free(LP);
    free(LM);
}

/* Spherical advection divergence (Sec. "Advection spatial schemes"):
 * [div(B v)]_jk = (s_{j+1/2} F^th_{j+1/2} - s_{j-1/2} F^th_{j-1/2}) / (s_j dth)
 *               + (F^ph_{k+1/2} - F^ph_{k-1/2}) / (s_j dph). */
/* Flow attenuation (eq. flow_attenuation): a face velocity is multiplied by
 * 1 - tanh(|B|/b0) with |B| read as the mean of |Batt| over the face's two
 * cells; Batt is the field at the start of the advection advance.  Batt =
 * NULL or b0 <= 0: no attenuation. */
static double att_factor(const double *Batt, double b0, size_t i0, size_t i1)
{
    if (!Batt || !(b0 > 0.0)) return 1.0;
    return 1.0 - tanh(0.5 * (fabs(Batt[i0]) + fabs(Batt[i1])) / b0);
}

void or_adv_operator_att(int nt, int np, const double *B, const double *vph_row,
                         const double *vth_face, int scheme, double eps_mode, const double *Batt,
                         double b0, double *out);

void or_adv_operator(int nt, int np, const double *B, const double *vph_row,
                     const double *vth_face, int scheme, double eps_mode, double *out)
{
    or_adv_operator_att(nt, np, B, vph_row, vth_face, scheme, eps_mode, NULL, 0.0, out);
}

void or_adv_operator_att(int nt, int np, const double *B, const double *vph_row,
                         const double *vth_face, int scheme, double eps_mode, const double *Batt,
                         double b0, double *out)
{
    or_geom g;
    geom_init(&g, nt, np);
    double *Fth = (double *)malloc(sizeof(double) * (size_t)(nt + 1) * np);
    double *Fph = (double *)malloc(sizeof(double) * (size_t)nt * (np + 1));

    /* phi sweeps, one per row */
    #pragma omp parallel
    {
        double *dxp = (double *)malloc(sizeof(double) * np);
        double *vp = (double *)malloc(sizeof(double) * (np + 1));
        #pragma omp for schedule(static)
        for (int j = 0; j < nt; ++j) {
            for (int k = 0; k < np; ++k) dxp[k] = g.dph;
            /* face k lies between cells k-1 and k (periodic) */
            for (int k = 0; k < np; ++k)
                vp[k] = vph_row[j] * att_factor(Batt, b0, (size_t)j * np + (k + np - 1) % np,
                                                (size_t)j * np + k);
            vp[np] = vp[0];
            or_line_flux(np, 1, B + (size_t)j * np, dxp, vp, scheme, eps_mode,
                         Fph + (size_t)j * (np + 1));
        }
        free(dxp);
        free(vp);
    }
    /* theta sweeps, one per column */
    #pragma omp parallel
    {
        double *dxt = (double *)malloc(sizeof(double) * nt);
        double *col = (double *)malloc(sizeof(double) * nt);
        double *Fc = (double *)malloc(sizeof(double) * (nt + 1));
        double *vt = (double *)malloc(sizeof(double) * (nt + 1));
        #pragma omp for schedule(static)
        for (int k = 0; k < np; ++k) {
            for (int j = 0; j < nt; ++j) {
                dxt[j] = g.dth;
                col[j] = B[(size_t)j * np + k];
            }
            /* face f lies between rows f-1 and f; the pole faces carry v = 0 */
            vt[0] = vth_face[0];
            vt[nt] = vth_face[nt];
            for (int f = 1; f < nt; ++f)
                vt[f] = vth_face[f] * att_factor(Batt, b0, (size_t)(f - 1) * np + k, (size_t)f * np + k);
            or_line_flux(nt, 0, col, dxt, vt, scheme, eps_mode, Fc);
            for (int f = 0; f <= nt; ++f) Fth[(size_t)f * np + k] = Fc[f];
        }
        free(dxt);
        free(col);
        free(Fc);
        free(vt);
    }
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nt; ++j) {
        for (int k = 0; k < np; ++k) {
            double dthf = (g.sf[j + 1] * Fth[(size_t)(j + 1) * np + k] -
                           g.sf[j] * Fth[(size_t)j * np + k]) / (g.st[j] * g.dth);
            double dphf = (Fph[(size_t)j * (np + 1) + k + 1] - Fph[(size_t)j * (np + 1) + k]) /
                          (g.st[j] * g.dph);
            out[(size_t)j * np + k] = dthf + dphf;
        }
    }
    free(Fth);
    free(Fph);
    geom_free(&g);
}

/* One advection step (Sec. "Advection temporal schemes").
 * time_scheme 0: SSPRK(4,3)
 *   f1 = fn - dt/2 A(fn); f2 = f1 - dt/2 A(f1);
 *   f3 = 2/3 fn + 1/3 f2 - dt/6 A(f2); fn+1 = f3 - dt/2 A(f3)
 * time_scheme 1: forward Euler (eq. adv_euler)
 * time_scheme 2: SSPRK(3,3)
 *   f1 = fn - dt A(fn); f2 = 3/4 fn + 1/4 f1 - dt/4 A(f1);
 *   fn+1 = 1/3 fn + 2/3 f2 - 2/3 dt A(f2)
 * A is the divergence operator above; B is updated in place. */
void or_adv_step_att(int nt, int np, double *B, const double *vph_row, const double *vth_face,
                     double dt, int scheme, int time_scheme, double eps_mode, double b0);

void or_adv_step(int nt, int np, double *B, const double *vph_row, const double *vth_face,
                 double dt, int scheme, int time_scheme, double eps_mode)
{
    or_adv_step_att(nt, np, B, vph_row, vth_face, dt, scheme, time_scheme, eps_mode, 0.0);
}

/* The same with flow attenuation b0 (gauss, <= 0: none), its factors taken
 * from the field at the start of the advance (fn) for every stage. */
void or_adv_step_att(int nt, int np, double *B, const double *vph_row, const double *vth_face,
                     double dt, int scheme, int time_scheme, double eps_mode, double b0)
{
    size_t n = (size_t)nt * np;
    double *fn = (double *)malloc(sizeof(double) * n);
    double *fa = (double *)malloc(sizeof(double) * n);
    double *fb = (double *)malloc(sizeof(double) * n);
    double *op = (double *)malloc(sizeof(double) * n);
    memcpy(fn, B, sizeof(double) * n);
    if (time_scheme == 1) {
        or_adv_operator_att(nt, np, fn, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) B[i] = fn[i] - dt * op[i];
    } else if (time_scheme == 2) {
        or_adv_operator_att(nt, np, fn, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) fa[i] = fn[i] - dt * op[i];
        or_adv_operator_att(nt, np, fa, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) fb[i] = 0.75 * fn[i] + 0.25 * fa[i] - 0.25 * dt * op[i];
        or_adv_operator_att(nt, np, fb, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i)
            B[i] = (1.0 / 3.0) * fn[i] + (2.0 / 3.0) * fb[i] - (2.0 / 3.0) * dt * op[i];
    } else {
        or_adv_operator_att(nt, np, fn, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) fa[i] = fn[i] - 0.5 * dt * op[i];          /* f1 */
        or_adv_operator_att(nt, np, fa, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) fb[i] = fa[i] - 0.5 * dt * op[i];          /* f2 */
        or_adv_operator_att(nt, np, fb, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i)
            fa[i] = (2.0 / 3.0) * fn[i] + (1.0 / 3.0) * fb[i] - (1.0 / 6.0) * dt * op[i]; /* f3 */
        or_adv_operator_att(nt, np, fa, vph_row, vth_face, scheme, eps_mode, fn, b0, op);
        for (size_t i = 0; i < n; ++i) B[i] = fa[i] - 0.5 * dt * op[i];
    }
    free(fn);
    free(fa);
    free(fb);
    free(op);
}

/* -------------------------------------------------------------- diffusion */
/* Eq. diffusion_matrix with a scalar diffusivity nu (R_sun^2/h): the
 * half-half averages of nu are nu itself.  Per row j:
 *   a_ph  = (nu+nu) / (2 dph dph sin^2 theta_j)              (k-1 and k+1)
 *   a_up  = (nu+nu) sin theta_{j-1/2} / (2 dth dth sin theta_j)   (j-1)
 *   a_dn  = (nu+nu) sin theta_{j+1/2} / (2 dth dth sin theta_j)   (j+1)
 *   a_d   = -(a_up + a_dn + a_ph + a_ph)
 * The pole faces have sin = 0, so a_up of row 0 and a_dn of the last row
 * vanish (App. A closure). */
/* The same table for a diffusivity that depends on colatitude only, given
 * at the cell corners: nu_face[f] is nu on theta face f (f = 0..nt, face f
 * between rows f-1 and f), the same at both corners of a face.  The corner
 * pairs of the table are then: phi neighbours (nu_face[j+1] + nu_face[j]),
 * theta neighbours (nu_face[j] + nu_face[j]) and (nu_face[j+1] +
 * nu_face[j+1]). */
void or_diff_coefs_face(int nt, int np, const double *nu_face, double *a_up, double *a_dn,
                        double *a_ph, double *a_d)
{
    or_geom g;
    geom_init(&g, nt, np);
    for (int j = 0; j < nt; ++j) {
        double s = g.st[j];
        a_ph[j] = (nu_face[j + 1] + nu_face[j]) / (2.0 * g.dph * g.dph * s * s);
        a_up[j] = (nu_face[j] + nu_face[j]) * g.sf[j] / (2.0 * g.dth * g.dth * s);
        a_dn[j] = (nu_face[j + 1] + nu_face[j + 1]) * g.sf[j + 1] / (2.0 * g.dth * g.dth * s);
        a_d[j] = -(a_up[j] + a_dn[j] + a_ph[j] + a_ph[j]);
    }
    geom_free(&g);
}

void or_diff_coefs(int nt, int np, double nu, double *a_up, double *a_dn, double *a_ph, double *a_d)
{
    double *nf = (double *)malloc(sizeof(double) * (nt + 1));
    for (int f = 0; f <= nt; ++f) nf[f] = nu;
    or_diff_coefs_face(nt, np, nf, a_up, a_dn, a_ph, a_d);
    free(nf);
}

/* Grid-based diffusivity of the flux-preserving smoother (eq. diffgrid):
 * nu_g = alpha [dth^2 + (dph sin(theta))^2] at the theta faces (the corners'
 * colatitudes; sin = 0 at the poles), alpha in 1/h so nu_g is in
 * R_sun^2 / h on the unit sphere. */
void or_nu_grid(int nt, int np, double alpha, double *nu_face)
{
    or_geom g;
    geom_init(&g, nt, np);
    for (int f = 0; f <= nt; ++f) {
        double x = g.dph * g.sf[f];
        nu_face[f] = alpha * (g.dth * g.dth + x * x);
    }
    geom_free(&g);
}

/* Apply the DIA operator: out = L(B), summing the five diagonals in the
 * table's order (k-1, j-1, centre, j+1, k+1). */
static void diff_apply(int nt, int np, const double *a_up, const double *a_dn, const double *a_ph,
                       const double *a_d, const double *B, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nt; ++j) {
        const double *row = B + (size_t)j * np;
        const double *up = j > 0 ? B + (size_t)(j - 1) * np : NULL;
        const double *dn = j < nt - 1 ? B + (size_t)(j + 1) * np : NULL;
        for (int k = 0; k < np; ++k) {
            int km = k == 0 ? np - 1 : k - 1;
            int kp = k == np - 1 ? 0 : k + 1;
            double v = a_ph[j] * row[km];
            if (up) v += a_up[j] * up[k];
            v += a_d[j] * row[k];
            if (dn) v += a_dn[j] * dn[k];
            v += a_ph[j] * row[kp];
            out[(size_t)j * np + k] = v;
        }
    }
}

void or_diff_operator_face(int nt, int np, const double *nu_face, const double *B, double *out)
{
    double *c = (double *)malloc(sizeof(double) * 4 * nt);
    or_diff_coefs_face(nt, np, nu_face, c, c + nt, c + 2 * nt, c + 3 * nt);
    diff_apply(nt, np, c, c + nt, c + 2 * nt, c + 3 * nt, B, out);
    free(c);
}

void or_diff_operator(int nt, int np, double nu, const double *B, double *out)
{
    double *c = (double *)malloc(sizeof(double) * 4 * nt);
    or_diff_coefs(nt, np, nu, c, c + nt, c + 2 * nt, c + 3 * nt);
    diff_apply(nt, np, c, c + nt, c + 2 * nt, c + 3 * nt, B, out);
    free(c);
}

/* Explicit Euler limit of the operator (Sec. "Diffusion temporal schemes";
 * the paper computes it from the DIA coefficients without giving the rule).
 * Reading: Gershgorin, |lambda| <= 2 max_j |a_d|, so dt_E = 1 / max_j |a_d|. */
double or_euler_limit(int nt, int np, double nu)
{
    double *c = (double *)malloc(sizeof(double) * 4 * nt);
    or_diff_coefs(nt, np, nu, c, c + nt, c + 2 * nt, c + 3 * nt);
    double m = 0.0;
    for (int j = 0; j < nt; ++j) {
        double a = fabs(c[3 * nt + j]);
        if (a > m) m = a;
    }
    free(c);
    return m > 0.0 ? 1.0 / m : INFINITY;
}

/* Super-time-stepping schemes (Sec. "Diffusion temporal schemes"; the
 * coefficients are those of the cited RKL2 and RKG2(3/2) schemes, restated
 * here from their Legendre / Gegenbauer stability polynomials):
 *   RKL2: R_s(z) = 1 - b_s + b_s P_s(1 + w1 z),  b_j = (j^2+j-2)/(2j(j+1)),
 *         w1 = 4/(s^2+s-2), stable for tau/dt_E <= (s^2+s-2)/4;
 *   RKG2: R_s(z) = 1 - b_s C_s(1) + b_s C^{3/2}_s(1 + w1 z),
 *         b_j = 4(j-1)(j+4)/(3j(j+1)(j+2)(j+3)), C_j(1) = (j+1)(j+2)/2,
 *         w1 = 6/((s+4)(s-1)), stable for tau/dt_E <= (s+4)(s-1)/6.
 * Stages: Y1 = Y0 + mut_1 tau L Y0, then for j = 2..s
 *   Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + (1-mu_j-nu_j) Y0
 *         + mut_j tau L Y_{j-1} + gamt_j tau L Y0,
 * with mu_j = c_j b_j/b_{j-1}, nu_j = -e_j b_j/b_{j-2}, mut_j = mu_j w1,
 * gamt_j = -a_{j-1} mut_j, a_j = 1 - b_j P_j(1) (P = Legendre or Gegenbauer),
 * and (c_j, e_j) = ((2j-1)/j, (j-1)/j) for RKL2, ((2j+1)/j, (j+1)/j) for RKG2.
 * b_0 and b_1 only change round-off, not R_s: RKL2 uses b_0 = b_1 = 1/3,
 * RKG2 uses b_0 = 1, b_1 = 1/3 (reading).
 * scheme: 0 = RKG2, 1 = RKL2. */
int or_sts_stages(double tau, double dt_euler, int scheme)
{
    double r = tau / dt_euler;
    double s;
    if (scheme == 1)
        s = ceil((sqrt(9.0 + 16.0 * r) - 1.0) / 2.0);
    else
        s = ceil((sqrt(25.0 + 24.0 * r) - 3.0) / 2.0);
    if (s < 2.0) s = 2.0;
    return (int)s;
}

static double sts_b(int j, int scheme)
{
    if (scheme == 1) {
        if (j < 2) return 1.0 / 3.0;
        return ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
    }
    if (j == 0) return 1.0;
    if (j == 1) return 1.0 / 3.0;
    return 4.0 * (j - 1.0) * (j + 4.0) / (3.0 * j * (j + 1.0) * (j + 2.0) * (j + 3.0));
}

static double sts_p1(int j, int scheme)   /* P_j(1) of the scheme's polynomial family */
{
    if (scheme == 1) return 1.0;
    return (j + 1.0) * (j + 2.0) / 2.0;
}

/* Fills mu, nu, mut, gamt for j = 0..s (entries 0 unused; entry 1 holds
 * mut_1 only). */
void or_sts_coefs(int s, int scheme, double *mu, double *nu, double *mut, double *gamt)
{
    double w1 = scheme == 1 ? 4.0 / ((double)s * s + s - 2.0) : 6.0 / ((s + 4.0) * (s - 1.0));
    for (int j = 0; j <= s; ++j) mu[j] = nu[j] = mut[j] = gamt[j] = 0.0;
    mut[1] = (scheme == 1 ? sts_b(1, scheme) : 3.0 * sts_b(1, scheme)) * w1;
    for (int j = 2; j <= s; ++j) {
        double bj = sts_b(j, scheme), bj1 = sts_b(j - 1, scheme), bj2 = sts_b(j - 2, scheme);
        double cj = scheme == 1 ? (2.0 * j - 1.0) / j : (2.0 * j + 1.0) / j;
        double ej = scheme == 1 ? (j - 1.0) / j : (j + 1.0) / j;
        double aj1 = 1.0 - bj1 * sts_p1(j - 1, scheme);
        mu[j] = cj * bj / bj1;
        nu[j] = -ej * bj / bj2;
        mut[j] = mu[j] * w1;
        gamt[j] = -aj1 * mut[j];
    }
}

/* One diffusion advance of length tau (Sec. "Diffusion temporal schemes").
 * dscheme: 0 = RKG2(3/2), 1 = RKL2, 2 = forward Euler with n = ceil(tau/dt_E)
 * equal sub-steps (the paper's reference scheme).  ptl_dt > 0 splits tau into
 * n = ceil(tau/ptl_dt) STS calls of equal length tau/n (Sec. "Diffusion
 * temporal schemes": the practical time step limit cycles the STS advance
 * over sub-steps; the rule that picks the limit is only cited there, so the
 * limit is an input).  Pinned: one advance equals R_s(tau/n A)^n Y0.
 * Returns the number of operator applications (stages). */
long or_diffuse_face(int nt, int np, double *B, const double *nu_face, double tau, int dscheme,
                     double ptl_dt);

long or_diffuse(int nt, int np, double *B, double nu, double tau, int dscheme, double ptl_dt)
{
    if (nu == 0.0 || tau <= 0.0) return 0;
    double *nf = (double *)malloc(sizeof(double) * (nt + 1));
    for (int f = 0; f <= nt; ++f) nf[f] = nu;
    long st = or_diffuse_face(nt, np, B, nf, tau, dscheme, ptl_dt);
    free(nf);
    return st;
}

/* The same with the colatitude-dependent corner diffusivity nu_face. */
long or_diffuse_face(int nt, int np, double *B, const double *nu_face, double tau, int dscheme,
                     double ptl_dt)
{
    if (tau <= 0.0) return 0;
    size_t n = (size_t)nt * np;
    double *c = (double *)malloc(sizeof(double) * 4 * nt);
    or_diff_coefs_face(nt, np, nu_face, c, c + nt, c + 2 * nt, c + 3 * nt);
    const double *a_up = c, *a_dn = c + nt, *a_ph = c + 2 * nt, *a_d = c + 3 * nt;
    double m = 0.0;
    for (int j = 0; j < nt; ++j) m = fabs(a_d[j]) > m ? fabs(a_d[j]) : m;
    double dtE = 1.0 / m;
    long stages = 0;
    double *L = (double *)malloc(sizeof(double) * n);

    if (dscheme == 2) {
        long nsub = (long)ceil(tau / dtE);
        double h = tau / nsub;
        for (long it = 0; it < nsub; ++it) {
            diff_apply(nt, np, a_up, a_dn, a_ph, a_d, B, L);
            for (size_t i = 0; i < n; ++i) B[i] = B[i] + h * L[i];
        }
        free(L);
        free(c);
        return nsub;
    }

    int ncall = 1;
    if (ptl_dt > 0.0 && tau > ptl_dt) ncall = (int)ceil(tau / ptl_dt);
    double tc = tau / ncall;
    int s = or_sts_stages(tc, dtE, dscheme);
    double *mu = (double *)malloc(sizeof(double) * (s + 1) * 4);
    double *nuc = mu + (s + 1), *mut = mu + 2 * (s + 1), *gamt = mu + 3 * (s + 1);
    or_sts_coefs(s, dscheme, mu, nuc, mut, gamt);

    double *Y0 = (double *)malloc(sizeof(double) * n);
    double *LY0 = (double *)malloc(sizeof(double) * n);
    double *Ym1 = (double *)malloc(sizeof(double) * n);
    double *Ym2 = (double *)malloc(sizeof(double) * n);
    double *Yj = (double *)malloc(sizeof(double) * n);
    for (int call = 0; call < ncall; ++call) {
        memcpy(Y0, B, sizeof(double) * n);
        diff_apply(nt, np, a_up, a_dn, a_ph, a_d, Y0, LY0);
        for (size_t i = 0; i < n; ++i) {
            Ym2[i] = Y0[i];
            Ym1[i] = Y0[i] + mut[1] * tc * LY0[i];
        }
        for (int j = 2; j <= s; ++j) {
            diff_apply(nt, np, a_up, a_dn, a_ph, a_d, Ym1, L);
            double cy0 = 1.0 - mu[j] - nuc[j];
            for (size_t i = 0; i < n; ++i)
                Yj[i] = mu[j] * Ym1[i] + nuc[j] * Ym2[i] + cy0 * Y0[i] + mut[j] * tc * L[i] +
                        gamt[j] * tc * LY0[i];
            double *t = Ym2;
            Ym2 = Ym1;
            Ym1 = Yj;
            Yj = t;
        }
        memcpy(B, Ym1, sizeof(double) * n);
        stages += s;
    }
    free(Y0);
    free(LY0);
    free(Ym1);
    free(Ym2);
    free(Yj);
    free(mu);
    free(L);
    free(c);
    return stages;
}

/* ------------------------------------------------------------ assimilation */
/* Observer cosine of the disk-centre angle for a sub-observer point at
 * latitude b0 and longitude l0 (radians): mu = cos of the great-circle
 * angle between the cell centre and the disk centre. */
void or_mu_disk(int nt, int np, double b0, double l0, double *mu)
{
    double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    for (int j = 0; j < nt; ++j) {
        double th = (j + 0.5) * dth;
        for (int k = 0; k < np; ++k) {
            double ph = (k + 0.5) * dph;
            mu[(size_t)j * np + k] = sin(b0) * cos(th) + cos(b0) * sin(th) * cos(ph - l0);
        }
    }
}

/* Eq. data_assim_f: F = mu^alpha where mu > mu_lim and |latitude| < lat_lim,
 * else 0.  alpha = 4 is evaluated as (mu mu)(mu mu); other exponents by pow. */
void or_weight_from_mu(int nt, int np, const double *mu, double alpha, double mu_lim,
                       double lat_lim_rad, double *F)
{
    double dth = M_PI / nt;
    for (int j = 0; j < nt; ++j) {
        double lat = M_PI / 2.0 - (j + 0.5) * dth;
        for (int k = 0; k < np; ++k) {
            size_t i = (size_t)j * np + k;
            double m = mu[i];
            double f = 0.0;
            if (m > mu_lim && fabs(lat) < lat_lim_rad) {
                if (alpha == 4.0) {
                    double m2 = m * m;
                    f = m2 * m2;
                } else {
                    f = pow(m, alpha);
                }
            }
            F[i] = f;
        }
    }
}

/* Eq. data_assim (flux_balance = 0):  B = F B_d + (1-F) B.
 * Eqs. data_assim_deltab and fluxbal (flux_balance = 1):
 *   dB = F (B_d - B); Phi+- = sum of dB w over dB > 0 and dB < 0;
 *   dB > 0 -> dB / sqrt|Phi+/Phi-|,  dB <= 0 -> dB * sqrt|Phi+/Phi-|;
 *   B = B + dB.
 * Reading: when Phi+ or Phi- is zero no balancing factor is applied. */
void or_assimilate(int nt, int np, double *B, const double *data, const double *F, int flux_balance)
{
    size_t n = (size_t)nt * np;
    if (!flux_balance) {
        for (size_t i = 0; i < n; ++i) B[i] = F[i] * data[i] + (1.0 - F[i]) * B[i];
        return;
    }
    double *w = (double *)malloc(sizeof(double) * nt);
    or_cell_weights(nt, np, w);
    double *dB = (double *)malloc(sizeof(double) * n);
    double pp = 0.0, pm = 0.0;
    for (int j = 0; j < nt; ++j) {
        for (int k = 0; k < np; ++k) {
            size_t i = (size_t)j * np + k;
            dB[i] = F[i] * (data[i] - B[i]);
            if (dB[i] > 0.0) pp += dB[i] * w[j];
            else if (dB[i] < 0.0) pm += dB[i] * w[j];
        }
    }
    double r = 1.0;
    int bal = (pp != 0.0 && pm != 0.0);
    if (bal) r = sqrt(fabs(pp / pm));
    for (size_t i = 0; i < n; ++i) {
        double d = dB[i];
        if (bal) d = d > 0.0 ? d / r : d * r;
        B[i] = B[i] + d;
    }
    free(dB);
    free(w);
}

/* ---------------------------------------------------- random flux emergence */
/* Counter-based generator for the random draws of Sec. "Flux emergence": the
 * Philox4x32 generator with 10 rounds (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), restated from that
 * publication.  A round multiplies counter words 0 and 2 by two fixed odd
 * constants; the new words are (high half of the second product) ^ word 1 ^
 * key 0, its low half, (high half of the first product) ^ word 3 ^ key 1 and
 * its low half.  The key grows by two Weyl constants before every round but
 * the first. */
void or_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Standard normal draws Y_i (Sec. "Flux emergence") of source map k of the
 * realization with key (seed, id): cells 2i and 2i+1 take the Box-Muller
 * pair (Box and Muller 1958) r cos(2 pi u2), r sin(2 pi u2), r =
 * sqrt(-2 ln u1), of the generator's output at counter (i, k low word,
 * k high word, 0); u1 comes from output words (0, 1) and u2 from (2, 3),
 * each as (top 53 bits of the 64-bit word + 1/2) / 2^53, inside (0, 1).
 * n must be even. */
void or_rfe_normals(long n, uint32_t seed, uint32_t id, int64_t k, double *Y)
{
    const uint32_t key[2] = {seed, id};
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n / 2; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(uint64_t)k, (uint32_t)((uint64_t)k >> 32), 0u};
        uint32_t x[4];
        or_philox4x32_10(ctr, key, x);
        uint64_t a = ((uint64_t)x[0] << 32) | x[1];
        uint64_t b = ((uint64_t)x[2] << 32) | x[3];
        double u1 = ((double)(a >> 11) + 0.5) * 0x1p-53;
        double u2 = ((double)(b >> 11) + 0.5) * 0x1p-53;
        double r = sqrt(-2.0 * log(u1));
        double t = 2.0 * M_PI * u2;
        Y[2 * i] = r * cos(t);
        Y[2 * i + 1] = r * sin(t);
    }
}

/* One random-flux source map S in gauss per hour (Sec. "Flux emergence"),
 * phi_hr the total unsigned flux per hour in Mx:
 *   model 1 (eq. rfe_m1): S_jk = phi_hr / (dA_j N_cells) sqrt(pi/2) Y_jk,
 *                         dA_j = R^2 sin(theta_j) dth dph, N_cells = nt np;
 *   model 2 (eq. rfe_m2): S = phi_hr / (4 pi R^2) sqrt(pi/2) Y;
 * R = 6.96e10 cm (Sec. "Units").  With balance != 0 the map is then flux
 * balanced as eq. fluxbal: positive values divided by, negative values
 * multiplied by sqrt(|Phi+ / Phi-|), Phi+- the surface integrals (sums of
 * S w_j) of the positive and negative parts; no change when either is 0. */
void or_rfe_map(int nt, int np, int model, double phi_hr, uint32_t seed, uint32_t id, int64_t k,
                int balance, double *S)
{
    const double R = OR_RSUN_M * 100.0;
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    const size_t n = (size_t)nt * np;
    or_rfe_normals((long)n, seed, id, k, S);
    for (int j = 0; j < nt; ++j) {
        double c;
        if (model == 1) {
            double dA = R * R * sin((j + 0.5) * dth) * dth * dph;
            c = phi_hr / (dA * (double)n) * sqrt(M_PI / 2.0);
        } else {
            c = phi_hr / (4.0 * M_PI * R * R) * sqrt(M_PI / 2.0);
        }
        for (int q = 0; q < np; ++q) S[(size_t)j * np + q] = c * S[(size_t)j * np + q];
    }
    if (!balance) return;
    double *w = (double *)malloc(sizeof(double) * nt);
    or_cell_weights(nt, np, w);
    double pp = 0.0, pm = 0.0;
    for (int j = 0; j < nt; ++j) {
        for (int q = 0; q < np; ++q) {
            double v = S[(size_t)j * np + q];
            if (v > 0.0) pp += v * w[j];
            else if (v < 0.0) pm += v * w[j];
        }
    }
    if (pp != 0.0 && pm != 0.0) {
        double r = sqrt(fabs(pp / pm));
        for (size_t i = 0; i < n; ++i) S[i] = S[i] > 0.0 ? S[i] / r : S[i] * r;
    }
    free(w);
}

/* Index k of the source-map interval [k tau, (k+1) tau) holding time t (a
 * time within 1e-10 h below a boundary counts as on it). */
int64_t or_rfe_interval(double t, double tau)
{
    int64_t k = (int64_t)floor(t / tau);
    if ((double)(k + 1) * tau - t < 1e-10) k += 1;
    if (t < (double)k * tau - 1e-10) k -= 1;
    return k;
}

/* Source sub-advance of length h from time ta (eqs. num_opsplit_nostrang /
 * num_opsplit_strang with eq. rfe_s): S(t) = (1 - a(t)) S_k + a(t) S_k+1,
 * a(t) = (t - k tau) / tau, is linear in t on the interval, so its integral
 * over [ta, ta + h] is h S(ta + h/2), added to B.  tau <= 0 (infinite
 * lifetime): S = S_k. */
static void rfe_apply(size_t n, double *B, const double *Sk, const double *Sk1, int64_t k, double tau,
                      double ta, double h)
{
    if (tau <= 0.0) {
        for (size_t i = 0; i < n; ++i) B[i] = B[i] + h * Sk[i];
        return;
    }
    double tm = ta + 0.5 * h;
    double a = (tm - (double)k * tau) / tau;
    for (size_t i = 0; i < n; ++i) B[i] = B[i] + h * ((1.0 - a) * Sk[i] + a * Sk1[i]);
}

/* ------------------------------------------------------------ diagnostics */
/* Sec. "Analysis": out = {Phi+, Phi-, net, h1, h2, D, min, max, min|B|}
 *   Phi+- = sum of B w over B > 0 / B < 0, net = their sum,
 *   h1 = 3/(4 pi) sum B sin(theta) cos(phi) w, h2 with sin(phi),
 *   D  = 3/(4 pi) sum B cos(theta) w.
 * Serial sums in (row, column) order. */
void or_diagnostics(int nt, int np, const double *B, double *out)
{
    double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    double pp = 0.0, pm = 0.0, h1 = 0.0, h2 = 0.0, d = 0.0;
    double mn = INFINITY, mx = -INFINITY, mabs = INFINITY;
    for (int j = 0; j < nt; ++j) {
        double th = (j + 0.5) * dth;
        double w = sin(th) * dth * dph;
        for (int k = 0; k < np; ++k) {
            double ph = (k + 0.5) * dph;
            double b = B[(size_t)j * np + k];
            if (b > 0.0) pp += b * w;
            else if (b < 0.0) pm += b * w;
            h1 += b * sin(th) * cos(ph) * w;
            h2 += b * sin(th) * sin(ph) * w;
            d += b * cos(th) * w;
            if (b < mn) mn = b;
            if (b > mx) mx = b;
            if (fabs(b) < mabs) mabs = fabs(b);
        }
    }
    double c = 3.0 / (4.0 * M_PI);
    out[0] = pp;
    out[1] = pm;
    out[2] = pp + pm;
    out[3] = c * h1;
    out[4] = c * h2;
    out[5] = c * d;
    out[6] = mn;
    out[7] = mx;
    out[8] = mabs;
}

/* Eq. hh: HH = sqrt( sum |X-Y|^2 / sum |X||Y| ). */
double or_hh(long n, const double *X, const double *Y)
{
    double a = 0.0, b = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = X[i] - Y[i];
        a += d * d;
        b += fabs(X[i]) * fabs(Y[i]);
    }
    return sqrt(a / b);
}

/* ------------------------------------------------------------- time loop */
/* Sec. "Time steps" and "Operator splitting": each step takes
 * dt = min(time left in the interval, safety * CFL limit, dt_max), then
 * without Strang splitting (eq. num_opsplit_nostrang) B* = A(B, dt),
 * B** = D(B*, dt); with Strang splitting (eq. num_opsplit_strang)
 * B* = A(B, dt/2), B** = D(B*, dt), B*** = A(B**, dt/2), and the CFL limit of
 * the step doubles because each advection advance is dt/2.  With random flux
 * emergence the source sub-advances close the step (B^{n+1} = S(B**, dt)) or,
 * under Strang splitting, open and close it over dt/2 each; each integrates
 * the interpolated source of eq. rfe_s exactly.  Reading: the time left is
 * measured from the start of the segment (elapsed time is accumulated from
 * zero, the segment length is its end minus its start), and a step that would
 * leave less than 1e-10 h before the segment's end is stretched to land on it.
 * prm = {d0, d2, d4, m1, m3, m5} (m/s), nu_km2_s scalar diffusivity.
 * opts = {adv_scheme, adv_time, diff_scheme, safety, dt_max, eps_mode, ptl_dt, strang, att_b0,
 *         rfe_model, rfe_phi_hr, rfe_tau, rfe_seed, rfe_id, nu_grid_alpha, dt_min, att_cfl}
 * (att_b0: flow attenuation saturation, gauss, 0 = none; with att_cfl = 0
 * the CFL limit is that of the unattenuated flow, an upper bound of the
 * attenuated speeds, with att_cfl = 1 that of the attenuated flow of the
 * field at the start of each step (eq. ssprk43_dt per step, doubled under
 * Strang splitting);
 * dt_min > 0: the step limit min(safety CFL, dt_max) is raised to dt_min
 * (Sec. "Time steps" lists a minimum step among the user's controls), the
 * step still ending no later than the segment's end;
 * rfe_model 0 = no source, 1 / 2 = eq. rfe_m1 / rfe_m2 maps of phi_hr Mx per
 * hour, lifetime rfe_tau hours (<= 0: infinite, one map), maps keyed by
 * (rfe_seed, rfe_id) and their index k, map k belonging to time k tau;
 * nu_grid_alpha > 0, in 1/h: the grid diffusivity of eq. diffgrid replaces
 * nu).
 * stats = {steps, diffusion stages, last dt}.  Returns 0. */
int or_advance(int nt, int np, double *B, const double *prm, double nu_km2_s, double t0,
               double t_end, const double *opts, double *stats)
{
    double ms, k2;
    or_units(&ms, &k2);
    double nu = nu_km2_s * k2;
    int adv_scheme = (int)opts[0], adv_time = (int)opts[1], dscheme = (int)opts[2];
    double safety = opts[3], dt_max = opts[4], eps_mode = opts[5], ptl_dt = opts[6];
    int strang = (int)opts[7];
    double att_b0 = opts[8];
    int rfe = (int)opts[9];
    double rfe_phi = opts[10], tau = opts[11];
    uint32_t seed = (uint32_t)opts[12], rid = (uint32_t)opts[13];
    double nu_alpha = opts[14];
    double dt_min = opts[15];
    int att_cfl = (int)opts[16];
    size_t n = (size_t)nt * np;
    /* eq. diffgrid replaces the scalar diffusivity when nu_alpha > 0 */
    double *nuf = NULL;
    if (nu_alpha > 0.0) {
        nuf = (double *)malloc(sizeof(double) * (nt + 1));
        or_nu_grid(nt, np, nu_alpha, nuf);
    }
    double *vph = (double *)malloc(sizeof(double) * nt);
    double *vth = (double *)malloc(sizeof(double) * (nt + 1));
    or_flows(nt, prm, vph, vth);
    int has_flow = 0;
    for (int j = 0; j < nt; ++j) has_flow |= vph[j] != 0.0;
    for (int f = 0; f <= nt; ++f) has_flow |= vth[f] != 0.0;
    double cfl = or_cfl_dt(nt, np, vph, vth, adv_time);
    if (strang) cfl *= 2.0;
    /* source maps S_k and S_k+1 of the current interval (Sec. "Flux emergence") */
    double *Sk = NULL, *Sk1 = NULL;
    int64_t have = -1;
    if (rfe) {
        Sk = (double *)malloc(sizeof(double) * n);
        Sk1 = (double *)malloc(sizeof(double) * n);
    }
    long steps = 0, stages = 0;
    double last = 0.0;
    /* Sec. "Time steps": with random flux emergence of finite lifetime tau,
     * steps also land on the map times k tau, so the advance splits into
     * segments at those times; each segment takes the greedy step rule. */
    double a = t0;
    for (;;) {
        double b = t_end;
        int64_t k = 0;
        if (rfe && tau > 0.0) {
            k = or_rfe_interval(a, tau);
            double nb = (double)(k + 1) * tau;
            if (nb < t_end - 1e-10) b = nb;
        }
        if (rfe && k != have) {
            or_rfe_map(nt, np, rfe, rfe_phi, seed, rid, k, 1, Sk);
            if (tau > 0.0) or_rfe_map(nt, np, rfe, rfe_phi, seed, rid, k + 1, 1, Sk1);
            have = k;
        }
        double len = b - a;
        double el = 0.0;
        while (el < len) {
            double rem = len - el;
            double lim = cfl;
            if (att_cfl && att_b0 > 0.0 && has_flow) {
                lim = or_cfl_dt_att(nt, np, vph, vth, B, att_b0, adv_time);
                if (strang) lim *= 2.0;
            }
            double cap = safety * lim;
            if (dt_max > 0.0 && dt_max < cap) cap = dt_max;
            if (dt_min > 0.0 && cap < dt_min) cap = dt_min;
            double dt = rem;
            if (cap < dt) dt = cap;
            int final = 0;
            if (rem - dt < 1e-10) {
                dt = rem;
                final = 1;
            }
            double ta = a + el;
            if (strang) {
                if (rfe) rfe_apply(n, B, Sk, Sk1, k, tau, ta, 0.5 * dt);
                if (has_flow) or_adv_step_att(nt, np, B, vph, vth, 0.5 * dt, adv_scheme, adv_time, eps_mode, att_b0);
                stages += nuf ? or_diffuse_face(nt, np, B, nuf, dt, dscheme, ptl_dt)
                              : or_diffuse(nt, np, B, nu, dt, dscheme, ptl_dt);
                if (has_flow) or_adv_step_att(nt, np, B, vph, vth, 0.5 * dt, adv_scheme, adv_time, eps_mode, att_b0);
                if (rfe) rfe_apply(n, B, Sk, Sk1, k, tau, ta + 0.5 * dt, 0.5 * dt);
            } else {
                if (has_flow) or_adv_step_att(nt, np, B, vph, vth, dt, adv_scheme, adv_time, eps_mode, att_b0);
                stages += nuf ? or_diffuse_face(nt, np, B, nuf, dt, dscheme, ptl_dt)
                              : or_diffuse(nt, np, B, nu, dt, dscheme, ptl_dt);
                if (rfe) rfe_apply(n, B, Sk, Sk1, k, tau, ta, dt);
            }
            el = final ? len : el + dt;
            last = dt;
            ++steps;
        }
        if (b == t_end) break;
        a = b;
    }
    stats[0] = (double)steps;
    stats[1] = (double)stages;
    stats[2] = last;
    free(Sk);
    free(Sk1);
    free(nuf);
    free(vph);
    free(vth);
    return 0;
}
