"""Plain FP64 CPU oracle of the surface-flux-transport hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_2501_06377_amd``) never imports it and shares no code with it.

The numerics live in ``sft_oracle.c`` (plain C, FP64, OpenMP over rows, built
with ``-ffp-contract=off``); this module only marshals numpy arrays through
ctypes and sequences whole runs (time loop, assimilation schedule, ensemble)
the way the paper describes them (Sec. "Time steps", "Operator splitting",
"Data assimilation", "Multiple Realizations").  The CNN surrogate's oracle is
``oracle.cnn`` (numpy FP64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# option codes (oracle-private; the GPU library defines its own)
WENO3CSH, UPWIND = 0, 1
SSPRK43, FE, SSPRK33 = 0, 1, 2
RKG2, RKL2, DIFF_FE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O3 (no FMA contraction, no reassociation:
    -ffp-contract=off -fno-fast-math keep every operation IEEE as written)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        i, d, l = ctypes.c_int, ctypes.c_double, ctypes.c_long
        U32P = ctypes.POINTER(ctypes.c_uint32)
        sig = {
            "or_units": (None, [P, P]),
            "or_num_threads": (i, []),
            "or_cell_weights": (None, [i, i, P]),
            "or_flows": (None, [i, P, P, P]),
            "or_cfl_dt": (d, [i, i, P, P, i]),
            "or_cfl_dt_att": (d, [i, i, P, P, P, d, i]),
            "or_line_flux": (None, [i, i, P, P, P, i, d, P]),
            "or_adv_operator": (None, [i, i, P, P, P, i, d, P]),
            "or_adv_operator_att": (None, [i, i, P, P, P, i, d, P, d, P]),
            "or_adv_step": (None, [i, i, P, P, P, d, i, i, d]),
            "or_diff_coefs": (None, [i, i, d, P, P, P, P]),
            "or_diff_operator": (None, [i, i, d, P, P]),
            "or_diff_operator_face": (None, [i, i, P, P, P]),
            "or_diff_coefs_face": (None, [i, i, P, P, P, P, P]),
            "or_nu_grid": (None, [i, i, d, P]),
            "or_diffuse_face": (l, [i, i, P, P, d, i, d]),
            "or_euler_limit": (d, [i, i, d]),
            "or_sts_stages": (i, [d, d, i]),
            "or_sts_coefs": (None, [i, i, P, P, P, P]),
            "or_diffuse": (l, [i, i, P, d, d, i, d]),
            "or_mu_disk": (None, [i, i, d, d, P]),
            "or_weight_from_mu": (None, [i, i, P, d, d, d, P]),
            "or_assimilate": (None, [i, i, P, P, P, i]),
            "or_diagnostics": (None, [i, i, P, P]),
            "or_hh": (d, [l, P, P]),
            "or_advance": (i, [i, i, P, P, d, d, d, P, P]),
            "or_philox4x32_10": (None, [U32P, U32P, U32P]),
            "or_rfe_normals": (None, [l, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, P]),
            "or_rfe_map": (None, [i, i, i, d, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, i, P]),
            "or_rfe_interval": (ctypes.c_int64, [d, d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle takes C-contiguous float64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------- primitives
def units():
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().or_units(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def num_threads() -> int:
    return int(lib().or_num_threads())


def cell_weights(nt, np_):
    w = np.empty(nt)
    lib().or_cell_weights(nt, np_, _p(w))
    return w


def flows(nt, prm):
    """prm = (d0, d2, d4, m1, m3, m5) in m/s -> (v_phi per row, v_theta per face) in Rsun/h."""
    vph, vth = np.empty(nt), np.empty(nt + 1)
    lib().or_flows(nt, _p(_f64(prm)), _p(vph), _p(vth))
    return vph, vth


def cfl_dt(nt, np_, vph, vth, time_scheme=SSPRK43):
    return lib().or_cfl_dt(nt, np_, _p(_f64(vph)), _p(_f64(vth)), time_scheme)


def cfl_dt_att(vph, vth, Batt, b0, time_scheme=SSPRK43):
    """CFL limit of the flow attenuated by the field Batt (eq. flow_attenuation)."""
    Batt = _f64(Batt)
    nt, np_ = Batt.shape
    return lib().or_cfl_dt_att(nt, np_, _p(_f64(vph)), _p(_f64(vth)), _p(Batt), float(b0), time_scheme)


def line_flux(B, dx, v, periodic, scheme=WENO3CSH, eps_mode=0.0):
    B, dx, v = _f64(B), _f64(dx), _f64(v)
    n = B.size
    F = np.empty(n + 1)
    lib().or_line_flux(n, int(periodic), _p(B), _p(dx), _p(v), scheme, eps_mode, _p(F))
    return F


def adv_operator(B, vph, vth, scheme=WENO3CSH, eps_mode=0.0, Batt=None, b0=0.0):
    """Flux divergence of eq. advection; with b0 > 0 the face velocities are
    attenuated (eq. flow_attenuation) by the field Batt."""
    B = _f64(B)
    out = np.empty_like(B)
    nt, np_ = B.shape
    att = _p(_f64(Batt)) if Batt is not None else None
    lib().or_adv_operator_att(nt, np_, _p(B), _p(_f64(vph)), _p(_f64(vth)), scheme, eps_mode, att,
                              float(b0), _p(out))
    return out


def adv_step(B, vph, vth, dt, scheme=WENO3CSH, time_scheme=SSPRK43, eps_mode=0.0):
    B = _f64(B).copy()
    nt, np_ = B.shape
    lib().or_adv_step(nt, np_, _p(B), _p(_f64(vph)), _p(_f64(vth)), dt, scheme, time_scheme,
                      eps_mode)
    return B


def diff_coefs(nt, np_, nu):
    c = [np.empty(nt) for _ in range(4)]
    lib().or_diff_coefs(nt, np_, nu, *[_p(x) for x in c])
    return tuple(c)  # a_up, a_dn, a_ph, a_d


def diff_operator(B, nu):
    B = _f64(B)
    out = np.empty_like(B)
    lib().or_diff_operator(B.shape[0], B.shape[1], nu, _p(B), _p(out))
    return out


def diff_operator_face(B, nu_face):
    """Eq. diffusion_matrix with a colatitude-dependent corner diffusivity
    (nu_face[f] on theta face f, R_sun^2/h)."""
    B = _f64(B)
    out = np.empty_like(B)
    lib().or_diff_operator_face(B.shape[0], B.shape[1], _p(_f64(nu_face)), _p(B), _p(out))
    return out


def diff_coefs_face(nt, np_, nu_face):
    c = [np.empty(nt) for _ in range(4)]
    lib().or_diff_coefs_face(nt, np_, _p(_f64(nu_face)), *[_p(x) for x in c])
    return tuple(c)  # a_up, a_dn, a_ph, a_d


def nu_grid(nt, np_, alpha):
    """Eq. diffgrid at the theta faces (alpha in 1/h -> R_sun^2/h)."""
    nf = np.empty(nt + 1)
    lib().or_nu_grid(nt, np_, float(alpha), _p(nf))
    return nf


def diffuse_face(B, nu_face, tau, scheme=RKG2, ptl_dt=0.0):
    B = _f64(B).copy()
    st = lib().or_diffuse_face(B.shape[0], B.shape[1], _p(B), _p(_f64(nu_face)), tau, scheme, ptl_dt)
    return B, int(st)


def euler_limit(nt, np_, nu):
    return lib().or_euler_limit(nt, np_, nu)


def sts_stages(tau, dt_euler, scheme=RKG2):
    return int(lib().or_sts_stages(tau, dt_euler, scheme))


def sts_coefs(s, scheme=RKG2):
    arrs = [np.empty(s + 1) for _ in range(4)]
    lib().or_sts_coefs(s, scheme, *[_p(a) for a in arrs])
    return tuple(arrs)  # mu, nu, mut, gamt


def diffuse(B, nu, tau, scheme=RKG2, ptl_dt=0.0):
    """One diffusion advance of length tau (nu in Rsun^2/h). Returns (B, stages)."""
    B = _f64(B).copy()
    st = lib().or_diffuse(B.shape[0], B.shape[1], _p(B), nu, tau, scheme, ptl_dt)
    return B, int(st)


def mu_disk(nt, np_, b0_rad, l0_rad):
    mu = np.empty((nt, np_))
    lib().or_mu_disk(nt, np_, b0_rad, l0_rad, _p(mu))
    return mu


def weight_from_mu(mu, alpha=4.0, mu_lim=0.0, lat_lim_rad=np.pi / 2):
    mu = _f64(mu)
    F = np.empty_like(mu)
    lib().or_weight_from_mu(mu.shape[0], mu.shape[1], _p(mu), alpha, mu_lim, lat_lim_rad, _p(F))
    return F


def assimilate(B, data, F, flux_balance=False):
    B = _f64(B).copy()
    lib().or_assimilate(B.shape[0], B.shape[1], _p(B), _p(_f64(data)), _p(_f64(F)),
                        int(bool(flux_balance)))
    return B


DIAG_KEYS = ("phi_pos", "phi_neg", "phi_net", "h1", "h2", "dax", "bmin", "bmax", "babs_min")


def diagnostics(B):
    B = _f64(B)
    out = np.empty(9)
    lib().or_diagnostics(B.shape[0], B.shape[1], _p(B), _p(out))
    return dict(zip(DIAG_KEYS, out.tolist()))


def hh(X, Y):
    X, Y = _f64(X).ravel(), _f64(Y).ravel()
    return lib().or_hh(X.size, _p(X), _p(Y))


def advance(B, prm, nu_km2_s, t0, t_end, adv_scheme=WENO3CSH, adv_time=SSPRK43,
            diff_scheme=RKG2, safety=0.9, dt_max=0.0, eps_mode=0.0, ptl_dt=0.0, strang=0, att_b0=0.0,
            rfe_model=0, rfe_phi_hr=0.0, rfe_tau=0.0, rfe_seed=0, rfe_id=0, nu_grid_alpha=0.0,
            dt_min=0.0, att_cfl=0):
    """Advance one realization from t0 to t_end (hours), operator split with
    or without Strang splitting, optionally with flow attenuation (att_b0 in
    gauss) and random flux emergence (model 1 / 2, phi_hr Mx per hour,
    lifetime rfe_tau hours, 0 = infinite; maps keyed by seed and id) and the
    smoother's grid diffusivity (nu_grid_alpha > 0 in 1/h replaces nu).
    dt_min > 0 raises the step limit to at least dt_min hours; att_cfl = 1
    takes each step's CFL limit from the attenuated flow of the field at the
    step's start.  Returns (B, stats)."""
    B = _f64(B).copy()
    opts = np.array([adv_scheme, adv_time, diff_scheme, safety, dt_max, eps_mode, ptl_dt, strang, att_b0,
                     rfe_model, rfe_phi_hr, rfe_tau, rfe_seed, rfe_id, nu_grid_alpha, dt_min, att_cfl],
                    dtype=np.float64)
    stats = np.zeros(3)
    lib().or_advance(B.shape[0], B.shape[1], _p(B), _p(_f64(prm)), float(nu_km2_s), float(t0),
                     float(t_end), _p(opts), _p(stats))
    return B, {"steps": int(stats[0]), "stages": int(stats[1]), "dt_last": float(stats[2])}


# ------------------------------------------------- random flux emergence
def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC 2011): 4 counter words,
    2 key words -> 4 output words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def rfe_normals(n, seed, rid, k):
    """Standard normal draws of source map k (n even)."""
    Y = np.empty(n)
    lib().or_rfe_normals(int(n), int(seed) & 0xFFFFFFFF, int(rid) & 0xFFFFFFFF, int(k), _p(Y))
    return Y


def rfe_map(nt, np_, model, phi_hr, seed, rid, k, balance=True):
    """Source map k (gauss per hour) of eq. rfe_m1 (model 1) or rfe_m2 (model 2),
    flux balanced as eq. fluxbal when balance is true."""
    S = np.empty((nt, np_))
    lib().or_rfe_map(nt, np_, int(model), float(phi_hr), int(seed) & 0xFFFFFFFF, int(rid) & 0xFFFFFFFF,
                     int(k), int(bool(balance)), _p(S))
    return S


def rfe_interval(t, tau):
    return int(lib().or_rfe_interval(float(t), float(tau)))
