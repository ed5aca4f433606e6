"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module only draws random numbers and lays out the workloads: initial
bipolar fields, hourly synthetic observations, realization parameter sets and
observer geometry.  It holds none of the transport method's arithmetic and
imports neither the GPU package nor the oracle.

Every stream derives from ``numpy.random.SeedSequence(250106377)`` with a
fixed spawn key per purpose, so each array is reproducible on any machine.

The paper's own workloads (an HMI Carrington map, MagMAP assimilation maps,
ConFlow flows) are not available; the recipes below stand in for them with
the paper's default grid and parameter ranges (diffusivity 100-600 km^2/s,
flows of tens of m/s):

* bipolar field: pairs of Gaussian spots (sigma = 2 deg, 6 deg apart) at
  latitudes U(-35, 35) deg, longitudes U(0, 360) deg, peak |B| U(50, 500) G,
  tilt 0.5|lat| + N(0, 10) deg (Joy's law, leading spot equatorward), Hale
  polarity (leading spot positive in the north, negative in the south);
* observations: a 'truth' field plus N(0, 5 G) noise per cell and hour; the
  truth is either the hourly state of a nominal realization evolved by a
  solver (the benchmark: the library's FP64 path for the GPU run, the oracle
  for the CPU baseline; truth_observation) or, where the observations only
  need to be plausible inputs (parity tests), the initial field sheared in
  longitude (each row shifted by a whole number of columns, -3 sin^2(lat)
  deg/day; observation); the weight of the visible disk is left to the
  library;
* observer: sub-observer latitude 0, longitude 180 deg - 13.2 deg/day * t.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

ROOT_SEED = 250106377
PURPOSE = {"field": 0, "obs_noise": 1, "params": 2, "cnn_init": 3, "shuffle": 4, "surrogate_data": 5,
           "test": 6}

# 1 deg/day of angular rate on the solar surface, in m/s (R_sun = 6.96e8 m)
DEG_PER_DAY_M_S = math.pi / 180.0 / 86400.0 * 6.96e8


def rng(purpose: str, *sub: int) -> np.random.Generator:
    key = (PURPOSE[purpose],) + tuple(int(s) for s in sub)
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=key))


# ------------------------------------------------------------ initial field
def bipolar_pairs(n_pairs: int, seed_sub: int = 0) -> np.ndarray:
    """Draw n_pairs bipolar regions; rows = (lat0, lon0, amp, tilt) in deg / G."""
    g = rng("field", seed_sub)
    lat = g.uniform(-35.0, 35.0, n_pairs)
    lon = g.uniform(0.0, 360.0, n_pairs)
    amp = g.uniform(50.0, 500.0, n_pairs)
    tilt = 0.5 * np.abs(lat) + g.normal(0.0, 10.0, n_pairs)
    return np.stack([lat, lon, amp, tilt], axis=1)


def _spot_centres(pairs: np.ndarray, sep_deg: float = 6.0):
    lat, lon, amp, tilt = pairs.T
    hemi = np.where(lat >= 0.0, 1.0, -1.0)
    # leading spot: prograde (east, +lon) and equatorward by the tilt angle
    t = np.radians(tilt)
    dlat = 0.5 * sep_deg * np.sin(t) * hemi
    dlon = 0.5 * sep_deg * np.cos(t) / np.maximum(np.cos(np.radians(lat)), 0.2)
    lead = np.stack([lat - dlat, lon + dlon], 1)
    trail = np.stack([lat + dlat, lon - dlon], 1)
    sign_lead = hemi            # Hale: leading polarity + in the north
    return lead, trail, sign_lead * amp


def bipolar_field(nt: int, np_: int, pairs: np.ndarray, sigma_deg: float = 2.0,
                  lon_shift_deg=None, dtype=np.float64) -> np.ndarray:
    """Sum of Gaussian spots on the cell-centred grid (great-circle distance).

    ``lon_shift_deg`` optionally shifts every spot by a longitude offset (deg).
    Spots are evaluated on rows within 8 sigma of their latitude (the
    neglected tail is below 1e-13 of the peak)."""
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(np_) + 0.5) * 2.0 * math.pi / np_
    lat_rows = 90.0 - np.degrees(th)
    B = np.zeros((nt, np_), dtype=np.float64)
    lead, trail, amp = _spot_centres(pairs)
    s2 = 2.0 * math.radians(sigma_deg) ** 2
    cos_ph, sin_ph = np.cos(ph), np.sin(ph)
    for centres, sgn in ((lead, 1.0), (trail, -1.0)):
        for (la, lo), a in zip(centres, amp):
            if lon_shift_deg is not None:
                lo = lo + lon_shift_deg
            rows = np.nonzero(np.abs(lat_rows - la) <= 8.0 * sigma_deg)[0]
            if rows.size == 0:
                continue
            la_r, lo_r = math.radians(la), math.radians(lo)
            # cos of the great-circle distance between each cell and the centre
            st, ct = np.sin(th[rows])[:, None], np.cos(th[rows])[:, None]
            cd = (ct * math.sin(la_r) +
                  st * math.cos(la_r) * (cos_ph[None, :] * math.cos(lo_r) + sin_ph[None, :] * math.sin(lo_r)))
            d = np.arccos(np.clip(cd, -1.0, 1.0))
            B[rows, :] += sgn * a * np.exp(-d * d / s2)
    return B.astype(dtype)


# ------------------------------------------------------------ observations
def observer(t_hours: float) -> Tuple[float, float]:
    """(b0, l0) in degrees for a synthetic observer at time t (hours)."""
    return 0.0, (180.0 - 13.2 * t_hours / 24.0) % 360.0


def observation(field0: np.ndarray, t_hours: float, hour_index: int, noise_g: float = 5.0,
                dtype=np.float64) -> np.ndarray:
    """Synthetic observed map at time t: the initial field sheared in
    longitude by -3 sin^2(lat) deg/day (whole-column shifts per row) plus
    seeded N(0, noise_g) noise."""
    nt, np_ = field0.shape
    th = (np.arange(nt) + 0.5) * math.pi / nt
    lat = math.pi / 2 - th
    drift = -3.0 * np.sin(lat) ** 2 * t_hours / 24.0               # degrees
    shift = np.rint(drift / (360.0 / np_)).astype(np.int64)
    k = (np.arange(np_)[None, :] - shift[:, None]) % np_
    truth = np.take_along_axis(field0, k, axis=1)
    noise = rng("obs_noise", hour_index).standard_normal((nt, np_)) * noise_g
    return (truth + noise).astype(dtype)


def nominal_truth_realization() -> "Realization":
    """Parameters of the 'truth' realization whose evolved field the
    synthetic observers see: the first configuration's eta = 500 km^2/s and
    15 m/s meridional amplitude, with the workloads' rotation profile."""
    return Realization(nu_km2_s=500.0, **dr_mf(amp_mf=15.0))


def truth_observation(truth_map: np.ndarray, hour_index: int, noise_g: float = 5.0,
                      dtype=np.float64) -> np.ndarray:
    """Observed map of one hour: the truth field at that hour (evolved by a
    solver elsewhere; this module only adds noise) plus seeded N(0, noise_g)
    per cell, from the same noise stream as synth.observation."""
    nt, np_ = truth_map.shape
    noise = rng("obs_noise", hour_index).standard_normal((nt, np_)) * noise_g
    return (truth_map + noise).astype(dtype)


# ---------------------------------------------------------- validation maps
def soccer_ball(nt: int, np_: int) -> np.ndarray:
    """The soccer-ball map of eq. soccerball at t = 0 on the cell centres,
    Y_6^0 + sqrt(14/11) Y_6^5 with orthonormal harmonics (the m = 5 term is
    the real part of the complex harmonic).  Its exact evolution under
    diffusivity nu is the same map times exp(-42 nu t), and a full rigid
    rotation brings it back unchanged."""
    import scipy.special as sps
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(np_) + 0.5) * 2.0 * math.pi / np_
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    return (sps.sph_harm_y(6, 0, TH, PH).real +
            math.sqrt(14.0 / 11.0) * sps.sph_harm_y(6, 5, TH, PH).real)


# ------------------------------------------------------------- realizations
@dataclasses.dataclass
class Realization:
    nu_km2_s: float
    d0: float = 0.0
    d2: float = -2.4 * DEG_PER_DAY_M_S
    d4: float = -1.8 * DEG_PER_DAY_M_S
    m1: float = 30.0
    m3: float = 0.0
    m5: float = 0.0
    alpha_mu: float = 4.0
    mu_lim: float = 0.0
    lat_lim_deg: float = 90.0
    flux_balance: int = 0
    att_b0: float = 0.0        # flow attenuation saturation field, gauss (0 = off)
    nu_grid_alpha: float = 0.0  # grid-diffusivity factor of the smoother, 1/h (0 = scalar nu)

    @property
    def flow(self):
        return (self.d0, self.d2, self.d4, self.m1, self.m3, self.m5)


def dr_mf(om2=-2.4, om4=-1.8, om0_minus_frame=0.0, amp_mf=15.0):
    """Eq. dr / eq. mf coefficients (m/s) of the workloads' flow forms:
    Omega(lat) = 13.2 + om2 sin^2 + om4 sin^4 deg/day minus a 13.2 deg/day
    frame, and a poleward meridional flow amp_mf sin(2 lat) (m1 = 2 amp)."""
    c = DEG_PER_DAY_M_S
    return dict(d0=om0_minus_frame * c, d2=om2 * c, d4=om4 * c, m1=2.0 * amp_mf, m3=0.0, m5=0.0)


@dataclasses.dataclass
class Workload:
    name: str
    classes: List[Tuple[int, int, List[Realization]]]   # (nt, np, realizations)
    hours: float
    precision: str            # "f64" or "f32"
    assim_every_h: float = 0.0
    n_pairs: int = 20

    @property
    def n_real(self):
        return sum(len(r) for _, _, r in self.classes)

    @property
    def cells(self):
        return sum(nt * np_ * len(r) for nt, np_, r in self.classes)


def config1() -> Workload:
    """Plain method, FP64, 1 realization at 180x360, 20 pairs, 7 days."""
    r = Realization(nu_km2_s=500.0, **dr_mf(amp_mf=15.0))
    return Workload("plain-f64-180x360-r1-7d", [(180, 360, [r])], 168.0, "f64", 0.0, 20)


def config2(hours: float = 655.2) -> Workload:
    """Ensemble FP64: 512x1024, 8 realizations, eta x MF amplitude grid,
    hourly mu^4 assimilation, 27.3 days."""
    rs = [Realization(nu_km2_s=eta, **dr_mf(amp_mf=a)) for eta in (250.0, 500.0, 750.0, 1000.0)
          for a in (10.0, 20.0)]
    return Workload("ensemble-f64-512x1024-r8-27.3d", [(512, 1024, rs)], hours, "f64", 1.0, 200)


def _jittered(n: int, sub: int) -> List[Realization]:
    g = rng("params", sub)
    eta = g.uniform(200.0, 800.0, n)
    fdr = g.uniform(0.8, 1.2, n)
    fmf = g.uniform(0.8, 1.2, n)
    return [Realization(nu_km2_s=float(e), **dr_mf(om2=-2.4 * a, om4=-1.8 * a, amp_mf=15.0 * b))
            for e, a, b in zip(eta, fdr, fmf)]


def config3(hours: float = 655.2, n: int = 32) -> Workload:
    """Precision: FP32 stencils + FP64 reductions, 1024x2048, 32 realizations."""
    return Workload("mixed-f32-1024x2048-r32-27.3d", [(1024, 2048, _jittered(n, 3))], hours, "f32",
                    1.0, 200)


def smoother(n_maps: int = 1, alpha: float = 0.5) -> Workload:
    """Flux-preserving smoothing: 512x1024 map(s), the grid diffusivity of
    eq. diffgrid with alpha = 0.5 (the paper's smoothing example), no flows,
    no assimilation; each hour of the advance smooths further."""
    rs = [Realization(nu_km2_s=0.0, d0=0.0, d2=0.0, d4=0.0, m1=0.0, nu_grid_alpha=alpha)
          for _ in range(n_maps)]
    return Workload(f"smoother-f64-512x1024-r{n_maps}-alpha{alpha:g}", [(512, 1024, rs)], 1.0, "f64", 0.0,
                    200)


def config4(hours: float = 168.0, n_each: int = 32) -> Workload:
    """Batching: 96 realizations of uneven sizes, FP32, 7 days, no assimilation."""
    return Workload("batched-f32-uneven-r96-7d",
                    [(256, 512, _jittered(n_each, 40)), (512, 1024, _jittered(n_each, 41)),
                     (1024, 2048, _jittered(n_each, 42))], hours, "f32", 0.0, 200)


# The paper's validation runs (Sec. "Test cases"): the soccer-ball map for
# 672 h with nu = 500 km^2/s, with or without a rigid rotation of
# 1.80766 km/s sin(theta) (one full turn in 672 h), on the default 512x1024
# grid.  Each case names the schemes and step rule it runs with.
SOCCER_HOURS = 672.0
SOCCER_NU_KM2_S = 500.0
RIGID_ROTATION_M_S = 1807.66


@dataclasses.dataclass
class SoccerCase:
    name: str
    flows: bool                 # rigid rotation on (advection + diffusion) or off (diffusion only)
    adv: str = "ssprk43"        # "ssprk43" | "ssprk33"
    diff: str = "rkg2"          # "rkg2" | "rkl2"
    strang: int = 0
    dt_max: float = 0.0         # hours; 0 = the CFL limit (or one step when there is no flow)

    def realization(self) -> Realization:
        return Realization(nu_km2_s=SOCCER_NU_KM2_S, d0=RIGID_ROTATION_M_S if self.flows else 0.0,
                           d2=0.0, d4=0.0, m1=0.0)


def soccer_cases() -> List[SoccerCase]:
    return [SoccerCase("diffusion, RKL2, one 672 h step", False, diff="rkl2"),
            SoccerCase("diffusion, RKG2, one 672 h step", False),
            SoccerCase("advection+diffusion, dt 0.5 h", True, dt_max=0.5),
            SoccerCase("advection+diffusion, dt 0.5 h, Strang", True, dt_max=0.5, strang=1),
            SoccerCase("advection+diffusion, max CFL dt", True),
            SoccerCase("advection+diffusion, max CFL dt, Strang", True, strang=1),
            SoccerCase("advection+diffusion, max CFL dt, SSPRK(3,3)", True, adv="ssprk33")]
