"""Pins of the oracle's random flux emergence (Sec. "Flux emergence", eqs.
rfe_m1, rfe_m2, rfe_s, fluxbal; Sec. "Operator splitting" with the source).

The generator is pinned by the published known-answer vectors, the normal
draws by their distribution (including eq. mean, <|Y|> = sqrt(2/pi)), the maps
by the unsigned flux the paper says each model realizes and by eq. fluxbal's
balance, and the time integration by closed forms of the piecewise-linear
source and the paper's qualitative result for finite lifetimes.
"""
import math
import os

import numpy as np
import pytest
import scipy.stats as sst

import oracle

KAT = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
R_CM = 6.96e10          # Sec. "Units": R_sun = 6.96e8 m
PHI = 1.0e23            # 100e21 Mx per hour, the rate of the paper's validation runs


def test_philox_known_answers():
    n = 0
    for line in open(KAT):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert oracle.philox4x32_10(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


def test_normals_distribution_and_independence():
    n = 1 << 20
    Y = oracle.rfe_normals(n, 7, 3, 11)
    se = 1.0 / math.sqrt(n)
    assert abs(Y.mean()) < 5 * se
    assert abs(Y.var() - 1.0) < 5 * math.sqrt(2.0) * se
    # eq. mean: <|Y|> = sqrt(2/pi)
    assert abs(np.abs(Y).mean() - math.sqrt(2 / math.pi)) < 5 * math.sqrt(1 - 2 / math.pi) * se
    p1 = math.erf(1 / math.sqrt(2))
    assert abs((np.abs(Y) < 1).mean() - p1) < 5 * math.sqrt(p1 * (1 - p1)) * se
    assert sst.kstest(Y, "norm").pvalue > 1e-4
    # the pair members (cos, sin) and draws of other maps / realizations / seeds are uncorrelated
    assert abs(np.corrcoef(Y[0::2], Y[1::2])[0, 1]) < 6 * math.sqrt(2) * se
    for args in ((7, 3, 12), (7, 4, 11), (8, 3, 11)):
        Z = oracle.rfe_normals(n, *args)
        assert abs(np.corrcoef(Y, Z)[0, 1]) < 6 * se
    assert np.array_equal(Y, oracle.rfe_normals(n, 7, 3, 11))
    # map k of a realization is a pure function of (seed, id, k): the first
    # pairs of a longer draw are the same draws
    assert np.array_equal(oracle.rfe_normals(64, 7, 3, 11), Y[:64])


def test_map_models_realize_the_unsigned_flux_rate():
    """Eqs. rfe_m1 / rfe_m2 set sigma so that the expected unsigned flux per
    hour of a map is phi_hr: model 1 per cell (phi_hr / N_cells each), model 2
    per unit area (phi_hr / (4 pi R^2)); model 1 is larger where cells are
    smaller (near the poles), model 2 is uniform."""
    nt, np_ = 256, 512
    w = oracle.cell_weights(nt, np_)[:, None] * R_CM ** 2        # cell areas, cm^2
    S1 = oracle.rfe_map(nt, np_, 1, PHI, 5, 0, 0, balance=False)
    S2 = oracle.rfe_map(nt, np_, 2, PHI, 5, 0, 0, balance=False)
    sd = math.sqrt(math.pi / 2 - 1)                             # sd(|Y|) / <|Y|>
    tol = 6 * sd / math.sqrt(nt * np_)
    # model 1: each cell's unsigned flux |S| dA has mean phi_hr / N
    assert abs((np.abs(S1) * w).sum() / PHI - 1.0) < tol
    # model 2: unsigned flux density mean phi_hr / (4 pi R^2), total phi_hr
    assert abs(np.abs(S2).mean() / (PHI / (4 * math.pi * R_CM ** 2)) - 1.0) < tol
    assert abs((np.abs(S2) * w).sum() / PHI - 1.0) < 1.5 * tol
    # same draws, model 1 / model 2 = (4 pi R^2) / (dA_j N): larger near the poles
    ratio = S1 / S2
    assert np.allclose(ratio, 4 * math.pi * R_CM ** 2 / (w * nt * np_), rtol=1e-13)
    assert ratio[0, 0] > 50 * ratio[nt // 2, 0]


def test_map_flux_balance():
    """Eq. fluxbal on a source map: positive parts divided, negative parts
    multiplied by one factor sqrt(|Phi+/Phi-|); afterwards Phi+ = -Phi- =
    sqrt(Phi+ |Phi-|) of the raw map, signs (neutral lines) kept."""
    nt, np_ = 48, 96
    w = oracle.cell_weights(nt, np_)[:, None]
    raw = oracle.rfe_map(nt, np_, 2, PHI, 9, 2, 5, balance=False)
    bal = oracle.rfe_map(nt, np_, 2, PHI, 9, 2, 5, balance=True)
    assert np.array_equal(np.sign(raw), np.sign(bal))
    pp, pm = (raw * w)[raw > 0].sum(), (raw * w)[raw < 0].sum()
    assert abs(pp + pm) > 1e-3 * pp            # the raw map is not balanced
    qp, qm = (bal * w)[bal > 0].sum(), (bal * w)[bal < 0].sum()
    assert abs(qp + qm) <= 1e-13 * qp
    assert qp == pytest.approx(math.sqrt(pp * -pm), rel=1e-13)
    fp = bal[raw > 0] / raw[raw > 0]
    fm = bal[raw < 0] / raw[raw < 0]
    assert np.ptp(fp) <= 1e-15 * fp[0] and np.ptp(fm) <= 1e-15 * fm[0]
    assert fp[0] * fm[0] == pytest.approx(1.0, rel=1e-14)


def _rfe_only(B0, t0, t1, **kw):
    opts = dict(rfe_model=2, rfe_phi_hr=PHI, rfe_tau=0.3, rfe_seed=4, rfe_id=1)
    opts.update(kw)
    return oracle.advance(B0, (0, 0, 0, 0, 0, 0), 0.0, t0, t1, **opts)


def test_source_integration_is_exact_and_lands_on_map_times():
    """No flow, no diffusion: B(T) is the integral of the piecewise-linear
    source of eq. rfe_s, whatever the steps.  Over [0, 1] h with tau = 0.3 h:
    steps 0.3, 0.3, 0.3, 0.1 (they land on the map times), and
    B(1) = tau (S0/2 + S1 + S2 + S3/2) + 0.1 (5/6 S3 + 1/6 S4)."""
    nt, np_ = 24, 48
    S = [oracle.rfe_map(nt, np_, 2, PHI, 4, 1, k) for k in range(5)]
    exact = 0.3 * (0.5 * S[0] + S[1] + S[2] + 0.5 * S[3]) + 0.1 * ((5 / 6) * S[3] + (1 / 6) * S[4])
    B0 = np.zeros((nt, np_))
    B, st = _rfe_only(B0, 0.0, 1.0)
    assert st["steps"] == 4 and st["dt_last"] == pytest.approx(0.1, abs=1e-12)
    scale = np.abs(exact).max()
    assert np.abs(B - exact).max() <= 1e-13 * scale
    for kw in ({"dt_max": 0.07}, {"strang": 1}, {"strang": 1, "dt_max": 0.045}):
        Bk, sk = _rfe_only(B0, 0.0, 1.0, **kw)
        assert np.abs(Bk - exact).max() <= 1e-13 * scale, kw
    # split advances restart from the maps of their own interval
    Ba, _ = _rfe_only(B0, 0.0, 0.45)
    Bb, _ = _rfe_only(Ba, 0.45, 1.0)
    assert np.abs(Bb - exact).max() <= 1e-13 * scale
    # mid-interval: int_0^{tau/2} ((1 - t/tau) S0 + (t/tau) S1) dt = 3 tau/8 S0 + tau/8 S1
    Bh, sh = _rfe_only(B0, 0.0, 0.15)
    assert sh["steps"] == 1
    assert np.abs(Bh - (0.1125 * S[0] + 0.0375 * S[1])).max() <= 1e-13 * scale


def test_interval_index():
    assert oracle.rfe_interval(0.0, 0.3) == 0
    assert oracle.rfe_interval(0.3, 0.3) == 1
    assert oracle.rfe_interval(0.8999999999999999, 0.3) == 3
    assert oracle.rfe_interval(0.9 - 5e-11, 0.3) == 3
    assert oracle.rfe_interval(0.9 - 5e-9, 0.3) == 2
    assert oracle.rfe_interval(1.0, 0.3) == 3


def test_infinite_lifetime_realizes_the_rate_finite_lifetime_cancels():
    """The paper's validation of the source (RFE only, zero start): with an
    infinite lifetime the total unsigned flux grows at the set rate phi_hr,
    with a finite lifetime much more slowly (samples cancel); the flux stays
    balanced in both cases."""
    nt, np_ = 128, 256
    w = oracle.cell_weights(nt, np_)[:, None] * R_CM ** 2
    B0 = np.zeros((nt, np_))
    T = 10.0
    Binf, _ = _rfe_only(B0, 0.0, T, rfe_tau=0.0)
    S0 = oracle.rfe_map(nt, np_, 2, PHI, 4, 1, 0)
    assert np.abs(Binf - T * S0).max() <= 1e-13 * np.abs(T * S0).max()
    unsigned = (np.abs(Binf) * w).sum()
    assert abs(unsigned / (T * PHI) - 1.0) < 0.02
    Bfin, st = _rfe_only(B0, 0.0, T, rfe_tau=0.3)
    assert st["steps"] == 34
    assert (np.abs(Bfin) * w).sum() < 0.3 * unsigned
    for B in (Binf, Bfin):
        assert abs((B * w).sum()) <= 1e-12 * (np.abs(B) * w).sum()


def test_source_with_transport_keeps_the_flux_balanced():
    """Flows, diffusion and the balanced source together: the net flux of a
    balanced start stays zero to round-off (the split operators conserve it,
    each source map is balanced)."""
    import synth
    nt, np_ = 32, 64
    w = oracle.cell_weights(nt, np_)[:, None]
    r = synth.Realization(nu_km2_s=500.0, **synth.dr_mf(amp_mf=15.0))
    B0 = synth.bipolar_field(nt, np_, synth.bipolar_pairs(4, 3))
    B0 = B0 - (B0 * w).sum() / (w.sum() * np_)
    for model, strang in ((1, 0), (2, 1)):
        B, _ = oracle.advance(B0, r.flow, r.nu_km2_s, 0.0, 6.0, strang=strang, rfe_model=model,
                              rfe_phi_hr=PHI, rfe_tau=0.7, rfe_seed=2, rfe_id=0)
        assert abs((B * w).sum()) <= 1e-12 * (np.abs(B) * w).sum()
        assert np.abs(B - B0).max() > 1.0
