"""The FP32 increment form of the super-time-stepping recurrence, modelled in
numpy (CPU): carried as the increment d and its last change e it is the same
recurrence as the three-term form (equal to the FP64 oracle in FP64), and in
FP32 its rounding error stays far below the three-term form's over a call of
about a thousand stages (the three-term form's errors grow with the square
of the stage count).  The GPU's FP32 kernels fold the stage coefficients
into the operator rows (per row and stage, formed in FP64 and rounded to
FP32: cL ph, cL up, cL dd - cy0, cL dn) and sum the two longitude neighbours
first; that arithmetic is modelled too.  This pins the arithmetic the GPU's
FP32 kernels use."""
import numpy as np
import pytest

import oracle

NT, NP = 128, 256


def operator(coefs, y):
    """The five-diagonal operator with the oracle's row coefficients (pole
    rows carry a zero pole-face coefficient; their clamped neighbour meets it)."""
    up, dn, ph, dd = coefs
    n = np.concatenate([y[:1], y[:-1]], axis=0)
    s = np.concatenate([y[1:], y[-1:]], axis=0)
    w, e = np.roll(y, 1, axis=1), np.roll(y, -1, axis=1)
    return ph[:, None] * w + up[:, None] * n + dd[:, None] * y + dn[:, None] * s + ph[:, None] * e


def folded_increment(c64, cl, cy0, nu_j, g, d, e, ly0, dtype):
    """e_j in the folded form: A (w + e) + U n + C d + S s - nu e + G L(Y0),
    with A, U, C, S formed per row in FP64 and rounded (dtype arithmetic)."""
    up, dn, ph, dd = c64
    A, U = (cl * ph).astype(dtype)[:, None], (cl * up).astype(dtype)[:, None]
    C, S = (cl * dd - cy0).astype(dtype)[:, None], (cl * dn).astype(dtype)[:, None]
    n = np.concatenate([d[:1], d[:-1]], axis=0)
    s = np.concatenate([d[1:], d[-1:]], axis=0)
    t = (np.roll(d, 1, axis=1) + np.roll(d, -1, axis=1)).astype(dtype)
    return A * t + U * n + C * d + S * s + dtype(-nu_j) * e + dtype(g) * ly0


def run(y0, nu, tau, s, dtype, carried, folded=False):
    mu, nv, mut, gamt = oracle.sts_coefs(s, oracle.RKG2)
    c64 = oracle.diff_coefs(NT, NP, nu)
    coefs = tuple(c.astype(dtype) for c in c64)
    ly0 = operator(oracle.diff_coefs(NT, NP, nu), y0).astype(dtype)   # L(Y0) formed in FP64
    d = (dtype(mut[1] * tau) * ly0).astype(dtype)
    e = d.copy()                               # d_1 - d_0, d_0 = 0
    dprev = np.zeros_like(d)
    for j in range(2, s + 1):
        L = operator(coefs, d)
        c1, c2 = dtype(mut[j] * tau), dtype((mut[j] + gamt[j]) * tau)
        if folded:
            en = folded_increment(c64, mut[j] * tau, 1.0 - mu[j] - nv[j], nv[j], (mut[j] + gamt[j]) * tau,
                                  d, e, ly0, dtype)
            d, e = (d + en).astype(dtype), en.astype(dtype)
        elif carried:
            en = dtype(mu[j] + nv[j] - 1.0) * d - dtype(nv[j]) * e + c1 * L + c2 * ly0
            d, e = (d + en).astype(dtype), en.astype(dtype)
        else:
            dn = dtype(mu[j]) * d + dtype(nv[j]) * dprev + c1 * L + c2 * ly0
            dprev, d = d, dn.astype(dtype)
    return y0 + d.astype(np.float64)


@pytest.fixture(scope="module")
def case():
    th = (np.arange(NT) + 0.5) * np.pi / NT
    ph = (np.arange(NP) + 0.5) * 2 * np.pi / NP
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    y0 = 300.0 * np.exp(-((TH - 1.2) ** 2 + (PH - 2.0) ** 2) / 0.05) - 200.0 * np.sin(TH) ** 3 * np.cos(3 * PH)
    _, k2 = oracle.units()
    nu = 500.0 * k2
    dte = oracle.euler_limit(NT, NP, nu)
    tau = 1.7e5 * dte
    s = oracle.sts_stages(tau, dte, oracle.RKG2)
    ref, st = oracle.diffuse(y0, nu, tau, oracle.RKG2)
    assert st == s and s > 900
    return y0, nu, tau, s, ref


def test_carried_form_is_the_same_recurrence(case):
    """In FP64 both forms land on the oracle's result (the same recurrence,
    rounded differently)."""
    y0, nu, tau, s, ref = case
    for carried, folded in ((False, False), (True, False), (True, True)):
        got = run(y0, nu, tau, s, np.float64, carried, folded)
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert e < 1e-11, (carried, folded, e)


def test_carried_form_keeps_fp32_rounding_small(case):
    """In FP32 the three-term form drifts by ~s^2 eps of the increment; the
    carried form stays orders of magnitude closer to the FP64 oracle."""
    y0, nu, tau, s, ref = case
    e3 = np.linalg.norm(run(y0, nu, tau, s, np.float32, False) - ref) / np.linalg.norm(ref)
    ec = np.linalg.norm(run(y0, nu, tau, s, np.float32, True) - ref) / np.linalg.norm(ref)
    ef = np.linalg.norm(run(y0, nu, tau, s, np.float32, True, True) - ref) / np.linalg.norm(ref)
    assert ec < 1e-6, ec
    assert ec < e3 / 30.0, (e3, ec)
    assert ef < 1e-6, ef
    assert ef < e3 / 30.0, (e3, ef)


def run_paper(y0, nu, tau, s, dtype):
    """The paper's three-term recurrence in Y itself, in the given precision."""
    mu, nv, mut, gamt = oracle.sts_coefs(s, oracle.RKG2)
    coefs = tuple(c.astype(dtype) for c in oracle.diff_coefs(NT, NP, nu))
    Y0 = y0.astype(dtype)
    ly0 = operator(coefs, Y0)
    ym2, ym1 = Y0, Y0 + dtype(mut[1] * tau) * ly0
    for j in range(2, s + 1):
        y = (dtype(mu[j]) * ym1 + dtype(nv[j]) * ym2 + dtype(1.0 - mu[j] - nv[j]) * Y0 +
             dtype(mut[j] * tau) * operator(coefs, ym1) + dtype(gamt[j] * tau) * ly0)
        ym2, ym1 = ym1, y
    return ym1


def test_fp64_paper_form_drifts_and_increment_form_does_not(case):
    """In FP64 the three-term recurrence in Y (the paper's form, which the
    oracle evaluates) drifts from an 80-bit run of the same recurrence by far
    more than rounding level over a ~1,000-stage call, while the carried
    increment form stays at rounding level: the FP64 oracle's own error on
    long calls is this drift (it grows with resolution and stage count)."""
    y0, nu, tau, s, ref = case
    ext = run_paper(y0, nu, tau, s, np.longdouble).astype(np.float64)
    paper = run_paper(y0, nu, tau, s, np.float64)
    inc = run(y0, nu, tau, s, np.float64, True, True)
    e_paper = np.linalg.norm(paper - ext) / np.linalg.norm(ext)
    e_inc = np.linalg.norm(inc - ext) / np.linalg.norm(ext)
    e_oracle = np.linalg.norm(ref - ext) / np.linalg.norm(ext)
    assert 1e-14 < e_paper < 1e-12, e_paper
    assert e_inc < 1e-14, e_inc
    assert abs(e_oracle - e_paper) < 0.1 * e_paper, (e_oracle, e_paper)
