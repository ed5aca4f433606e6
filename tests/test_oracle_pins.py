"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/paper_constants.txt), closed-form solutions,
invariants, library routines (scipy spherical harmonics, Legendre and
Gegenbauer polynomials, dense eigen-decompositions) or brute force on tiny
grids.  None of these tests needs a GPU.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden():
    out = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, val = line.split()[:2]
        out[name] = float(val)
    return out


def grid(nt, np_):
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = (np.arange(np_) + 0.5) * 2 * np.pi / np_
    return np.meshgrid(th, ph, indexing="ij")


def weights(nt, np_):
    th = (np.arange(nt) + 0.5) * np.pi / nt
    return np.sin(th) * (np.pi / nt) * (2 * np.pi / np_)


def dense(op, nt, np_):
    """Dense matrix of a linear grid operator by applying it to unit vectors."""
    n = nt * np_
    M = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, i] = op(e.reshape(nt, np_)).ravel()
    return M


# ------------------------------------------------------------------ units
def test_units_match_paper():
    g = golden()
    ms, k2 = oracle.units()
    assert ms == pytest.approx(g["m_s_to_rs_hr"], rel=1e-15)
    assert k2 == pytest.approx(g["km2_s_to_rs2_hr"], rel=1e-14)


def test_rigid_rotation_period_from_flow_form():
    """eq. dr with d0 = 1807.66 m/s and d2 = d4 = 0 turns once in 672 h."""
    g = golden()
    nt = 16
    vph, vth = oracle.flows(nt, (g["rigid_rotation_km_s"] * 1000.0, 0, 0, 0, 0, 0))
    th = (np.arange(nt) + 0.5) * np.pi / nt
    omega = vph / np.sin(th)          # rad/h on the unit sphere
    assert np.allclose(omega, omega[0], rtol=1e-14)
    assert 2 * np.pi / omega[0] == pytest.approx(g["rigid_rotation_period_h"], rel=1e-5)
    assert np.all(vth == 0.0)


def test_flow_shapes():
    nt = 32
    d = (46.0, -262.0, -379.0, 22.0, 11.0, -28.0)     # the paper's defaults
    vph, vth = oracle.flows(nt, d)
    ms, _ = oracle.units()
    # DR symmetric about the equator, MF antisymmetric and zero at the poles
    assert np.allclose(vph, vph[::-1], rtol=1e-13, atol=0)
    assert np.allclose(vth, -vth[::-1], atol=1e-18)
    assert vth[0] == 0.0 and vth[-1] == 0.0
    # equator face: v_theta = 0, v_phi at the row nearest the equator ~ d0
    assert abs(vth[nt // 2]) < 1e-20
    # poleward flow for positive m1 (northern faces move towards theta = 0)
    d1 = (0, 0, 0, 30.0, 0, 0)
    _, v1 = oracle.flows(nt, d1)
    assert np.all(v1[1:nt // 2] < 0) and np.all(v1[nt // 2 + 1:-1] > 0)
    # the m1 term alone peaks at 45 degrees with amplitude m1/2 (sin 2 lambda form)
    f = np.arange(nt + 1) * np.pi / nt
    assert np.allclose(v1, -30.0 * ms * np.cos(f) * np.sin(f) * (f > 0) * (f < np.pi), atol=1e-18)


def test_cfl_limits_rigid_rotation():
    nt, np_ = 24, 48
    omega = 2 * np.pi / 672.0
    th = (np.arange(nt) + 0.5) * np.pi / nt
    vph = omega * np.sin(th)
    vth = np.zeros(nt + 1)
    dph = 2 * np.pi / np_
    lim = oracle.cfl_dt(nt, np_, vph, vth, oracle.SSPRK43)
    assert lim == pytest.approx(dph / omega, rel=1e-13)
    assert oracle.cfl_dt(nt, np_, vph, vth, oracle.FE) == pytest.approx(0.5 * dph / omega, rel=1e-13)
    assert oracle.cfl_dt(nt, np_, vph * 0, vth, oracle.SSPRK43) == math.inf



@pytest.mark.parametrize("case", ["top", "bottom"])
def test_cfl_takes_the_larger_flanking_theta_speed(case):
    """Eq. ssprk43_dt evaluates each velocity at a cell as the larger of its
    two flanking staggered values.  One row carries azimuthal speed and its
    two theta faces carry different speeds (the larger one on top, then on
    the bottom); every other face is at rest, so that row binds and the limit
    is 1/(max(a, b)/dth + vp/(sin(theta) dph)).  Reading one face only, or the
    mean of the two, gives a different number in one of the two cases."""
    nt, np_ = 24, 48
    dth, dph = np.pi / nt, 2 * np.pi / np_
    j = 7
    a, b = (3.0, 1.0) if case == "top" else (1.0, 3.0)
    vth = np.zeros(nt + 1)
    vth[j], vth[j + 1] = -a, b
    vph = np.zeros(nt)
    vph[j] = 0.8
    s = math.sin((j + 0.5) * dth)
    want = 1.0 / (3.0 / dth + 0.8 / (s * dph))
    lim = oracle.cfl_dt(nt, np_, vph, vth, oracle.SSPRK43)
    assert lim == pytest.approx(want, rel=1e-14)
    for wrong in (1.0 / (2.0 / dth + 0.8 / (s * dph)),                       # mean of the flanks
                  1.0 / max(1.0 / dth + 0.8 / (s * dph), 3.0 / dth)):        # the other face only
        assert abs(lim - wrong) > 1e-3 * want
    # forward Euler and SSPRK(3,3) take half of it (eq. advection_timestep)
    assert oracle.cfl_dt(nt, np_, vph, vth, oracle.FE) == pytest.approx(0.5 * want, rel=1e-14)
    assert oracle.cfl_dt(nt, np_, vph, vth, oracle.SSPRK33) == pytest.approx(0.5 * want, rel=1e-14)


def test_cfl_closed_form_for_the_workload_flows():
    """Eq. mf with m1 only is v_theta = -m1 cos(theta) sin(theta), whose
    largest speed m1/2 sits on the face at 45 degrees (a face of the grid when
    nt is a multiple of 4).  Alone it gives dth/(m1/2); with rigid rotation
    added (eq. dr with d0 only, so v_phi/(sin(theta) dph) is the same Omega/dph
    in every row) the limit is 1/((m1/2)/dth + Omega/dph).  The mean of two
    flanks never reaches the peak, so that reading fails both."""
    nt, np_ = 40, 80
    dth, dph = np.pi / nt, 2 * np.pi / np_
    ms, _ = oracle.units()
    m1, d0 = 24.0, 140.0
    for with_dr in (False, True):
        vph, vth = oracle.flows(nt, (d0 if with_dr else 0.0, 0, 0, m1, 0, 0))
        omega = d0 * ms if with_dr else 0.0
        want = 1.0 / (0.5 * m1 * ms / dth + omega / dph)
        assert oracle.cfl_dt(nt, np_, vph, vth, oracle.SSPRK43) == pytest.approx(want, rel=1e-13)
        # the factor 1/2 of forward Euler and SSPRK(3,3)
        for ts in (oracle.FE, oracle.SSPRK33):
            assert oracle.cfl_dt(nt, np_, vph, vth, ts) == pytest.approx(0.5 * want, rel=1e-13)
        mean_flank = np.maximum(0.5 * (np.abs(vth[:-1]) + np.abs(vth[1:])), 0.0).max()
        assert mean_flank < 0.5 * m1 * ms * (1 - 1e-3)

# --------------------------------------------------------------- WENO3
@pytest.mark.parametrize("nonuniform", [False, True])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_weno_exact_for_linear_data(nonuniform, sign):
    """Both WENO3 candidate reconstructions are exact for linear data, on any
    grid, whatever the nonlinear weights: the face value is the line through
    the cell centres.  This pins the D-factor index reading of App. B."""
    rng = np.random.default_rng(1)
    n = 24
    dx = 1.0 + 0.4 * rng.random(n) if nonuniform else np.ones(n)
    dx *= 0.01
    xf = np.concatenate([[0.0], np.cumsum(dx)])
    xc = 0.5 * (xf[1:] + xf[:-1])
    a, b = 0.7, 3.0
    B = a + b * xc
    v = np.full(n + 1, 0.3 * sign)
    F = oracle.line_flux(B, dx, v, periodic=False)
    exact = 0.3 * sign * (a + b * xf)
    assert np.allclose(F[2:n - 1], exact[2:n - 1], rtol=1e-13, atol=1e-15)
    # pole-adjacent faces are upwind, pole faces carry nothing
    up = 0.3 * sign * (B[0] if sign > 0 else B[1])
    assert F[1] == pytest.approx(up, rel=1e-15)
    assert F[0] == 0.0 and F[n] == 0.0


def test_weno_linear_weights_when_smoothness_equal():
    """With beta0 = beta1 on a uniform grid the nonlinear weights equal the
    linear ones (1/3, 2/3) and the reconstruction is -1/6, 5/6, 1/3."""
    n = 16
    B = np.zeros(n)
    B[7] = 1.0       # LM_{i-2}=0, LM_{i-1}=1, LM_i=0 at face 8 -> beta0 = beta1
    dx = np.full(n, 0.05)
    v = np.full(n + 1, 2.0)
    F = oracle.line_flux(B, dx, v, periodic=True)
    assert F[8] == pytest.approx(2.0 * 5.0 / 6.0, rel=1e-14)
    # mirror: leftward flow reconstructs from the right
    F2 = oracle.line_flux(B, dx, -v, periodic=True)
    assert F2[7] == pytest.approx(-2.0 * 5.0 / 6.0, rel=1e-14)


def test_weno_mirror_symmetry():
    """Reversing a periodic line and the flow direction mirrors the fluxes."""
    rng = np.random.default_rng(2)
    n = 20
    B = rng.standard_normal(n)
    dx = np.full(n, 0.1)
    v = np.full(n + 1, 0.8)
    F = oracle.line_flux(B, dx, v, periodic=True)
    Fr = oracle.line_flux(B[::-1].copy(), dx, -v, periodic=True)
    assert np.allclose(Fr[::-1], -F, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------ advection
def test_advection_conserves_flux_and_constants():
    nt, np_ = 20, 40
    rng = np.random.default_rng(3)
    B = rng.standard_normal((nt, np_))
    vph, vth = oracle.flows(nt, (46.0, -262.0, -379.0, 22.0, 11.0, -28.0))
    w = weights(nt, np_)
    for scheme in (oracle.WENO3CSH, oracle.UPWIND):
        A = oracle.adv_operator(B, vph, vth, scheme)
        assert abs((A * w[:, None]).sum()) < 1e-14 * (np.abs(A) * w[:, None]).sum()
    # differential rotation is divergence free: a constant stays constant
    A = oracle.adv_operator(np.full((nt, np_), 3.0), vph, 0 * vth)
    assert np.abs(A).max() < 1e-15


def test_upwind_euler_courant_one_is_a_shift():
    nt, np_ = 8, 32
    omega = 2 * np.pi / 672.0
    th = (np.arange(nt) + 0.5) * np.pi / nt
    vph, vth = omega * np.sin(th), np.zeros(nt + 1)
    dt = (2 * np.pi / np_) / omega
    B = np.random.default_rng(4).standard_normal((nt, np_))
    B1 = oracle.adv_step(B, vph, vth, dt, oracle.UPWIND, oracle.FE)
    assert np.allclose(B1, np.roll(B, 1, axis=1), atol=1e-13)


@pytest.mark.parametrize("time_scheme,coefs", [
    (oracle.SSPRK43, [1, 1, 1 / 2, 1 / 6, 1 / 48]),
    (oracle.SSPRK33, [1, 1, 1 / 2, 1 / 6]),
    (oracle.FE, [1, 1]),
])
def test_ssprk_stability_polynomial(time_scheme, coefs):
    """On a linear operator one step is P(-dt M) with the scheme's stability
    polynomial: Taylor coefficients of exp up to third order, and z^4/48 for
    SSPRK(4,3).  M is the dense upwind operator (with both flows)."""
    nt, np_ = 6, 10
    vph, vth = oracle.flows(nt, (800.0, -300.0, 0.0, 400.0, 0.0, 0.0))
    M = dense(lambda x: oracle.adv_operator(x, vph, vth, oracle.UPWIND), nt, np_)
    dt = 0.3 * oracle.cfl_dt(nt, np_, vph, vth)
    Z = -dt * M
    P = np.zeros_like(Z)
    Zk = np.eye(Z.shape[0])
    for c in coefs:
        P += c * Zk
        Zk = Zk @ Z
    B = np.random.default_rng(5).standard_normal((nt, np_))
    got = oracle.adv_step(B, vph, vth, dt, oracle.UPWIND, time_scheme)
    assert np.allclose(got.ravel(), P @ B.ravel(), rtol=1e-12, atol=1e-13)


def blob_field(th, ph, t, vth_c, om, sigma=0.03):
    """Eq. testblob (App. C exact solution), with periodic phi distance."""
    def d(a):
        return (a + np.pi) % (2 * np.pi) - np.pi
    g = th - np.pi / 4 - vth_c * t
    e1 = np.exp(-g ** 2 / sigma - d(ph - np.pi / 2 - om * t) ** 2 / sigma)
    e2 = np.exp(-g ** 2 / sigma - d(ph - 3 * np.pi / 2 - om * t) ** 2 / sigma)
    return (-e1 + e2) / np.sin(th)


def run_blob(nt, np_, vth_c, om, T, scheme=oracle.WENO3CSH, eps_mode=0.0):
    TH, PH = grid(nt, np_)
    B = blob_field(TH, PH, 0.0, vth_c, om)
    th = (np.arange(nt) + 0.5) * np.pi / nt
    vph = om * np.sin(th)
    vth = np.full(nt + 1, vth_c)
    vth[0] = vth[-1] = 0.0
    cfl = 0.9 * oracle.cfl_dt(nt, np_, vph, vth)
    nsteps = int(math.ceil(T / cfl))
    dt = T / nsteps
    for _ in range(nsteps):
        B = oracle.adv_step(B, vph, vth, dt, scheme, oracle.SSPRK43, eps_mode)
    return oracle.hh(B, blob_field(TH, PH, T, vth_c, om))


def order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]


def test_phi_rotation_convergence_orders():
    """App. B: WENO3-CS(h) converges at third order on the phi-rotation
    Gaussian test; WENO3 with a constant eps = 1e-12 loses that order and
    upwinding is far less accurate (first order, pre-asymptotic here)."""
    om = 2 * np.pi / 672.0
    ns = [256, 512, 1024]
    e_h = [run_blob(16, n, 0.0, om, 672.0) for n in ns]
    e_e = [run_blob(16, n, 0.0, om, 672.0, eps_mode=1e-12) for n in ns]
    e_u = [run_blob(16, n, 0.0, om, 672.0, oracle.UPWIND) for n in ns]
    o_h, o_e, o_u = order(e_h, ns), order(e_e, ns), order(e_u, ns)
    assert o_h[-1] > 2.7, (e_h, o_h)
    assert 1.2 < o_e[-1] < 2.3, (e_e, o_e)
    assert e_e[-1] > 5 * e_h[-1]
    assert 0.3 < o_u[-1] < 1.2 and e_u[-1] > 50 * e_h[-1], (e_u, o_u)


def test_theta_advection_exact_solution():
    """App. C: (1/sin theta) B0(theta - v t) is exact for constant v_theta;
    the pair moves from 45 degrees north to 45 degrees south in 672 h and
    the error falls at high order."""
    vt = (np.pi / 2) / 672.0
    ns = [128, 256, 512]
    e = [run_blob(n, 64, vt, 0.0, 672.0) for n in ns]
    assert e[-1] < 1e-3
    assert order(e, ns)[-1] > 2.7, e


# ------------------------------------------------------------ diffusion
def test_diffusion_matrix_symmetry_and_constants():
    nt, np_ = 12, 24
    nu = 3.7e-6
    a_up, a_dn, a_ph, a_d = oracle.diff_coefs(nt, np_, nu)
    w = weights(nt, np_)
    # weighted symmetry w_j a_{j,j+1} = w_{j+1} a_{j+1,j}
    assert np.allclose(w[:-1] * a_dn[:-1], w[1:] * a_up[1:], rtol=1e-14)
    assert a_up[0] == 0.0 and a_dn[-1] == 0.0
    L = oracle.diff_operator(np.full((nt, np_), 2.5), nu)
    assert np.abs(L).max() < 1e-12 * np.abs(a_d).max()
    # self-adjoint in the weighted inner product, negative semi-definite
    M = dense(lambda x: oracle.diff_operator(x, nu), nt, np_)
    W = np.repeat(w, np_)
    S = np.sqrt(W)[:, None] * M / np.sqrt(W)[None, :]
    assert np.allclose(S, S.T, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.max() < 1e-9 * abs(ev.min())
    # Euler limit reading: dt_E * spectral radius <= 2 (forward Euler stable)
    dtE = oracle.euler_limit(nt, np_, nu)
    assert dtE == pytest.approx(1.0 / np.abs(a_d).max(), rel=1e-15)
    assert dtE * abs(ev.min()) <= 2.0 + 1e-12


def real_ylm(l, m, th, ph):
    y = sps.sph_harm_y(l, abs(m), th, ph)
    return y.real if m >= 0 else y.imag


def soccer(th, ph):
    return real_ylm(6, 0, th, ph) + math.sqrt(14.0 / 11.0) * real_ylm(6, 5, th, ph)


@pytest.mark.parametrize("scheme", [oracle.RKG2, oracle.RKL2])
def test_soccer_ball_decay_second_order(scheme):
    """Eq. soccerball: exp(-42 nu t) decay of an l = 6 mode; the spatial error
    falls as O(h^2)."""
    _, k2 = oracle.units()
    nu = 500.0 * k2
    tau, ncall = 168.0, 80      # 20 rotations in short calls: time error small
    errs = []
    ns = [24, 48]
    for nt in ns:
        TH, PH = grid(nt, 2 * nt)
        u0 = soccer(TH, PH)
        u = u0
        for _ in range(ncall):
            u, st = oracle.diffuse(u, nu, tau, scheme)
        exact = math.exp(-42.0 * nu * tau * ncall) * u0
        errs.append(oracle.hh(u, exact))
    assert math.exp(-42.0 * nu * tau * ncall) < 0.2
    assert errs[-1] < 5e-2
    assert order(errs, ns)[0] > 1.8, errs


def test_y10_decay_and_flux_conservation():
    _, k2 = oracle.units()
    nu = 600.0 * k2
    nt, np_ = 64, 128
    TH, PH = grid(nt, np_)
    u0 = np.cos(TH)
    T = 5000.0
    u, _ = oracle.diffuse(u0, nu, T)
    ratio = (u * u0).sum() / (u0 * u0).sum()
    assert ratio == pytest.approx(math.exp(-2.0 * nu * T), rel=2e-3)
    w = weights(nt, np_)
    v0 = (np.random.default_rng(6).standard_normal((nt, np_)))
    v1, _ = oracle.diffuse(v0, nu, 3.0)
    assert abs(((v1 - v0) * w[:, None]).sum()) < 1e-13 * (np.abs(v0) * w[:, None]).sum()


def sts_poly(s, scheme):
    """The STS stability polynomial from its defining conditions: R(z) = a +
    b P_s(1 + w z) with R(0) = R'(0) = R''(0) = 1, P = Legendre (RKL2) or
    Gegenbauer(3/2) (RKG2), evaluated with scipy's polynomial routines."""
    if scheme == oracle.RKL2:
        P = sps.legendre(s)
    else:
        P = sps.gegenbauer(s, 1.5)
    p1, d1, d2 = P(1.0), P.deriv(1)(1.0), P.deriv(2)(1.0)
    w = d1 / d2
    b = 1.0 / (w * d1)
    a = 1.0 - b * p1
    return (lambda z: a + b * P(1.0 + w * z)), w


@pytest.mark.parametrize("scheme", [oracle.RKG2, oracle.RKL2])
@pytest.mark.parametrize("tau", [0.05, 0.7, 9.0])
def test_sts_matches_stability_polynomial_brute_force(scheme, tau):
    """One STS call equals R_s(tau M) Y0 for the dense operator M of a tiny
    grid (eigen-decomposition), with s the fewest stages whose stability
    interval [-2/w, 0] covers the Gershgorin bound."""
    nt, np_ = 6, 12
    _, k2 = oracle.units()
    nu = 400.0 * k2 * 1e3
    M = dense(lambda x: oracle.diff_operator(x, nu), nt, np_)
    dtE = oracle.euler_limit(nt, np_, nu)
    s = oracle.sts_stages(tau, dtE, scheme)
    R, w = sts_poly(s, scheme)
    lam_bound = 2.0 / dtE
    assert 2.0 / w >= tau * lam_bound * (1 - 1e-12)
    if s > 2:
        _, w_prev = sts_poly(s - 1, scheme)
        assert 2.0 / w_prev < tau * lam_bound
    ev, V = sla.eig(M)
    ev, V = ev.real, V.real
    Y0 = np.random.default_rng(7).standard_normal(nt * np_)
    exact = V @ (R(tau * ev) * np.linalg.solve(V, Y0))
    got, st = oracle.diffuse(Y0.reshape(nt, np_), nu, tau, scheme)
    assert st == s
    assert np.allclose(got.ravel(), exact, rtol=1e-11, atol=1e-11 * np.abs(Y0).max())
    assert np.all(np.abs(R(tau * ev)) <= 1 + 1e-12)



def _fewest_stages(tau, dtE, scheme):
    """Fewest stages (>= 2) whose stability interval [-2/w, 0] covers the
    Gershgorin bound 2/dtE of the operator's spectrum, from the polynomials."""
    s = 2
    while 2.0 / sts_poly(s, scheme)[1] < tau * (2.0 / dtE) * (1 - 1e-12):
        s += 1
    return s


@pytest.mark.parametrize("scheme", [oracle.RKG2, oracle.RKL2])
@pytest.mark.parametrize("tau,ptl", [(9.0, 2.5), (9.0, 3.0), (0.7, 2.0)])
def test_ptl_hook_splits_into_equal_sts_calls(scheme, tau, ptl):
    """With a step limit ptl_dt the diffusion advance of length tau runs as
    n = ceil(tau/ptl_dt) super-time-stepping calls of the same length tau/n
    (one call when tau <= ptl_dt), so the result is R_s(tau/n M)^n Y0 with s
    the fewest stages for tau/n, and n s stages are counted (dense
    eigen-decomposition on a 6 x 12 grid).  A floor instead of the ceiling,
    or unequal calls (full ptl_dt steps and a remainder), land elsewhere."""
    nt, np_ = 6, 12
    _, k2 = oracle.units()
    nu = 400.0 * k2 * 1e3
    M = dense(lambda x: oracle.diff_operator(x, nu), nt, np_)
    dtE = oracle.euler_limit(nt, np_, nu)
    n = math.ceil(tau / ptl) if tau > ptl else 1
    tc = tau / n
    s = _fewest_stages(tc, dtE, scheme)
    R, _ = sts_poly(s, scheme)
    ev, V = sla.eig(M)
    ev, V = ev.real, V.real
    Y0 = np.random.default_rng(11).standard_normal(nt * np_)
    Vi = np.linalg.inv(V)

    def run(lengths):
        y = Y0.copy()
        for h in lengths:
            Rh, _ = sts_poly(_fewest_stages(h, dtE, scheme), scheme)
            y = V @ (Rh(h * ev) * (Vi @ y))
        return y

    exact = V @ (R(tc * ev) ** n * (Vi @ Y0))
    got, st = oracle.diffuse(Y0.reshape(nt, np_), nu, tau, scheme, ptl_dt=ptl)
    assert st == n * s
    scale = np.abs(Y0).max()
    assert np.allclose(got.ravel(), exact, rtol=1e-10, atol=1e-10 * scale)
    if n > 1:
        nf = math.floor(tau / ptl)
        for wrong in (run([tau / nf] * nf) if nf * ptl != tau else None,
                      run([ptl] * nf + ([tau - nf * ptl] if tau > nf * ptl else []))):
            if wrong is not None and not np.allclose(wrong, exact, rtol=1e-10, atol=1e-10 * scale):
                assert np.abs(got.ravel() - wrong).max() > 1e-6 * scale
    # the grid-diffusivity path (eq. diffgrid) runs the same hook
    nf_face = np.full(nt + 1, nu)
    got_f, st_f = oracle.diffuse_face(Y0.reshape(nt, np_), nf_face, tau, scheme, ptl_dt=ptl)
    assert st_f == n * s
    assert np.array_equal(got_f, got)

def test_forward_euler_diffusion_reference():
    nt, np_ = 6, 12
    nu = 0.3
    M = dense(lambda x: oracle.diff_operator(x, nu), nt, np_)
    dtE = oracle.euler_limit(nt, np_, nu)
    tau = 3.3 * dtE
    n = math.ceil(tau / dtE)
    Y0 = np.random.default_rng(8).standard_normal(nt * np_)
    exact = np.linalg.matrix_power(np.eye(nt * np_) + (tau / n) * M, n) @ Y0
    got, st = oracle.diffuse(Y0.reshape(nt, np_), nu, tau, oracle.DIFF_FE)
    assert st == n
    assert np.allclose(got.ravel(), exact, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------- assimilation
def test_mu_disk_is_cosine_of_angle_to_disk_centre():
    nt, np_ = 18, 36
    b0, l0 = math.radians(7.0), math.radians(100.0)
    TH, PH = grid(nt, np_)
    cell = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    lat0 = b0
    centre = np.array([math.cos(lat0) * math.cos(l0), math.cos(lat0) * math.sin(l0), math.sin(lat0)])
    assert np.allclose(oracle.mu_disk(nt, np_, b0, l0), cell @ centre, atol=1e-15)


def test_weight_function():
    nt, np_ = 18, 36
    mu = oracle.mu_disk(nt, np_, 0.0, math.pi)
    F = oracle.weight_from_mu(mu, 4.0, 0.0, math.pi / 2)
    assert np.allclose(F, np.where(mu > 0, mu ** 4, 0.0), rtol=1e-14)
    TH, _ = grid(nt, np_)
    lat = np.pi / 2 - TH
    F2 = oracle.weight_from_mu(mu, 2.0, 0.3, math.radians(60))
    ref = np.where((mu > 0.3) & (np.abs(lat) < math.radians(60)), mu ** 2, 0.0)
    assert np.allclose(F2, ref, rtol=1e-13)


def test_assimilation_limits_and_balance():
    nt, np_ = 16, 32
    rng = np.random.default_rng(9)
    B = rng.standard_normal((nt, np_)) * 50
    D = rng.standard_normal((nt, np_)) * 50 + 5.0
    assert np.array_equal(oracle.assimilate(B, D, np.ones_like(B)), D)
    assert np.array_equal(oracle.assimilate(B, D, np.zeros_like(B)), B)
    F = rng.random((nt, np_))
    Bn = oracle.assimilate(B, D, F, flux_balance=True)
    dB = Bn - B
    raw = F * (D - B)
    w = weights(nt, np_)[:, None]
    pp, pm = (dB * w)[dB > 0].sum(), (dB * w)[dB < 0].sum()
    assert pp == pytest.approx(-pm, rel=1e-12)
    assert np.array_equal(np.sign(dB), np.sign(raw))
    rp, rm = (raw * w)[raw > 0].sum(), (raw * w)[raw < 0].sum()
    assert pp == pytest.approx(math.sqrt(abs(rp * rm)), rel=1e-12)


# ----------------------------------------------------------- diagnostics
def test_diagnostics_dipoles_and_fluxes():
    nt, np_ = 90, 180
    TH, PH = grid(nt, np_)
    d = oracle.diagnostics(np.cos(TH))
    assert d["dax"] == pytest.approx(1.0, abs=5e-4)
    assert d["phi_pos"] == pytest.approx(np.pi, rel=5e-4)
    assert d["phi_neg"] == pytest.approx(-np.pi, rel=5e-4)
    assert abs(d["phi_net"]) < 1e-12
    d1 = oracle.diagnostics(np.sin(TH) * np.cos(PH))
    assert d1["h1"] == pytest.approx(1.0, abs=5e-4) and abs(d1["h2"]) < 1e-12
    d2 = oracle.diagnostics(np.sin(TH) * np.sin(PH))
    assert d2["h2"] == pytest.approx(1.0, abs=5e-4) and abs(d2["h1"]) < 1e-12
    B = np.zeros((nt, np_))
    B[3, 4], B[10, 7] = -7.0, 9.0
    d3 = oracle.diagnostics(B)
    assert d3["bmin"] == -7.0 and d3["bmax"] == 9.0 and d3["babs_min"] == 0.0


def test_hh_metric():
    assert oracle.hh(np.array([1.0, 2.0]), np.array([1.0, 1.0])) == pytest.approx(math.sqrt(1 / 3))


# -------------------------------------------------------------- time loop
def test_time_loop_dt_rule_and_conservation():
    nt, np_ = 32, 64
    prm = (0.0, -337.4, -253.1, 30.0, 0.0, 0.0)
    vph, vth = oracle.flows(nt, prm)
    cfl = oracle.cfl_dt(nt, np_, vph, vth)
    B0 = np.random.default_rng(10).standard_normal((nt, np_)) * 30
    T = 3.7 * cfl
    B, st = oracle.advance(B0, prm, 500.0, 0.0, T)
    assert st["steps"] == math.ceil(T / (0.9 * cfl))
    assert st["dt_last"] == pytest.approx(T - (st["steps"] - 1) * 0.9 * cfl, rel=1e-9)
    w = weights(nt, np_)[:, None]
    assert abs(((B - B0) * w).sum()) < 1e-13 * (np.abs(B0) * w).sum()
    # the same interval in two calls lands at the same state up to the split
    Ba, _ = oracle.advance(B0, prm, 500.0, 0.0, 0.5 * T)
    Ba, _ = oracle.advance(Ba, prm, 500.0, 0.5 * T, T)
    assert np.allclose(Ba, B, atol=1e-2 * np.abs(B0).max())


def test_time_loop_minimum_step():
    """A minimum step (Sec. "Time steps" lists it among the user's controls)
    raises the step limit min(0.9 CFL, dt_max) to dt_min; the step still ends
    on the interval's end.  Below the limit it changes nothing."""
    nt, np_ = 24, 48
    prm = (0.0, -337.4, -253.1, 30.0, 0.0, 0.0)
    vph, vth = oracle.flows(nt, prm)
    lim = 0.9 * oracle.cfl_dt(nt, np_, vph, vth)
    B0 = np.random.default_rng(12).standard_normal((nt, np_)) * 30
    T = 7.3 * lim
    ref, st0 = oracle.advance(B0, prm, 300.0, 0.0, T)
    same, st1 = oracle.advance(B0, prm, 300.0, 0.0, T, dt_min=0.5 * lim)
    assert np.array_equal(ref, same) and st1 == st0
    dmin = 2.5 * lim
    _, st = oracle.advance(B0, prm, 300.0, 0.0, T, dt_min=dmin)
    assert st["steps"] == math.ceil(T / dmin) == 3
    assert st["dt_last"] == pytest.approx(T - 2 * dmin, rel=1e-12)
    # dt_min also overrides a smaller dt_max
    _, st = oracle.advance(B0, prm, 300.0, 0.0, T, dt_max=0.3 * lim, dt_min=dmin)
    assert st["steps"] == 3
    # and never carries a step past the end
    _, st = oracle.advance(B0, prm, 300.0, 0.0, 0.4 * lim, dt_min=dmin)
    assert st["steps"] == 1 and st["dt_last"] == pytest.approx(0.4 * lim, rel=1e-15)


def test_attenuated_cfl_closed_forms():
    """CFL limit of the attenuated flow (eq. flow_attenuation inside eq.
    ssprk43_dt): a zero field leaves the flow and the limit as they are; a
    field of uniform magnitude c scales every speed by 1 - tanh(c/B0), so the
    limit by its inverse; a field saturating everywhere except two adjacent
    rows j, j+1 stops every face but the phi faces of those rows and the
    theta face between them, leaving 1/(|v_theta(face j+1)|/dth + Omega/dph)
    under rigid rotation (Omega/dph the same in every row)."""
    nt, np_ = 24, 48
    dth, dph = np.pi / nt, 2 * np.pi / np_
    ms, _ = oracle.units()
    d0, m1, b0 = 14.0, 240.0, 50.0
    vph, vth = oracle.flows(nt, (d0, 0, 0, m1, 0, 0))
    plain = oracle.cfl_dt(nt, np_, vph, vth)
    assert oracle.cfl_dt_att(vph, vth, np.zeros((nt, np_)), b0) == plain
    c = 37.0
    for sign in (1.0, -1.0):
        lim = oracle.cfl_dt_att(vph, vth, np.full((nt, np_), sign * c), b0)
        assert lim == pytest.approx(plain / (1.0 - math.tanh(c / b0)), rel=1e-13)
    for ts in (oracle.FE, oracle.SSPRK33):
        assert (oracle.cfl_dt_att(vph, vth, np.full((nt, np_), c), b0, ts) ==
                pytest.approx(0.5 * plain / (1.0 - math.tanh(c / b0)), rel=1e-13))
    j = 1
    Batt = np.full((nt, np_), 1e4 * b0)
    Batt[j:j + 2] = 0.0
    want = 1.0 / (abs(vth[j + 1]) / dth + d0 * ms / dph)
    assert oracle.cfl_dt_att(vph, vth, Batt, b0) == pytest.approx(want, rel=1e-13)
    assert want > 1.5 * plain


def test_time_loop_attenuated_cfl_step_count():
    """Under rigid rotation a constant field stays constant (the flow is
    divergence-free and constants are a fixed point of diffusion), so with
    the per-step attenuated limit every step is 0.9 dph/(Omega (1 - tanh(c/B0)))
    long, and the interval takes the closed-form number of steps; the static
    (unattenuated) limit takes more, shorter steps."""
    nt, np_ = 16, 32
    dph = 2 * np.pi / np_
    ms, _ = oracle.units()
    d0, b0, c = 1807.66, 40.0, 30.0
    omega = d0 * ms
    f = 1.0 - math.tanh(c / b0)
    B0 = np.full((nt, np_), c)
    T = 40.0
    B, st = oracle.advance(B0, (d0, 0, 0, 0, 0, 0), 500.0, 0.0, T, att_b0=b0, att_cfl=1)
    step = 0.9 * dph / (omega * f)
    assert st["steps"] == math.ceil(T / step)
    assert st["dt_last"] == pytest.approx(T - (st["steps"] - 1) * step, rel=1e-9)
    assert np.allclose(B, c, rtol=1e-12)
    _, st_static = oracle.advance(B0, (d0, 0, 0, 0, 0, 0), 500.0, 0.0, T, att_b0=b0)
    assert st_static["steps"] == math.ceil(T / (0.9 * dph / omega)) > st["steps"]
    # under Strang splitting each advection advance is half a step: the limit doubles
    _, st2 = oracle.advance(B0, (d0, 0, 0, 0, 0, 0), 500.0, 0.0, T, att_b0=b0, att_cfl=1, strang=1)
    assert st2["steps"] == math.ceil(T / (2.0 * step))

def test_rigid_rotation_returns_map():
    """A full rigid rotation (Sec. "Test cases", v_phi = 1.80766 km/s sin
    theta for 672 h) through the full time loop returns the soccer-ball map
    with third-order convergence."""
    g = golden()
    errs, ns = [], [128, 256]
    for np_ in ns:
        TH, PH = grid(16, np_)
        u0 = soccer(TH, PH)
        B, st = oracle.advance(u0, (g["rigid_rotation_km_s"] * 1000.0, 0, 0, 0, 0, 0), 0.0, 0.0,
                               g["rigid_rotation_period_h"])
        errs.append(oracle.hh(B, u0))
    assert errs[-1] < 3e-3
    assert order(errs, ns)[0] > 2.7, errs


def test_meridional_divergence_converges():
    """With the LLF split read literally (one-sided face velocities, per-cell
    alpha over a six-face window), the divergence of a constant field under
    the meridional flow of eq. mf converges to the analytic
    (1/sin) d(sin v_theta)/dtheta at second order away from the pole-adjacent
    rows and the equator.  At the equator v_theta changes sign and the
    per-cell alpha has a kink, which leaves an error confined to a few rows
    whose area-weighted L1 norm still falls at first order."""
    ms, _ = oracle.units()
    m1 = 30.0
    e_max, e_l1, ns = [], [], [64, 128, 256]
    for nt in ns:
        vph, vth = oracle.flows(nt, (0, 0, 0, m1, 0, 0))
        A = oracle.adv_operator(np.ones((nt, 8)), vph, vth)
        th = (np.arange(nt) + 0.5) * np.pi / nt
        exact = m1 * ms * (np.sin(th) ** 2 - 2 * np.cos(th) ** 2)
        err = np.abs(A[:, 0] - exact) / np.abs(exact).max()
        keep = np.ones(nt, bool)
        keep[:3] = keep[-3:] = False
        keep[nt // 2 - 4:nt // 2 + 4] = False
        e_max.append(err[keep].max())
        e_l1.append((err * np.sin(th)).sum() / np.sin(th).sum())
    assert e_max[-1] < 1e-3
    assert order(e_max, ns)[-1] > 0.9, e_max
    assert order(e_l1, ns)[-1] > 0.9, e_l1


def test_strang_splitting_is_second_order():
    """Eq. num_opsplit_strang vs eq. num_opsplit_nostrang on a linear problem
    (upwind advection, diffusion) whose exact solution is the matrix
    exponential of the summed operators: with fixed steps, the plain split
    converges at first order and the Strang split at second order; with the
    CFL-limited step, the Strang step is twice as long."""
    import scipy.linalg as sl
    nt, np_ = 12, 24
    r = synth.Realization(nu_km2_s=2000.0, **synth.dr_mf(om2=-40.0, om4=-30.0, amp_mf=300.0))
    vph, vth = oracle.flows(nt, r.flow)
    nu = r.nu_km2_s * oracle.units()[1]
    n = nt * np_
    MA, MD = np.zeros((n, n)), np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        MA[:, i] = oracle.adv_operator(e.reshape(nt, np_), vph, vth, oracle.UPWIND).ravel()
        MD[:, i] = oracle.diff_operator(e.reshape(nt, np_), nu).ravel()
    B0 = np.random.default_rng(1).standard_normal((nt, np_))
    T = 4.0
    exact = (sl.expm(T * (MD - MA)) @ B0.ravel()).reshape(nt, np_)
    order = {}
    for strang in (0, 1):
        errs = []
        for N in (16, 32, 64):
            B, _ = oracle.advance(B0, r.flow, r.nu_km2_s, 0.0, T, adv_scheme=oracle.UPWIND, dt_max=T / N,
                                  strang=strang)
            errs.append(np.linalg.norm(B - exact) / np.linalg.norm(exact))
        order[strang] = np.log2(errs[-2] / errs[-1])
    assert 0.9 < order[0] < 1.2, order
    assert 1.8 < order[1] < 2.3, order
    # CFL-limited steps: the Strang step (two half advections) is twice as long
    cfl = oracle.cfl_dt(nt, np_, vph, vth, oracle.SSPRK43)
    T2 = 40.0
    _, s0 = oracle.advance(B0, r.flow, r.nu_km2_s, 0.0, T2, adv_scheme=oracle.UPWIND)
    _, s1 = oracle.advance(B0, r.flow, r.nu_km2_s, 0.0, T2, adv_scheme=oracle.UPWIND, strang=1)
    assert s0["steps"] == int(np.ceil(T2 / (0.9 * cfl) - 1e-9))
    assert s1["steps"] == int(np.ceil(T2 / (2 * 0.9 * cfl) - 1e-9))


def _att_setup(nt=24, np_=48, seed=3):
    r = synth.Realization(nu_km2_s=0.0, **synth.dr_mf(amp_mf=15.0))
    vph, vth = oracle.flows(nt, r.flow)
    g = np.random.default_rng(seed)
    return r, vph, vth, g


def test_flow_attenuation_limits_and_scaling():
    """Eq. flow_attenuation: b0 -> infinity leaves the operator unchanged; a
    field of uniform magnitude c attenuates every face by 1 - tanh(c/b0), so
    with upwind fluxes (linear in the velocity) the operator scales by it."""
    nt, np_ = 24, 48
    r, vph, vth, g = _att_setup(nt, np_)
    B = g.standard_normal((nt, np_)) * 100
    for scheme in (oracle.WENO3CSH, oracle.UPWIND):
        A0 = oracle.adv_operator(B, vph, vth, scheme)
        assert np.array_equal(oracle.adv_operator(B, vph, vth, scheme, Batt=B, b0=1e300), A0)
    S = np.sign(g.standard_normal((nt, np_))) * 300.0
    f = 1.0 - math.tanh(300.0 / 500.0)
    Au = oracle.adv_operator(S, vph, vth, oracle.UPWIND)
    Aa = oracle.adv_operator(S, vph, vth, oracle.UPWIND, Batt=S, b0=500.0)
    assert np.abs(Aa - f * Au).max() <= 1e-14 * np.abs(Au).max()


def test_flow_attenuation_face_reading():
    """Each face velocity is scaled by 1 - tanh(mean(|B| of its two cells)/b0)
    of the attenuating field (not of the advected one): with a meridional
    flow only, and an attenuating field whose magnitude is constant along
    rows, the operator equals the plain one with the theta-face velocities
    scaled row by row; with a zonal flow only and a magnitude constant along
    columns, the phi sweep equals the line flux with the phi-face velocities
    scaled column by column."""
    nt, np_, b0 = 24, 48, 400.0
    r, vph, vth, g = _att_setup(nt, np_)
    B = g.standard_normal((nt, np_)) * 100
    mag_r = g.uniform(0, 900, nt)
    Batt = mag_r[:, None] * np.sign(g.standard_normal((nt, np_)))
    ft = np.ones(nt + 1)
    ft[1:nt] = 1.0 - np.tanh(0.5 * (mag_r[:-1] + mag_r[1:]) / b0)
    zero = np.zeros(nt)
    for scheme in (oracle.WENO3CSH, oracle.UPWIND):
        got = oracle.adv_operator(B, zero, vth, scheme, Batt=Batt, b0=b0)
        ref = oracle.adv_operator(B, zero, vth * ft, scheme)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    mag_c = g.uniform(0, 900, np_)
    Batt = mag_c[None, :] * np.sign(g.standard_normal((nt, np_)))
    fp = 1.0 - np.tanh(0.5 * (np.roll(mag_c, 1) + mag_c) / b0)   # face k between cells k-1, k
    dph = 2 * math.pi / np_
    th = (np.arange(nt) + 0.5) * math.pi / nt
    got = oracle.adv_operator(B, vph, np.zeros(nt + 1), oracle.WENO3CSH, Batt=Batt, b0=b0)
    for j in (0, 5, nt // 2):
        v = np.append(vph[j] * fp, vph[j] * fp[0])
        F = oracle.line_flux(B[j], np.full(np_, dph), v, True)
        ref = (F[1:np_ + 1] - F[:np_]) / (math.sin(th[j]) * dph)
        assert np.abs(got[j] - ref).max() <= 1e-13 * np.abs(ref).max(), j


def test_flow_attenuation_conserves_and_holds_factors_over_a_step():
    """The attenuated flux divergence still conserves sum(B w); one advection
    advance takes its attenuation from the field at its start for every
    stage (SSPRK(4,3) composed from the operator with that fixed field)."""
    nt, np_, b0 = 24, 48, 250.0
    r, vph, vth, g = _att_setup(nt, np_)
    B0 = g.standard_normal((nt, np_)) * 200
    w = oracle.cell_weights(nt, np_)
    A = oracle.adv_operator(B0, vph, vth, Batt=B0, b0=b0)
    assert abs((A * w[:, None]).sum()) <= 1e-13 * (np.abs(A) * w[:, None]).sum()
    dt = 0.3
    op = lambda f: oracle.adv_operator(f, vph, vth, Batt=B0, b0=b0)
    f1 = B0 - 0.5 * dt * op(B0)
    f2 = f1 - 0.5 * dt * op(f1)
    f3 = (2.0 / 3.0) * B0 + (1.0 / 3.0) * f2 - (1.0 / 6.0) * dt * op(f2)
    ref = f3 - 0.5 * dt * op(f3)
    got, st = oracle.advance(B0, r.flow, 0.0, 0.0, dt, att_b0=b0)
    assert st["steps"] == 1
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    plain, _ = oracle.advance(B0, r.flow, 0.0, 0.0, dt)
    assert np.abs(got - plain).max() > 1e-6 * np.abs(B0).max()
