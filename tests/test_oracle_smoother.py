"""Pins of the oracle's flux-preserving smoother: the diffusion operator of
eq. diffusion_matrix with a colatitude-dependent diffusivity at the cell
corners, and the grid diffusivity of eq. diffgrid (Sec. "Surface
diffusion", Sec. "Flux-preserving smoothing tool")."""
import math

import numpy as np

import oracle
import synth


def dense(nt, np_, nu_face):
    n = nt * np_
    M = np.empty((n, n))
    E = np.zeros(n)
    for i in range(n):
        E[i] = 1.0
        M[:, i] = oracle.diff_operator_face(E.reshape(nt, np_), nu_face).ravel()
        E[i] = 0.0
    return M


def test_constant_corner_diffusivity_is_the_scalar_operator():
    nt, np_ = 20, 40
    B = np.random.default_rng(1).standard_normal((nt, np_))
    nu = 0.0123
    assert np.array_equal(oracle.diff_operator_face(B, np.full(nt + 1, nu)), oracle.diff_operator(B, nu))


def test_variable_operator_conserves_and_is_self_adjoint():
    """With nu varying in colatitude the operator still conserves sum(B w),
    is self-adjoint in the w-weighted inner product and negative
    semidefinite with the constants as its null space."""
    nt, np_ = 10, 20
    nf = oracle.nu_grid(nt, np_, 0.5)
    assert np.ptp(nf) >= 0.49 * nf.max()           # really variable (pole: half the equator)
    M = dense(nt, np_, nf)
    w = np.repeat(oracle.cell_weights(nt, np_), np_)
    WM = w[:, None] * M
    assert np.abs(WM - WM.T).max() <= 1e-13 * np.abs(WM).max()
    assert np.abs(w @ M).max() <= 1e-13 * np.abs(WM).max()
    sw = np.sqrt(w)
    ev = np.linalg.eigvalsh((sw[:, None] * M) / sw[None, :])
    assert ev.max() <= 1e-12 * np.abs(ev).max()
    assert np.sum(np.abs(ev) <= 1e-10 * np.abs(ev).max()) == 1


def _analytic(nt, np_, a, b):
    """(1/sin) d/dth (nu sin dB/dth) + nu/sin^2 d2B/dph2 for nu = a + b sin^2(theta)
    and B = cos(theta) + sin^2(theta) cos(2 phi), at the cell centres."""
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(np_) + 0.5) * 2 * math.pi / np_
    T, P = np.meshgrid(th, ph, indexing="ij")
    s, c = np.sin(T), np.cos(T)
    nu = a + b * s * s
    dnu = 2 * b * s * c
    B = c + s * s * np.cos(2 * P)
    L1 = -dnu * s - 2 * nu * c
    L2 = 2 * np.cos(2 * P) * (dnu * s * c + nu * (2 * c * c - s * s) - 2 * nu)
    return B, L1 + L2


def test_variable_operator_is_second_order():
    a, b = 0.02, 0.05
    errs = []
    for nt in (24, 48, 96):
        np_ = 2 * nt
        B, L = _analytic(nt, np_, a, b)
        f = np.arange(nt + 1) * math.pi / nt
        nf = a + b * np.sin(f) ** 2
        got = oracle.diff_operator_face(B, nf)
        w = oracle.cell_weights(nt, np_)[:, None]
        errs.append(math.sqrt(((got - L) ** 2 * w).sum() / (L ** 2 * w).sum()))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.8, (errs, orders)


def test_grid_diffusivity_spreads_at_its_scale():
    """A unit spike at the equator spreads with variance 2 nu_g t in theta
    and in phi (times sin^2 = 1 there), nu_g = alpha (dth^2 + dph^2) at the
    equator (eq. diffgrid)."""
    nt, np_, alpha, t = 64, 128, 0.5, 4.0
    dth, dph = math.pi / nt, 2 * math.pi / np_
    B = np.zeros((nt, np_))
    j0, k0 = nt // 2, np_ // 2                   # cell centre just south of the equator
    B[j0, k0] = 1.0
    out, _ = oracle.diffuse_face(B, oracle.nu_grid(nt, np_, alpha), t, scheme=oracle.RKG2, ptl_dt=0.25)
    w = oracle.cell_weights(nt, np_)[:, None]
    m = out * w
    th = (np.arange(nt) + 0.5) * dth
    ph = (np.arange(np_) + 0.5) * dph
    var_th = (m.sum(1) * (th - th[j0]) ** 2).sum() / m.sum()
    var_ph = (m.sum(0) * (ph - ph[k0]) ** 2).sum() / m.sum()
    nu_eq = alpha * (dth * dth + dph * dph)
    assert abs(var_th / (2 * nu_eq * t) - 1) < 0.05
    assert abs(var_ph / (2 * nu_eq * t) - 1) < 0.05
    # the scalar diffusivity of the same equatorial value spreads alike
    ref, _ = oracle.diffuse(B, nu_eq, t, ptl_dt=0.25)
    assert abs((ref * w).sum(1) @ (th - th[j0]) ** 2 / (ref * w).sum() / var_th - 1) < 0.05


def test_smoother_preserves_flux_and_smooths():
    nt, np_ = 64, 128
    B0 = synth.bipolar_field(nt, np_, synth.bipolar_pairs(20, 5))
    w = oracle.cell_weights(nt, np_)[:, None]
    B, st = oracle.advance(B0, (0, 0, 0, 0, 0, 0), 0.0, 0.0, 2.0, nu_grid_alpha=0.5)
    assert st["stages"] > 0
    assert abs(((B - B0) * w).sum()) <= 1e-13 * (np.abs(B0) * w).sum()
    assert (np.abs(B) * w).sum() < (np.abs(B0) * w).sum()
    assert np.abs(B).max() < 0.9 * np.abs(B0).max()
    # the same as one diffusion advance with the grid diffusivity
    D, _ = oracle.diffuse_face(B0, oracle.nu_grid(nt, np_, 0.5), 2.0)
    assert np.array_equal(B, D)
