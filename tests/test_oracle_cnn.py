"""Pins of the FP64 CNN oracle (oracle/cnn.py): padding by index arithmetic,
delta-kernel shifts, the dense-operator adjoint identity, central finite
differences for every gradient, Adam's first step in closed form, and the
bfloat16 rounding against torch's conversion."""
import numpy as np
import pytest

from oracle import cnn


def test_pad_sphere_by_index():
    rng = np.random.default_rng(0)
    H, W = 5, 8
    x = rng.standard_normal((1, 2, H, W))
    xp = cnn.pad_sphere(x)
    for j in range(-1, H + 1):
        for k in range(-1, W + 1):
            kk = k % W
            if j == -1:
                want = x[0, :, 0, (kk + W // 2) % W]
            elif j == H:
                want = x[0, :, H - 1, (kk + W // 2) % W]
            else:
                want = x[0, :, j, kk]
            assert np.array_equal(xp[0, :, j + 1, k + 1], want), (j, k)


@pytest.mark.parametrize("dy,dx", [(0, 0), (0, 2), (2, 1), (1, 1), (2, 2)])
def test_delta_kernel_is_a_shift(dy, dx):
    """A kernel with a single 1 at tap (dy, dx) shifts the input by
    (dy-1, dx-1) with periodic longitude and across-pole rows."""
    rng = np.random.default_rng(1)
    H, W = 6, 10
    x = rng.standard_normal((2, 1, H, W))
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, dy, dx] = 1.0
    y = cnn.conv3x3(x, w, np.zeros(1))
    for j in range(H):
        for k in range(W):
            sj, sk = j + dy - 1, (k + dx - 1) % W
            if sj < 0:
                sj, sk = 0, (sk + W // 2) % W
            elif sj >= H:
                sj, sk = H - 1, (sk + W // 2) % W
            assert y[0, 0, j, k] == x[0, 0, sj, sk] and y[1, 0, j, k] == x[1, 0, sj, sk]


def test_conv_adjoint_identity():
    """<conv(x), g> = <x, conv_backward_input(g)> for the bias-free conv."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 4, 6))
    w = rng.standard_normal((5, 3, 3, 3))
    g = rng.standard_normal((2, 5, 4, 6))
    y = cnn.conv3x3(x, w, np.zeros(5))
    gx, _, _ = cnn.conv3x3_backward(x, w, g)
    assert np.vdot(y, g) == pytest.approx(np.vdot(x, gx), rel=1e-12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(3)
    params = cnn.init_params(3, rng, channels=(4, 4, 1))
    params[-1][0] = rng.standard_normal(params[-1][0].shape) * 0.3   # non-zero last layer
    for layer in params:
        layer[1] = rng.standard_normal(layer[1].shape) * 0.1
    x = rng.standard_normal((2, 3, 4, 6))
    t = rng.standard_normal((2, 1, 4, 6))
    loss, grads = cnn.loss_and_grads(params, x, t)
    h = 1e-6
    worst = 0.0
    for li, layer in enumerate(params):
        for pi, p in enumerate(layer):
            flat = p.reshape(-1)
            idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
            for i in idx:
                old = flat[i]
                flat[i] = old + h
                lp, _ = cnn.loss_and_grads(params, x, t)
                flat[i] = old - h
                lm, _ = cnn.loss_and_grads(params, x, t)
                flat[i] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][pi].reshape(-1)[i]
                worst = max(worst, abs(fd - an) / max(abs(fd), abs(an), 1e-8))
    assert worst < 1e-6, worst


def test_adam_first_step_closed_form():
    """After one step with bias correction, each parameter moves by
    -lr g / (|g| + eps)."""
    p = [[np.array([1.0, -2.0, 0.5]), np.array([0.0])]]
    g = [[np.array([0.3, -4.0, 1e-3]), np.array([2.0])]]
    opt = cnn.Adam(p, lr=0.01)
    before = p[0][0].copy()
    opt.step(p, g)
    want = before - 0.01 * g[0][0] / (np.abs(g[0][0]) + 1e-8)
    assert np.allclose(p[0][0], want, rtol=1e-12)


def test_untrained_net_is_identity_and_features():
    rng = np.random.default_rng(4)
    params = cnn.init_params(6, rng)
    nt, np_ = 4, 8
    Bf = rng.standard_normal((2, nt, np_)) * 100
    x = cnn.features(Bf, nt, np.array([[0.5, 1.0, 0.75], [1.0, 0.9, 0.5]]))
    assert x.shape == (2, 6, nt, np_)
    assert np.allclose(x[:, 0], Bf / 500.0) and np.all(x[1, 2] == 0.9)
    th = (np.arange(nt) + 0.5) * np.pi / nt
    assert np.allclose(x[0, 4, :, 3], np.cos(th))
    assert np.all(cnn.forward(params, x) == 0.0)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    a = rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000)
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), ref)
