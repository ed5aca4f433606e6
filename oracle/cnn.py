"""FP64 CPU oracle of the spherical-padded CNN surrogate (numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The paper has no learned
component; this network follows the workload definition of the surrogate:
five 3x3 convolution layers (C_in -> 64 -> 64 -> 64 -> 64 -> 1), ReLU after
the first four, a residual output B_out = B_in + 5 G * y (about one
hour's typical change, so y is of order one), padding that
wraps periodically in longitude and reflects across the pole in colatitude
(the ghost row above row 0 at column k is row 0 at column k + n_phi/2, and
likewise below the last row), MSE loss on the scaled increment, and Adam with
the usual defaults.

Tensors are NCHW float64: x[b, c, j, k] with j the colatitude row and k the
longitude column.  Weights w[l] have shape (C_out, C_in, 3, 3) with tap
(dy, dx) reading the padded input at (j + dy - 1, k + dx - 1).  A matrix
product (numpy.tensordot) is the only library primitive used; each layer is a
loop over the nine taps.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (64, 64, 64, 64, 1)
OUT_SCALE = 5.0       # gauss per unit of network output
B_SCALE = 500.0       # gauss per unit of the field input channel


def pad_sphere(x: np.ndarray) -> np.ndarray:
    """Pad one cell on every side: periodic in longitude, across-pole in colatitude."""
    B, C, H, W = x.shape
    assert W % 2 == 0
    xp = np.zeros((B, C, H + 2, W + 2), dtype=x.dtype)
    xp[:, :, 1:H + 1, 1:W + 1] = x
    half = W // 2
    src = (np.arange(W) + half) % W
    xp[:, :, 0, 1:W + 1] = x[:, :, 0, src]            # across the north pole
    xp[:, :, H + 1, 1:W + 1] = x[:, :, H - 1, src]    # across the south pole
    xp[:, :, :, 0] = xp[:, :, :, W]                   # periodic longitude (incl. ghost rows)
    xp[:, :, :, W + 1] = xp[:, :, :, 1]
    return xp


def pad_sphere_adjoint(gp: np.ndarray) -> np.ndarray:
    """Adjoint of pad_sphere: fold the gradient of the padded array back."""
    B, C, Hp, Wp = gp.shape
    H, W = Hp - 2, Wp - 2
    g = gp.copy()
    g[:, :, :, W] += g[:, :, :, 0]
    g[:, :, :, 1] += g[:, :, :, W + 1]
    out = g[:, :, 1:H + 1, 1:W + 1].copy()
    half = W // 2
    src = (np.arange(W) + half) % W
    np.add.at(out, (slice(None), slice(None), 0, src), g[:, :, 0, 1:W + 1])
    np.add.at(out, (slice(None), slice(None), H - 1, src), g[:, :, H + 1, 1:W + 1])
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[b, o, j, k] = bias[o] + sum_{c, dy, dx} w[o, c, dy, dx] xp[b, c, j+dy, k+dx]."""
    B, C, H, W = x.shape
    xp = pad_sphere(x)
    out = np.zeros((B, w.shape[0], H, W))
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + H, dx:dx + W]                 # B C H W
            out += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], patch, optimize=True)
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, gout):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    B, C, H, W = x.shape
    xp = pad_sphere(x)
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + H, dx:dx + W]
            gw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", gout, patch, optimize=True)
            gxp[:, :, dy:dy + H, dx:dx + W] += np.einsum("oc,bohw->bchw", w[:, :, dy, dx], gout,
                                                         optimize=True)
    gb = gout.sum(axis=(0, 2, 3))
    return pad_sphere_adjoint(gxp), gw, gb


def init_params(c_in: int, rng: np.random.Generator, channels=CHANNELS):
    """He-normal weights, zero biases (the last layer starts at zero so the
    untrained surrogate is the identity map)."""
    params = []
    cin = c_in
    for i, cout in enumerate(channels):
        std = np.sqrt(2.0 / (9 * cin))
        w = rng.standard_normal((cout, cin, 3, 3)) * std
        if i == len(channels) - 1:
            w = w * 0.0
        params.append([w, np.zeros(cout)])
        cin = cout
    return params


def forward(params, x, keep=False):
    """Network output y (B, 1, H, W); with keep=True also the layer inputs."""
    acts = [x]
    h = x
    for i, (w, b) in enumerate(params):
        h = conv3x3(h, w, b)
        if i < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return (h, acts) if keep else h


def loss_and_grads(params, x, target):
    """MSE loss mean((y - target)^2) and gradients for every (w, b)."""
    y, acts = forward(params, x, keep=True)
    n = y.size
    loss = float(np.mean((y - target) ** 2))
    g = 2.0 * (y - target) / n
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        w, b = params[i]
        if i < len(params) - 1:
            g = g * (acts[i + 1] > 0.0)
        gx, gw, gb = conv3x3_backward(acts[i], w, g)
        grads[i] = [gw, gb]
        g = gx
    return loss, grads


class Adam:
    """Adam (lr, beta1 = 0.9, beta2 = 0.999, eps = 1e-8) with bias correction."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros_like(p) for p in layer] for layer in params]
        self.v = [[np.zeros_like(p) for p in layer] for layer in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for li, layer in enumerate(params):
            for pi, p in enumerate(layer):
                g = grads[li][pi]
                m = self.m[li][pi] = self.b1 * self.m[li][pi] + (1.0 - self.b1) * g
                v = self.v[li][pi] = self.b2 * self.v[li][pi] + (1.0 - self.b2) * g * g
                p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def features(B, nt, feats):
    """Network input (B, 6, H, W): field/500, three per-sample parameter
    features broadcast over the grid, cos(theta), sin(theta)."""
    B = np.asarray(B, dtype=np.float64)
    nb = B.shape[0]
    th = (np.arange(nt) + 0.5) * np.pi / nt
    x = np.zeros((nb, 6) + B.shape[1:])
    x[:, 0] = B / B_SCALE
    for c in range(3):
        x[:, 1 + c] = np.asarray(feats, dtype=np.float64)[:, c][:, None, None]
    x[:, 4] = np.cos(th)[None, :, None]
    x[:, 5] = np.sin(th)[None, :, None]
    return x


def split_bf16(f: np.ndarray):
    """A float32 value as a pair of bfloat16 values: hi = bf16(f),
    lo = bf16(f - hi) (exact difference), so hi + lo carries 16 significant bits."""
    f32 = np.asarray(f, dtype=np.float32).astype(np.float64)
    hi = bf16_round(f32)
    return hi, bf16_round(f32 - hi)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
