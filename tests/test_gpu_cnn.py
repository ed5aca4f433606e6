"""CNN surrogate kernels (BF16 MFMA, FP32 accumulate) vs the FP64 oracle.

Each layer is checked on identical operands: the oracle is fed the GPU's own
bf16 activations of the previous layer and the bf16-rounded weights, so only
the FP32 accumulation order differs before the final bf16 rounding (at most
one bf16 ulp, on a small fraction of elements).  Gradients are checked with
the oracle emulating the same bf16 storage points.  The surrogate advance is
checked for its fallback (tolerance 0 gives the plain solver's field bit for
bit) and its accept path.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import random_field, rel_l2, say
from oracle import cnn

pytestmark = pytest.mark.gpu


def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def bf16_to_f64(t):
    """bf16 bits in an int16 tensor -> float64 numpy array."""
    a = t.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32).astype(np.float64)


def random_params(rng, scale_last=0.3):
    params = cnn.init_params(6, rng)
    params[-1][0] = rng.standard_normal(params[-1][0].shape) * scale_last / 24.0
    for layer in params:
        layer[1] = rng.standard_normal(layer[1].shape) * 0.05
    return params


def flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def unflat(vec, like):
    out, o = [], 0
    for w, b in like:
        nw, nb = w.size, b.size
        out.append([vec[o:o + nw].reshape(w.shape).astype(np.float64),
                    vec[o + nw:o + nw + nb].astype(np.float64)])
        o += nw + nb
    return out


def nchw(a, c=None):
    x = np.transpose(a, (0, 3, 1, 2))
    return x[:, :c] if c else x


def close_bf16(gpu, ref, atol=1e-30):
    """At most one bf16 ulp apart (or atol), and identical almost everywhere."""
    diff = np.abs(gpu - ref)
    tol = 2.0 ** -7 * np.maximum(np.abs(gpu), np.abs(ref)) + atol
    frac = float(np.mean((gpu != ref) & (diff > atol)))
    return bool(np.all(diff <= tol)), frac


def x6_from_x0(x0):
    """The 6-channel network input seen by the first layer: the field as
    hi + lo (its two bf16 slots share one weight), then the five others."""
    return np.concatenate([x0[:, 0:1] + x0[:, 1:2], x0[:, 2:7]], axis=1)


def setup_net(H, W, batch, seed):
    torch = torch_cuda()
    import paper_2501_06377_amd as sft
    rng = np.random.default_rng(seed)
    params = random_params(rng)
    # round the master weights to float32 as the library stores them
    params = unflat(flat(params), params)
    net = sft.Net(H, W, batch)
    net.set_params(flat(params))
    B = torch.tensor(rng.standard_normal((batch, H, W)) * 200.0, dtype=torch.float64, device="cuda")
    feats = torch.tensor(rng.uniform(0.2, 1.2, (batch, 3)), dtype=torch.float32, device="cuda")
    return torch, net, params, B, feats


def get_acts(torch, net, batch, H, W):
    acts = []
    for layer in range(5):
        c = 16 if layer == 0 else 64
        t = torch.empty((batch, H, W, c), dtype=torch.int16, device="cuda")
        net.activation(layer, t)
        acts.append(nchw(bf16_to_f64(t)))
    return acts


@pytest.mark.parametrize("H,W,batch,cap", [(20, 40, 2, 0), (13, 64, 2, 0), (20, 40, 2, 4), (48, 96, 3, 7)])
def test_cnn_forward_layers_match_oracle(H, W, batch, cap):
    """Each layer against the oracle.  With a grid limit (cap > 0) every
    persistent block walks several tiles (the last round ragged), so the
    loads of the next tiles issued during a tile's matrix products are
    checked as well; the output does not depend on the grid."""
    say(f"case cnn forward {H}x{W} batch {batch} grid limit {cap}")
    torch, net, params, B, feats = setup_net(H, W, batch, 11)
    y = torch.empty((batch, H, W), dtype=torch.float32, device="cuda")
    if cap:
        y0 = torch.empty_like(y)
        net.forward(B, feats, y0)
        net.set_grid_limit(cap)
    net.forward(B, feats, y)
    torch.cuda.synchronize()
    if cap:
        assert torch.equal(y, y0)
    acts = get_acts(torch, net, batch, H, W)
    ref6 = cnn.features(B.cpu().numpy(), H, feats.cpu().numpy().astype(np.float64))
    hi, lo = cnn.split_bf16(ref6[:, 0])
    assert np.array_equal(acts[0][:, 0], hi) and np.array_equal(acts[0][:, 1], lo)
    # cos(theta) of an equator row is ~1e-17 on either side: compare it absolutely
    ok, frac = close_bf16(acts[0][:, 2:7], cnn.bf16_round(ref6[:, 1:]), atol=1e-12)
    say(f"  input features: within 1 ulp {ok}, differing {frac:.2e}")
    assert ok and frac < 1e-3 and np.all(acts[0][:, 7:] == 0)
    for l in range(1, 5):
        w, b = params[l - 1]
        xin = x6_from_x0(acts[0]) if l == 1 else acts[l - 1]
        ref = cnn.bf16_round(np.maximum(cnn.conv3x3(xin, cnn.bf16_round(w), b), 0.0))
        # outputs near zero come from cancelling sums: FP32 accumulation error
        # is relative to the layer's scale there, not to the tiny result
        ok, frac = close_bf16(acts[l], ref, atol=1e-5 * np.abs(ref).max())
        say(f"  layer {l}: within 1 ulp {ok}, differing {frac:.2e}")
        assert ok and frac < 2e-2, l
    w5, b5 = params[4]
    yref = cnn.conv3x3(acts[4], cnn.bf16_round(w5), b5)[:, 0]
    e = float(np.abs(y.cpu().numpy() - yref).max() / np.abs(yref).max())
    say(f"  output layer: max rel {e:.2e}")
    assert e < 1e-5


@pytest.mark.parametrize("H,W,batch,cap", [(20, 40, 2, 0), (13, 64, 3, 0), (48, 96, 5, 0), (48, 96, 5, 3),
                                           (20, 40, 2, 5)])
def test_predict_is_forward_bitwise(H, W, batch, cap):
    """The inference path (input channels formed while the first layer stages
    its tiles; the last hidden layer and the output layer's tap products in
    one pass) gives the forward pass's output bit for bit, over partial and
    several tiles, from FP64 and FP32 fields; afterwards the input and layer-4
    activations are reported unavailable until the next forward pass, and a
    smaller batch on the same network matches too."""
    import paper_2501_06377_amd as sft
    say(f"case cnn predict {H}x{W} batch {batch} grid limit {cap}")
    torch, net, params, B, feats = setup_net(H, W, batch, 21)
    y1 = torch.empty((batch, H, W), dtype=torch.float32, device="cuda")
    y2 = torch.full((batch, H, W), float("nan"), dtype=torch.float32, device="cuda")
    net.forward(B, feats, y1)      # on the default grid
    net.set_grid_limit(cap)
    net.predict(B, feats, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    t = torch.empty((batch, H, W, 64), dtype=torch.int16, device="cuda")
    for layer in (0, 4):
        with pytest.raises(sft.SftError) as ex:
            net.activation(layer, t)
        assert ex.value.status == sft.SFT_ERR_STATE
    net.activation(3, t)                      # the hidden layers before the last are held
    net.forward(B, feats, y1)
    net.activation(4, t)
    net.predict(B[:1], feats[:1], y2[:1])
    net.forward(B[:1], feats[:1], y1[:1])
    torch.cuda.synchronize()
    assert torch.equal(y1[:1], y2[:1])
    B32 = B.float()
    net.forward(B32, feats, y1)
    net.predict(B32, feats, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    net.close()


@pytest.mark.parametrize("H,W,batch,cap", [(16, 32, 2, 0), (32, 128, 3, 2), (40, 192, 2, 5)])
def test_cnn_gradients_match_oracle(H, W, batch, cap):
    """Weight and bias gradients of every layer against the oracle's
    backward pass.  With a grid limit each weight-gradient block accumulates
    several work items (16-row strips of a 64-pixel column segment) and each
    data-gradient block several tiles."""
    say(f"case cnn gradients {H}x{W} batch {batch} grid limit {cap}")
    torch, net, params, B, feats = setup_net(H, W, batch, 12)
    rng = np.random.default_rng(13)
    Bt = B + torch.tensor(rng.standard_normal((batch, H, W)) * 3.0, dtype=torch.float64, device="cuda")
    net.set_grid_limit(cap)
    loss = net.train_step(B, Bt, feats, lr=0.0, apply=False)
    g = unflat(net.get_grads(), params)
    acts = get_acts(torch, net, batch, H, W)
    w5, b5 = params[4]
    y = cnn.conv3x3(acts[4], cnn.bf16_round(w5), b5)
    t = ((Bt - B).cpu().numpy() / cnn.OUT_SCALE)[:, None]
    n = y.size
    loss_ref = float(np.mean((y - t) ** 2))
    assert loss == pytest.approx(loss_ref, rel=1e-4)
    # the output gradient is stored as bf16 for the matrix cores
    gy = cnn.bf16_round(2.0 * (y - t) / n)
    ref = [None] * 5
    gx, gw, gb = cnn.conv3x3_backward(acts[4], cnn.bf16_round(w5), gy)
    ref[4] = (gw, gb)
    dz = cnn.bf16_round(gx * (acts[4] > 0))
    for l in range(4, 0, -1):
        w, _ = params[l - 1]
        xin = x6_from_x0(acts[0]) if l == 1 else acts[l - 1]
        gx, gw, gb = cnn.conv3x3_backward(xin, cnn.bf16_round(w), dz)
        ref[l - 1] = (gw, gb)
        if l > 1:
            dz = cnn.bf16_round(gx * (acts[l - 1] > 0))
    for l in range(5):
        ew = rel_l2(g[l][0], ref[l][0])
        eb = rel_l2(g[l][1], ref[l][1])
        say(f"  layer {l + 1}: weight-grad rel-L2 {ew:.2e}, bias-grad rel-L2 {eb:.2e}")
        assert ew < 3e-3 and eb < 3e-3, l


def test_training_reduces_loss():
    torch = torch_cuda()
    import paper_2501_06377_amd as sft
    H, W, batch = 16, 32, 4
    say("case cnn training smoke")
    rng = np.random.default_rng(14)
    params = cnn.init_params(6, rng)
    net = sft.Net(H, W, batch)
    net.set_params(flat(params))
    # targets: a fixed smooth map of the input, so a small net can learn it
    B = torch.tensor(rng.standard_normal((batch, H, W)) * 100.0, dtype=torch.float32, device="cuda")
    Bt = B + 0.05 * torch.roll(B, 1, dims=2)
    feats = torch.full((batch, 3), 0.5, dtype=torch.float32, device="cuda")
    losses = [net.train_step(B, Bt, feats, lr=1e-3) for _ in range(60)]
    say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.2 * losses[0]


def test_surrogate_fallback_is_plain_bitwise_and_accept_path():
    torch = torch_cuda()
    import paper_2501_06377_amd as sft
    from gpu_helpers import random_field
    nt, np_ = 32, 64
    say("case surrogate fallback / accept")
    reals = [synth.Realization(nu_km2_s=500.0, **synth.dr_mf(amp_mf=15.0)),
             synth.Realization(nu_km2_s=800.0, **synth.dr_mf(amp_mf=20.0))]
    B0 = np.stack([random_field(nt, np_, 6, 80 + i) for i in range(2)])
    feats = np.array([[0.5, 1.0, 0.75], [0.8, 1.0, 1.0]], np.float32)
    rng = np.random.default_rng(15)
    params = random_params(rng, scale_last=0.01)
    net = sft.Net(nt, np_, 2)
    net.set_params(flat(params))

    plain = sft.Ensemble()
    g = plain.add_grid(nt, np_, reals)
    plain.set_states(g, B0)
    plain.advance(1.0)
    ref = plain.get_states(g)

    ens = sft.Ensemble()
    g = ens.add_grid(nt, np_, reals)
    ens.set_states(g, B0)
    err = sft.surrogate_advance(ens, g, net, feats, 1.0, 0.0)
    got = ens.get_states(g)
    assert np.array_equal(got, ref)
    assert ens.diagnostics(0)["surr_reject"] == 1 and ens.time() == 1.0
    say(f"  rejected at tol 0, distances {err}")

    # accept path: the state becomes B + 5 G y of the network
    y = torch.empty((2, nt, np_), dtype=torch.float32, device="cuda")
    net.forward(torch.tensor(B0, device="cuda"), torch.tensor(feats, device="cuda"), y)
    pred = B0 + cnn.OUT_SCALE * y.cpu().numpy().astype(np.float64)
    ens2 = sft.Ensemble()
    g = ens2.add_grid(nt, np_, reals)
    ens2.set_states(g, B0)
    err2 = sft.surrogate_advance(ens2, g, net, feats, 1.0, 1e30)
    assert np.array_equal(ens2.get_states(g), pred)
    assert np.allclose(err2, [rel_l2(pred[r], ref[r]) for r in range(2)], rtol=1e-10)
    assert ens2.diagnostics(1)["surr_accept"] == 1


def test_trained_surrogate_gain():
    """The shipped trained network on held-out realizations of its training
    distribution (512 x 1024, no assimilation): its one-hour prediction is
    checked against the plain solver every interval.  It must beat the
    method without it (the identity map, i.e. no transport) by a clear
    factor, every accepted interval must be within the tolerance, and every
    rejected one must leave the plain solver's field."""
    import os
    import paper_2501_06377_amd as sft
    from paper_2501_06377_amd import surrogate as S
    nt, np_ = 512, 1024
    path = S.weights_path(nt, np_)
    assert os.path.exists(path), "trained weights are shipped with the package"
    params = np.load(path).astype(np.float32)
    n, hours, tol = 4, 3, 1e-3
    reals, feats = S.sample_realizations(n, 7)
    f0 = S.initial_fields(nt, np_, n, 7)
    say(f"case trained surrogate gain: {n} held-out realizations x {hours} h")
    net = sft.Net(nt, np_, n)
    net.set_params(params)
    ens = sft.Ensemble()
    g = ens.add_grid(nt, np_, reals)
    ens.set_states(g, f0)
    plain = sft.Ensemble()
    gp = plain.add_grid(nt, np_, reals)
    plain.set_states(gp, f0)
    prev = f0
    errs, ident = [], []
    for h in range(1, hours + 1):
        # both start the interval from the same state
        plain.set_states(gp, prev)
        plain.set_time(h - 1.0)
        plain.advance(float(h))
        ref = plain.get_states(gp)
        e = sft.surrogate_advance(ens, g, net, feats, float(h), tol)
        got = ens.get_states(g)
        for r in range(n):
            if e[r] <= tol:
                assert rel_l2(got[r], ref[r]) <= tol
            else:
                assert np.array_equal(got[r], ref[r])
            ident.append(rel_l2(prev[r], ref[r]))
        errs += e.tolist()
        prev = got
    errs, ident = np.array(errs), np.array(ident)
    acc = float(np.mean(errs <= tol))
    gain = float(np.median(ident) / np.median(errs))
    say(f"  surrogate rel-L2 median {np.median(errs):.3e} (max {errs.max():.3e}), identity median "
        f"{np.median(ident):.3e}, gain {gain:.1f}x, accepted {acc:.0%} at {tol}")
    assert gain > 5.0 and acc >= 0.5


def test_surrogate_strided_checks_and_escalation():
    """Throughput mode (check = K = 3): a realization is checked on its 1st,
    4th, 7th... surrogate interval and takes the surrogate field unverified
    in between; a rejection switches it to a check every interval until one
    passes.  Realizations 0 and 1 pass every check (tol 1e30): their fields
    equal the unchecked surrogate's bit for bit and the plain solver ran only
    on their checked intervals.  Realization 2 holds a zero field, which the
    plain solver keeps exactly and the network does not (relative distance
    inf): it is rejected every interval, stays escalated and stays zero."""
    import paper_2501_06377_amd as sft
    nt, np_ = 24, 48
    say("case surrogate strided checks K = 3, 7 intervals, one realization always rejected")
    reals = [synth.Realization(nu_km2_s=(500.0, 800.0, 300.0)[i], **synth.dr_mf(amp_mf=15.0 + 5 * i))
             for i in range(3)]
    B0 = np.stack([random_field(nt, np_, 6, 90 + i) for i in range(2)] + [np.zeros((nt, np_))])
    feats = np.array([[0.5, 1.0, 0.75], [0.8, 1.0, 1.0], [0.3, 1.0, 1.0]], np.float32)
    params = random_params(np.random.default_rng(16), scale_last=0.01)
    net = sft.Net(nt, np_, 3)
    net.set_params(flat(params))

    def run(check, hours=7):
        e = sft.Ensemble()
        g = e.add_grid(nt, np_, reals)
        e.set_states(g, B0)
        errs = [sft.surrogate_advance(e, g, net, feats, float(h), 1e30, check) for h in range(1, hours + 1)]
        return e, g, np.array(errs)

    ens, g, errs = run(3)
    free, gf, _ = run(0)
    got, ref = ens.get_states(g), free.get_states(gf)
    assert np.array_equal(got[:2], ref[:2])
    assert np.array_equal(got[2], np.zeros((nt, np_))) and np.abs(ref[2]).max() > 0
    checked = [0, 3, 6]
    for h in range(7):
        for r in range(2):
            assert (errs[h, r] >= 0) == (h in checked), (h, r, errs[h])
        assert errs[h, 2] == np.inf
    c = [sft.surrogate_counts(ens, r) for r in range(3)]
    say(f"  counters {c}")
    for r in range(2):
        assert c[r] == {"accepted": 3, "rejected": 0, "unchecked": 4, "escalated": 0}
    assert c[2] == {"accepted": 0, "rejected": 7, "unchecked": 0, "escalated": 1}
    # the plain solver advanced realization r only on its checked intervals
    one = sft.Ensemble()
    g1 = one.add_grid(nt, np_, reals)
    one.set_states(g1, B0)
    one.advance(1.0)
    per_hour = [one.counts(r)["steps"] for r in range(3)]
    assert [ens.counts(r)["steps"] for r in range(3)] == [3 * per_hour[0], 3 * per_hour[1], 7 * per_hour[2]]
    # a check that passes clears the escalation: realization 2 from a nonzero field
    ens.set_states(g, np.stack([got[0], got[1], B0[0]]))
    e8 = sft.surrogate_advance(ens, g, net, feats, 8.0, 1e30, 3)
    assert 0 <= e8[2] < np.inf and sft.surrogate_counts(ens, 2)["escalated"] == 0
    assert e8[0] == -1.0 and e8[1] == -1.0   # their 8th interval is not a checked one
    # one surrogate evaluation stands in for one hour, no other length
    with pytest.raises(sft.SftError):
        sft.surrogate_advance(ens, g, net, feats, 10.0, 1e30, 1)
    assert ens.time() == 8.0
    with pytest.raises(sft.SftError):
        sft.surrogate_advance(ens, g, net, feats, 9.0, 1e30, -1)
