"""Training data, training and evaluation of the CNN surrogate of one 1-hour
transport interval.

Everything numerical runs in the HIP library through its C ABI: the plain
solver generates the trajectories (advection + RKG2 diffusion, no
assimilation), ``sft_net_train_step`` trains, ``sft_surrogate_advance`` infers
and judges each interval against the plain solver.  torch only holds device
memory (trajectory snapshots, batches).

Data: n_traj realizations with diffusivity U(250, 1000) km^2/s, meridional
amplitude U(10, 20) m/s and differential-rotation shear factor U(0.8, 1.2),
each starting from its own seeded bipolar field, stepped hourly; the network
features are (eta/1000, shear factor, amplitude/20).

Command line (on a GPU):
    python -m paper_2501_06377_amd.surrogate train --out W.npy [--traj 40 --hours 500 ...]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import Ensemble, Net, surrogate_advance  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
FLOP_PER_PIXEL = 2 * 9 * (6 * 64 + 3 * 64 * 64 + 64)   # multiply-adds of the five layers, x2


def sample_realizations(n: int, sub: int):
    g = synth.rng("surrogate_data", sub)
    eta = g.uniform(250.0, 1000.0, n)
    amp = g.uniform(10.0, 20.0, n)
    fdr = g.uniform(0.8, 1.2, n)
    reals = [synth.Realization(nu_km2_s=float(e), **synth.dr_mf(om2=-2.4 * f, om4=-1.8 * f, amp_mf=float(a)))
             for e, a, f in zip(eta, amp, fdr)]
    feats = np.stack([eta / 1000.0, fdr, amp / 20.0], 1).astype(np.float32)
    return reals, feats


def initial_fields(nt, np_, n, sub, n_pairs=200):
    def one(i):
        return synth.bipolar_field(nt, np_, synth.bipolar_pairs(n_pairs, 100000 + 1000 * sub + i))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return np.stack(list(ex.map(one, range(n))))


def generate(nt, np_, n_traj, hours, sub=0, n_pairs=200, log=print):
    """Hourly snapshots [n_traj][hours+1][nt][np] (FP32, device) and features."""
    import torch
    reals, feats = sample_realizations(n_traj, sub)
    f0 = initial_fields(nt, np_, n_traj, sub, n_pairs)
    ens = Ensemble()
    gid = ens.add_grid(nt, np_, reals)
    cur = torch.tensor(f0, dtype=torch.float64, device="cuda")
    snaps = torch.empty((n_traj, hours + 1, nt, np_), dtype=torch.float32, device="cuda")
    ens.set_states(gid, cur)
    snaps[:, 0] = cur.float()
    t0 = time.perf_counter()
    for h in range(1, hours + 1):
        ens.advance(float(h))
        ens.get_states(gid, cur)
        ens.sync()
        snaps[:, h] = cur.float()
    torch.cuda.synchronize()
    log(f"generated {n_traj} x {hours} intervals at {nt}x{np_} in {time.perf_counter() - t0:.1f} s")
    ens.close()
    return snaps, feats, reals


def train(net, snaps, feats, epochs=2, batch=16, lr=1e-3, lr_min=1e-5, log=print, log_every=200,
          seconds=0.0, save=None, save_every=120.0):
    """Adam with a cosine learning-rate schedule over shuffled (trajectory,
    hour) pairs.  With seconds > 0 the number of steps is set from the
    measured step time so that training ends after about that long (epochs
    is then ignored); save(params) is called every save_every seconds."""
    import torch
    n_traj, hp1 = snaps.shape[0], snaps.shape[1]
    pairs = np.array([(t, h) for t in range(n_traj) for h in range(hp1 - 1)], dtype=np.int64)
    fdev = torch.tensor(feats, device="cuda")
    order_rng = synth.rng("shuffle", 0)
    steps_per_epoch = len(pairs) // batch
    total = epochs * steps_per_epoch
    step = 0
    t0 = time.perf_counter()
    last_save = t0
    hist = []
    order = order_rng.permutation(len(pairs))
    i = 0
    while step < total:
        if i == steps_per_epoch:
            order = order_rng.permutation(len(pairs))
            i = 0
        sel = pairs[order[i * batch:(i + 1) * batch]]
        i += 1
        ti = torch.tensor(sel[:, 0], device="cuda")
        hi = torch.tensor(sel[:, 1], device="cuda")
        b_in = snaps[ti, hi].contiguous()
        b_out = snaps[ti, hi + 1].contiguous()
        f = fdev[ti].contiguous()
        cur_lr = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(total, 1)))
        want = (step % log_every == 0) or step == total - 1
        loss = net.train_step(b_in, b_out, f, cur_lr, want_loss=want)
        if seconds > 0 and step == 20:
            torch.cuda.synchronize()
            per = (time.perf_counter() - t0) / 21
            total = max(int(seconds / per), 21)
            log(f"step time {per * 1e3:.1f} ms -> {total} steps ({total * batch / len(pairs):.2f} epochs)")
        if want:
            el = time.perf_counter() - t0
            log(f"step {step}/{total} loss {loss:.4e} lr {cur_lr:.2e} ({el:.1f} s)")
            hist.append((step, loss))
        if save and time.perf_counter() - last_save > save_every:
            save(net.get_params())
            last_save = time.perf_counter()
        step += 1
    torch.cuda.synchronize()
    return {"steps": total, "seconds": time.perf_counter() - t0, "loss_history": hist,
            "epochs": total * batch / len(pairs)}


def evaluate(net_params, nt, np_, n_real, hours, sub, tol=1e-3, log=print):
    """Held-out realizations stepped with the surrogate (checked against the
    plain solver every interval, falling back when above tol).  Returns error
    statistics, the identity baseline and the acceptance rate."""
    import torch
    reals, feats = sample_realizations(n_real, sub)
    f0 = initial_fields(nt, np_, n_real, sub)
    net = Net(nt, np_, n_real)
    net.set_params(net_params)
    ens = Ensemble()
    gid = ens.add_grid(nt, np_, reals)
    ens.set_states(gid, np.ascontiguousarray(f0))
    errs, ident = [], []
    prev = f0.copy()
    for h in range(1, hours + 1):
        err = surrogate_advance(ens, gid, net, feats, float(h), tol)
        cur = ens.get_states(gid)
        ident.extend(np.linalg.norm((cur - prev).reshape(n_real, -1), axis=1) /
                     np.linalg.norm(cur.reshape(n_real, -1), axis=1))
        errs.extend(err.tolist())
        prev = cur
    errs, ident = np.array(errs), np.array(ident)
    acc = sum(ens.diagnostics(r)["surr_accept"] for r in range(n_real))
    rej = sum(ens.diagnostics(r)["surr_reject"] for r in range(n_real))
    out = {"intervals": int(errs.size), "tol": tol, "accept_rate": acc / max(acc + rej, 1),
           "err_median": float(np.median(errs)), "err_p90": float(np.quantile(errs, 0.9)),
           "err_max": float(errs.max()), "identity_median": float(np.median(ident)),
           "gain_over_identity": float(np.median(ident) / max(np.median(errs), 1e-300))}
    log(json.dumps(out))
    net.close()
    ens.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--nt", type=int, default=512)
    t.add_argument("--np", type=int, default=1024)
    t.add_argument("--traj", type=int, default=40)
    t.add_argument("--hours", type=int, default=500)
    t.add_argument("--epochs", type=int, default=2)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--init", default="")
    t.add_argument("--out", required=True)
    t.add_argument("--eval-real", type=int, default=4)
    t.add_argument("--eval-hours", type=int, default=24)
    t.add_argument("--minutes", type=float, default=0.0, help="train for about this long (sets the steps)")
    t.add_argument("--lr-min", type=float, default=1e-5)
    return ap.parse_args(argv)


def run_train(a):
    snaps, feats, _ = generate(a.nt, a.np, a.traj, a.hours, sub=0)
    net = Net(a.nt, a.np, a.batch)
    if a.init:
        net.set_params(np.load(a.init).astype(np.float32))
    else:
        net.set_params(init_params(7))
    info = train(net, snaps, feats, a.epochs, a.batch, a.lr, a.lr_min, seconds=60.0 * a.minutes,
                 save=lambda p: np.save(a.out, p))
    params = net.get_params()
    np.save(a.out, params)
    del snaps
    ev = evaluate(params, a.nt, a.np, a.eval_real, a.eval_hours, sub=1)
    print(json.dumps({"train": {k: v for k, v in info.items() if k != "loss_history"}, "eval": ev}))


def weights_path(nt: int, np_: int) -> str:
    return os.path.join(WEIGHTS, f"surrogate_{nt}x{np_}.npy")


def load_weights(nt: int, np_: int):
    """(parameters, description): the trained weights shipped with the
    package for this grid, else the untrained identity-map initialisation."""
    path = weights_path(nt, np_)
    if os.path.exists(path):
        return np.load(path).astype(np.float32), os.path.relpath(path, ROOT)
    return init_params(7), "untrained (identity-map initialisation)"


def init_params(seed: int) -> np.ndarray:
    """He-normal initial weights in the library's parameter layout (last
    layer zero: the untrained surrogate is the identity map)."""
    g = synth.rng("cnn_init", seed)
    chans = [(6, 64), (64, 64), (64, 64), (64, 64), (64, 1)]
    parts = []
    for i, (cin, cout) in enumerate(chans):
        w = g.standard_normal((cout, cin, 3, 3)) * math.sqrt(2.0 / (9 * cin))
        if i == len(chans) - 1:
            w = w * 0.0
        parts += [w.ravel(), np.zeros(cout)]
    return np.concatenate(parts).astype(np.float32)


if __name__ == "__main__":
    run_train(main())
