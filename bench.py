#!/usr/bin/env python3
"""Benchmark of the surface-flux-transport hot path on one MI355X.

Workload (the ensemble configuration): 8 realizations on a 512 x 1024 grid,
FP64, diffusivity {250, 500, 750, 1000} km^2/s x meridional amplitude
{10, 20} m/s, differential rotation 13.2 - 2.4 sin^2 - 1.8 sin^4 deg/day minus
a 13.2 deg/day frame, a seeded 200-pair bipolar initial field, and hourly
assimilation of synthetic observations (observed map + N(0, 5 G)) weighted
mu^4 on the visible disk.  One step = one 1-hour interval for all
realizations: advection (WENO3-CS(h) + SSPRK(4,3)), RKG2 diffusion,
assimilation and the FP64 analysis reductions.  The default --steps 655
covers the configuration's 27.3 days (655 one-hour intervals).

Inputs (initial fields and every observation map) are resident in HBM
before the timed region, which runs without per-launch events.  A second
pass over the first intervals of the same workload, in a one-lane context,
brackets every kernel launch with HIP events on the stream it is launched
on; the roofline object reports the dominant kernel family from those
events.  The CPU baseline times the FP64 oracle (as is) on the first hours
of the same workload.

Other workloads (--workload): the FP32-mixed precision configuration (with
its per-realization difference from the FP64 path), the uneven batch, the
flux-preserving smoother, the paper's timed soccer-ball validation runs, and
the plain single-realization configuration.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "realization-cell-updates/s + sim-days/s at 1 GPU; surrogate vs plain @1e-3"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="1-hour intervals (default: 655 for the "
                    "ensemble workload, 24 for the others)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("ensemble", "precision", "batching", "smoother", "soccer", "plain"),
                    default="ensemble",
                    help="ensemble: 8 x 512x1024 FP64 with hourly assimilation (the headline); "
                         "precision: 32 x 1024x2048 FP32-mixed with hourly assimilation; "
                         "batching: 96 realizations in three size classes, FP32-mixed, graphs; "
                         "smoother: 512x1024 map(s) smoothed with the grid diffusivity (alpha 0.5); "
                         "soccer: the paper's timed validation runs (soccer-ball map, 512x1024, 672 h; "
                         "--steps runs per case, default 3); plain: one 180x360 FP64 realization through 168 h "
                         "in one call (--steps runs, default 10)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graphs", action="store_true", help="replay captured graphs (no per-kernel timing)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--att-b0", type=float, default=0.0,
                    help="flow attenuation saturation field B0 in gauss for every realization (0: off)")
    ap.add_argument("--smooth-maps", type=int, default=1, help="maps smoothed together (smoother workload)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="concurrent sub-batches per grid class in the timed region (0: library default)")
    ap.add_argument("--timing-steps", type=int, default=100,
                    help="intervals of the per-kernel event-timing pass (0: none)")
    ap.add_argument("--rfe-model", type=int, default=0, choices=(0, 1, 2),
                    help="random flux emergence model (eq. rfe_m1 / rfe_m2; 0: off)")
    ap.add_argument("--rfe-phi", type=float, default=1.0e23, help="unsigned flux per hour of a map, Mx")
    ap.add_argument("--rfe-tau", type=float, default=1.0, help="source-map lifetime, hours (0: infinite)")
    ap.add_argument("--sts-tile", type=int, default=-1, help="blocked STS shape (-1: autotuned)")
    ap.add_argument("--surr-batch", type=int, default=64)
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate measurement (inference batch, plain vs surrogate intervals)")
    ap.add_argument("--no-f64-compare", action="store_true",
                    help="precision workload: skip the FP64 run that the FP32-mixed result is compared with")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def make_obs(f0, hours, dtype=np.float64):
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        maps = list(ex.map(lambda h: synth.observation(f0, float(h), h, dtype=dtype), hours))
    return np.stack(maps)


def cpu_baseline(nt, np_, reals, f0, obs_first, max_seconds, rfe=None):
    """FP64 oracle on the first realization-hours of a workload class (hour
    by hour, all realizations of an hour in turn), stopped after about
    max_seconds of CPU work."""
    import math

    import oracle
    B = [f0.copy() for _ in reals]
    updates = 0
    done = 0
    t0 = time.perf_counter()
    h = 0
    el = 0.0
    while el < max_seconds:
        h += 1
        if obs_first is not None:
            if h > len(obs_first):
                break
            b0, l0 = synth.observer(float(h))
            mu = oracle.mu_disk(nt, np_, math.radians(b0), math.radians(l0))
        for r, real in enumerate(reals):
            extra = dict(rfe, rfe_id=r) if rfe else {}
            B[r], st = oracle.advance(B[r], real.flow, real.nu_km2_s, float(h - 1), float(h),
                                      att_b0=real.att_b0, nu_grid_alpha=real.nu_grid_alpha, **extra)
            n = st["stages"] + 4 * st["steps"]
            if obs_first is not None:
                F = oracle.weight_from_mu(mu, real.alpha_mu, real.mu_lim, math.radians(real.lat_lim_deg))
                B[r] = oracle.assimilate(B[r], obs_first[h - 1], F, real.flux_balance)
                n += 1
            updates += nt * np_ * n
            done += 1
            el = time.perf_counter() - t0
            if el >= max_seconds:
                break
    return {"value": updates / el, "unit": "realization-cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {done} realization-hours ({nt}x{np_}, hour by hour over {len(reals)} "
                      f"realizations; {el:.1f} s of CPU work, FP64 C oracle, OpenMP over rows)",
            "sim_days_per_s": done / len(reals) / 24.0 / el}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def surrogate_bench(sft, torch, batch, n_real=16, hours=3, tol=1e-3):
    """The learned surrogate at 512 x 1024: BF16-MFMA inference throughput of
    a batch, then plain and surrogate intervals on the same realizations
    (drawn from the surrogate's training distribution: no assimilation),
    with the acceptance rate of the checked surrogate at tol."""
    from paper_2501_06377_amd import surrogate as S
    nt, np_ = 512, 1024
    params, wname = S.load_weights(nt, np_)
    reals, feats = S.sample_realizations(n_real, 2)
    f0 = S.initial_fields(nt, np_, n_real, 2)
    reps = (batch + n_real - 1) // n_real
    net = sft.Net(nt, np_, batch)
    net.set_params(params)
    B = torch.tensor(np.concatenate([f0] * reps)[:batch], dtype=torch.float64, device="cuda")
    F = torch.tensor(np.concatenate([feats] * reps)[:batch], device="cuda")
    y = torch.empty((batch, nt, np_), dtype=torch.float32, device="cuda")
    net.predict(B, F, y)
    net.sync()
    iters = 5
    t0 = time.perf_counter()
    for _ in range(iters):
        net.predict(B, F, y)
    net.sync()
    ms = (time.perf_counter() - t0) / iters * 1e3
    flop = S.FLOP_PER_PIXEL * nt * np_ * batch
    tflops = flop / (ms * 1e-3) / 1e12
    net.close()
    del B, F, y
    log(f"surrogate inference: batch {batch} in {ms:.2f} ms ({tflops:.1f} TFLOP/s)")

    net = sft.Net(nt, np_, n_real)
    net.set_params(params)
    ens = sft.Ensemble()
    gid = ens.add_grid(nt, np_, reals)
    ens.set_states(gid, f0)
    ens.advance(1.0)
    ens.sync()
    t0 = time.perf_counter()
    ens.advance(2.0)
    ens.sync()
    plain = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    sft.surrogate_advance(ens, gid, net, feats, 3.0, tol, check_=False)
    ens.sync()
    unchecked = (time.perf_counter() - t0) * 1e3
    # checked intervals from a plain state
    ens.set_states(gid, f0)
    ens.set_time(0.0)
    errs, ident = [], []
    prev = f0
    checked = 0.0
    for h in range(1, hours + 1):
        t0 = time.perf_counter()
        e = sft.surrogate_advance(ens, gid, net, feats, float(h), tol)
        ens.sync()
        checked += (time.perf_counter() - t0) * 1e3
        cur = ens.get_states(gid)
        ident += list(np.linalg.norm((cur - prev).reshape(n_real, -1), axis=1) /
                      np.linalg.norm(cur.reshape(n_real, -1), axis=1))
        errs += e.tolist()
        prev = cur
    acc = sum(ens.diagnostics(r)["surr_accept"] for r in range(n_real))
    rej = sum(ens.diagnostics(r)["surr_reject"] for r in range(n_real))
    net.close()
    ens.close()
    errs = np.array(errs)
    return {"weights": wname, "grid": f"{nt}x{np_}",
            "inference": {"batch": batch, "ms_per_batch": ms, "flop_per_batch": flop, "TFLOP_s": tflops,
                          "peak_TFLOP_s": 2500.0, "mfma_frac": tflops / 2500.0, "dtype": "bf16 (fp32 acc)"},
            "ms_per_realization_interval": {"plain_f64": plain / n_real, "surrogate_unchecked": unchecked / n_real,
                                            "surrogate_checked": checked / hours / n_real},
            "speedup_unchecked_vs_plain": plain / unchecked,
            "tol_rel_l2": tol, "checked_intervals": int(errs.size), "accept_rate": acc / max(acc + rej, 1),
            "err_median": float(np.median(errs)), "err_max": float(errs.max()),
            "identity_err_median": float(np.median(ident)),
            "gain_over_identity": float(np.median(ident) / max(np.median(errs), 1e-300))}


def copy_probe(mib):
    """A plain device-to-device copy of known size, five times: the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))


def traffic_from_profiles(family, tile_index):
    """HBM bytes per launch of a kernel family from the committed rocprofv3
    counter summary, if it was taken on the same kernel (tile shape) and the
    current kernel sources (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(family)
    if not rec or rec.get("tile_index") != tile_index:
        return None
    for f, h in rec["sources_sha256"].items():
        src = open(os.path.join(ROOT, "paper_2501_06377_amd", "csrc", f), "rb").read()
        if hashlib.sha256(src).hexdigest() != h:
            return None
    return rec["hbm_bytes_per_launch"]


def roofline_fields(fams, traffic, how):
    """The roofline object of the dominant kernel family (by event time) and
    the per-family table, from the library's per-launch event timing."""
    dom = max(fams, key=lambda k: fams[k]["ms"])
    f = fams[dom]
    achieved = f["bytes"] / (f["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "avg_launch_us": f["ms"] / max(f["launches"], 1) * 1e3,
            "alg_bytes_per_launch": f["bytes"] / max(f["launches"], 1),
            "launches": f["launches"], "timing_pass": how,
            # bytes a fused multi-stage launch must move at least
            # (one read of its inputs, one write of its outputs)
            "min_hbm_GB_s": f["min_bytes"] / (f["ms"] * 1e-3) / 1e9,
            "min_hbm_frac": f["min_bytes"] / (f["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    kernels = {k: {"ms": v["ms"], "launches": v["launches"],
                   "GB_s": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
               for k, v in fams.items() if v["launches"]}
    return {"roofline": roof, "kernels": kernels}


# Wall clock and HH error the paper reports for its validation runs at
# 512x1024 on an RTX 3090 Ti (precision not stated): the Strang table, the
# SSPRK(3,3) comparison of Sec. "Advection time" and the diffusion-only
# RKL2 / RKG2 timings.  Context only: another machine, another grid layout.
PAPER_SOCCER = {
    "diffusion, RKL2, one 672 h step": (0.45, 8.0e-5),
    "diffusion, RKG2, one 672 h step": (0.55, 6.3e-5),
    "advection+diffusion, dt 0.5 h": (23.8, 4.4e-5),
    "advection+diffusion, dt 0.5 h, Strang": (26.7, 4.0e-5),
    "advection+diffusion, max CFL dt": (21.1, 4.8e-5),
    "advection+diffusion, max CFL dt, Strang": (15.6, 4.8e-5),
    "advection+diffusion, max CFL dt, SSPRK(3,3)": (38.5, 4.3e-5),
}
SOCCER_DEFAULT = "advection+diffusion, max CFL dt"


def soccer_bench(sft, torch, args, K, W):
    """The paper's timed validation runs on one 512x1024 realization: each
    case advances the soccer-ball map through 672 h in one call, W untimed
    and K timed times from the same initial map; the HH metric compares the
    final map with the analytic one (the initial map times exp(-42 nu t))."""
    import math
    nt, np_ = 512, 1024
    u0 = synth.soccer_ball(nt, np_)
    nu_code = synth.SOCCER_NU_KM2_S * 3.6e9 / 6.96e8 ** 2          # km^2/s -> R_sun^2/h
    exact = u0 * math.exp(-42.0 * nu_code * synth.SOCCER_HOURS)
    x0 = torch.from_numpy(u0[None].copy()).cuda()
    gopt = {"ssprk43": sft.SFT_SSPRK43, "ssprk33": sft.SFT_SSPRK33, "rkg2": sft.SFT_RKG2, "rkl2": sft.SFT_RKL2}
    graphs = bool(args.graphs)

    def make(c, timing=False):
        e = sft.Ensemble(precision=0, use_graphs=0 if timing else int(graphs), adv_time=gopt[c.adv],
                         diff_time=gopt[c.diff], strang=c.strang, dt_max=c.dt_max, sts_tile=args.sts_tile)
        return e, e.add_grid(nt, np_, [c.realization()])

    def once(e, g):
        e.set_states(g, x0)
        e.set_time(0.0)
        a = e.counts(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.advance(synth.SOCCER_HOURS)
        e.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b = e.counts(0)
        return dt, {k: b[k] - a[k] for k in ("steps", "stages", "adv_stages")}

    cases, default = [], None
    for c in synth.soccer_cases():
        e, g = make(c)
        for _ in range(W):
            once(e, g)
        walls = []
        for _ in range(K):
            w_s, cnt = once(e, g)
            walls.append(w_s)
        B = e.get_states(g)[0]
        ti = e.tile_choice(g)
        tile = {"index": ti, "shape_tx_ty_k_threads": sft.tile_info(0, ti) if ti >= 0 else None}
        hh = float(np.sqrt(np.sum((B - exact) ** 2) / np.sum(np.abs(B) * np.abs(exact))))
        e.close()
        wall = float(np.mean(walls))
        upd = nt * np_ * (cnt["stages"] + cnt["adv_stages"])
        pw, ph = PAPER_SOCCER[c.name]
        row = {"case": c.name, "wall_s": wall, "wall_s_min": float(np.min(walls)), "steps": cnt["steps"],
               "sts_stages": cnt["stages"], "adv_stages": cnt["adv_stages"], "sts_tile": tile,
               "dt_h": synth.SOCCER_HOURS / cnt["steps"], "hh": hh,
               "realization_cell_updates_per_s": upd / wall,
               "paper_rtx3090ti": {"wall_s": pw, "hh": ph}, "paper_wall_over_this": pw / wall}
        log(f"soccer: {c.name}: {wall * 1e3:.1f} ms, {cnt['steps']} steps, {cnt['stages']} STS stages, "
            f"HH {hh:.2e} (paper {pw} s, HH {ph:.1e})")
        cases.append(row)
        if c.name == SOCCER_DEFAULT:
            default = (c, row, upd)
    c, row, upd = default
    out = {
        "metric": METRIC, "value": upd / row["wall_s"], "unit": "realization-cell-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": row["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (analytic soccer-ball map)",
        "config": {"workload": "soccer-ball-512x1024-672h", "grid": [f"{nt}x{np_}x1"], "realizations": 1,
                   "step": "one 672 h advance of the soccer-ball map with a full rigid rotation and "
                           "nu = 500 km^2/s (WENO3-CS(h) + SSPRK(4,3), RKG2, max CFL dt), the paper's "
                           "default schemes; the other validation runs are in 'cases'",
                   "simulated_hours": synth.SOCCER_HOURS, "graphs": graphs},
        "sim_days_per_s": synth.SOCCER_HOURS / 24.0 / row["wall_s"],
        "cases": cases,
    }
    if args.timing_steps > 0:
        e, g = make(c, timing=True)
        once(e, g)
        e.set_timing(True)
        once(e, g)
        out.update(roofline_fields(e.timing(), None, "one 672 h run of the same case, HIP events around "
                                   "every launch"))
        e.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = soccer_cpu_baseline(u0, c, args.cpu_seconds)
    return out


def soccer_cpu_baseline(u0, c, max_seconds):
    """FP64 oracle on the default validation case, advanced in 10.5 h
    calls (1/64 of the run) until about max_seconds of CPU work."""
    import oracle
    nt, np_ = u0.shape
    real = c.realization()
    B, t, updates, el, chunk = u0.copy(), 0.0, 0, 0.0, synth.SOCCER_HOURS / 64.0
    t0 = time.perf_counter()
    while el < max_seconds and t < synth.SOCCER_HOURS:
        B, st = oracle.advance(B, real.flow, real.nu_km2_s, t, t + chunk)
        t += chunk
        updates += nt * np_ * (st["stages"] + 4 * st["steps"])
        el = time.perf_counter() - t0
    return {"value": updates / el, "unit": "realization-cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {t:g} h of the default case ({nt}x{np_}, calls of {chunk:g} h; {el:.1f} s of CPU "
                      f"work, FP64 C oracle, OpenMP over rows)",
            "sim_days_per_s": t / 24.0 / el}


def plain_bench(sft, torch, args, K, W):
    """The plain single-realization configuration: one 180x360 FP64
    realization (20 bipolar pairs, eta = 500 km^2/s, the workloads' flow
    forms) advanced through 168 h in one call, W untimed and K timed times
    from the same initial field.  Few cells per launch: the cost is launch
    latency, which replayed graphs remove from the host side."""
    w = synth.config1()
    nt, np_, reals = w.classes[0]
    f0 = synth.bipolar_field(nt, np_, synth.bipolar_pairs(w.n_pairs, 0))
    x0 = torch.from_numpy(f0[None].copy()).cuda()
    graphs = bool(args.graphs)

    def make(timing=False):
        e = sft.Ensemble(precision=0, use_graphs=0 if timing else int(graphs), sts_tile=args.sts_tile)
        return e, e.add_grid(nt, np_, reals)

    def once(e, g):
        e.set_states(g, x0)
        e.set_time(0.0)
        a = e.counts(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.advance(w.hours)
        e.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b = e.counts(0)
        return dt, {k: b[k] - a[k] for k in ("steps", "stages", "adv_stages")}

    e, g = make()
    for _ in range(W):
        once(e, g)
    walls = []
    for _ in range(K):
        w_s, cnt = once(e, g)
        walls.append(w_s)
    ti = e.tile_choice(g)
    tile = {"index": ti, "shape_tx_ty_k_threads": sft.tile_info(0, ti) if ti >= 0 else None}
    e.close()
    wall = float(np.mean(walls))
    upd = nt * np_ * (cnt["stages"] + cnt["adv_stages"])
    log(f"{w.name}: {wall * 1e3:.2f} ms per run, {cnt['steps']} steps, {cnt['stages']} STS stages")
    out = {
        "metric": METRIC, "value": upd / wall, "unit": "realization-cell-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "grid": [f"{nt}x{np_}x1"], "realizations": 1,
                   "step": "one 168 h advance in one call: advection (WENO3-CS(h) + SSPRK(4,3)) + RKG2 "
                           "diffusion at the CFL step, no assimilation",
                   "simulated_hours": w.hours, "graphs": graphs, "sts_tiles": [tile],
                   "run_steps": cnt["steps"], "run_sts_stages": cnt["stages"],
                   "wall_ms_min": float(np.min(walls)) * 1e3},
        "sim_days_per_s": w.hours / 24.0 / wall,
    }
    if args.timing_steps > 0:
        e, g = make(timing=True)
        once(e, g)
        e.set_timing(True)
        once(e, g)
        out.update(roofline_fields(e.timing(), None, "one 168 h run, HIP events around every launch"))
        e.close()
    if not args.no_cpu_baseline:
        import oracle
        real = reals[0]
        B, t, updates, el, chunk = f0.copy(), 0.0, 0, 0.0, w.hours / 8.0
        t0 = time.perf_counter()
        while el < args.cpu_seconds and t < w.hours:
            B, st = oracle.advance(B, real.flow, real.nu_km2_s, t, t + chunk)
            t += chunk
            updates += nt * np_ * (st["stages"] + 4 * st["steps"])
            el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": updates / el, "unit": "realization-cell-updates/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"first {t:g} h of the run ({nt}x{np_}, calls of {chunk:g} h; "
                                         f"{el:.2f} s of CPU work, FP64 C oracle, OpenMP over rows)",
                               "sim_days_per_s": t / 24.0 / el}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(realizations would shard across GPUs)"}))
        sys.exit(2)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    import torch

    import paper_2501_06377_amd as sft

    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_bench(sft, torch, args.surr_batch)}), flush=True)
        return
    if args.workload == "plain":
        print(json.dumps(plain_bench(sft, torch, args, args.steps or 10, args.warmup)), flush=True)
        return
    if args.workload == "soccer":
        print(json.dumps(soccer_bench(sft, torch, args, args.steps or 3, args.warmup)), flush=True)
        return
    w = {"ensemble": synth.config2, "precision": synth.config3, "batching": synth.config4,
         "smoother": lambda: synth.smoother(args.smooth_maps)}[args.workload]()
    K = args.steps if args.steps is not None else (655 if args.workload == "ensemble" else 24)
    if args.att_b0 > 0.0:
        for _, _, reals in w.classes:
            for r in reals:
                r.att_b0 = args.att_b0
        w.name += f"+attenuation-B0-{args.att_b0:g}G"
    rfe_gpu, rfe_cpu = {}, None
    if args.rfe_model:
        rfe_gpu = dict(rfe_model=args.rfe_model, rfe_phi_hr=args.rfe_phi, rfe_lifetime_h=args.rfe_tau, rfe_seed=1)
        rfe_cpu = dict(rfe_model=args.rfe_model, rfe_phi_hr=args.rfe_phi, rfe_tau=args.rfe_tau, rfe_seed=1)
        w.name += f"+flux-emergence-m{args.rfe_model}-tau{args.rfe_tau:g}h"
    W = args.warmup
    prec = 0 if w.precision == "f64" else 1
    graphs = args.graphs or args.workload == "batching"
    assim = w.assim_every_h > 0
    dev = torch.device("cuda:0")
    inits, obs_d, f0s, obs0 = [], [], [], None
    for ci, (nt, np_, reals) in enumerate(w.classes):
        f0 = synth.bipolar_field(nt, np_, synth.bipolar_pairs(w.n_pairs, ci))
        f0s.append(f0)
        if assim:
            obs = make_obs(f0, range(1, max(K, W) + 1))
            if ci == 0:
                obs0 = obs[:24]
            obs_d.append(torch.from_numpy(obs).to(dev))
            del obs
        inits.append(torch.from_numpy(np.ascontiguousarray(np.broadcast_to(f0, (len(reals), nt, np_)))).to(dev))
    R = w.n_real

    def make(lanes):
        e = sft.Ensemble(precision=prec, use_graphs=1 if graphs else 0, sts_tile=args.sts_tile, lanes=lanes,
                         **rfe_gpu)
        return e, [e.add_grid(nt, np_, reals) for nt, np_, reals in w.classes]

    def run(ens, gids, n_steps):
        for h in range(1, n_steps + 1):
            ens.advance(float(h))
            if assim:
                b0, l0 = synth.observer(float(h))
                for g, o in zip(gids, obs_d):
                    ens.assimilate(g, o[h - 1], None, sft.SFT_WEIGHT_DISK, b0, l0)

    def reset(ens, gids):
        for g, x in zip(gids, inits):
            ens.set_states(g, x)
        ens.set_time(0.0)

    ens, gids = make(args.lanes)
    torch.cuda.synchronize()
    log(f"{w.name}: inputs resident, {K} timed intervals")
    reset(ens, gids)
    run(ens, gids, W)
    ens.sync()
    # timed region starts from the initial state at t = 0
    reset(ens, gids)
    c0 = [ens.counts(r) for r in range(R)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(ens, gids, K)
    ens.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = [ens.counts(r) for r in range(R)]
    # per-kernel timing: a second pass over the first intervals of the same
    # workload in a one-lane context (every launch covers the whole class, as
    # in the counter record), with HIP events around every launch; the events
    # themselves cost wall time, so the timed region above runs without them
    Kt = min(K, args.timing_steps)
    fams = {}
    if Kt > 0:
        ens_t, gids_t = make(1)
        reset(ens_t, gids_t)
        run(ens_t, gids_t, 1)
        ens_t.sync()
        reset(ens_t, gids_t)
        ens_t.set_timing(True)
        run(ens_t, gids_t, Kt)
        ens_t.sync()
        fams = ens_t.timing()
        ens_t.close()
    tiles = []
    for g in gids:
        ti = ens.tile_choice(g)
        desc = sft.tile_info(prec, ti) if ti >= 0 else None
        tiles.append({"index": ti, "shape_tx_ty_k_threads": desc})

    cells = [nt * np_ for nt, np_, reals in w.classes for _ in reals]
    updates = sum(n * ((b["stages"] - a["stages"]) + (b["adv_stages"] - a["adv_stages"]) +
                       (b["assim"] - a["assim"])) for n, a, b in zip(cells, c0, c1))
    value = updates / wall
    diag = ens.diagnostics(0)
    out = {
        "metric": METRIC, "value": value, "unit": "realization-cell-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": wall / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": w.precision, "data": "synthetic",
        "config": {"workload": w.name, "grid": [f"{nt}x{np_}x{len(r)}" for nt, np_, r in w.classes],
                   "realizations": R,
                   "step": ("1 h of smoothing: RKG2 diffusion with the grid diffusivity of eq. diffgrid "
                            "(alpha 0.5 / h)" if args.workload == "smoother" else
                            "1 h interval: advection" +
                            (f" (flow attenuation, B0 = {args.att_b0:g} G)" if args.att_b0 > 0.0 else "") +
                            " + RKG2 diffusion") +
                           (f" + flux emergence (model {args.rfe_model}, {args.rfe_phi:g} Mx/h, "
                            f"lifetime {args.rfe_tau:g} h)" if args.rfe_model else "") +
                           (" + mu^4 assimilation" if assim else "") + " + diagnostics",
                   "simulated_hours": K, "graphs": bool(graphs), "sts_tiles": tiles,
                   "lanes": args.lanes or "library default (min(2, realizations per class))"},
        "sim_days_per_s": K / 24.0 / wall,
    }
    if fams:
        dom = max(fams, key=lambda k: fams[k]["ms"])
        # the counter record was taken on the ensemble workload's launches
        traffic = (traffic_from_profiles(dom, tiles[0]["index"])
                   if len(tiles) == 1 and args.workload == "ensemble" else None)
        out.update(roofline_fields(fams, traffic,
                                   f"{Kt} intervals of the same workload, HIP events around every launch"))
        # kernel time per interval in the timing pass, against the timed region's
        # interval time (the difference is launch gaps and the events' own cost)
        out["kernel_ms_per_interval_timing_pass"] = sum(v["ms"] for v in fams.values()) / Kt
    out["final_diag_r0"] = {k: diag[k] for k in ("phi_pos", "phi_neg", "dax", "bmin", "bmax")}
    if w.precision == "f32":
        out["state_dtype"] = "f64 (state, flux and weight reductions)"
    if w.precision == "f32" and args.workload == "precision" and not args.no_f64_compare:
        # the FP32-mixed result of the timed region against the FP64 path on
        # the same inputs (the FP64 path is itself held to the FP64 oracle)
        got = [ens.get_states(g) for g in gids]
        log(f"{w.name}: the same {K} intervals on the FP64 path")
        e64 = sft.Ensemble(precision=0, sts_tile=-1, lanes=args.lanes)
        g64 = [e64.add_grid(nt, np_, reals) for nt, np_, reals in w.classes]
        reset(e64, g64)
        run(e64, g64, K)
        e64.sync()
        ref = [e64.get_states(g) for g in g64]
        e64.close()
        rel, mx = [], []
        for a, b in zip(got, ref):
            for r in range(a.shape[0]):
                rel.append(float(np.linalg.norm(a[r] - b[r]) / np.linalg.norm(b[r])))
                mx.append(float(np.abs(a[r] - b[r]).max()))
        out["f32_vs_f64"] = {"hours": K, "reference": "the library's FP64 path on the same inputs",
                             "rel_l2_per_realization": rel, "max_abs_G_per_realization": mx,
                             "rel_l2_max": max(rel), "tolerance": 1e-5}
        log(f"{w.name}: FP32-mixed vs FP64 after {K} h: rel-L2 max {max(rel):.3e}, "
            f"max-abs max {max(mx):.3e} G")
    ens.close()
    del obs_d, inits
    log(f"{w.name}: {wall:.2f} s for {K} intervals")
    if not args.no_surrogate and args.workload == "ensemble":
        out["surrogate"] = surrogate_bench(sft, torch, args.surr_batch)
    if not args.no_cpu_baseline:
        nt, np_, reals = w.classes[-1]
        out["cpu_baseline"] = cpu_baseline(nt, np_, reals, f0s[-1], obs0 if len(w.classes) == 1 else None,
                                           args.cpu_seconds, rfe_cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
