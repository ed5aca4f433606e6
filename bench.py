#!/usr/bin/env python3
"""Benchmark of the surface-flux-transport hot path on one MI355X.

Default workload (the precision configuration, the largest that the
configurations define): 32 realizations on a 1024 x 2048 grid, FP32 stencil
arithmetic with FP64 state, flux and weight reductions, diffusivity
U(200, 800) km^2/s, differential rotation 13.2 - 2.4 f sin^2 - 1.8 f sin^4
deg/day minus a 13.2 deg/day frame and a poleward meridional flow 15 g
sin(2 lat) m/s with f, g ~ U(0.8, 1.2) per realization, a seeded 200-pair
bipolar initial field, and hourly assimilation, weighted mu^4 on the visible
disk, of observed maps: the hourly state of a nominal realization (eta = 500
km^2/s, 15 m/s) evolved from the same field by the library's FP64 path, plus
N(0, 5 G).  One step = one 1-hour interval for all realizations: advection
(WENO3-CS(h) + SSPRK(4,3)), RKG2 diffusion, assimilation and the FP64
analysis reductions.  The FP64 path is timed on the same inputs, and the
FP32-mixed result is compared with it per realization.

Inputs (initial fields and every observation map) are resident in HBM
before the timed region.  Per-launch HIP events on the launch stream give
the roofline of the dominant kernel: inside the timed region for this
workload (one lane; its launches are long), in a second, one-lane pass for
the others.  The learned surrogate (512 x 1024, BF16 MFMA) is measured
against the plain solver in FP64 and FP32-mixed, with checks every K-th
interval (throughput mode).  The CPU baseline times the FP64 oracle (as is)
on the first hours of the same workload.

Other workloads (--workload): the FP64 ensemble configuration, the uneven
batch, the flux-preserving smoother, the paper's timed soccer-ball
validation runs, and the plain single-realization configuration.

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
                    default="precision",
                    help="precision (default, the largest configuration): 32 x 1024x2048 FP32-mixed with "
                         "hourly assimilation, with the FP64 path timed on the same inputs; "
                         "ensemble: 8 x 512x1024 FP64 with hourly assimilation; "
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
    ap.add_argument("--lanes", type=int, default=None,
                    help="concurrent sub-batches per grid class in the timed region (0: library default; "
                         "default 1 for the precision workload, whose launches each fill the GPU, else 0)")
    ap.add_argument("--events-in-region", type=int, default=None, choices=(0, 1),
                    help="1: HIP events around every launch inside the timed region itself (the roofline "
                         "then comes from the timed run; default for the precision workload, whose launches "
                         "are long enough that the events cost nothing); 0: a separate timing pass")
    ap.add_argument("--timing-steps", type=int, default=100,
                    help="intervals of the per-kernel event-timing pass (0: none)")
    ap.add_argument("--rfe-model", type=int, default=0, choices=(0, 1, 2),
                    help="random flux emergence model (eq. rfe_m1 / rfe_m2; 0: off)")
    ap.add_argument("--rfe-phi", type=float, default=1.0e23, help="unsigned flux per hour of a map, Mx")
    ap.add_argument("--rfe-tau", type=float, default=1.0, help="source-map lifetime, hours (0: infinite)")
    ap.add_argument("--sts-tile", type=int, default=-1, help="blocked STS shape (-1: autotuned)")
    ap.add_argument("--surr-batch", type=int, default=64)
    ap.add_argument("--inference-only", action="store_true",
                    help="only the batch inference timing of the surrogate (few launches: counter runs)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the surrogate measurement (inference batch, plain vs surrogate intervals)")
    ap.add_argument("--no-f64-compare", action="store_true",
                    help="precision workload: skip the FP64 run that the FP32-mixed result is compared with")
    ap.add_argument("--sts-fuse", type=int, default=0, choices=(0, 1),
                    help="1: one diffusion stage per launch (the unfused kernel)")
    ap.add_argument("--class-tiles", default=None,
                    help="comma-separated diffusion tile shape per grid class, in class order "
                         "(sft_set_class_tile; -1 = one stage per launch), instead of the autotuner's")
    ap.add_argument("--att-cfl", type=int, default=0, choices=(0, 1),
                    help="with --att-b0: 1 = per-step CFL limit of the attenuated flow")
    ap.add_argument("--obs", choices=("truth", "sheared"), default="truth",
                    help="observations: truth = hourly maps of a nominal realization run by the library's "
                         "FP64 path plus N(0, 5 G); sheared = the initial field sheared in longitude plus "
                         "N(0, 5 G)")
    ap.add_argument("--surr-stride", type=int, default=8, help="surrogate throughput mode: check every K-th interval")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def make_obs(f0, hours, dtype=np.float64):
    """Sheared-field observations (synth.observation) for the given hours."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        maps = list(ex.map(lambda h: synth.observation(f0, float(h), h, dtype=dtype), hours))
    return np.stack(maps)


def truth_obs_gpu(sft, torch, f0, n_hours):
    """Observed maps of hours 1..n_hours on the device: a nominal realization
    (eta = 500 km^2/s, meridional 15 m/s, the workloads' rotation) evolved
    from the initial field by the library's FP64 path, plus seeded N(0, 5 G)
    per cell and hour (synth.truth_observation).  Untimed input preparation."""
    nt, np_ = f0.shape
    ens = sft.Ensemble(precision=0)
    g = ens.add_grid(nt, np_, [synth.nominal_truth_realization()])
    ens.set_states(g, f0[None].copy())
    out = torch.empty((n_hours, nt, np_), dtype=torch.float64, device="cuda")
    cur = torch.empty((1, nt, np_), dtype=torch.float64, device="cuda")
    for h in range(1, n_hours + 1):
        ens.advance(float(h))
        ens.get_states(g, cur)
        ens.sync()
        out[h - 1] = torch.from_numpy(synth.truth_observation(cur[0].cpu().numpy(), h)).to(out.device)
    ens.close()
    return out


def oracle_truth_stream(f0):
    """obs(h): the same observed map of hour h with the truth run by the
    oracle, hour after hour, for the CPU baseline (the oracle takes no input
    from the GPU path)."""
    import oracle
    r = synth.nominal_truth_realization()
    st = {"B": f0.copy(), "h": 0}

    def obs(h):
        while st["h"] < h:
            st["B"], _ = oracle.advance(st["B"], r.flow, r.nu_km2_s, float(st["h"]), float(st["h"] + 1))
            st["h"] += 1
        return synth.truth_observation(st["B"], h)
    return obs


def cpu_baseline(nt, np_, reals, f0, obs_first, max_seconds, rfe=None, obs_fn=None):
    """FP64 oracle on the first realization-hours of a workload class (hour
    by hour, all realizations of an hour in turn), stopped after about
    max_seconds of CPU work.  obs_fn(h) gives the observed map of hour h
    when obs_first is None (its own cost is not counted)."""
    import math

    import oracle
    B = [f0.copy() for _ in reals]
    updates = 0
    done = 0
    t0 = time.perf_counter()
    h = 0
    el = 0.0
    obs_h = None
    while el < max_seconds:
        h += 1
        if obs_fn is not None:
            t_obs = time.perf_counter()
            obs_h = obs_fn(h)
            t0 += time.perf_counter() - t_obs
        elif obs_first is not None:
            if h > len(obs_first):
                break
            obs_h = obs_first[h - 1]
        if obs_h is not None:
            b0, l0 = synth.observer(float(h))
            mu = oracle.mu_disk(nt, np_, math.radians(b0), math.radians(l0))
        for r, real in enumerate(reals):
            extra = dict(rfe, rfe_id=r) if rfe else {}
            B[r], st = oracle.advance(B[r], real.flow, real.nu_km2_s, float(h - 1), float(h),
                                      att_b0=real.att_b0, nu_grid_alpha=real.nu_grid_alpha, **extra)
            n = st["stages"] + 4 * st["steps"]
            if obs_h is not None:
                F = oracle.weight_from_mu(mu, real.alpha_mu, real.mu_lim, math.radians(real.lat_lim_deg))
                B[r] = oracle.assimilate(B[r], obs_h, F, real.flux_balance)
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


def surrogate_bench(sft, torch, batch, n_real=64, hours=16, stride=8, tol=1e-3, inference_only=False):
    """The learned surrogate at 512 x 1024 on realizations of its training
    distribution (no assimilation): BF16-MFMA inference throughput of a
    batch, then the cost of a realization-interval over `hours` one-hour
    intervals from the same initial fields, for the plain solver (FP64 and
    FP32-mixed) and for the surrogate unverified, checked every `stride`-th
    interval per realization (throughput mode, every interval after a
    rejection), and checked every interval (validation).  A checked interval
    runs the context's plain solver (FP64 or FP32-mixed) as the arbiter."""
    from paper_2501_06377_amd import surrogate as S
    nt, np_ = 512, 1024
    params, wname = S.load_weights(nt, np_)
    reals, feats = S.sample_realizations(n_real, 2)
    f0 = S.initial_fields(nt, np_, n_real, 2)
    x0 = torch.tensor(f0, dtype=torch.float64, device="cuda")
    net = sft.Net(nt, np_, max(batch, n_real))
    net.set_params(params)
    B = x0[torch.arange(batch, device="cuda") % n_real].contiguous()
    F = torch.tensor(feats[np.arange(batch) % n_real], device="cuda")
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
    del B, F, y
    log(f"surrogate inference: batch {batch} in {ms:.2f} ms ({tflops:.1f} TFLOP/s)")
    if inference_only:
        net.close()
        return {"weights": wname, "grid": f"{nt}x{np_}",
                "inference": {"batch": batch, "ms_per_batch": ms, "flop_per_batch": flop, "TFLOP_s": tflops,
                              "peak_TFLOP_s": 2500.0, "mfma_frac": tflops / 2500.0, "dtype": "bf16 (fp32 acc)"}}

    def context(prec):
        ens = sft.Ensemble(precision=prec)
        gid = ens.add_grid(nt, np_, reals)
        return ens, gid

    def plain(prec):
        ens, gid = context(prec)
        ens.set_states(gid, x0)
        ens.advance(1.0)             # first interval: the tile autotuner
        ens.set_states(gid, x0)
        ens.set_time(0.0)
        ens.sync()
        t0 = time.perf_counter()
        for h in range(1, hours + 1):
            ens.advance(float(h))
        ens.sync()
        wall = time.perf_counter() - t0
        out = ens.get_states(gid)
        ens.close()
        return wall, out

    def surrogate(check, prec=0):
        ens, gid = context(prec)
        ens.set_states(gid, x0)
        ens.advance(1.0)             # the tile autotuner, outside the timed intervals
        ens.set_states(gid, x0)
        ens.set_time(0.0)
        # one untimed surrogate interval (first-call allocations), from the initial state again
        sft.surrogate_advance(ens, gid, net, feats, 1.0, tol, check)
        ens.set_states(gid, x0)
        ens.set_time(0.0)
        c0 = [sft.surrogate_counts(ens, r) for r in range(n_real)]
        ens.sync()
        errs = []
        t0 = time.perf_counter()
        for h in range(1, hours + 1):
            errs.append(sft.surrogate_advance(ens, gid, net, feats, float(h), tol, check))
        ens.sync()
        wall = time.perf_counter() - t0
        c1 = [sft.surrogate_counts(ens, r) for r in range(n_real)]
        cnt = {k: sum(b[k] - a[k] for a, b in zip(c0, c1)) for k in ("accepted", "rejected", "unchecked")}
        out = ens.get_states(gid)
        ens.close()
        return wall, out, np.array(errs), cnt

    def per(wall):
        return wall / hours / n_real * 1e3

    w64, ref64 = plain(0)
    w32, ref32 = plain(1)
    wun, fin_un, _, _ = surrogate(0)
    wst, fin_st, err_st, cnt_st = surrogate(stride)
    wst32, fin_st32, err_st32, cnt_st32 = surrogate(stride, 1)
    wck, fin_ck, err_ck, cnt_ck = surrogate(1)
    net.close()

    def drift(a):
        return [float(np.linalg.norm(a[r] - ref64[r]) / np.linalg.norm(ref64[r])) for r in range(n_real)]

    d_st, d_un, d_ck = drift(fin_st), drift(fin_un), drift(fin_ck)
    # the method without the surrogate: the identity map over one interval
    e1 = sft.Ensemble()
    g1 = e1.add_grid(nt, np_, reals)
    e1.set_states(g1, x0)
    e1.advance(1.0)
    one = e1.get_states(g1)
    e1.close()
    ident = [float(np.linalg.norm(one[r] - f0[r]) / np.linalg.norm(one[r])) for r in range(n_real)]
    chk = err_st[err_st >= 0]
    log(f"surrogate: ms per realization-interval plain f64 {per(w64):.4f}, plain f32 {per(w32):.4f}, "
        f"unchecked {per(wun):.4f}, every {stride}th checked {per(wst):.4f} (f32 arbiter {per(wst32):.4f}), "
        f"every interval checked {per(wck):.4f}")
    return {"weights": wname, "grid": f"{nt}x{np_}", "realizations": n_real, "intervals": hours,
            "data": "synthetic (the training distribution: seeded 200-pair fields, eta U(250, 1000) km^2/s, "
                    "MF U(10, 20) m/s, DR shear U(0.8, 1.2); no assimilation)",
            "inference": {"batch": batch, "ms_per_batch": ms, "flop_per_batch": flop, "TFLOP_s": tflops,
                          "peak_TFLOP_s": 2500.0, "mfma_frac": tflops / 2500.0, "dtype": "bf16 (fp32 acc)"},
            "ms_per_realization_interval": {
                "plain_f64": per(w64), "plain_f32_mixed": per(w32), "surrogate_unchecked": per(wun),
                f"surrogate_checked_every_{stride}": per(wst),
                f"surrogate_checked_every_{stride}_f32_arbiter": per(wst32),
                "surrogate_checked_every_interval": per(wck)},
            "speedup_checked_every_%d_vs_plain_f64" % stride: w64 / wst,
            "speedup_checked_every_%d_vs_plain_f32_mixed" % stride: w32 / wst,
            "speedup_checked_every_%d_f32_arbiter_vs_plain_f32_mixed" % stride: w32 / wst32,
            "speedup_unchecked_vs_plain_f64": w64 / wun,
            "tol_rel_l2": tol, "check_stride": stride,
            "strided_counts": cnt_st, "strided_counts_f32_arbiter": cnt_st32, "every_interval_counts": cnt_ck,
            "strided_checked_err_median": float(np.median(chk)) if chk.size else None,
            "strided_checked_err_max": float(chk.max()) if chk.size else None,
            "every_interval_err_median": float(np.median(err_ck)), "every_interval_err_max": float(err_ck.max()),
            "accept_rate_every_interval": cnt_ck["accepted"] / max(cnt_ck["accepted"] + cnt_ck["rejected"], 1),
            "trajectory_rel_l2_vs_plain_f64_after": {
                "hours": hours, f"checked_every_{stride}_median": float(np.median(d_st)),
                f"checked_every_{stride}_max": float(np.max(d_st)),
                "unchecked_median": float(np.median(d_un)), "every_interval_median": float(np.median(d_ck)),
                "plain_f32_mixed_max": float(max(np.linalg.norm(ref32[r] - ref64[r]) / np.linalg.norm(ref64[r])
                                                 for r in range(n_real)))},
            "identity_err_median": float(np.median(ident)),
            "gain_over_identity": float(np.median(ident) / max(np.median(err_ck), 1e-300))}


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


def traffic_from_profiles(family, tile_index, workload, precision, sts_fuse):
    """HBM bytes per launch of a kernel family from the committed rocprofv3
    counter record (profiles/traffic.json) taken on the same workload, kernel
    (precision, tile shape) and kernel sources; None without one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    for rec in json.load(open(path)).get("records", []):
        if (rec.get("family") != family or rec.get("workload") != workload or
                rec.get("precision") != precision or rec.get("sts_fuse", 0) != sts_fuse or
                (not sts_fuse and rec.get("tile_index") != tile_index)):
            continue
        ok = True
        for f, h in rec["sources_sha256"].items():
            src = open(os.path.join(ROOT, "paper_2501_06377_amd", "csrc", f), "rb").read()
            ok &= hashlib.sha256(src).hexdigest() == h
        if ok:
            return rec["hbm_bytes_per_launch"]
    return None


def roofline_fields(fams, traffic, how):
    """The roofline object of the dominant kernel family (by event time) and
    the per-family table, from the library's per-launch event timing.

    achieved: the bytes a launch must move (its inputs read once, its outputs
    written once; for a launch that fuses k diffusion stages, the
    algorithm's bytes of one k-stage pass) over the average launch time, so
    frac <= 1.  effective_GB_s: the method's bytes per stage (e.g. 16 B per
    cell and FP32-mixed diffusion stage) over the same time; it exceeds the
    peak when stages are fused.  traffic: measured HBM bytes per launch from
    the committed counter record of this workload and kernel, else null."""
    dom = max(fams, key=lambda k: fams[k]["ms"])
    f = fams[dom]
    n = max(f["launches"], 1)
    t = f["ms"] * 1e-3
    achieved = f["min_bytes"] / t / 1e9
    eff = f["bytes"] / t / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "avg_launch_us": f["ms"] / n * 1e3,
            "alg_bytes_per_launch": f["min_bytes"] / n,
            "launches": f["launches"], "timing_pass": how,
            "traffic_GB_s": traffic / (t / n) / 1e9 if traffic else None,
            "traffic_frac": traffic / (t / n) / 1e9 / HBM_PEAK_GBS if traffic else None,
            "effective_GB_s": eff, "effective_frac": eff / HBM_PEAK_GBS,
            "method_bytes_per_launch": f["bytes"] / n}
    kernels = {k: {"ms": v["ms"], "launches": v["launches"],
                   "GB_s": (v["min_bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None,
                   "effective_GB_s": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
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

    if args.surrogate_only or args.inference_only:
        print(json.dumps({"surrogate": surrogate_bench(sft, torch, args.surr_batch,
                                                       inference_only=args.inference_only)}), flush=True)
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
    if args.lanes is None:
        args.lanes = 1 if args.workload == "precision" else 0
    in_region = (args.events_in_region if args.events_in_region is not None
                 else int(args.workload == "precision"))
    prec = 0 if w.precision == "f64" else 1
    graphs = args.graphs or args.workload == "batching"
    assim = w.assim_every_h > 0
    dev = torch.device("cuda:0")
    inits, obs_d, f0s, obs0 = [], [], [], None
    for ci, (nt, np_, reals) in enumerate(w.classes):
        f0 = synth.bipolar_field(nt, np_, synth.bipolar_pairs(w.n_pairs, ci))
        f0s.append(f0)
        if assim:
            if args.obs == "truth":
                obs_d.append(truth_obs_gpu(sft, torch, f0, max(K, W)))
            else:
                obs = make_obs(f0, range(1, max(K, W) + 1))
                if ci == 0:
                    obs0 = obs[:24]
                obs_d.append(torch.from_numpy(obs).to(dev))
                del obs
        inits.append(torch.from_numpy(np.ascontiguousarray(np.broadcast_to(f0, (len(reals), nt, np_)))).to(dev))
    R = w.n_real
    okw = dict(sts_fuse=args.sts_fuse, att_cfl=args.att_cfl)

    class_tiles = [int(x) for x in args.class_tiles.split(",")] if args.class_tiles else None
    if class_tiles is not None and len(class_tiles) != len(w.classes):
        raise SystemExit(f"--class-tiles needs {len(w.classes)} values, one per grid class")

    def make(lanes, tile=None):
        e = sft.Ensemble(precision=prec, use_graphs=1 if graphs and not in_region else 0,
                         sts_tile=args.sts_tile if tile is None else tile, lanes=lanes, **rfe_gpu, **okw)
        gids = [e.add_grid(nt, np_, reals) for nt, np_, reals in w.classes]
        for g, t in zip(gids, class_tiles or []):
            e.set_class_tile(g, t)
        return e, gids

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
    if in_region:
        ens.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(ens, gids, K)
    ens.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = [ens.counts(r) for r in range(R)]
    # per-kernel timing: the timed region's own events, or a second pass
    # over the first intervals of the same workload in a one-lane context
    # with the same tile shape (every launch covers the whole class), with
    # HIP events around every launch; where the events would cost wall time
    # (short launches), the timed region above runs without them
    Kt = K if in_region else min(K, args.timing_steps)
    fams = {}
    if in_region:
        fams = ens.timing()
        ens.set_timing(False)
    elif Kt > 0:
        one_tile = ens.tile_choice(gids[0]) if len(gids) == 1 else None
        ens_t, gids_t = make(1, one_tile)
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
                   "sts_fuse": args.sts_fuse, "att_cfl": args.att_cfl,
                   "observations": (("hourly maps of a nominal realization (eta 500 km^2/s, MF 15 m/s) run by "
                                     "the library's FP64 path from the same initial field, + N(0, 5 G)")
                                    if args.obs == "truth" else
                                    "the initial field sheared in longitude, + N(0, 5 G)") if assim else None,
                   "lanes": args.lanes or "library default (min(2, realizations per class))",
                   "events_in_timed_region": bool(in_region)},
        "sim_days_per_s": K / 24.0 / wall,
    }
    if fams:
        dom = max(fams, key=lambda k: fams[k]["ms"])
        # a counter record applies when taken on this workload's launches of
        # the same kernel (tile shape) and sources
        traffic = (traffic_from_profiles(dom, tiles[0]["index"], w.name, prec, args.sts_fuse)
                   if len(tiles) == 1 and not (args.att_b0 or args.rfe_model) else None)
        out.update(roofline_fields(fams, traffic,
                                   f"the timed region's {Kt} intervals, HIP events around every launch on its "
                                   f"stream" if in_region else
                                   f"{Kt} intervals of the same workload in one lane, HIP events around every "
                                   f"launch"))
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
        e64 = sft.Ensemble(precision=0, sts_tile=-1, lanes=args.lanes, **okw)
        g64 = [e64.add_grid(nt, np_, reals) for nt, np_, reals in w.classes]
        reset(e64, g64)
        run(e64, g64, W)
        e64.sync()
        reset(e64, g64)
        a64 = [e64.counts(r) for r in range(R)]
        torch.cuda.synchronize()
        t64 = time.perf_counter()
        run(e64, g64, K)
        e64.sync()
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t64
        b64 = [e64.counts(r) for r in range(R)]
        upd64 = sum(n * ((b["stages"] - a["stages"]) + (b["adv_stages"] - a["adv_stages"]) +
                         (b["assim"] - a["assim"])) for n, a, b in zip(cells, a64, b64))
        ref = [e64.get_states(g) for g in g64]
        e64.close()
        out["f64_path"] = {"value": upd64 / wall64, "unit": "realization-cell-updates/s",
                           "ms_per_step": wall64 / K * 1e3, "sim_days_per_s": K / 24.0 / wall64,
                           "steps": K, "warmup": W, "inputs": "the same initial fields and observations",
                           "f32_mixed_speedup": wall64 / wall}
        log(f"{w.name}: FP64 path {wall64 / K * 1e3:.2f} ms per interval ({upd64 / wall64:.3e} "
            f"realization-cell-updates/s)")
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
    if not args.no_surrogate and args.workload in ("ensemble", "precision"):
        out["surrogate"] = surrogate_bench(sft, torch, args.surr_batch, stride=args.surr_stride)
    if not args.no_cpu_baseline:
        nt, np_, reals = w.classes[-1]
        one = len(w.classes) == 1
        out["cpu_baseline"] = cpu_baseline(nt, np_, reals, f0s[-1], obs0 if one else None, args.cpu_seconds,
                                           rfe_cpu, oracle_truth_stream(f0s[-1]) if (one and assim and
                                                                                      args.obs == "truth") else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
