"""Shared helpers of the GPU parity tests: run one workload through the HIP
library (via its C ABI binding) and through the CPU oracle on identical
seeded inputs."""
import math
import sys

import numpy as np

import oracle
import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_weight(nt, np_, real, kind, weight, b0_deg, l0_deg):
    """F map of eq. data_assim_f for one realization, computed by the oracle."""
    if kind == 0:
        return weight
    if kind == 1:
        mu = weight
    else:
        mu = oracle.mu_disk(nt, np_, math.radians(b0_deg), math.radians(l0_deg))
    return oracle.weight_from_mu(mu, real.alpha_mu, real.mu_lim, math.radians(real.lat_lim_deg))


def oracle_run(B0, reals, schedule, opts=None):
    """Run each realization through the oracle.

    schedule: list of ("advance", t_end) / ("assim", data, kind, weight, b0, l0).
    Returns the array of final fields [R, nt, np] and per-realization stats."""
    opts = dict(opts or {})
    first_id = opts.pop("rfe_first_id", 0)
    out, stats = [], []
    R, nt, np_ = B0.shape
    for r, real in enumerate(reals):
        if opts.get("rfe_model", 0):
            opts["rfe_id"] = first_id + r       # the generator's key word 1: the realization id
        B = B0[r].copy()
        t = 0.0
        st = {"steps": 0, "stages": 0}
        for ev in schedule:
            if ev[0] == "advance":
                B, s = oracle.advance(B, real.flow, real.nu_km2_s, t, ev[1],
                                      att_b0=getattr(real, "att_b0", 0.0),
                                      nu_grid_alpha=getattr(real, "nu_grid_alpha", 0.0), **opts)
                st["steps"] += s["steps"]
                st["stages"] += s["stages"]
                t = ev[1]
            else:
                _, data, kind, weight, b0, l0 = ev
                F = oracle_weight(nt, np_, real, kind, weight, b0, l0)
                B = oracle.assimilate(B, data, F, real.flux_balance)
        out.append(B)
        stats.append(st)
    return np.stack(out), stats


def gpu_run(B0, reals, schedule, **optkw):
    """Run the same schedule through the HIP library; returns (fields, ensemble)."""
    import paper_2501_06377_amd as sft
    ens = sft.Ensemble(**optkw)
    R, nt, np_ = B0.shape
    gid = ens.add_grid(nt, np_, reals)
    ens.set_states(gid, np.ascontiguousarray(B0))
    for ev in schedule:
        if ev[0] == "advance":
            ens.advance(ev[1])
        else:
            _, data, kind, weight, b0, l0 = ev
            ens.assimilate(gid, data, weight, kind, b0, l0)
    out = ens.get_states(gid)
    return out, ens


def random_field(nt, np_, n_pairs=20, sub=0):
    return synth.bipolar_field(nt, np_, synth.bipolar_pairs(n_pairs, sub))
