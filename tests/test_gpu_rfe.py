"""Random flux emergence (Sec. "Flux emergence") on the GPU vs the FP64 oracle.

Source maps are drawn on the device (Philox4x32-10 + Box-Muller, eqs.
rfe_m1 / rfe_m2, eq. fluxbal balance); steps land on the map times; the
source sub-advances close each step (or open and close it under Strang
splitting).  Bars as for the plain path: FP64 rel-L2 <= 1e-12, FP32 mixed
rel-L2 <= 1e-5.  The maps are a pure function of (seed, realization id, map
index), so restarts and graph replays reproduce them bit for bit.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, max_rel, oracle_run, random_field, rel_l2, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
PHI = 1.0e23          # Mx per hour, the rate of the paper's validation runs


def gpu_opts(model, tau, seed=11, **kw):
    return dict(rfe_model=model, rfe_phi_hr=PHI, rfe_lifetime_h=tau, rfe_seed=seed, **kw)


def oracle_opts(model, tau, seed=11, **kw):
    return dict(rfe_model=model, rfe_phi_hr=PHI, rfe_tau=tau, rfe_seed=seed, **kw)


def reals_mix(n):
    out = []
    for i in range(n):
        r = synth.Realization(nu_km2_s=(250.0, 500.0, 0.0, 750.0)[i % 4],
                              **synth.dr_mf(amp_mf=(10.0, 20.0)[i % 2]))
        out.append(r)
    return out


@pytest.mark.parametrize("nt,np_,model,tau", [(24, 48, 2, 0.3), (21, 40, 1, 0.3), (36, 72, 2, 0.0),
                                              (64, 128, 1, 0.45)])
def test_source_only_f64(nt, np_, model, tau):
    """No flow, no diffusion, zero start: the field is the time integral of the
    device's source maps, against the oracle's maps."""
    say(f"case rfe source only {nt}x{np_} model {model} tau {tau}")
    reals = [synth.Realization(nu_km2_s=0.0, d0=0, d2=0, d4=0, m1=0) for _ in range(3)]
    B0 = np.zeros((3, nt, np_))
    sched = [("advance", 0.5), ("advance", 1.0), ("advance", 2.2)]
    ref, st = oracle_run(B0, reals, sched, oracle_opts(model, tau))
    got, ens = gpu_run(B0, reals, sched, **gpu_opts(model, tau))
    for r in range(3):
        assert ens.counts(r)["steps"] == st[r]["steps"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e} max-rel {max_rel(got[r], ref[r]):.3e}")
        assert e <= TOL64
    # realizations draw different maps
    assert rel_l2(got[0], got[1]) > 0.5


@pytest.mark.parametrize("opts", [{}, {"strang": 1}, {"adv_time": 2}, {"strang": 1, "adv_time": 1}])
def test_transport_with_source_f64(opts):
    nt, np_ = 48, 96
    say(f"case rfe with flows and diffusion f64 {opts}")
    reals = reals_mix(4)
    B0 = np.stack([random_field(nt, np_, 6, 300 + i) for i in range(4)])
    sched = [("advance", 1.0), ("advance", 2.3), ("advance", 4.0)]
    b0, l0 = synth.observer(4.0)
    sched.append(("assim", synth.observation(B0[0], 4.0, 4), 2, None, b0, l0))
    sched.append(("advance", 5.0))
    okw = {"adv_time": opts.get("adv_time", 0), "strang": opts.get("strang", 0)}
    ref, st = oracle_run(B0, reals, sched, {**okw, **oracle_opts(2, 0.7)})
    got, ens = gpu_run(B0, reals, sched, **opts, **gpu_opts(2, 0.7))
    for r in range(4):
        c = ens.counts(r)
        assert c["steps"] == st[r]["steps"] and c["stages"] == st[r]["stages"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e}")
        assert e <= TOL64


@pytest.mark.parametrize("strang", [0, 1])
def test_source_mixed_precision(strang):
    nt, np_ = 64, 128
    say(f"case rfe fp32 mixed 64x128, 12 h hourly assimilation, strang {strang}")
    reals = reals_mix(4)
    B0 = np.stack([random_field(nt, np_, 12, 310 + i) for i in range(4)])
    sched = []
    for h in range(1, 13):
        sched.append(("advance", float(h)))
        b0, l0 = synth.observer(h)
        sched.append(("assim", synth.observation(B0[0], h, h), 2, None, b0, l0))
    ref, _ = oracle_run(B0, reals, sched, {"strang": strang, **oracle_opts(1, 0.3)})
    got, _ = gpu_run(B0, reals, sched, precision=1, strang=strang, **gpu_opts(1, 0.3))
    for r in range(4):
        e, m = rel_l2(got[r], ref[r]), max_rel(got[r], ref[r])
        say(f"  realization {r}: rel-L2 {e:.3e}  max-abs / max|B| {m:.3e}")
        assert e <= TOL32 and m <= TOL32


def test_graph_replay_and_restart_bitwise():
    """Hourly advances with tau = 0.5 h reuse one plan and one graph while the
    device's map index advances; eager, graph and a restarted context (new
    maps drawn for the restart time) agree bit for bit, and with the oracle."""
    import paper_2501_06377_amd as sft
    nt, np_ = 32, 64
    say("case rfe graphs / restart")
    reals = reals_mix(3)
    B0 = np.stack([random_field(nt, np_, 6, 320 + i) for i in range(3)])
    sched = [("advance", float(h)) for h in range(1, 7)]
    eager, _ = gpu_run(B0, reals, sched, **gpu_opts(2, 0.5))
    graph, _ = gpu_run(B0, reals, sched, use_graphs=1, **gpu_opts(2, 0.5))
    assert np.array_equal(eager, graph)
    half, ens = gpu_run(B0, reals, sched[:3], **gpu_opts(2, 0.5))
    e2 = sft.Ensemble(**gpu_opts(2, 0.5))
    g = e2.add_grid(nt, np_, reals)
    e2.set_states(g, half)
    e2.set_time(3.0)
    for h in range(4, 7):
        e2.advance(float(h))
    assert np.array_equal(e2.get_states(g), eager)
    ref, _ = oracle_run(B0, reals, sched, oracle_opts(2, 0.5))
    assert rel_l2(eager, ref) <= TOL64


def test_incommensurate_lifetime_many_advances():
    """tau = 0.37 h with hourly advances: every advance starts at a new phase
    of its interval, so plans are not reused and the library drops its plan
    cache when it fills; the result still matches the oracle."""
    nt, np_ = 16, 32
    say("case rfe tau 0.37 h over 70 hourly advances")
    reals = reals_mix(2)
    B0 = np.stack([random_field(nt, np_, 4, 330 + i) for i in range(2)])
    sched = [("advance", float(h)) for h in range(1, 71)]
    ref, st = oracle_run(B0, reals, sched, oracle_opts(2, 0.37))
    got, ens = gpu_run(B0, reals, sched, **gpu_opts(2, 0.37))
    for r in range(2):
        assert ens.counts(r)["steps"] == st[r]["steps"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e}")
        assert e <= TOL64


def test_full_size_ensemble_first_hours():
    """512x1024, the ensemble workload's 8 realizations with model-2 emergence
    (1e23 Mx/h, tau = 0.3 h) over 2 h, against the oracle."""
    w = synth.config2()
    nt, np_, reals = w.classes[0]
    say(f"case {w.name} with flux emergence: 2 h")
    f0 = random_field(nt, np_, w.n_pairs)
    B0 = np.stack([f0] * len(reals))
    sched = [("advance", 1.0), ("advance", 2.0)]
    ref, st = oracle_run(B0, reals, sched, oracle_opts(2, 0.3))
    got, _ = gpu_run(B0, reals, sched, **gpu_opts(2, 0.3))
    for r in range(len(reals)):
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e}")
        assert e <= TOL64
