"""Flow attenuation (eq. flow_attenuation) on the GPU vs the FP64 oracle.

Each advection advance scales every face velocity by 1 - tanh(m/B0), m the
mean of |B| over the face's two cells of the field at the start of the
advance; B0 is a per-realization parameter (0 = off), so one grid class can
mix attenuated and plain realizations.  Bars as for the plain path: FP64
rel-L2 <= 1e-12, FP32 mixed rel-L2 <= 1e-5.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, max_rel, oracle_run, random_field, rel_l2, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def att_reals(b0s, nu=(500.0, 0.0, 750.0, 250.0), amps=(15.0, 25.0)):
    out = []
    for i, b0 in enumerate(b0s):
        r = synth.Realization(nu_km2_s=nu[i % len(nu)], **synth.dr_mf(amp_mf=amps[i % len(amps)]))
        if i % 2:
            r.d0 = 250.0          # a zonal drift in the rotating frame, so phi faces carry flow
        r.att_b0 = float(b0)
        out.append(r)
    return out


def okw_of(opts):
    return {"adv_scheme": opts.get("adv_scheme", 0), "adv_time": opts.get("adv_time", 0),
            "strang": opts.get("strang", 0)}


@pytest.mark.parametrize("nt,np_,opts", [
    (36, 72, {}), (21, 40, {}), (64, 128, {"adv_scheme": 1}), (36, 72, {"adv_time": 2}),
    (24, 48, {"adv_time": 1}), (48, 96, {"strang": 1}), (40, 200, {})])
def test_attenuation_f64(nt, np_, opts):
    say(f"case attenuation f64 {nt}x{np_} {opts}")
    reals = att_reals((500.0, 100.0, 0.0))
    B0 = np.stack([random_field(nt, np_, 8, 200 + i) for i in range(3)])
    sched = [("advance", 2.0), ("advance", 4.5)]
    ref, st = oracle_run(B0, reals, sched, okw_of(opts))
    got, ens = gpu_run(B0, reals, sched, **opts)
    for r in range(3):
        c = ens.counts(r)
        assert c["steps"] == st[r]["steps"] and c["stages"] == st[r]["stages"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r} (B0 {reals[r].att_b0}): rel-L2 {e:.3e}  max-rel {max_rel(got[r], ref[r]):.3e}")
        assert e <= TOL64
    # the attenuated realizations really differ from the plain flow
    plain = [synth.Realization(**{**vars(x), "att_b0": 0.0}) for x in reals[:2]]
    ref0, _ = oracle_run(B0[:2], plain, sched, okw_of(opts))
    for r in range(2):
        assert rel_l2(ref0[r], ref[r]) > 1e-6


@pytest.mark.parametrize("strang", [0, 1])
def test_attenuation_mixed_precision(strang):
    nt, np_ = 64, 128
    say(f"case attenuation fp32 mixed 64x128, 12 h hourly assimilation, strang {strang}")
    reals = att_reals((500.0, 250.0, 0.0, 1000.0))
    B0 = np.stack([random_field(nt, np_, 12, 210 + i) for i in range(4)])
    sched = []
    for h in range(1, 13):
        sched.append(("advance", float(h)))
        b0, l0 = synth.observer(h)
        sched.append(("assim", synth.observation(B0[0], h, h), 2, None, b0, l0))
    ref, _ = oracle_run(B0, reals, sched, {"strang": strang})
    got, _ = gpu_run(B0, reals, sched, precision=1, strang=strang)
    for r in range(4):
        e, m = rel_l2(got[r], ref[r]), max_rel(got[r], ref[r])
        say(f"  realization {r}: rel-L2 {e:.3e}  max-abs / max|B| {m:.3e}")
        assert e <= TOL32 and m <= TOL32


def test_attenuation_graph_replay_bitwise():
    nt, np_ = 48, 96
    say("case attenuation graph replay vs eager")
    reals = att_reals((500.0, 0.0, 300.0))
    B0 = np.stack([random_field(nt, np_, 6, 220 + i) for i in range(3)])
    sched = [("advance", float(h)) for h in range(1, 5)]
    for prec in (0, 1):
        a, _ = gpu_run(B0, reals, sched, precision=prec)
        b, _ = gpu_run(B0, reals, sched, precision=prec, use_graphs=1)
        assert np.array_equal(a, b), prec


def test_attenuation_full_size_first_hour():
    """512x1024, the ensemble workload's 8 realizations with B0 = 500 G (the
    paper's default), first hour against the oracle."""
    w = synth.config2()
    nt, np_, reals = w.classes[0]
    for r in reals:
        r.att_b0 = 500.0
    say(f"case {w.name} with attenuation: first hour")
    f0 = random_field(nt, np_, w.n_pairs)
    B0 = np.stack([f0] * len(reals))
    sched = [("advance", 1.0)]
    ref, st = oracle_run(B0, reals, sched)
    got, _ = gpu_run(B0, reals, sched)
    for r in range(len(reals)):
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e}")
        assert e <= TOL64


def test_negative_or_nonfinite_b0_rejected():
    import paper_2501_06377_amd as sft
    for bad in (-1.0, float("inf"), float("nan")):
        ens = sft.Ensemble()
        with pytest.raises(sft.SftError):
            ens.add_grid(16, 32, att_reals((bad,)))


def fast_reals(b0s):
    """Flows ten times the workloads' (meridional 150 / 250 m/s, ten times the
    rotation shear, a 2500 m/s drift on odd realizations), so that an hour
    takes several CFL steps even on small grids."""
    out = []
    for i, b0 in enumerate(b0s):
        r = synth.Realization(nu_km2_s=(500.0, 0.0, 750.0, 250.0)[i % 4],
                              **synth.dr_mf(amp_mf=(150.0, 250.0)[i % 2]))
        r.d2 *= 10.0
        r.d4 *= 10.0
        if i % 2:
            r.d0 = 2500.0
        r.att_b0 = float(b0)
        out.append(r)
    return out


def polar_field(nt, np_, sub):
    """A bipolar field on a 300 G axial dipole, so that the flow is strongly
    attenuated towards the poles and the CFL limit moves with the field."""
    th = (np.arange(nt) + 0.5) * np.pi / nt
    return random_field(nt, np_, 8, sub) + 300.0 * np.cos(th)[:, None]


@pytest.mark.parametrize("nt,np_,opts", [
    (36, 72, {}), (48, 96, {"strang": 1}), (24, 48, {"adv_time": 2}), (40, 80, {"lanes": 2}),
    (32, 64, {"adv_scheme": 1, "adv_time": 1})])
def test_attenuated_cfl_per_step_f64(nt, np_, opts):
    """att_cfl = 1: every step of an attenuated realization takes eq.
    ssprk43_dt of the attenuated flow of the field at the step's start (a
    device max-reduction read back per step).  Same steps, stages and fields
    as the oracle's per-step rule; the strongly attenuated realizations take
    fewer steps than under the static limit."""
    say(f"case attenuated per-step CFL f64 {nt}x{np_} {opts}")
    reals = fast_reals((100.0, 60.0, 0.0, 500.0))
    B0 = np.stack([polar_field(nt, np_, 230 + i) for i in range(4)])
    sched = [("advance", 10.0), ("advance", 25.5)]
    ok = {k: v for k, v in opts.items() if k != "lanes"}
    ref, st = oracle_run(B0, reals, sched, {**okw_of(ok), "att_cfl": 1})
    got, ens = gpu_run(B0, reals, sched, att_cfl=1, **opts)
    for r in range(4):
        c = ens.counts(r)
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r} (B0 {reals[r].att_b0}): steps {c['steps']} / oracle {st[r]['steps']}, "
            f"rel-L2 {e:.3e}")
        assert c["steps"] == st[r]["steps"] and c["stages"] == st[r]["stages"]
        assert e <= TOL64
    _, st0 = oracle_run(B0, reals, sched, okw_of(ok))
    for r in (0, 1, 3):
        assert st[r]["steps"] < st0[r]["steps"]
    assert st[2]["steps"] == st0[2]["steps"]      # B0 = 0: the static limit


def test_attenuated_cfl_per_step_mixed_and_full_grid():
    """The same rule in the FP32-mixed path (the limit is taken from the FP64
    state), and on the ensemble workload's 512x1024 grid for one hour."""
    nt, np_ = 64, 128
    say("case attenuated per-step CFL fp32 mixed 64x128, 6 h")
    reals = fast_reals((100.0, 60.0, 0.0))
    B0 = np.stack([polar_field(nt, np_, 240 + i) for i in range(3)])
    sched = [("advance", float(h)) for h in range(1, 7)]
    ref, st = oracle_run(B0, reals, sched, {"att_cfl": 1})
    got, ens = gpu_run(B0, reals, sched, precision=1, att_cfl=1)
    for r in range(3):
        e, m = rel_l2(got[r], ref[r]), max_rel(got[r], ref[r])
        say(f"  realization {r}: steps {ens.counts(r)['steps']} / {st[r]['steps']}, rel-L2 {e:.3e}, "
            f"max-abs / max|B| {m:.3e}")
        assert e <= TOL32 and m <= TOL32
    nt, np_ = 512, 1024
    reals = fast_reals((100.0, 500.0, 60.0, 0.0))
    say(f"case attenuated per-step CFL f64 {nt}x{np_}, 4 realizations, first hour")
    B0 = np.stack([polar_field(nt, np_, 250 + i) for i in range(4)])
    ref, st = oracle_run(B0, reals, [("advance", 1.0)], {"att_cfl": 1})
    got, ens = gpu_run(B0, reals, [("advance", 1.0)], att_cfl=1)
    for r in range(4):
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {ens.counts(r)['steps']} / {st[r]['steps']}, rel-L2 {e:.3e}")
        assert ens.counts(r)["steps"] == st[r]["steps"]
        assert e <= TOL64
