"""Edge cases of the HIP library against the FP64 oracle: the smallest grids
the library accepts (odd row counts, fewer columns than one tile), the
degenerate realizations (no flow, no diffusion; zero field), a zero-length
advance, a very stiff diffusivity (over a hundred STS stages in one call), a
long single advance, and the state / argument errors of the C ABI."""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, max_rel, oracle_run, random_field, rel_l2, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def mix(n):
    return [synth.Realization(nu_km2_s=(400.0, 900.0, 150.0)[i % 3], **synth.dr_mf(amp_mf=(12.0, 20.0)[i % 2]))
            for i in range(n)]


@pytest.mark.parametrize("nt,np_", [(8, 8), (9, 16), (13, 10), (8, 70)])
@pytest.mark.parametrize("prec", [0, 1])
def test_smallest_grids(nt, np_, prec):
    say(f"case smallest grid {nt}x{np_} precision {prec}")
    reals = mix(3)
    B0 = np.stack([random_field(nt, np_, 2, 500 + i) for i in range(3)])
    sched = [("advance", 2.0)]
    b0, l0 = synth.observer(2.0)
    sched.append(("assim", synth.observation(B0[0], 2.0, 2), 2, None, b0, l0))
    sched.append(("advance", 5.5))
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched, precision=prec)
    for r in range(3):
        assert ens.counts(r)["steps"] == st[r]["steps"] and ens.counts(r)["stages"] == st[r]["stages"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: rel-L2 {e:.3e}  max-abs / max|B| {max_rel(got[r], ref[r]):.3e}")
        assert e <= (TOL64 if prec == 0 else TOL32)
        assert prec == 0 or max_rel(got[r], ref[r]) <= TOL32


def test_degenerate_realizations():
    """No flow and no diffusion leaves the field bit for bit (one step per
    advance, no stages); a zero-length advance changes nothing and takes no
    step; a zero field stays exactly zero under every operator and under the
    assimilation of zero data."""
    nt, np_ = 24, 48
    say("case degenerate realizations")
    still = synth.Realization(nu_km2_s=0.0, d0=0.0, d2=0.0, d4=0.0, m1=0.0)
    B0 = np.stack([random_field(nt, np_, 4, 510)])
    zeros = np.zeros((2, nt, np_))
    b0, l0 = synth.observer(1.0)
    for prec in (0, 1):
        got, ens = gpu_run(B0, [still], [("advance", 1.0), ("advance", 1.0), ("advance", 3.0)], precision=prec)
        assert np.array_equal(got[0], B0[0]), prec
        c = ens.counts(0)
        assert c["steps"] == 2 and c["stages"] == 0 and c["adv_stages"] == 0, c
        got, _ = gpu_run(zeros, mix(2), [("advance", 1.0), ("assim", zeros[0], 2, None, b0, l0),
                                         ("advance", 2.5)], precision=prec)
        assert np.array_equal(got, zeros), prec


def test_stiff_diffusivity_many_stages():
    """Diffusivities 100-200x the workloads' take over a hundred RKG2 stages
    in one call (every blocked launch full, many groups); FP64 against the
    oracle."""
    nt, np_ = 64, 128
    say("case stiff diffusivity")
    reals = [synth.Realization(nu_km2_s=2.0e5, d0=0.0, d2=0.0, d4=0.0, m1=0.0),
             synth.Realization(nu_km2_s=1.0e5, **synth.dr_mf(amp_mf=10.0))]
    B0 = np.stack([random_field(nt, np_, 6, 520 + i) for i in range(2)])
    sched = [("advance", 1.0)]
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched)
    assert st[0]["stages"] > 100
    for r in range(2):
        assert ens.counts(r)["stages"] == st[r]["stages"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: stages {st[r]['stages']} rel-L2 {e:.3e}")
        assert e <= TOL64


def test_long_single_advance():
    """One 120 h advance (many CFL-limited steps, one plan) against the oracle."""
    nt, np_ = 21, 40
    say("case long single advance")
    reals = mix(2)
    B0 = np.stack([random_field(nt, np_, 4, 530 + i) for i in range(2)])
    ref, st = oracle_run(B0, reals, [("advance", 120.0)])
    got, ens = gpu_run(B0, reals, [("advance", 120.0)])
    for r in range(2):
        assert ens.counts(r)["steps"] == st[r]["steps"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {st[r]['steps']} rel-L2 {e:.3e}")
        assert e <= TOL64


def test_state_and_argument_errors():
    import paper_2501_06377_amd as sft
    ens = sft.Ensemble()
    with pytest.raises(sft.SftError) as ex:
        ens.advance(1.0)                                  # no realizations yet
    assert ex.value.status == sft.SFT_ERR_STATE
    for nt, np_ in ((7, 16), (16, 15), (16, 6)):
        with pytest.raises(sft.SftError):
            ens.add_grid(nt, np_, mix(1))                 # below the minimum or odd phi count
    g = ens.add_grid(16, 32, mix(2))
    ens.set_states(g, np.stack([random_field(16, 32, 2, 540 + i) for i in range(2)]))
    ens.advance(1.0)
    with pytest.raises(sft.SftError) as ex:
        ens.advance(0.5)                                  # backwards in time
    assert ex.value.status == sft.SFT_ERR_ARG
    with pytest.raises(sft.SftError) as ex:
        ens.add_grid(16, 32, mix(1))                      # after the first advance
    assert ex.value.status == sft.SFT_ERR_STATE
    ens.close()


def test_fp32_long_sts_call_stays_accurate():
    """One FP32-mixed STS call of ~1,800 stages at 1024 x 2048 (diffusivity
    800 km^2/s over 1 h) against the FP64 oracle: carried as the increment
    and its last change, the FP32 rounding does not grow with the stage
    count, so the result holds 1e-7 rel-L2 (the three-term form drifted to
    ~2e-5 here)."""
    nt, np_ = 1024, 2048
    say("case FP32 long STS call 1024x2048")
    reals = [synth.Realization(nu_km2_s=800.0, d0=0.0, d2=0.0, d4=0.0, m1=0.0)]
    B0 = np.stack([random_field(nt, np_, 200, 560)])
    sched = [("advance", 1.0)]
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched, precision=1)
    assert st[0]["stages"] > 1500 and ens.counts(0)["stages"] == st[0]["stages"]
    e = rel_l2(got[0], ref[0])
    say(f"  stages {st[0]['stages']} rel-L2 {e:.3e}")
    assert e <= 1e-7


@pytest.mark.parametrize("prec", [0, 1])
def test_minimum_step_matches_oracle(prec):
    """dt_min raises the step limit min(0.9 CFL, dt_max) (here above the CFL
    limit and over a smaller dt_max): the same fewer, longer steps as the
    oracle's rule, each advance still ending on its t_end."""
    import oracle
    nt, np_ = 64, 128
    say(f"case minimum step, precision {prec}")
    reals = mix(3)
    vph, vth = oracle.flows(nt, reals[1].flow)
    lim = 0.9 * oracle.cfl_dt(nt, np_, vph, vth)
    dmin = 1.3 * lim
    B0 = np.stack([random_field(nt, np_, 6, 520 + i) for i in range(3)])
    sched = [("advance", 9.0), ("advance", 9.0 + 0.4 * dmin), ("advance", 31.0)]
    ref, st = oracle_run(B0, reals, sched, {"dt_min": dmin, "dt_max": 0.5 * lim})
    got, ens = gpu_run(B0, reals, sched, precision=prec, dt_min=dmin, dt_max=0.5 * lim)
    _, st0 = oracle_run(B0, reals, sched)
    for r in range(3):
        c = ens.counts(r)
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: steps {c['steps']} / oracle {st[r]['steps']} (without dt_min "
            f"{st0[r]['steps']}), rel-L2 {e:.3e}")
        assert c["steps"] == st[r]["steps"] and c["stages"] == st[r]["stages"]
        assert e <= (TOL64 if prec == 0 else TOL32)
        assert prec == 0 or max_rel(got[r], ref[r]) <= TOL32
    assert st[1]["steps"] < st0[1]["steps"]
