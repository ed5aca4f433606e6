"""GPU (HIP library through its C ABI) vs FP64 CPU oracle, element by element.

FP64 path: the kernels evaluate the paper's formulas in the oracle's order;
the diffusion stages use fused multiply-adds where the oracle rounds each
product, and reduction orders differ (flux-balance sums, device cosine of
the observer geometry), so fields agree to rounding level.  The bar is
rel-L2 <= 1e-12 (stated in the tests), and the measured error is printed.
FP32 mixed path: rel-L2 <= 1e-5.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import gpu_run, max_rel, oracle_run, random_field, rel_l2, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def reals_mix(n, nu=(250.0, 500.0, 750.0, 1000.0), amps=(10.0, 20.0)):
    out = []
    for i in range(n):
        out.append(synth.Realization(nu_km2_s=nu[i % len(nu)],
                                     **synth.dr_mf(amp_mf=amps[(i // len(nu)) % len(amps)])))
    return out


@pytest.mark.parametrize("nt,np_", [(64, 128), (36, 72), (21, 40)])
def test_diffusion_only_f64(nt, np_):
    say(f"case diffusion-only f64 {nt}x{np_}")
    reals = [synth.Realization(nu_km2_s=nu, d0=0, d2=0, d4=0, m1=0) for nu in (200.0, 600.0, 1000.0)]
    B0 = np.stack([random_field(nt, np_, 10, i) for i in range(3)])
    sched = [("advance", 5.0), ("advance", 7.5)]
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched)
    for r in range(3):
        c = ens.counts(r)
        assert c["stages"] == st[r]["stages"] and c["steps"] == st[r]["steps"]
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.3e}  max-rel {max_rel(got, ref):.3e}  bitwise {np.array_equal(got, ref)}")
    assert e <= TOL64


@pytest.mark.parametrize("nt,np_,scheme", [(64, 128, 0), (36, 72, 0), (21, 40, 0), (36, 72, 1)])
def test_advection_only_f64(nt, np_, scheme):
    say(f"case advection-only f64 {nt}x{np_} scheme {scheme}")
    reals = [synth.Realization(nu_km2_s=0.0, **synth.dr_mf(amp_mf=a)) for a in (10.0, 25.0)]
    reals[1].d0 = 300.0
    B0 = np.stack([random_field(nt, np_, 10, 5 + i) for i in range(2)])
    sched = [("advance", 30.0)]
    ref, _ = oracle_run(B0, reals, sched, {"adv_scheme": scheme})
    got, _ = gpu_run(B0, reals, sched, adv_scheme=scheme)
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.3e}  bitwise {np.array_equal(got, ref)}")
    assert e <= TOL64


def test_config1_plain_f64():
    """180x360, one realization, 20 pairs, eta = 500, MF 15 m/s, 7 days."""
    w = synth.config1()
    nt, np_, reals = w.classes[0]
    say(f"case {w.name}")
    B0 = random_field(nt, np_, w.n_pairs)[None]
    sched = [("advance", w.hours)]
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched)
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.3e}  max-rel {max_rel(got, ref):.3e}  stages {st[0]['stages']}")
    assert e <= TOL64
    d = ens.diagnostics(0)
    od = oracle.diagnostics(ref[0])
    for k in ("phi_pos", "phi_neg", "h1", "h2", "dax"):
        assert d[k] == pytest.approx(od[k], rel=1e-11, abs=1e-9 * abs(od["phi_pos"])), k
    assert d["bmin"] == pytest.approx(od["bmin"], rel=TOL64)
    assert d["bmax"] == pytest.approx(od["bmax"], rel=TOL64)


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("balance", [0, 1])
def test_assimilation_f64(kind, balance):
    nt, np_ = 40, 80
    say(f"case assimilation kind {kind} balance {balance}")
    reals = reals_mix(3)
    for i, r in enumerate(reals):
        r.flux_balance = balance
        r.alpha_mu = (4.0, 2.5, 4.0)[i]
        r.mu_lim = (0.0, 0.1, 0.2)[i]
        r.lat_lim_deg = (90.0, 60.0, 75.0)[i]
    B0 = np.stack([random_field(nt, np_, 8, 10 + i) for i in range(3)])
    obs = synth.observation(B0[0], 2.0, 0)
    mu = oracle.mu_disk(nt, np_, math.radians(5.0), math.radians(100.0))
    weight = {0: np.clip(mu, 0, None) ** 3, 1: mu, 2: None}[kind]
    sched = [("advance", 2.0), ("assim", obs, kind, weight, 5.0, 100.0), ("advance", 3.0)]
    ref, _ = oracle_run(B0, reals, sched)
    got, _ = gpu_run(B0, reals, sched)
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.3e}")
    assert e <= TOL64


@pytest.mark.parametrize("opts", [
    {"adv_time": 1}, {"adv_time": 2}, {"diff_time": 1}, {"diff_time": 2, "dt_max": 0.05}, {"ptl_dt": 0.3},
    {"dt_max": 0.7, "cfl_safety": 0.5}, {"strang": 1}, {"strang": 1, "adv_time": 1}])
def test_scheme_options_f64(opts):
    nt, np_ = 24, 48
    say(f"case options {opts}")
    reals = reals_mix(2)
    B0 = np.stack([random_field(nt, np_, 6, 20 + i) for i in range(2)])
    sched = [("advance", 1.0), ("advance", 2.3)]
    okw = {"adv_time": opts.get("adv_time", 0), "diff_scheme": opts.get("diff_time", 0),
           "dt_max": opts.get("dt_max", 0.0), "ptl_dt": opts.get("ptl_dt", 0.0),
           "safety": opts.get("cfl_safety", 0.9), "strang": opts.get("strang", 0)}
    ref, _ = oracle_run(B0, reals, sched, okw)
    got, _ = gpu_run(B0, reals, sched, **opts)
    e = rel_l2(got, ref)
    say(f"  rel-L2 {e:.3e}")
    assert e <= TOL64


@pytest.mark.parametrize("adv_time,strang", [(0, 0), (2, 0), (0, 1)])
def test_mixed_precision_matches_oracle(adv_time, strang):
    nt, np_ = 64, 128
    say(f"case fp32 mixed 64x128, 24 h with hourly assimilation, advection scheme {adv_time}, strang {strang}")
    reals = reals_mix(4)
    B0 = np.stack([random_field(nt, np_, 12, 30 + i) for i in range(4)])
    sched = []
    for h in range(1, 25):
        sched.append(("advance", float(h)))
        b0, l0 = synth.observer(h)
        sched.append(("assim", synth.observation(B0[0], h, h), 2, None, b0, l0))
    ref, _ = oracle_run(B0, reals, sched, {"adv_time": adv_time, "strang": strang})
    got, _ = gpu_run(B0, reals, sched, precision=1, adv_time=adv_time, strang=strang)
    for r in range(4):
        e, m = rel_l2(got[r], ref[r]), max_rel(got[r], ref[r])
        say(f"  realization {r}: rel-L2 {e:.3e}  max-abs {np.abs(got[r] - ref[r]).max():.3e} G "
            f"({m:.3e} of max|B|)")
        assert e <= TOL32 and m <= TOL32


def test_graph_replay_is_bitwise_equal_to_eager():
    nt, np_ = 48, 96
    say("case graph replay vs eager")
    reals = reals_mix(3)
    B0 = np.stack([random_field(nt, np_, 6, 40 + i) for i in range(3)])
    sched = []
    for h in range(1, 6):
        sched.append(("advance", float(h)))
        b0, l0 = synth.observer(h)
        sched.append(("assim", synth.observation(B0[0], h, h), 2, None, b0, l0))
    for prec in (0, 1):
        a, _ = gpu_run(B0, reals, sched, precision=prec)
        b, _ = gpu_run(B0, reals, sched, precision=prec, use_graphs=1)
        assert np.array_equal(a, b), prec


def test_checkpoint_restart_bitwise():
    nt, np_ = 32, 64
    say("case checkpoint / restart")
    import paper_2501_06377_amd as sft
    reals = reals_mix(2)
    B0 = np.stack([random_field(nt, np_, 6, 50 + i) for i in range(2)])
    full, _ = gpu_run(B0, reals, [("advance", 3.0), ("advance", 6.0)])
    half, ens = gpu_run(B0, reals, [("advance", 3.0)])
    t = ens.time()
    e2 = sft.Ensemble()
    g = e2.add_grid(nt, np_, reals)
    e2.set_states(g, half)
    e2.set_time(t)
    e2.advance(6.0)
    assert np.array_equal(e2.get_states(g), full)


def test_nonfinite_is_reported():
    nt, np_ = 16, 32
    say("case non-finite guard")
    import paper_2501_06377_amd as sft
    reals = reals_mix(1)
    B0 = random_field(nt, np_, 3, 60)[None].copy()
    B0[0, 5, 7] = np.nan
    ens = sft.Ensemble()
    g = ens.add_grid(nt, np_, reals)
    ens.set_states(g, B0)
    ens.advance(1.0)
    d = ens.diagnostics(0)
    assert d["status"] == sft.SFT_ERR_NOT_FINITE and d["nonfinite"] > 0


def test_full_size_ensemble_first_hour_f64():
    """512x1024, 8 realizations (the ensemble workload's grid and parameter
    set), first hour plus one assimilation, against the oracle."""
    w = synth.config2()
    nt, np_, reals = w.classes[0]
    say(f"case {w.name}: first hour")
    f0 = random_field(nt, np_, w.n_pairs)
    B0 = np.stack([f0] * len(reals))
    b0, l0 = synth.observer(1.0)
    sched = [("advance", 1.0), ("assim", synth.observation(f0, 1.0, 1), 2, None, b0, l0)]
    ref, st = oracle_run(B0, reals, sched)
    got, ens = gpu_run(B0, reals, sched)
    for r in range(len(reals)):
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: stages {st[r]['stages']} rel-L2 {e:.3e}")
        assert e <= TOL64


@pytest.mark.parametrize("prec,nt,np_", [(0, 70, 150), (1, 70, 150), (1, 300, 256), (1, 257, 130)])
def test_blocked_tiles_bitwise_equal_unfused(prec, nt, np_):
    """Every blocked tile shape (temporal blocking in LDS / registers) gives
    bitwise the same fields as one stage per launch: the grids span several
    column tiles with ragged tails (and, at 300 and 257 rows, several
    pole-aligned row tiles for the FP32 shapes), realizations with different stage counts end in
    different launches, and advection increments feed the mixed path."""
    import paper_2501_06377_amd as sft
    say(f"case tile invariance precision {prec} grid {nt}x{np_}")
    reals = [synth.Realization(nu_km2_s=nu, **synth.dr_mf(amp_mf=a))
             for nu, a in ((200.0, 10.0), (600.0, 20.0), (1000.0, 15.0))]
    B0 = np.stack([random_field(nt, np_, 8, 70 + i) for i in range(3)])
    sched = [("advance", 6.0), ("advance", 13.0)]
    ref, ens = gpu_run(B0, reals, sched, precision=prec, sts_fuse=1)
    assert ens.tile_choice(0) == -1
    i = 0
    while sft.tile_info(prec, i) is not None:
        got, e2 = gpu_run(B0, reals, sched, precision=prec, sts_tile=i)
        assert e2.tile_choice(0) == i
        same = np.array_equal(got, ref)
        say(f"  tile {i} {sft.tile_info(prec, i)}: bitwise {same}")
        assert same, i
        i += 1
    assert i >= 3
    auto, e3 = gpu_run(B0, reals, sched, precision=prec)
    say(f"  autotuned choice {e3.tile_choice(0)}")
    assert np.array_equal(auto, ref)
    oref, _ = oracle_run(B0, reals, sched)
    e = rel_l2(ref, oref)
    say(f"  one stage per launch vs oracle: rel-L2 {e:.3e}")
    assert e <= (TOL64 if prec == 0 else TOL32)


def run_classes(classes, fields, hours, **optkw):
    """All size classes in one context (one plan / graph per interval)."""
    import paper_2501_06377_amd as sft
    ens = sft.Ensemble(**optkw)
    gids = []
    for (nt, np_, reals), B0 in zip(classes, fields):
        g = ens.add_grid(nt, np_, reals)
        ens.set_states(g, B0)
        gids.append(g)
    for h in hours:
        ens.advance(float(h))
    return [ens.get_states(g) for g in gids], ens


@pytest.mark.parametrize("prec,graphs", [(0, 0), (0, 1), (1, 1)])
def test_uneven_classes_in_one_context(prec, graphs):
    """Three grid classes of uneven sizes advanced together (per-realization
    dt and stage counts, one graph per interval), each realization against
    the oracle."""
    say(f"case uneven classes precision {prec} graphs {graphs}")
    classes = [(24, 48, reals_mix(2)), (40, 80, reals_mix(3)), (64, 128, reals_mix(2, nu=(900.0, 300.0)))]
    fields = [np.stack([random_field(nt, np_, 6, 90 + 10 * c + i) for i in range(len(rs))])
              for c, (nt, np_, rs) in enumerate(classes)]
    hours = [1.0, 2.0, 3.5]
    got, ens = run_classes(classes, fields, hours, precision=prec, use_graphs=graphs)
    tol = TOL64 if prec == 0 else TOL32
    for c, ((nt, np_, rs), B0) in enumerate(zip(classes, fields)):
        ref, _ = oracle_run(B0, rs, [("advance", h) for h in hours])
        for r in range(len(rs)):
            e = rel_l2(got[c][r], ref[r])
            say(f"  class {nt}x{np_} realization {r}: rel-L2 {e:.3e}")
            assert e <= tol
            assert prec == 0 or max_rel(got[c][r], ref[r]) <= TOL32


@pytest.mark.parametrize("prec", [0, 1])
def test_class_tiles_bitwise_equal_autotuned(prec):
    """sft_set_class_tile fixes each class's diffusion kernel (a blocked shape,
    one stage per launch, another blocked shape) after a first advance has
    captured graphs with the autotuner's choices: the fields stay bitwise
    those of the autotuned run, the choices read back, and an index past the
    table is refused."""
    import paper_2501_06377_amd as sft
    say(f"case per-class tiles precision {prec}")
    classes = [(24, 48, reals_mix(2)), (40, 80, reals_mix(3)), (64, 128, reals_mix(2, nu=(900.0, 300.0)))]
    fields = [np.stack([random_field(nt, np_, 6, 190 + 10 * c + i) for i in range(len(rs))])
              for c, (nt, np_, rs) in enumerate(classes)]
    hours = [1.0, 2.0, 3.5]
    ref, _ = run_classes(classes, fields, hours, precision=prec, use_graphs=1)
    n = 0
    while sft.tile_info(prec, n) is not None:
        n += 1
    pick = [n - 1, -1, 0]
    ens = sft.Ensemble(precision=prec, use_graphs=1)
    gids = []
    for (nt, np_, rs), B0 in zip(classes, fields):
        g = ens.add_grid(nt, np_, rs)
        ens.set_states(g, B0)
        gids.append(g)
    ens.advance(hours[0])
    for g, t in zip(gids, pick):
        ens.set_class_tile(g, t)
    for h in hours[1:]:
        ens.advance(h)
    for g, t, (nt, np_, _), want in zip(gids, pick, classes, ref):
        assert ens.tile_choice(g) == t
        same = np.array_equal(ens.get_states(g), want)
        say(f"  class {nt}x{np_} tile {t}: bitwise {same}")
        assert same
    with pytest.raises(sft.SftError):
        ens.set_class_tile(gids[0], n)
    with pytest.raises(sft.SftError):
        ens.set_class_tile(len(gids), 0)


def test_full_size_flux_balanced_assimilation_f64():
    """Flux-balanced mu^4 assimilation (eqs. data_assim_deltab, fluxbal) on
    the ensemble workload's 512 x 1024 grid, where the FP64 sums of the
    increment's positive and negative flux run over many blocks: against the
    oracle at the FP64 bar, after an hour of transport and the assimilation,
    and the balanced increment carries no net flux (to round-off of its
    unsigned flux)."""
    w = synth.config2()
    nt, np_, reals = w.classes[0]
    reals = reals[:3]
    for i, r in enumerate(reals):
        r.flux_balance = 1
        r.alpha_mu = (4.0, 2.0, 4.0)[i]
    say(f"case {w.name}: flux-balanced assimilation at full size, 3 realizations")
    f0 = random_field(nt, np_, w.n_pairs)
    B0 = np.stack([f0] * len(reals))
    b0, l0 = synth.observer(1.0)
    obs = synth.observation(f0, 1.0, 1)
    ref1, _ = oracle_run(B0, reals, [("advance", 1.0)])
    ref, _ = oracle_run(B0, reals, [("advance", 1.0), ("assim", obs, 2, None, b0, l0)])
    import paper_2501_06377_amd as sft
    ens = sft.Ensemble()
    g = ens.add_grid(nt, np_, reals)
    ens.set_states(g, B0)
    ens.advance(1.0)
    before = [ens.diagnostics(r)["phi_net"] for r in range(3)]
    ens.assimilate(g, obs, None, sft.SFT_WEIGHT_DISK, b0, l0)
    got = ens.get_states(g)
    wgt = np.sin((np.arange(nt) + 0.5) * np.pi / nt)[:, None] * (np.pi / nt) * (2 * np.pi / np_)
    for r in range(3):
        e = rel_l2(got[r], ref[r])
        dnet = ens.diagnostics(r)["phi_net"] - before[r]
        unsigned = float((np.abs(ref[r] - ref1[r]) * wgt).sum())
        say(f"  realization {r}: rel-L2 {e:.3e}, net flux of the increment {dnet:.3e} "
            f"(unsigned {unsigned:.3e})")
        assert e <= TOL64
        assert abs(dnet) <= 1e-12 * unsigned and unsigned > 0


def test_full_size_mixed_precision_first_hour():
    """The precision workload's grid (1024 x 2048, FP32 stencils with FP64
    state and reductions): two of its realizations, first hour plus one
    mu^4 assimilation, against the FP64 oracle."""
    w = synth.config3(n=2)
    nt, np_, reals = w.classes[0]
    say(f"case {w.name}: first hour, 2 realizations")
    f0 = random_field(nt, np_, w.n_pairs)
    B0 = np.stack([f0] * len(reals))
    b0, l0 = synth.observer(1.0)
    sched = [("advance", 1.0), ("assim", synth.observation(f0, 1.0, 1), 2, None, b0, l0)]
    ref, st = oracle_run(B0, reals, sched)
    got, _ = gpu_run(B0, reals, sched, precision=1)
    for r in range(len(reals)):
        e, m = rel_l2(got[r], ref[r]), max_rel(got[r], ref[r])
        say(f"  realization {r}: stages {st[r]['stages']} rel-L2 {e:.3e} "
            f"max-abs {np.abs(got[r] - ref[r]).max():.3e} G ({m:.3e} of max|B|)")
        assert e <= TOL32 and m <= TOL32


def test_full_size_precision_grid_f64_first_hour():
    """The FP64 path on the precision workload's 1024 x 2048 grid against the
    FP64 oracle over its first hour: a realization of that workload and a
    pure-diffusion one at 800 km^2/s whose single STS call is ~1,800 stages
    long (the longest calls of the workloads)."""
    nt, np_ = 1024, 2048
    w = synth.config3(n=1)
    reals = [w.classes[0][2][0], synth.Realization(nu_km2_s=800.0, d0=0.0, d2=0.0, d4=0.0, m1=0.0)]
    say("case 1024x2048 FP64 first hour")
    f0 = random_field(nt, np_, w.n_pairs, 570)
    B0 = np.stack([f0, f0])
    ref, st = oracle_run(B0, reals, [("advance", 1.0)])
    got, ens = gpu_run(B0, reals, [("advance", 1.0)])
    assert st[1]["stages"] > 1500
    for r in range(2):
        assert ens.counts(r)["stages"] == st[r]["stages"]
        e = rel_l2(got[r], ref[r])
        say(f"  realization {r}: stages {st[r]['stages']} rel-L2 {e:.3e}")
        assert e <= TOL64


def test_full_size_uneven_batch_first_hour():
    """The batching workload's three size classes (256x512, 512x1024,
    1024x2048; one realization each here) in one graph-captured context,
    FP32 stencils, first hour, against the FP64 oracle."""
    w = synth.config4(n_each=1)
    say(f"case {w.name}: first hour, one realization per class")
    fields = [random_field(nt, np_, w.n_pairs, 7)[None].copy() for nt, np_, _ in w.classes]
    got, _ = run_classes(w.classes, fields, [1.0], precision=1, use_graphs=1)
    for c, ((nt, np_, rs), B0) in enumerate(zip(w.classes, fields)):
        ref, st = oracle_run(B0, rs, [("advance", 1.0)])
        e, m = rel_l2(got[c][0], ref[0]), max_rel(got[c][0], ref[0])
        say(f"  class {nt}x{np_}: stages {st[0]['stages']} rel-L2 {e:.3e}  max-abs / max|B| {m:.3e}")
        assert e <= TOL32 and m <= TOL32


def test_strang_step_count_and_counters():
    """With Strang splitting the CFL-limited step is twice as long (half as
    many steps and diffusion calls) and each step runs two advection advances;
    the fields match the oracle's Strang sequence."""
    nt, np_ = 48, 96
    say("case strang counters")
    reals = reals_mix(2)
    B0 = np.stack([random_field(nt, np_, 6, 110 + i) for i in range(2)])
    sched = [("advance", 12.0)]
    plain, e0 = gpu_run(B0, reals, sched)
    got, e1 = gpu_run(B0, reals, sched, strang=1)
    ref, st = oracle_run(B0, reals, sched, {"strang": 1})
    for r in range(2):
        c0, c1 = e0.counts(r), e1.counts(r)
        say(f"  realization {r}: steps {c0['steps']} -> {c1['steps']}, adv stages {c0['adv_stages']} -> "
            f"{c1['adv_stages']}, rel-L2 vs oracle {rel_l2(got[r], ref[r]):.3e}")
        assert c1["steps"] == st[r]["steps"]
        assert c1["steps"] <= (c0["steps"] + 1) // 2 + 1
        assert c1["adv_stages"] == 2 * 4 * c1["steps"]
        assert rel_l2(got[r], ref[r]) <= TOL64



@pytest.mark.parametrize("prec", [0, 1])
def test_lanes_give_identical_results(prec):
    """Realizations split into concurrent sub-batches on their own streams
    (lanes) give bit-identical fields and counters for any lane count, eager
    and in graphs, with flux emergence and assimilation in the interval."""
    nt, np_ = 40, 80
    say(f"case lanes invariance precision {prec}")
    reals = reals_mix(5)
    B0 = np.stack([random_field(nt, np_, 6, 120 + i) for i in range(5)])
    sched = []
    for h in (1.0, 2.0, 3.5):
        sched.append(("advance", h))
        b0, l0 = synth.observer(h)
        sched.append(("assim", synth.observation(B0[0], h, int(h)), 2, None, b0, l0))
    kw = dict(precision=prec, rfe_model=2, rfe_phi_hr=1e23, rfe_lifetime_h=0.6, rfe_seed=3)
    ref, e1 = gpu_run(B0, reals, sched, lanes=1, **kw)
    for lanes, graphs in ((2, 0), (3, 1), (4, 0), (5, 1), (0, 0)):
        got, e2 = gpu_run(B0, reals, sched, lanes=lanes, use_graphs=graphs, **kw)
        same = np.array_equal(got, ref)
        say(f"  lanes {lanes} graphs {graphs}: bitwise {same}")
        assert same
        for r in range(5):
            assert e2.counts(r) == e1.counts(r)
    if prec == 0:
        okw = {"rfe_model": 2, "rfe_phi_hr": 1e23, "rfe_tau": 0.6, "rfe_seed": 3}
        oref, _ = oracle_run(B0, reals, sched, okw)
        assert rel_l2(ref, oref) <= TOL64
