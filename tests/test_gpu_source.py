"""Continuous cathode source on the GPU: parity with the oracle, and the
steady-state beam weight of Sec. II.B.

The source repeats the seeding of Sec. IV (electrons at rest at x = 0) every
step at the physical rate per_step w_j0 / dt; the tail kernel injects the
markers after the particle kernel's outputs, with the step's population
control."""

import math

import numpy as np
import pytest

import oracle
import synth
from synth import configs, xsec
from synth.constants import QE, ME
from parity import compare_populations, STAT_INT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402


def _gap(n_seed=200, n_target=3000, **kw):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=n_seed,
                            n_target=n_target, capacity=configs.capacity_for(n_target, n_seed))
    for k, v in kw.items():
        setattr(inst, k, v)
    return inst


def test_fp64_source_with_population_control_matches_oracle_step_by_step(xs_argon):
    """Full physics plus a source of 37.5 markers per step: splitting first
    (w_j halves, 75 injections a step), then roulette (w_j doubles back,
    37 or 38 a step).  FP64: every step's integer statistics equal, the
    final markers (ids included) and fields equal."""
    inst = _gap()
    run = configs.Run(precision=64)
    gpu = slpic.Sim([inst], run, xs_argon)
    ref = oracle.Sim(inst, run, xs_argon)
    ions = synth.markers.ions(11, 1000, inst.cells, cell_hi=8, e_beam_hi=1500.0)
    gpu.load(1, ions)
    ref.load(1, ions)
    gpu.set_source(37.5)
    ref.set_source(37.5)
    v0 = gpu.scalars()["v0"]
    roul = split = 0
    for n in range(80):
        gpu.step(1)
        ref.step(1)
        sg, so = gpu.stats(), ref.stats()
        for k in STAT_INT:
            assert sg[k] == so[k], (n, k, sg[k], so[k])
        assert sg["w_j"] == so["w_j"]
        assert sg["w_e"] == pytest.approx(so["w_e"], rel=1e-9)
        roul += so["roulette"]
        split += so["split"]
    assert gpu.sync() == 0
    assert roul > 0 and split > 0
    for sp in (0, 1):
        compare_populations(gpu.read(sp), ref.read(sp), 1e-12 * inst.cells, 1e-12, v0,
                            label=f"species {sp}")
    assert np.allclose(gpu.fields()[2], ref.fields()[2], rtol=1e-11)


def test_sources_of_a_batch_under_graph_replay_match_oracles(xs_argon):
    """Three instances with their own sources (off, fractional, whole) in
    one handle stepped by graph replays, one source switched off and one on
    between replays: each instance equals its own oracle."""
    insts = [_gap(n_seed=300, n_target=0, capacity=20000),
             _gap(n_seed=500, n_target=800, V=350.0),
             _gap(n_seed=0, n_target=0, capacity=20000, cells=100)]
    run = configs.Run(precision=64)
    gpu = slpic.Sim(insts, run, xs_argon)
    gpu.use_graph(True)
    refs = [oracle.Sim(x, run, xs_argon, instance_index=k) for k, x in enumerate(insts)]
    plan = [(0.0, 12.25, 3.0), (0.0, 0.0, 3.0), (5.0, 0.0, 3.0)]
    for rates in plan:
        for k, r in enumerate(rates):
            gpu.set_source(r, inst=k)
            refs[k].set_source(r)
        gpu.step(16)
        for ref in refs:
            ref.step(16)
        assert gpu.sync() == 0
        for k, ref in enumerate(refs):
            sg, so = gpu.stats(inst=k), ref.stats()
            for key in STAT_INT:
                assert sg[key] == so[key], (rates, k, key, sg[key], so[key])
    for k, (x, ref) in enumerate(zip(insts, refs)):
        v0 = gpu.scalars(k)["v0"]
        for sp in (0, 1):
            compare_populations(gpu.read(sp, k), ref.read(sp), 1e-12 * x.cells, 1e-12, v0,
                                label=f"inst {k} sp {sp}")
    assert gpu.count(0, 2) > 0


@pytest.mark.parametrize("precision", [64, 32])
def test_steady_beam_weighs_the_physical_beam(precision):
    """Sec. II.B: a steady collisionless beam from the cathode weighs, in
    density weight beta w_j, what the physical beam holds below x: the rate
    per_step w_j0 / dt times the physical time sqrt(2 x / a) to reach x.
    The markers of a steady state have ages 0, 1, 2, ... steps; beta does
    not grow along an orbit that speeds up, so the weight lies within one
    step's injection above that value (FP32 positions may move a marker
    across x: one more step either way).  One handle runs the SLPIC gap
    (v0 = v_max / 10) and the PIC gap."""
    V, d, cells, per_step = 300.0, 0.01, 256, 4
    v_max = math.sqrt(2 * QE * V / ME)
    insts = [configs.Instance(d=d, p_torr=1.0, V=V, cells=cells, gamma_se=0.0, v_limit=vl,
                              seed_mode=configs.SEED_NONE, capacity=20000)
             for vl in (0.1 * v_max, math.inf)]
    run = configs.Run(precision=precision, area=1e30, cfl=0.5, w_j0=3.0)
    sim = slpic.Sim(insts, run, xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0))
    for k in range(2):
        sim.set_source(per_step, inst=k)
    steps = 1400  # the PIC beam crosses in 1024 steps, the SLPIC beam in about 520
    sim.step(steps)
    assert sim.sync() == 0
    a = QE * V / (ME * d)
    slack = 0.0 if precision == 64 else 1.0
    for k in range(2):
        h = sim.history(steps - 40, 40, inst=k)
        assert np.all(h["abs_e_anode"] == per_step) and np.all(h["abs_e_cathode"] == 0)
        sc = sim.scalars(k)
        pop = sim.read(0, k)
        x = (pop["cell"] + pop["off"]) * sc["dx"]
        speed = np.sqrt(pop["vx"] ** 2 + pop["vy"] ** 2 + pop["vz"] ** 2)
        with np.errstate(divide="ignore"):
            beta = np.minimum(1.0, sc["v0"] / speed) if math.isfinite(sc["v0"]) else np.ones_like(speed)
        rate = per_step * run.w_j0 / sc["dt"]
        for frac in (0.07, 0.23, 0.51, 0.77, 0.999):
            S = run.w_j0 * beta[x < frac * d].sum()
            excess = (S - rate * math.sqrt(2 * frac * d / a)) / (per_step * run.w_j0)
            print(f"inst {k} fp{precision} x = {frac:.2f} d: excess {excess:.3f} steps")
            # rounding, relative to the weight below x (in steps of injection)
            tol = (1e-9 if precision == 64 else 1e-5) * S / (per_step * run.w_j0)
            assert -slack - tol <= excess < 1.0 + slack + tol, (k, frac, excess)
        # the deposit carries the same weight: total electron charge of the
        # statistics row
        assert sim.stats(inst=k)["w_e"] == pytest.approx(run.w_j0 * beta.sum(),
                                                         rel=1e-12 if precision == 64 else 1e-5)


def test_set_source_rejects_bad_arguments(xs_argon):
    sim = slpic.Sim([_gap()], configs.Run(precision=32), xs_argon)
    for inst, rate in ((1, 1.0), (-1, 1.0), (0, -1.0), (0, math.nan), (0, math.inf), (0, 2.0 ** 25)):
        with pytest.raises(slpic.SlpicError):
            sim.set_source(rate, inst=inst)
    sim.set_source(0.0)
    sim.step(2)
    assert sim.sync() == 0


def test_source_overflowing_the_capacity_is_reported_and_stays_in_bounds():
    """A source larger than the instance holds: the injections that do not
    fit are dropped (never written past a partition), the step reports
    SLPIC_CAPACITY_EXCEEDED, and a neighbouring instance in the same batch
    is untouched (it equals the same instance stepped alone)."""
    import dataclasses
    small = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.0,
                             seed_mode=configs.SEED_NONE, capacity=1000)
    other = _gap(n_seed=500, n_target=0, capacity=20000)
    xs = xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0)
    run = configs.Run(precision=32)
    sim = slpic.Sim([small, other], run, xs)
    sim.set_source(700.0, inst=0)      # more than the capacity within two steps
    alone = slpic.Sim([dataclasses.replace(other, stream=1)], run, xs)
    sim.step(6)
    alone.step(6)
    with pytest.raises(slpic.SlpicError) as ei:
        sim.sync()
    assert ei.value.code == -3
    assert alone.sync() == 0
    occ, cap_p = sim.partitions(0, inst=0)
    assert np.all(np.asarray(occ) <= cap_p)
    assert sim.count(0, 0) <= len(occ) * cap_p
    # the neighbour is exactly what it is alone
    for sp in (0, 1):
        compare_populations(alone.read(sp), sim.read(sp, 1), 0.0, 0.0,
                            alone.scalars()["v0"], label=f"neighbour sp {sp}")


def test_source_and_flux_with_the_cell_sort_equal_an_unsorted_run(xs_argon):
    """FP64: a run with a cathode source and the flux diagnostic, cell-sorted
    every 4 steps, equals the same run unsorted bit for bit (the sort moves
    markers, including injected ones, without changing them, and nothing in
    a step depends on their order)."""
    inst = _gap(n_seed=800, n_target=1500)
    sims = []
    for rp in (0, 4):
        sim = slpic.Sim([inst], configs.Run(precision=64, resort_period=rp), xs_argon,
                        flags=slpic.FLAG_FLUX)
        sim.set_source(20.5)
        sim.step(24)
        assert sim.sync() == 0
        sims.append(sim)
    a, b = sims
    ha, hb = a.history(0, 24), b.history(0, 24)
    for f in STAT_INT + ["w_e", "w_i", "w_j"]:
        assert np.array_equal(ha[f], hb[f]), f
    for sp in (0, 1):
        compare_populations(a.read(sp), b.read(sp), 0.0, 0.0, a.scalars()["v0"],
                            label=f"species {sp}")
        assert np.array_equal(a.flux(sp), b.flux(sp))
    assert np.array_equal(a.fields()[2], b.fields()[2])
