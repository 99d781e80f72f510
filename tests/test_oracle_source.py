"""Pins of the oracle's continuous cathode source.

Sec. IV seeds electrons at rest at the cathode; the source repeats that
seeding every step at a fixed physical rate, per_step w_j0 / dt.  Sec. II.B:
the speed-limited equations are exact in steady state, because a marker slowed
by beta carries density weight beta w_j (Eq. 7, the passage after Eq. 11), so
a steady beam must weigh what the physical beam holds: the rate times the
physical time its particles spend in a region.
"""

import math

import numpy as np
import pytest

import oracle
from synth import configs, xsec
from synth.constants import QE, ME


def _beam_gap(v_limit, cells, V=300.0, d=0.01):
    # no collisions (zero fixed probabilities), no seeds, no secondary
    # emission; a huge electrode area makes the space charge negligible, so
    # the field is the vacuum field V / d
    return configs.Instance(d=d, p_torr=1.0, V=V, cells=cells, gamma_se=0.0,
                            v_limit=v_limit, seed_mode=configs.SEED_NONE,
                            capacity=200000)


def _collisionless():
    return xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0)


def _run_to_steady_state(sim, per_step, max_steps):
    # steady once every step absorbs at the anode what a step injects
    calm = 0
    for n in range(max_steps):
        sim.step(1)
        st = sim.stats()
        assert st["abs_e_cathode"] == 0 and st["err"] == 0
        calm = calm + 1 if st["abs_e_anode"] == per_step else 0
        if calm == 40:
            return n + 1
    raise AssertionError("no steady state")


@pytest.mark.parametrize("v_frac", [0.1, math.inf])
def test_steady_beam_weighs_the_physical_beam(v_frac):
    # Electrons from rest in a uniform field: a particle reaches x after the
    # physical time T(x) = sqrt(2 x / a).  In steady state the markers at the
    # end of a step have ages 0, 1, 2, ... steps, per_step of each, and the
    # age-m markers sit where the physical orbit is after the physical time
    # of m steps of proper time, t(m dt) = integral of beta over them.  beta
    # does not grow along an orbit that speeds up, so the sum of beta over
    # the ages found below x (a left Riemann sum) lies within one step of
    # T(x) / dt, from above:
    #   0 <= w_j0 sum_{x_p < x} beta_p - (per_step w_j0 / dt) T(x) < per_step w_j0.
    # Weighting markers by w_j instead of beta w_j would break this by the
    # factor 1 / beta (up to 10 here).
    V, d, cells, per_step = 300.0, 0.01, 256, 4
    v_max = math.sqrt(2 * QE * V / ME)
    inst = _beam_gap(v_frac * v_max, cells, V, d)
    run = configs.Run(precision=64, area=1e30, cfl=0.5, w_j0=3.0)
    sim = oracle.Sim(inst, run, _collisionless())
    sim.set_source(per_step)
    sc = sim.scalars()
    dt, v0 = sc["dt"], sc["v0"]
    steps = _run_to_steady_state(sim, per_step, 4000)
    pop = sim.read(0)
    x = (pop["cell"] + pop["off"]) * sc["dx"]
    speed = np.sqrt(pop["vx"] ** 2 + pop["vy"] ** 2 + pop["vz"] ** 2)
    with np.errstate(divide="ignore"):  # the age-0 markers are at rest: beta = 1
        beta = np.minimum(1.0, v0 / speed) if math.isfinite(v0) else np.ones_like(speed)
    assert np.all(pop["vy"] == 0) and np.all(pop["vz"] == 0)
    a = QE * V / (ME * d)
    rate = per_step * run.w_j0 / dt
    # the beam crosses the gap in T(d) = 2 d / v_max: about 0.2 (cells / cfl)
    # SLPIC steps or 2 (cells / cfl) PIC steps, so the bound is a few percent
    # of the beam's weight or less
    assert math.sqrt(2 * d / a) / dt > 100
    # (fractions whose physical times are not whole PIC steps)
    for frac in (0.07, 0.23, 0.51, 0.77, 0.999):
        xx = frac * d
        S = run.w_j0 * beta[x < xx].sum()
        excess = S - rate * math.sqrt(2 * xx / a)
        tol = 1e-9 * S
        print(f"x = {frac:.3f} d: weight {S:.1f}, excess {excess / (per_step * run.w_j0):.3f} step(s)")
        assert -tol <= excess < per_step * run.w_j0 + tol, (frac, S, excess, steps)
    # the statistics row holds the same weight
    assert sim.stats()["w_e"] == pytest.approx(run.w_j0 * beta.sum(), rel=1e-12)


def test_fractional_rate_injects_floor_or_one_more():
    # per_step = 2.25: each step injects 2 or 3 electrons, 3 with
    # probability 1/4.  Collisionless electrons only leave at the anode, so
    # the injections of step k are n_e(k) - n_e(k-1) + absorbed(k).
    inst = _beam_gap(0.0, 32)
    run = configs.Run(precision=64, area=1e30)
    sim = oracle.Sim(inst, run, _collisionless())
    sim.set_source(2.25)
    prev, inj = 0, []
    for _ in range(1600):
        sim.step(1)
        st = sim.stats()
        inj.append(st["n_e"] - prev + st["abs_e_anode"] + st["abs_e_cathode"])
        prev = st["n_e"]
    inj = np.array(inj)
    assert set(np.unique(inj)) == {2.0, 3.0}
    k = (inj == 3).sum()
    n = len(inj)
    assert abs(k - n / 4) < 4 * math.sqrt(n * 0.25 * 0.75), k


def test_source_keeps_its_physical_rate_under_population_control():
    # Roulette doubles w_j and splitting halves it; the source then injects
    # per_step w_j0 / w_j markers, so that markers times weight stays
    # per_step w_j0 per step.  Per step, injections = n_out - n_in +
    # absorbed + roulette removals - split clones.
    per_step = 3.0
    inst = _beam_gap(0.0, 32)
    inst.n_target = 40
    run = configs.Run(precision=64, area=1e30, w_j0=1.0)
    sim = oracle.Sim(inst, run, _collisionless())
    sim.set_source(per_step)
    w_prev, wants, got, roul, split = run.w_j0, [], [], 0, 0
    for _ in range(3000):
        sim.step(1)
        st = sim.stats()
        n = st["n_e"] - st["n_in"] + st["abs_e_anode"] + st["abs_e_cathode"] + st["roulette"] - st["split"]
        want = per_step * run.w_j0 / w_prev
        # the step's injections, before its own population control
        assert n in (math.floor(want), math.floor(want) + 1), (want, n)
        wants.append(want)
        got.append(n)
        roul += st["roulette"]
        split += st["split"]
        w_prev = st["w_j"]
    wants, got = np.array(wants), np.array(got)
    assert roul > 0 and split > 0
    assert np.any(wants != np.floor(wants)), "never a fractional rate"
    # the extra marker is a Bernoulli draw of the fraction
    f = wants - np.floor(wants)
    sd = math.sqrt((f * (1 - f)).sum())
    assert abs((got - wants).sum()) < 4 * sd + 1e-9


def test_set_source_rejects_bad_rates():
    sim = oracle.Sim(_beam_gap(0.0, 16), configs.Run(precision=64), _collisionless())
    for bad in (-1.0, math.inf, math.nan, 2.0 ** 25):
        with pytest.raises(ValueError):
            sim.set_source(bad)
    sim.set_source(0.0)
    sim.step(3)
    assert sim.count(oracle.ELECTRON) == 0
