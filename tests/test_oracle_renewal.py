"""Pins of the oracle's electron multiplication, and of the breakdown voltage
it implies, against the renewal equation of the Townsend test gas.

The breakdown condition of Sec. I (a generation of ions reproduces itself
through secondary emission, gamma (M - 1) = 1) is evaluated for a gas whose
multiplication M has an independent solution: one ionization channel with a
constant cross section above I = 15.76 eV, products at rest (tests/renewal.py
states both the continuous and the time-stepped process).  The oracle's
Monte Carlo must follow the stepped process it implements, and the stepped
process must converge to the continuous one as the step shrinks; together
they show where the oracle's breakdown voltage at the workload's step
(672.8 V at 128 cells and CFL 0.5) departs from the continuum value
(639.9 V) and why.
"""

import math

import numpy as np
import pytest

import oracle
from synth import configs, xsec
from renewal import (breakdown_voltage, continuum_multiplication,
                     discrete_multiplication, gas_density)

SIGMA, I_EV, D, P_TORR, GAMMA = 1e-20, 15.76, 0.01, 1.0, 0.07


def test_continuum_solver_matches_closed_forms_on_short_gaps():
    # on d < 2 l_I the delay term is 1: A(0) = 2 - exp(-c (d - l_I)); on
    # 2 l_I <= d < 3 l_I it is the first piece again, which integrates to
    # A = 4 - (2 + exp(-c l_I)) exp(-c s) - 2 c s exp(-c s), s = d - 2 l_I
    c = gas_density(P_TORR) * SIGMA
    for V in (672.0, 300.0):
        lI = I_EV * D / V
        for frac in (1.4, 1.9):
            d = frac * lI
            got = continuum_multiplication(V * d / D, d, P_TORR, SIGMA, I_EV)
            # V scaled with d keeps the field, hence l_I
            assert got == pytest.approx(2 - math.exp(-c * (d - lI)), rel=1e-7)
        for frac in (2.3, 2.9):
            d = frac * lI
            s = d - 2 * lI
            want = 4 - (2 + math.exp(-c * lI)) * math.exp(-c * s) - 2 * c * s * math.exp(-c * s)
            got = continuum_multiplication(V * d / D, d, P_TORR, SIGMA, I_EV)
            assert got == pytest.approx(want, rel=1e-7)


def test_stepped_multiplication_converges_to_the_continuum():
    # at the workload's grid (128 cells) the multiplication of the stepped
    # process approaches the continuum at first order as the step halves
    V = 672.0
    cont = continuum_multiplication(V, D, P_TORR, SIGMA, I_EV)
    errs = []
    for k in range(5):
        disc = discrete_multiplication(V, D, P_TORR, SIGMA, I_EV, 128, 0.5 / 2 ** k)
        errs.append(cont - disc)
    print("continuum", cont, "errors", errs)
    assert all(e > 0 for e in errs)
    for a, b in zip(errs, errs[1:]):
        assert 0.4 < b / a < 0.6, errs
    assert errs[-1] < 0.002 * cont


def test_breakdown_voltage_at_the_workload_step_and_in_the_continuum():
    # the end-of-step threshold test delays the first ionization by up to a
    # step; at 128 cells and CFL 0.5 (the statistics workload) that moves
    # the breakdown voltage from the continuum value up by about 33 V
    def stepped(V):
        return discrete_multiplication(V, D, P_TORR, SIGMA, I_EV, 128, 0.5)

    def cont(V):
        return continuum_multiplication(V, D, P_TORR, SIGMA, I_EV)
    vb_step = breakdown_voltage(stepped, GAMMA, 600.0, 760.0, xtol=0.01)
    vb_cont = breakdown_voltage(cont, GAMMA, 600.0, 700.0, xtol=0.01)
    print("V_b stepped", vb_step, "continuum", vb_cont)
    assert vb_step == pytest.approx(672.8, abs=0.2)
    assert vb_cont == pytest.approx(639.9, abs=0.2)
    # first-order convergence of V_b is masked by the staircase of the
    # threshold step count, but the error shrinks with the step
    errs = [abs(breakdown_voltage(
        lambda V, f=0.5 / 2 ** k: discrete_multiplication(V, D, P_TORR, SIGMA, I_EV, 128, f),
        GAMMA, 560.0, 760.0, xtol=0.01) - vb_cont) for k in (0, 2, 4)]
    print("V_b errors at CFL 0.5, 0.125, 0.03125:", errs)
    assert errs[0] > 25 and errs[1] < errs[0] / 2 and errs[2] < errs[1] / 2


def _oracle_multiplication(cells, cfl, V, batches=10, seeds=2000):
    xs = xsec.constant([(xsec.IONIZATION, SIGMA)], [I_EV])
    inst = configs.Instance(d=D, p_torr=P_TORR, V=V, cells=cells, gamma_se=0.0,
                            seed_mode=configs.SEED_CATHODE, n_seed=seeds)
    run = configs.Run(precision=64, area=1e30, cfl=cfl)
    means = []
    for b in range(batches):
        sim = oracle.Sim(inst, run, xs, instance_index=b, flags=oracle.FLAG_PRODUCTS_AT_REST)
        anode = 0
        for _ in range(40 * cells):
            sim.step(1)
            anode += sim.stats()["abs_e_anode"]
            if sim.count(oracle.ELECTRON) == 0:
                break
        assert sim.count(oracle.ELECTRON) == 0
        means.append(anode / seeds)
    m = np.array(means)
    return m.mean(), m.std(ddof=1) / math.sqrt(batches)


@pytest.mark.parametrize("cells,cfl,V", [(32, 1.0, 500.0), (32, 1.0, 672.0), (64, 0.5, 672.0)])
def test_oracle_multiplication_follows_the_stepped_process(cells, cfl, V):
    # grids coarse enough that the stepped process differs from the
    # continuum by 5-20 %: the oracle's Monte Carlo must give the stepped
    # value (end-of-step threshold test, null-collision probability per
    # step, the short first step from rest) and not the continuum's
    mean, se = _oracle_multiplication(cells, cfl, V)
    disc = discrete_multiplication(V, D, P_TORR, SIGMA, I_EV, cells, cfl)
    cont = continuum_multiplication(V, D, P_TORR, SIGMA, I_EV)
    print(cells, cfl, V, "oracle", mean, "+-", se, "stepped", disc, "continuum", cont)
    assert abs(mean - disc) < 4 * se
    assert abs(mean - cont) > 4 * se
