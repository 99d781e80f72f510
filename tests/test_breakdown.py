"""Host logic of the breakdown classification and V_b search (Sec. IV)."""

import math

import numpy as np
import pytest

from paper_2103_12194_amd import breakdown as bd
from synth.constants import QE, M_AR


def test_crossing_time_and_table_one_step_count():
    # Sec. IV: 30 ion crossing times of sqrt(2 m_Ar d / (e E)), E = V/d; with
    # dt = dx / v0 (CFL 1) and v0 = sqrt(2 e V / m_Ar) that is 60 steps per
    # cell whatever V, as in Table I
    d, V = 0.01, 170.0
    tc = bd.crossing_time(d, V)
    assert tc == pytest.approx(math.sqrt(2 * M_AR * d / (QE * V / d)), rel=1e-15)
    cells = 219
    v0 = math.sqrt(2 * QE * V / M_AR)
    assert 30 * tc / ((d / cells) / v0) == pytest.approx(60 * cells, rel=1e-12)


def test_growth_rate_recovers_an_exponential():
    tc = 2e-6
    t = np.arange(1, 4001) * (40 * tc / 4000)
    for lam in (-0.7, 0.0, 0.31):
        pop = 123.0 * np.exp(lam * t / tc)
        assert bd.growth_rate(t, pop, tc) == pytest.approx(lam, abs=1e-12)
    # only the window counts: a different early slope does not matter
    pop = np.where(t < 15 * tc, np.exp(3.0 * t / tc), np.exp(45.0) * np.exp(0.2 * (t / tc - 15)))
    assert bd.growth_rate(t, pop, tc) == pytest.approx(0.2, abs=1e-10)


def test_growth_rate_extinction_and_short_windows():
    tc = 1.0
    t = np.arange(0, 40, 0.5)
    pop = np.exp(-t)
    pop[t > 20] = 0.0
    assert bd.growth_rate(t, pop, tc) == -math.inf
    with pytest.raises(ValueError):
        bd.growth_rate(np.array([1.0, 2.0, 16.0]), np.ones(3), tc)


def test_growth_rate_is_least_squares_slope():
    rng = np.random.default_rng(5)
    tc = 1.0
    t = np.linspace(0, 40, 801)
    pop = np.exp(0.1 * t + rng.normal(0, 0.3, t.size))
    sel = (t >= 15) & (t <= 30)
    want = np.polyfit(t[sel], np.log(pop[sel]), 1)[0]
    assert bd.growth_rate(t, pop, tc) == pytest.approx(want, rel=1e-10)


def test_ensemble_mean_and_standard_error():
    r = np.array([0.1, 0.3, -0.2, 0.05, 0.12])
    m, se = bd.ensemble(r)
    assert m == pytest.approx(r.mean())
    assert se == pytest.approx(r.std(ddof=1) / math.sqrt(5))
    assert bd.ensemble([0.1, -math.inf])[0] == -math.inf


def test_zero_crossing_of_a_linear_rate():
    V = [500.0, 600.0, 700.0]
    lam = [0.002 * (v - 640.0) for v in V]
    Vb, s = bd.zero_crossing(V, lam, [0.0, 0.0, 0.0])
    assert Vb == pytest.approx(640.0, abs=1e-9)
    assert s == 0.0
    # order of the inputs does not matter; no sign change gives None
    assert bd.zero_crossing(V[::-1], lam[::-1], [0, 0, 0])[0] == pytest.approx(640.0)
    assert bd.zero_crossing(V, [0.1, 0.2, 0.3], [0, 0, 0]) is None
    # an extinct (below) point next to the crossing is skipped
    assert bd.zero_crossing([400.0] + V, [-math.inf] + lam, [0, 0, 0, 0])[0] == pytest.approx(640.0)


def test_zero_crossing_error_matches_monte_carlo():
    rng = np.random.default_rng(11)
    V = [600.0, 700.0]
    lam = np.array([-0.06, 0.09])
    se = np.array([0.004, 0.006])
    Vb, s = bd.zero_crossing(V, lam, se)
    draws = []
    for _ in range(200000 // 100):
        la = lam[0] + se[0] * rng.standard_normal(100)
        lb = lam[1] + se[1] * rng.standard_normal(100)
        draws.append(V[0] - la * 100.0 / (lb - la))
    draws = np.concatenate(draws)
    assert Vb == pytest.approx(draws.mean(), abs=0.05)
    assert s == pytest.approx(draws.std(), rel=0.03)


def test_bracket_and_bisection_round():
    lo, hi = bd.bracket([300, 400, 500, 600], [False, False, True, True])
    assert (lo, hi) == (400, 500)
    assert bd.bracket([300], [True]) == (None, 300)
    v = bd.bisection_voltages(400.0, 500.0, 8)
    assert len(v) == 8 and v[0] == 400.0 and v[-1] == 500.0
    assert np.allclose(np.diff(v), 100.0 / 7)
    # six rounds of eight points shrink a bracket by 7^6
    lo, hi, Vb = 100.0, 1000.0, 643.21
    for _ in range(6):
        vs = bd.bisection_voltages(lo, hi, 8)
        lo, hi = bd.bracket(vs, [x > Vb for x in vs])
    assert lo < Vb < hi and hi - lo == pytest.approx(900.0 / 7 ** 6)


def test_paired_difference_cancels_shared_noise():
    # two ensembles that share replica noise: the paired standard error
    # sees only the part that differs
    rng = np.random.default_rng(3)
    common = rng.normal(0.0, 1.0, 400)
    a = common + 0.01 + rng.normal(0.0, 0.001, 400)
    b = common
    d, se = bd.paired_difference(a, b)
    assert d == pytest.approx(0.01, abs=4 * 0.001 / 20)
    assert se == pytest.approx(0.001 / 20, rel=0.2)
    # replicas extinct on both sides drop out; on one side only, +-inf
    a2 = np.append(a, -math.inf)
    b2 = np.append(b, -math.inf)
    assert bd.paired_difference(a2, b2)[0] == pytest.approx(d)
    assert bd.paired_difference(np.append(a, -math.inf), np.append(b, 0.0))[0] == -math.inf


def test_paired_breakdown_difference_on_linear_rates():
    # lambda(V) = (V - 600) / 200 + replica noise shared by both sides, and
    # side a shifted by 0.01 (so V_b moves down by 2 V)
    rng = np.random.default_rng(4)
    V = [500.0, 700.0]
    noise = rng.normal(0.0, 0.05, (2, 50))
    b = np.array([[(v - 600.0) / 200.0] * 50 for v in V]) + noise
    a = b + 0.01
    d, se = bd.paired_breakdown_difference(V, a, b)
    vb_b = bd.zero_crossing(V, b.mean(1), [0, 0])[0]
    vb_a = bd.zero_crossing(V, a.mean(1), [0, 0])[0]
    assert d == pytest.approx(vb_a - vb_b) and d == pytest.approx(-2.0, abs=0.01)
    # the shared noise cancels: the paired error is far below either
    # ensemble's own (propagated from the replica spread)
    own = bd.zero_crossing(V, b.mean(1), b.std(1, ddof=1) / math.sqrt(50))[1]
    assert own > 1.0 and se < own / 20
