"""Pins of the oracle's speed-limited push (Eqs. 8-11) and time step rules."""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth
from synth import configs
from synth.constants import QE, ME, M_AR
from conftest import golden_rows

V0 = 3.807e4
DT = 2.052e-9


def test_beta_worked_example():
    # Sec. II.B: v = 10 v0 gives beta = 0.1; w_j = 100 gives w_p = 10
    for v_over, b_want, wj, wp in golden_rows("worked_example_flux_weight.txt"):
        b = oracle.beta(float(v_over) * V0, V0)
        assert b == pytest.approx(float(b_want), rel=1e-15)
        assert b * float(wj) == pytest.approx(float(wp), rel=1e-15)


def test_beta_piecewise():
    assert oracle.beta(V0, V0) == 1.0            # v >= v0 branch, v0/v0
    assert oracle.beta(0.0, V0) == 1.0           # slow branch
    assert oracle.beta(0.5 * V0, V0) == 1.0
    assert oracle.beta(4 * V0, V0) == 0.25
    assert oracle.beta(1e9, math.inf) == 1.0     # beta == 1: PIC


def _ode_flight(vx, vperp, a, dt, v0):
    """Integrate Eqs. (8)-(9) with beta from Eq. (11) numerically."""
    def f(t, y):
        v = math.hypot(y[1], vperp)
        b = v0 / v if v >= v0 else 1.0
        return [b * y[1], b * a]
    scale = max(abs(vx), abs(a) * dt, v0)
    r = solve_ivp(f, [0, dt], [0.0, vx], method="DOP853", rtol=1e-12,
                  atol=[1e-18, 1e-12 * scale], max_step=dt / 64)
    return r.y[0, -1], r.y[1, -1]


def test_free_flight_matches_ode():
    rng = np.random.default_rng(11)
    a0 = QE / ME * 3e4
    cases = [(0.0, 0.0, a0), (0.0, 0.0, -a0), (1e6, 0.0, -a0),
             (-2e5, 3e5, a0), (3e4, 1e4, a0 * 1e-3)]
    for _ in range(25):
        vx, vp = rng.normal(0, 1, 2) * 10 ** rng.uniform(3, 7)
        cases.append((vx, abs(vp), a0 * rng.choice([1, -1, 0.02])))
    for vx, vp, a in cases:
        tau, dx, vx1 = oracle.free_flight(vx, vp, a, DT, V0)
        xo, vo = _ode_flight(vx, vp, a, DT, V0)
        assert dx == pytest.approx(xo, rel=2e-8, abs=1e-14)
        assert vx1 == pytest.approx(vo, rel=2e-8, abs=1e-6 * V0)
        assert 0 < tau <= DT


def test_free_flight_phase_path_invariants():
    # in a uniform field the SLPIC orbit is the PIC phase path (Sec. II.B):
    # v_x^2 - 2 a x is conserved, and the pseudo speed never exceeds v0
    rng = np.random.default_rng(5)
    a0 = QE / ME * 3e4
    for _ in range(200):
        vx, vp = rng.normal(0, 1, 2) * 10 ** rng.uniform(2, 7)
        a = a0 * rng.uniform(-1, 1)
        tau, dx, vx1 = oracle.free_flight(vx, abs(vp), a, DT, V0)
        assert abs(dx) <= V0 * DT * (1 + 1e-12)
        lhs = vx1 * vx1 - vx * vx
        assert lhs == pytest.approx(2 * a * dx, rel=1e-9,
                                    abs=1e-9 * (vx * vx + vx1 * vx1))


def test_free_flight_time_closed_form():
    # for |v| > v0 throughout, dt = [s|v| + c^2 ln(s + |v|)] / (2 a v0)
    # evaluated between the end points (s = v_x, c = |v_perp|)
    def t_of(s, c, a):
        w = math.hypot(s, c)
        return (s * w + c * c * math.log(s + w)) / (2 * a * V0)
    a = QE / ME * 3e4
    for vx, c in [(2e6, 1e5), (5e5, 4e5), (1e7, 3e6), (1e5, 2e5)]:
        tau, dx, vx1 = oracle.free_flight(vx, c, a, DT, V0)
        assert t_of(vx1, c, a) - t_of(vx, c, a) == pytest.approx(DT, rel=1e-10)


def test_pic_limit_is_exact_parabola():
    # v0 = +inf: beta == 1 and the flight is x = v t + a t^2 / 2 exactly
    for vx, a in [(1e5, 3e15), (-2e6, 5e14), (0.0, -1e16)]:
        tau, dx, vx1 = oracle.free_flight(vx, 1e5, a, DT, math.inf)
        assert tau == DT
        assert dx == vx * DT + 0.5 * a * DT * DT
        assert vx1 == vx + a * DT


def _collisionless(v_limit=0.0, V=300.0, cells=64):
    inst = configs.Instance(d=0.01, p_torr=0.0, V=V, cells=cells,
                            gamma_se=0.0, v_limit=v_limit,
                            seed_mode=configs.SEED_NONE)
    # a huge electrode area makes the markers' own space charge negligible,
    # so E = -V/d to rounding
    return inst, configs.Run(precision=64, area=1e30)


def test_ballistic_orbits_pic_uniform_field():
    inst, run = _collisionless(v_limit=math.inf)
    sim = oracle.Sim(inst, run, synth.argon_like())
    sc = sim.scalars()
    dt, dx = sc["dt"], sc["dx"]
    assert dt == pytest.approx(run.cfl * dx / math.sqrt(2 * QE * 300 / ME))
    pop = synth.markers.electrons(1, 200, 64, e_lo=0.01, e_hi=5.0,
                                  cell_lo=20, cell_hi=30)
    sim.load(oracle.ELECTRON, pop)
    a = QE / ME * 300 / 0.01   # E = -V/d exactly without space charge
    x0 = (pop["cell"] + pop["off"]) * dx
    n = 7
    sim.step(n)
    out = sim.read(oracle.ELECTRON)
    order = np.argsort(out["id"])
    ref = np.argsort(pop["id"])
    t = n * dt
    x_want = x0[ref] + pop["vx"][ref] * t + 0.5 * a * t * t
    x_got = (out["cell"][order] + out["off"][order]) * dx
    # the few markers that reached a wall are absent on both sides
    keep = np.isin(pop["id"][ref], out["id"])
    assert keep.sum() == len(out["id"])
    np.testing.assert_allclose(x_got, x_want[keep], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["vx"][order],
                               (pop["vx"][ref] + a * t)[keep], rtol=1e-13)


def test_slpic_multi_step_keeps_phase_path():
    inst, run = _collisionless()
    sim = oracle.Sim(inst, run, synth.argon_like())
    dx = sim.scalars()["dx"]
    pop = synth.markers.electrons(2, 300, 64, e_lo=0.001, e_hi=50.0,
                                  cell_lo=10, cell_hi=20)
    sim.load(oracle.ELECTRON, pop)
    a = QE / ME * 300 / 0.01
    sim.step(40)
    out = sim.read(oracle.ELECTRON)
    m = {int(i): k for k, i in enumerate(pop["id"])}
    for k in range(len(out["id"])):
        j = m[int(out["id"][k])]
        x0 = (pop["cell"][j] + pop["off"][j]) * dx
        x1 = (out["cell"][k] + out["off"][k]) * dx
        inv0 = pop["vx"][j] ** 2 - 2 * a * x0
        inv1 = out["vx"][k] ** 2 - 2 * a * x1
        assert inv1 == pytest.approx(inv0, rel=1e-9, abs=1e-9 * out["vx"][k] ** 2)
        assert abs(x1 - x0) <= 40 * 0.5 * dx * (1 + 1e-12)


def test_time_step_rules_reproduce_table_one():
    # Sec. IV: dt_SLPIC = dx / v0, v0 = sqrt(2 e V / m_Ar); runs last 30 ion
    # crossing times 30 sqrt(2 m_Ar d / (e E)); dt_PIC = dx / sqrt(2 e V/m_e)
    ratio = math.sqrt(M_AR / ME)
    for p, V, cells, nts, ntp in golden_rows("table1_steps.txt"):
        inst = configs.Instance(d=0.01, p_torr=float(p), V=float(V),
                                cells=int(cells), seed_mode=0)
        run = configs.Run(cfl=1.0)
        sim = oracle.Sim(inst, run, synth.argon_like())
        dt = sim.scalars()["dt"]
        E = float(V) / 0.01
        t_cross = math.sqrt(2 * M_AR * 0.01 / (QE * E))
        n_slpic = 30 * t_cross / dt
        assert n_slpic == pytest.approx(60 * int(cells), rel=1e-12)
        # Table I quotes two significant digits
        assert n_slpic == pytest.approx(float(nts), rel=0.03)
        if ntp != "NA":
            pic = oracle.Sim(configs.Instance(d=0.01, p_torr=float(p),
                                              V=float(V), cells=int(cells),
                                              v_limit=math.inf, seed_mode=0),
                             run, synth.argon_like())
            r = dt / pic.scalars()["dt"]
            assert r == pytest.approx(ratio, rel=1e-12)
            assert float(ntp) / float(nts) == pytest.approx(ratio, rel=0.03)
