"""Pins of the oracle's weight-splitting collision strategy (Sec. III).

The paper states the flux-weight bookkeeping of a collision,
w_j,p0 = w_j,p1 + W_j,c with the collided part W_j,c carried by the
scattered primary and by every product, and that strategies which collide
whole markers with a reduced probability give the same expected W_c.  The
oracle writes both through one split fraction s (its collide_electron):
candidates with probability q = min(1, P/s), collided
fraction f = max(s, P).  These tests check, against closed forms and exact
conservation laws rather than the oracle's own formulas, that

  - flux weight is conserved in every event;
  - the expected collided weight per step equals the whole-marker one (the
    unscattered weight of a beam decays as exp(-x/lambda) for every s, the
    mean-free-path rule of Sec. III), while splitting lowers its variance;
  - the marker bookkeeping of split events balances exactly;
  - s = 1 is the whole-marker strategy, bit for bit.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from synth import configs, xsec


def _gap(V=0.0, v_limit=1e4, cells=64, p=1.0):
    return configs.Instance(d=0.01, p_torr=p, V=V, cells=cells, gamma_se=0.0,
                            v_limit=v_limit, seed_mode=configs.SEED_NONE,
                            capacity=1 << 22)


def _beam(n, speed, cell=30, seed=0):
    rng = np.random.default_rng(seed)
    z = np.zeros(n)
    return {"cell": np.full(n, cell, np.int32), "off": rng.uniform(0.0, 1.0, n),
            "vx": z + speed, "vy": z, "vz": z,
            "id": np.arange(1, n + 1, dtype=np.uint64)}


@pytest.mark.parametrize("s", [0.5, 0.1])
def test_split_events_conserve_flux_weight(s):
    # field-free, fixed events: elastic and excitation keep the electrons'
    # total flux weight, each ionization adds its collided weight to the
    # electrons and the same to the ions, charge exchange keeps the ions'
    xs = xsec.fixed_event([0.2, 0.1, 0.05], probs_cx=0.2)
    sim = oracle.Sim(_gap(), configs.Run(precision=64, area=1e30, split_frac=s), xs)
    e = _beam(2000, 2.0e6)
    i = _beam(1000, 100.0, seed=1)
    i["id"] += np.uint64(1 << 40)
    sim.load(oracle.ELECTRON, e)
    sim.load(oracle.ION, i)
    we0 = sim.read(0)["w"].sum()
    wi0 = sim.read(1)["w"].sum()
    for n in range(6):
        sim.step(1)
        ew, iw = sim.read(0)["w"], sim.read(1)["w"]
        st = sim.stats()
        assert st["abs_e_cathode"] + st["abs_e_anode"] + st["abs_i_cathode"] + st["abs_i_anode"] == 0
        assert np.all(ew > 0) and np.all(ew <= 1) and np.all(iw > 0) and np.all(iw <= 1)
        # electrons gain exactly what the ions gain: the ionized weight
        assert ew.sum() - we0 == pytest.approx(iw.sum() - wi0, abs=1e-9 * ew.sum())
    assert sim.count(0) > 2000 and ew.sum() > we0
    # expected ionized weight per step: P_ioniz of the electron weight
    # (f q = P for every candidate), within a loose statistical bound
    assert (iw.sum() - wi0) / we0 == pytest.approx(1.05 ** 6 - 1, rel=0.25)


def test_split_bookkeeping_balances_with_full_physics(xs_argon):
    # every real collision of a split run adds one marker (its scattered
    # part), an ionization one more electron and one ion; population control
    # (which splits add to: at 1 Torr P_null = 0.35 > s, so every electron
    # is a candidate every step) then removes or clones
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=3000,
                            n_target=3000, capacity=1 << 22)
    sim = oracle.Sim(inst, configs.Run(precision=64, split_frac=0.3), xs_argon)
    ions = synth.markers.ions(5, 1500, 64, cell_hi=8, e_beam_hi=500.0)
    sim.load(oracle.ION, ions)
    n_prev = sim.count(0) + sim.count(1)
    roulette = 0
    for n in range(40):
        sim.step(1)
        st = sim.stats()
        coll = st["elastic"] + st["excitation"] + st["ionization"] + st["cx"]
        absorbed = (st["abs_e_cathode"] + st["abs_e_anode"] + st["abs_i_cathode"]
                    + st["abs_i_anode"])
        pre = n_prev - absorbed + coll + 2 * st["ionization"] + st["see"]
        assert st["n_e"] + st["n_i"] == pre - st["roulette"] + st["split"], n
        n_prev = st["n_e"] + st["n_i"]
        roulette += st["roulette"]
        assert st["err"] == 0
        for sp in (0, 1):
            w = sim.read(sp)["w"]
            assert np.all((w > 0) & (w <= 1))
    assert roulette > 0
    assert sim.read(0)["w"].mean() < 0.9  # weights below 1 after splits


def _beam_survival(s, steps=10, n=20000, sigma=4e-20):
    # a speed-limited beam (v = 100 v0) in a field-free gap with a constant
    # elastic cross section: per step every marker is at the null-collision
    # bound, so its unscattered weight decays exactly as exp(-v0 dt / lambda)
    xs = xsec.constant([(xsec.ELASTIC, sigma)], [0.0])
    sim = oracle.Sim(_gap(v_limit=2e4, cells=400), configs.Run(precision=64, area=1e30,
                                                              split_frac=s), xs)
    beam = _beam(n, 2e6, cell=5)
    sim.load(oracle.ELECTRON, beam)
    sim.step(steps)
    out = sim.read(oracle.ELECTRON)
    # the uncollided part of original marker k keeps its id and velocity
    keep = (out["id"] <= np.uint64(n)) & (out["vy"] == 0.0) & (out["vz"] == 0.0)
    r = np.zeros(n)
    r[(out["id"][keep] - np.uint64(1)).astype(np.int64)] = out["w"][keep]
    sc = sim.scalars()
    lam = 1.0 / (sc["n_g"] * sigma)
    want = math.exp(-steps * sc["v0"] * sc["dt"] / lam)
    total = out["w"].sum()
    return r, want, total


@pytest.mark.parametrize("s", [1.0, 0.5, 0.1])
def test_split_keeps_the_mean_free_path(s):
    r, want, total = _beam_survival(s)
    se = r.std(ddof=1) / math.sqrt(r.size)
    print(s, "unscattered weight", r.mean(), "+-", se, "exact", want)
    assert abs(r.mean() - want) < 4 * se
    # elastic scattering only: no weight is created or lost
    assert total == pytest.approx(r.size, rel=1e-12)


def test_splitting_lowers_the_variance_of_the_unscattered_weight():
    r1, want, _ = _beam_survival(1.0)
    r2, _, _ = _beam_survival(0.1)
    assert r2.std() < 0.5 * r1.std()


def test_split_fraction_one_is_the_whole_marker_strategy(xs_argon):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=2000,
                            n_target=1500, capacity=1 << 20)
    a = oracle.Sim(inst, configs.Run(precision=64, split_frac=0.0), xs_argon)
    b = oracle.Sim(inst, configs.Run(precision=64, split_frac=1.0), xs_argon)
    a.step(30)
    b.step(30)
    for sp in (0, 1):
        pa, pb = a.read(sp), b.read(sp)
        for k in ("cell", "off", "vx", "vy", "vz", "id", "w"):
            assert np.array_equal(pa[k], pb[k]), (sp, k)
        assert np.all(pa["w"] == 1.0)
