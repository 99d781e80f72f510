"""The oracle taken over mid-run (set_clock + load), which the full-size
GPU comparison uses: a run continued from its own markers, step counter and
flux weight repeats the uninterrupted run, through population control (the
flux weight changes) and the draws keyed by step: every statistic and id
exactly, states within 1e-12 (the oracle keeps positions in metres, and
reading them out as cell and offset and loading them back rounds them)."""

import numpy as np
import pytest

import oracle
import synth
from synth import configs


def _inst(seed_mode, n_seed):
    return configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=seed_mode, n_seed=n_seed, n_target=800,
                            capacity=40000)


def test_a_run_continued_from_its_clock_repeats_itself():
    xs = synth.argon_like()
    run = configs.Run(precision=64)
    a = oracle.Sim(_inst(configs.SEED_MAXWELL_CELL0, 2000), run, xs, instance_index=3)
    a.step(30)
    sc = a.scalars()
    assert sc["w_j"] != run.w_j0  # population control has acted
    b = oracle.Sim(_inst(configs.SEED_NONE, 0), run, xs, instance_index=3)
    b.set_clock(int(sc["step"]), sc["w_j"])
    b.load(0, a.read(0))
    b.load(1, a.read(1))
    assert np.array_equal(a.fields()[2], b.fields()[2])
    for _ in range(5):
        a.step(1)
        b.step(1)
        assert a.stats() == b.stats()
    for sp in (0, 1):
        ra, rb = a.read(sp), b.read(sp)
        ia, ib = np.argsort(ra["id"]), np.argsort(rb["id"])
        for key in ("id", "cell"):
            assert np.array_equal(ra[key][ia], rb[key][ib]), (sp, key)
        for key in ("off", "vx", "vy", "vz"):
            x, y = ra[key][ia], rb[key][ib]
            assert np.allclose(x, y, rtol=1e-12, atol=1e-12 * np.abs(x).max()), (sp, key)
    # a different clock draws differently
    c = oracle.Sim(_inst(configs.SEED_NONE, 0), run, xs, instance_index=3)
    c.set_clock(int(sc["step"]) + 1, sc["w_j"])
    c.load(0, a.read(0))
    c.load(1, a.read(1))
    d = oracle.Sim(_inst(configs.SEED_NONE, 0), run, xs, instance_index=3)
    d.set_clock(int(sc["step"]), sc["w_j"])
    d.load(0, a.read(0))
    d.load(1, a.read(1))
    c.step(1)
    d.step(1)
    assert c.stats() != d.stats()


def test_set_clock_rejects_a_bad_weight():
    xs = synth.argon_like()
    s = oracle.Sim(_inst(configs.SEED_NONE, 0), configs.Run(precision=64), xs)
    with pytest.raises(ValueError):
        s.set_clock(10, 0.0)
    with pytest.raises(ValueError):
        s.set_clock(10, float("inf"))
