"""Parity of the weight-splitting collision strategy (Sec. III) with the
oracle: markers carry their own flux weights, a colliding candidate splits
into an uncollided remainder and a collided part that carries the fraction
f = max(s, P) of its weight, and products carry f (see slpic_config's
split_frac)."""

import numpy as np
import pytest

import oracle
import synth
from synth import configs, xsec
from parity import compare_populations, STAT_INT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402


def _gaps():
    return [configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.2,
                             seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=3000,
                             n_target=4000, capacity=40000),
            configs.Instance(d=0.02, p_torr=3.0, V=450.0, cells=400, gamma_se=0.1,
                             seed_mode=configs.SEED_CATHODE, n_seed=500,
                             n_target=3000, capacity=60000)]


@pytest.mark.parametrize("s", [0.5, 0.1])
def test_fp64_split_strategy_matches_oracle_step_by_step(s, xs_argon):
    """Two uneven instances in one batch, full physics with charge exchange,
    emission (emitted electrons carry their ion's weight) and population
    control: every integer statistic bit-exact every step, totals within
    1e-9, and at the end markers, their flux weights and fields within
    1e-12."""
    insts = _gaps()
    run = configs.Run(precision=64, split_frac=s)
    gpu = slpic.Sim(insts, run, xs_argon)
    refs = [oracle.Sim(x, run, xs_argon, instance_index=k) for k, x in enumerate(insts)]
    ions = synth.markers.ions(21, 2000, 64, cell_hi=10, e_beam_hi=800.0)
    gpu.load(1, ions, inst=0)
    refs[0].load(1, ions)
    split_seen = 0
    for n in range(40):
        gpu.step(1)
        for r in refs:
            r.step(1)
        for k in range(len(insts)):
            sg, so = gpu.stats(inst=k), refs[k].stats()
            for key in STAT_INT:
                assert sg[key] == so[key], (n, k, key, sg[key], so[key])
            assert sg["w_j"] == so["w_j"]
            assert sg["w_e"] == pytest.approx(so["w_e"], rel=1e-9)
            assert sg["w_i"] == pytest.approx(so["w_i"], rel=1e-9, abs=1e-9)
    assert gpu.sync() == 0
    for k, x in enumerate(insts):
        v0 = gpu.scalars(k)["v0"]
        for sp in (0, 1):
            ref = refs[k].read(sp)
            split_seen += int(np.count_nonzero(ref["w"] < 1.0))
            w = compare_populations(gpu.read(sp, k), ref, 1e-12 * x.cells, 1e-12, v0,
                                    tol_w=1e-12, label=f"s={s} inst {k} sp {sp}")
            print("split", s, k, sp, w["n"], w["x_cells"], w["vx"], w["w"])
        E_g, E_o = gpu.fields(inst=k)[2], refs[k].fields()[2]
        assert np.allclose(E_g, E_o, rtol=0, atol=1e-11 * np.abs(E_o).max())
    assert split_seen > 1000


def test_fp64_split_fixed_events_match_oracle():
    """Fixed-event mode with splitting: candidates by the split threshold,
    channels by the second word."""
    xs = xsec.fixed_event([0.1, 0.05, 0.03], probs_cx=0.1)
    inst = _gaps()[0]
    run = configs.Run(precision=64, split_frac=0.3)
    gpu = slpic.Sim([inst], run, xs)
    ref = oracle.Sim(inst, run, xs)
    for n in range(25):
        gpu.step(1)
        ref.step(1)
        sg, so = gpu.stats(), ref.stats()
        for key in STAT_INT:
            assert sg[key] == so[key], (n, key, sg[key], so[key])
    assert gpu.sync() == 0
    v0 = gpu.scalars()["v0"]
    for sp in (0, 1):
        compare_populations(gpu.read(sp), ref.read(sp), 1e-12 * inst.cells, 1e-12, v0,
                            tol_w=1e-12, label=f"fixed sp {sp}")


def test_fp32_split_single_step(xs_argon):
    """FP32 particles with splitting: one step from a loaded state, states
    within 1e-5, weights within 1e-6, ties within 1e-6 excused."""
    cells = 64
    inst = configs.Instance(d=0.01, p_torr=3.0, V=300.0, cells=cells, gamma_se=0.3,
                            seed_mode=configs.SEED_NONE, capacity=60000)
    e, i = synth.markers.mixed(7, 9000, 4100, cells)
    gpu = slpic.Sim([inst], configs.Run(precision=32, split_frac=0.4), xs_argon)
    ref = oracle.Sim(inst, configs.Run(precision=64, split_frac=0.4), xs_argon)
    for sim in (gpu, ref):
        sim.load(0, e)
        sim.load(1, i)
    gpu.step(1)
    ref.step(1)
    assert gpu.sync() == 0
    v0 = gpu.scalars()["v0"]
    tied = 0
    for sp in (0, 1):
        n = ref.count(sp)
        w = compare_populations(gpu.read(sp), ref.read(sp), 1e-5 * cells, 1e-5, v0,
                                tie_tol=1e-6, max_tied=n // 1000, tol_w=1e-6,
                                label=f"fp32 split sp {sp}")
        tied += w["tied"]
    sg, so = gpu.stats(), ref.stats()
    for k in STAT_INT:
        assert abs(sg[k] - so[k]) <= tied, (k, sg[k], so[k])


def test_split_with_the_flux_diagnostic_is_rejected(xs_argon):
    with pytest.raises(slpic.SlpicError):
        slpic.Sim(_gaps()[:1], configs.Run(precision=64, split_frac=0.5), xs_argon,
                  flags=slpic.FLAG_FLUX)
