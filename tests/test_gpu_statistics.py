"""Statistical parity of the HIP path with the oracle: ensemble growth rates
of the ion population and the breakdown voltage (Sec. IV classification).

Test gas: one ionization channel with a constant cross section (1e-20 m^2,
threshold 15.76 eV), both electrons of an ionization restarting at rest,
gamma_se = 0.07, d = 1 cm at 1 Torr, 128 cells (a step of 0.04 mm, several
steps to the threshold energy, so that the discrete process resolves the
field dependence).  Each voltage runs R replicas seeded at the cathode with
population control around 600 markers; replica k uses Philox key (seed, k)
on both sides, so the FP64 GPU run repeats the oracle's histories and the
FP32 run follows them until near-tie decisions part them.  Growth rates are
fitted over [15, 30] ion crossing times (30 crossing times = 120 steps per
cell at CFL 0.5).
"""

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from synth import configs, xsec
from paper_2103_12194_amd import breakdown as bd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402

VOLTS = (500.0, 750.0, 1100.0)
R = 12
CELLS = 128
STEPS = 120 * CELLS
EVERY = 8   # oracle samples of the ion population


def _gap(V):
    return configs.Instance(d=0.01, p_torr=1.0, V=V, cells=CELLS, gamma_se=0.07,
                            seed_mode=configs.SEED_CATHODE, n_seed=300,
                            n_target=600, capacity=8192)


def _gas():
    return xsec.constant([(xsec.IONIZATION, 1e-20)], [15.76])


@pytest.fixture(scope="module")
def setup():
    insts = [_gap(V) for V in VOLTS for _ in range(R)]
    xs = _gas()

    def one(k):
        sim = oracle.Sim(insts[k], configs.Run(precision=64), xs, instance_index=k,
                         flags=oracle.FLAG_PRODUCTS_AT_REST)
        w = np.empty(STEPS // EVERY)
        for n in range(STEPS // EVERY):
            sim.step(EVERY)
            w[n] = sim.stats()["w_i"]
        t = np.arange(1, STEPS // EVERY + 1) * EVERY * sim.scalars()["dt"]
        return bd.growth_rate(t, w, bd.crossing_time(insts[k].d, insts[k].V))

    with ThreadPoolExecutor(8) as ex:
        ref = np.array(list(ex.map(one, range(len(insts)))))
    return insts, xs, ref


def _gpu_rates(insts, xs, precision):
    sim = slpic.Sim(insts, configs.Run(precision=precision), xs,
                    flags=slpic.FLAG_PRODUCTS_AT_REST)
    steps, pops = bd.step_and_record(sim, STEPS)
    assert sim.sync() == 0
    keep = steps % EVERY == 0   # the oracle's sampling
    rates = bd.instance_rates(sim, insts, steps[keep], pops[:, keep])
    sim.close()
    return rates


def _per_voltage(rates):
    return [bd.ensemble(rates[v * R:(v + 1) * R]) for v in range(len(VOLTS))]


def test_fp64_replicas_repeat_the_oracle(setup):
    insts, xs, ref = setup
    got = _gpu_rates(insts, xs, 64)
    assert np.all(np.isfinite(ref))
    assert np.allclose(got, ref, rtol=0, atol=1e-9), np.abs(got - ref).max()


def test_fp32_growth_rates_and_breakdown_voltage_within_two_sigma(setup):
    insts, xs, ref = setup
    got = _gpu_rates(insts, xs, 32)
    eg, eo = _per_voltage(got), _per_voltage(ref)
    for V, (mg, sg), (mo, so) in zip(VOLTS, eg, eo):
        print(f"V={V:.0f}: lambda t_c GPU {mg:+.4f} +- {sg:.4f}, oracle {mo:+.4f} +- {so:.4f}")
        assert abs(mg - mo) <= 2 * math.hypot(sg, so), V
    # below at the lowest voltage, above at the highest
    assert eo[0][0] < 0 < eo[-1][0] and eg[0][0] < 0 < eg[-1][0]
    vg = bd.zero_crossing(VOLTS, [m for m, _ in eg], [s for _, s in eg])
    vo = bd.zero_crossing(VOLTS, [m for m, _ in eo], [s for _, s in eo])
    assert vg is not None and vo is not None
    print(f"V_b GPU {vg[0]:.1f} +- {vg[1]:.1f} V, oracle {vo[0]:.1f} +- {vo[1]:.1f} V")
    assert abs(vg[0] - vo[0]) <= 2 * math.hypot(vg[1], vo[1])
