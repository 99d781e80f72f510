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

Because replica k is run from the same seeds on both sides, the FP32 and
FP64 ensembles are compared as paired samples: the mean of the
replica-by-replica differences against twice its standard error (with a
floor of 1e-6 per crossing time, far below any statistical error, for
replicas whose histories never parted).  The breakdown voltages are compared
the same way, by a paired bootstrap over replicas.

The same comparison runs on the argon-shaped gas of the sweeps at two of the
64-point sweep's pd values (0.52 and 1.0 Torr cm, 114 and 219 cells by the
quarter-mean-free-path rule), at voltages on either side of the synthetic
gas's breakdown (about 182 V and 175 V from an FP32 scan).
"""

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
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


FLOOR = 1e-6   # per crossing time: FP32 rounding of the fitted log population


def _paired_check(volts, got, ref, label):
    """Paired 2-sigma comparison of growth rates per voltage and of the
    breakdown voltage; got/ref: [n_v, R] growth rates."""
    eg = [bd.ensemble(r) for r in got]
    eo = [bd.ensemble(r) for r in ref]
    for V, g, o, (mg, sg), (mo, so) in zip(volts, got, ref, eg, eo):
        d, se = bd.paired_difference(g, o)
        print(f"{label} V={V:.0f}: lambda t_c GPU {mg:+.4f} +- {sg:.4f}, "
              f"oracle {mo:+.4f} +- {so:.4f}, paired difference {d:+.2e} +- {se:.1e}")
        assert math.isfinite(d) and abs(d) <= max(2 * se, FLOOR), (label, V)
        # the same classification on both sides
        assert (mg > 0) == (mo > 0), (label, V)
    vg = bd.zero_crossing(volts, [m for m, _ in eg], [s for _, s in eg])
    vo = bd.zero_crossing(volts, [m for m, _ in eo], [s for _, s in eo])
    assert vg is not None and vo is not None, label
    dv = bd.paired_breakdown_difference(volts, got, ref)
    assert dv is not None, label
    print(f"{label} V_b GPU {vg[0]:.1f} +- {vg[1]:.1f} V, oracle {vo[0]:.1f} +- {vo[1]:.1f} V, "
          f"paired difference {dv[0]:+.3f} +- {dv[1]:.3f} V")
    assert abs(dv[0]) <= max(2 * dv[1], 0.01), label
    return eg, eo, vg, vo


def test_fp32_growth_rates_and_breakdown_voltage_within_two_sigma(setup):
    insts, xs, ref = setup
    got = _gpu_rates(insts, xs, 32)
    g = got.reshape(len(VOLTS), R)
    o = ref.reshape(len(VOLTS), R)
    eg, eo, vg, vo = _paired_check(VOLTS, g, o, "constant-sigma gas")
    # below at the lowest voltage, above at the highest
    assert eo[0][0] < 0 < eo[-1][0] and eg[0][0] < 0 < eg[-1][0]


# argon-shaped gas: (pd [Torr cm], voltages below and above breakdown)
ARGON = [(0.1 * 1000.0 ** (15 / 63), (145.0, 215.0)), (1.0, (145.0, 210.0))]
R_AR = 12


def _argon_gap(pd, V, sigma_max):
    cells = configs.cells_quarter_mfp(0.01, pd, sigma_max)
    return configs.Instance(d=0.01, p_torr=pd, V=V, cells=cells, gamma_se=0.07,
                            seed_mode=configs.SEED_CATHODE, n_seed=300,
                            n_target=600, capacity=8192)


def test_fp32_argon_gas_breakdown_within_two_sigma():
    xs = synth.argon_like()
    smax = xs.sigma_total_max()
    insts = [_argon_gap(pd, V, smax) for pd, volts in ARGON for V in volts for _ in range(R_AR)]
    steps = [120 * i.cells for i in insts]

    def one(k):
        sim = oracle.Sim(insts[k], configs.Run(precision=64), xs, instance_index=k)
        n = steps[k] // EVERY
        w = np.empty(n)
        for j in range(n):
            sim.step(EVERY)
            w[j] = sim.stats()["w_i"]
        t = np.arange(1, n + 1) * EVERY * sim.scalars()["dt"]
        return bd.growth_rate(t, w, bd.crossing_time(insts[k].d, insts[k].V))

    print("argon-shaped gas: oracle ensembles", flush=True)
    with ThreadPoolExecutor(8) as ex:
        ref = np.array(list(ex.map(one, range(len(insts)))))
    print("argon-shaped gas: GPU ensembles", flush=True)
    sim = slpic.Sim(insts, configs.Run(precision=32), xs)
    st, pops = bd.step_and_record(sim, max(steps))
    assert sim.sync() == 0
    keep = st % EVERY == 0
    got = bd.instance_rates(sim, insts, st[keep], pops[:, keep])
    sim.close()
    per = 2 * R_AR
    for a, (pd, volts) in enumerate(ARGON):
        g = got[a * per:(a + 1) * per].reshape(2, R_AR)
        o = ref[a * per:(a + 1) * per].reshape(2, R_AR)
        eg, eo, vg, vo = _paired_check(volts, g, o, f"argon pd={pd:.2f}")
        assert eo[0][0] < 0 < eo[1][0], pd
