"""Work distribution of the particle kernel: workgroups that claim runs of
tiles from the step's pool counters compute exactly what equal contiguous
shares compute.  Nothing in a step depends on which workgroup takes a tile
or in what order (draws are keyed by marker id and step, deposits are exact
fixed-point sums), so statistics, markers and fields must agree bit for bit.

A grid of 64 workgroups makes the batched sweep at 2 % of its marker counts
(about 4e5 markers, 1.6e3 tiles) run with many tiles per workgroup, so the
claims shrink to single tiles, move between the eight pools and run out,
every step, with population control, ionization and charge exchange.  The
same holds for the weight-splitting collision strategy (Sec. III), whose
markers carry flux weights and whose kernel is a variant of its own."""

import dataclasses

import numpy as np
import pytest

import synth
from synth import configs
from parity import compare_populations, STAT_INT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402

GRID = 64
STEPS = 48


def _sweep(claimed, graph=False, split_frac=0.0):
    xs = synth.argon_like()
    w = configs.scaled(configs.c4(xs.sigma_total_max(), precision=32), 0.02)
    w = dataclasses.replace(w, run=dataclasses.replace(w.run, split_frac=split_frac))
    if split_frac:
        # a split collision adds a marker: room for the larger populations
        w = dataclasses.replace(w, instances=[dataclasses.replace(i, capacity=3 * i.capacity)
                                              for i in w.instances])
    sim = slpic.Sim(w.instances, w.run, xs)
    # the weight-splitting kernel has one register budget (waves per SIMD: 0)
    sim.set_launch_shape(GRID, 0 if split_frac else 5)
    sim.set_work_distribution(claimed)
    if graph:
        sim.use_graph(True)
    sim.step(STEPS)
    assert sim.sync() == 0
    return w, sim


@pytest.mark.parametrize("split_frac", [0.0, 0.4])
def test_claimed_runs_equal_equal_shares_bit_for_bit(split_frac):
    w, a = _sweep(1, split_frac=split_frac)
    _, b = _sweep(0, split_frac=split_frac)
    _, c = _sweep(1, graph=True, split_frac=split_frac)
    assert a.work_distribution() == 1 and b.work_distribution() == 0
    print(f"claimed runs vs equal shares, split_frac={split_frac}:", len(w.instances), "instances,",
          sum(a.count(0, k) + a.count(1, k) for k in range(len(w.instances))), "markers",
          flush=True)
    for other in (b, c):
        for k in range(len(w.instances)):
            ha = a.history(0, STEPS, inst=k)
            ho = other.history(0, STEPS, inst=k)
            for key in STAT_INT + ["w_e", "w_i", "w_j"]:
                assert np.array_equal(ha[key], ho[key]), (k, key)
            for sp in (0, 1):
                pa, po = a.read(sp, k), other.read(sp, k)
                compare_populations(pa, po, 0.0, 0.0, a.scalars(k)["v0"], label=f"inst {k} sp {sp}")
                if split_frac:
                    # flux weights follow the markers (sorted by id as the comparison does)
                    ia, io = np.argsort(pa["id"]), np.argsort(po["id"])
                    assert np.array_equal(pa["w"][ia], po["w"][io]), (k, sp)
            assert np.array_equal(a.fields(inst=k)[2], other.fields(inst=k)[2]), k
    # the run collided, ionized and exchanged charge
    tot = {key: sum(int(a.history(0, STEPS, inst=k)[key].sum()) for k in range(len(w.instances)))
           for key in ("elastic", "ionization", "cx")}
    assert all(v > 0 for v in tot.values()), tot
    if split_frac:
        parts = sum(int(np.count_nonzero(a.read(sp, k)["w"] < 1.0))
                    for k in range(len(w.instances)) for sp in (0, 1))
        assert parts > 1000, parts


def test_work_distribution_defaults():
    xs = synth.argon_like()
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=1000,
                            n_target=0, capacity=4000)
    plain = slpic.Sim([inst], configs.Run(precision=32), xs)
    sorted_ = slpic.Sim([inst], configs.Run(precision=32, resort_period=16), xs)
    # claimed runs unless the markers are cell-sorted
    assert plain.work_distribution() == 1
    assert sorted_.work_distribution() == 0
    with pytest.raises(slpic.SlpicError):
        plain.set_work_distribution(-1)
