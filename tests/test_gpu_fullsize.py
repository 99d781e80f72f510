"""FP64 parity with the oracle at the grid sizes and partition counts the
batched sweeps run: gaps of 1024 to 8192 cells in one batch, markers spread
over each whole gap, with space charge strong enough that the deposit and
the Poisson solve shape the field (Eq. (7) deposit with density weight
w_p = beta w_j, Sec. III).

This exercises the paths small gaps never reach: deposits outside a
workgroup's 1856-node LDS window (of the species its tiles hold; products of
the other species always go outside), the window re-anchored per (instance,
species), the
tail kernel's scans with several nodes per thread (N + 1 > 1024) and its
second accumulator round (N + 1 > 5120), 8 and 16 output partitions per
(instance, species), population control at that size, and (with
resort_period 4) the cell sort, each against an independent oracle run per
instance.
"""

import dataclasses

import numpy as np
import pytest

import oracle
import synth
from synth import configs
from parity import compare_populations, STAT_INT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402

# cells, p [Torr] (a quarter mean free path per cell), V (Eq. (1) estimate
# at that pd), electrons, ions, population target, capacity per species
SPEC = [(1024, 4.7, 280.0, 20000, 8000, 0, 140000),
        (2048, 9.4, 450.0, 24000, 9000, 12000, 90000),
        (4096, 18.7, 750.0, 20000, 8000, 0, 300000),
        (8192, 37.4, 1300.0, 16000, 6000, 0, 70000)]
STEPS = 10


def _setup():
    insts, pops = [], []
    for k, (cells, p, V, ne, ni, nt, cap) in enumerate(SPEC):
        insts.append(configs.Instance(d=0.01, p_torr=p, V=V, cells=cells, gamma_se=0.2,
                                      seed_mode=configs.SEED_NONE, n_target=nt,
                                      capacity=cap))
        pops.append(synth.markers.mixed(100 + k, ne, ni, cells, e_hi=100.0))
    return insts, pops


@pytest.mark.parametrize("resort_period", [0, 4])
def test_large_gaps_match_independent_oracles_step_by_step(resort_period, xs_argon):
    _large_gaps(resort_period, xs_argon)


@pytest.mark.parametrize("resort_period", [0, 4])
def test_large_gaps_with_claimed_runs_match_independent_oracles(resort_period, xs_argon):
    """The same on a grid of 32 workgroups, so that the particle kernel's
    workgroups claim runs of tiles from the step's pool counters (at least
    four tiles per workgroup), with and without the cell sort."""
    _large_gaps(resort_period, xs_argon, grid=32, claimed=1)


def test_large_gaps_with_weight_splitting_match_independent_oracles(xs_argon):
    """Weight splitting (Sec. III, split fraction 0.3) on the same four gaps:
    every collision keeps the uncollided part and adds a marker carrying the
    collided part's flux weight, so each marker deposits its own weight,
    inside and outside the workgroups' LDS windows.  Capacities at 16 times
    the loaded markers (the populations grow about tenfold); 8 steps against
    an oracle per gap, flux weights within 1e-12."""
    _large_gaps(0, xs_argon, split=0.3, steps=8, cap_factor=16)


def _large_gaps(resort_period, xs_argon, grid=None, claimed=None, split=0.0, steps=STEPS,
                cap_factor=None):
    insts, pops = _setup()
    if cap_factor is not None:
        insts = [dataclasses.replace(x, capacity=cap_factor * (len(e["id"]) + len(i["id"])))
                 for x, (e, i) in zip(insts, pops)]
    # a flux weight at which the markers' space charge moves the field by
    # 0.1-3 % of V/d: about 1e8 times the field tolerance below
    run = configs.Run(precision=64, w_j0=2e7, resort_period=resort_period, split_frac=split)
    print(f"full-size parity, resort_period={resort_period}, grid={grid}, claimed={claimed}, "
          f"split={split}", flush=True)
    gpu = slpic.Sim(insts, run, xs_argon)
    if grid is not None:
        gpu.set_launch_shape(grid, 0)
    if claimed is not None:
        gpu.set_work_distribution(claimed)
        assert gpu.work_distribution() == claimed
    refs = [oracle.Sim(x, run, xs_argon, instance_index=k) for k, x in enumerate(insts)]
    for k, (e, i) in enumerate(pops):
        for sim, kw in ((gpu, {"inst": k}), (refs[k], {})):
            sim.load(0, e, **kw)
            sim.load(1, i, **kw)
    parts = [gpu.partitions(0, k)[0].size for k in range(len(insts))]
    if cap_factor is None:
        assert parts == [16, 8, 16, 8], parts
    for k, x in enumerate(insts):
        E_g, E_o = gpu.fields(inst=k)[2], refs[k].fields()[2]
        vac = x.V / x.d
        # the space charge is felt, and the loaded field agrees
        assert np.abs(E_o + vac).max() > 1e-3 * vac, k
        assert np.allclose(E_g, E_o, rtol=0, atol=1e-11 * np.abs(E_o).max()), k
    roulette = 0
    for n in range(steps):
        gpu.step(1)
        for r in refs:
            r.step(1)
        for k in range(len(insts)):
            sg, so = gpu.stats(inst=k), refs[k].stats()
            for key in STAT_INT:
                assert sg[key] == so[key], (n, k, key, sg[key], so[key])
            assert sg["w_j"] == so["w_j"]
            assert sg["w_e"] == pytest.approx(so["w_e"], rel=1e-9)
            assert sg["w_i"] == pytest.approx(so["w_i"], rel=1e-9)
            roulette += so["roulette"]
        if n in (0, steps - 1):
            for k in range(len(insts)):
                rho_g, _, E_g = gpu.fields(inst=k)
                rho_o, _, E_o = refs[k].fields()
                assert np.allclose(rho_g, rho_o, rtol=0, atol=1e-11 * np.abs(rho_o).max()), (n, k)
                assert np.allclose(E_g, E_o, rtol=0, atol=1e-11 * np.abs(E_o).max()), (n, k)
    assert gpu.sync() == 0
    assert roulette > 0
    for k, x in enumerate(insts):
        v0 = gpu.scalars(k)["v0"]
        for sp in (0, 1):
            w = compare_populations(gpu.read(sp, k), refs[k].read(sp), 1e-12 * x.cells,
                                    1e-12, v0, label=f"inst {k} sp {sp}",
                                    tol_w=1e-12 if split > 0.0 else None)
            print("full size", resort_period, split, k, sp, w)


@pytest.mark.parametrize("grid", [None, 32])
def test_fp32_large_gaps_single_step_from_loaded_state(grid, xs_argon):
    """FP32 particles with FP64 Poisson and totals on the same four gaps: one
    step from the loaded state against the FP64 oracle.  States agree within
    1e-5 (positions relative to the gap), decisions whose margin is below
    1e-6 are excused (at most 1 in 1000 markers), counts are equal up to the
    excused markers, and the deposit and field after the step agree within
    1e-6 of their largest magnitude (FP32 positions and weights, 31-bit fixed
    point).  With grid 32 the workgroups claim runs of tiles."""
    insts, pops = _setup()
    run32 = configs.Run(precision=32, w_j0=2e7)
    run64 = configs.Run(precision=64, w_j0=2e7)
    print(f"full-size FP32 step, grid={grid}", flush=True)
    gpu = slpic.Sim(insts, run32, xs_argon)
    if grid is not None:
        gpu.set_launch_shape(grid, 5)
        gpu.set_work_distribution(1)
    refs = [oracle.Sim(x, run64, xs_argon, instance_index=k) for k, x in enumerate(insts)]
    for k, (e, i) in enumerate(pops):
        for sim, kw in ((gpu, {"inst": k}), (refs[k], {})):
            sim.load(0, e, **kw)
            sim.load(1, i, **kw)
    gpu.step(1)
    for r in refs:
        r.step(1)
    assert gpu.sync() == 0
    for k, x in enumerate(insts):
        v0 = gpu.scalars(k)["v0"]
        tied = 0
        for sp in (0, 1):
            n = refs[k].count(sp)
            w = compare_populations(gpu.read(sp, k), refs[k].read(sp), 1e-5 * x.cells, 1e-5,
                                    v0, tie_tol=1e-6, max_tied=n // 1000,
                                    label=f"inst {k} sp {sp}")
            tied += w["tied"]
            print("full size fp32", grid, k, sp, w)
        sg, so = gpu.stats(inst=k), refs[k].stats()
        for key in STAT_INT:
            assert abs(sg[key] - so[key]) <= tied, (k, key, sg[key], so[key], tied)
        rho_g, _, E_g = gpu.fields(inst=k)
        rho_o, _, E_o = refs[k].fields()
        assert np.allclose(rho_g, rho_o, rtol=0, atol=1e-6 * np.abs(rho_o).max()), k
        assert np.allclose(E_g, E_o, rtol=0, atol=1e-6 * np.abs(E_o).max()), k


# cells, electron cells [lo, hi), ion cells [lo, hi), electrons, ions
DENSE = [(4096, (3300, 4090), (1000, 1500), 24000, 12000),
         (2048, (900, 1100), (0, 2048), 20000, 8000),
         (1024, (100, 300), (600, 900), 12000, 6000)]


def test_dense_regions_away_from_the_cathode_match_independent_oracles():
    """Each species' LDS deposit window sits where that species deposited
    most (chosen on every field refresh and every 16 steps): here a 4096-cell
    gap with its electrons packed against the anode (the window then starts
    at its last possible node) and its ions in the middle, a 2048-cell gap
    with electrons packed mid-gap, and a 1024-cell gap that fits one window,
    in one FP64 batch against an oracle per gap for 40 steps (three window
    choices).  A window reaching past its gap would add into the next gap's
    nodes; every integer statistic must stay bit-exact every step, the
    deposit and field within 1e-11, states within 1e-12."""
    xs = synth.argon_like()
    insts, pops = [], []
    for k, (cells, (elo, ehi), (ilo, ihi), ne, ni) in enumerate(DENSE):
        insts.append(configs.Instance(d=0.01, p_torr=4.7 * cells / 1024, V=300.0 + cells / 10,
                                      cells=cells, gamma_se=0.2, seed_mode=configs.SEED_NONE,
                                      capacity=8 * (ne + ni)))
        e, i = synth.markers.mixed(300 + k, ne, ni, cells, cell_lo=elo, cell_hi=ehi, e_hi=60.0)
        rng = np.random.default_rng([300 + k, 9])
        i["cell"] = rng.integers(ilo, ihi, size=ni).astype(np.int32)
        pops.append((e, i))
    run = configs.Run(precision=64, w_j0=2e7)
    print("dense regions away from the cathode", flush=True)
    gpu = slpic.Sim(insts, run, xs)
    refs = [oracle.Sim(x, run, xs, instance_index=k) for k, x in enumerate(insts)]
    for k, (e, i) in enumerate(pops):
        for sim, kw in ((gpu, {"inst": k}), (refs[k], {})):
            sim.load(0, e, **kw)
            sim.load(1, i, **kw)
    for n in range(40):
        gpu.step(1)
        for r in refs:
            r.step(1)
        for k in range(len(insts)):
            sg, so = gpu.stats(inst=k), refs[k].stats()
            for key in STAT_INT:
                assert sg[key] == so[key], (n, k, key, sg[key], so[key])
            assert sg["w_e"] == pytest.approx(so["w_e"], rel=1e-9)
            assert sg["w_i"] == pytest.approx(so["w_i"], rel=1e-9)
        if n in (0, 17, 39):
            for k in range(len(insts)):
                rho_g, _, E_g = gpu.fields(inst=k)
                rho_o, _, E_o = refs[k].fields()
                assert np.allclose(rho_g, rho_o, rtol=0, atol=1e-11 * np.abs(rho_o).max()), (n, k)
                assert np.allclose(E_g, E_o, rtol=0, atol=1e-11 * np.abs(E_o).max()), (n, k)
    assert gpu.sync() == 0
    for k, x in enumerate(insts):
        v0 = gpu.scalars(k)["v0"]
        for sp in (0, 1):
            compare_populations(gpu.read(sp, k), refs[k].read(sp), 1e-12 * x.cells, 1e-12, v0,
                                label=f"dense inst {k} sp {sp}")
