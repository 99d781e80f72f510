"""Pins of the oracle's flux diagnostic (Eq. (12) and the passage after it:
the time-integrated flux through a surface is the sum of the flux weights
w_j of the markers crossing it, whatever their speed)."""

import math

import numpy as np
import pytest

import oracle
from synth import configs, markers, xsec
from synth.constants import QE, ME
from test_oracle_collisions import _renewal_mean


def _gap(V=300.0, cells=64, **kw):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=V, cells=cells, gamma_se=0.0,
                            seed_mode=configs.SEED_NONE, capacity=200000)
    for k, v in kw.items():
        setattr(inst, k, v)
    return inst


def _ge(cells_of_markers, n_nodes):
    """Markers at or above each node: count of cell >= k for k = 0 .. N."""
    return np.array([(cells_of_markers >= k).sum() for k in range(n_nodes)])


def test_net_crossings_are_the_change_of_the_population_above_each_node():
    # Collisionless markers of both species that stay inside the gap: the net
    # number crossing node k upward equals the change of the number of
    # markers in cells >= k (an integer identity).
    inst = _gap()
    xs = xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0)
    run = configs.Run(precision=64, area=1e30, w_j0=3.0)
    sim = oracle.Sim(inst, run, xs, flags=oracle.FLAG_FLUX)
    e, i = markers.mixed(5, 4000, 3000, inst.cells)
    # keep them away from the electrodes: |dx| <= v0 dt = dx / 2 per step
    for pop in (e, i):
        pop["cell"] = 8 + pop["cell"] % (inst.cells - 16)
    sim.load(0, e)
    sim.load(1, i)
    n_nodes = inst.cells + 1
    before = [_ge(sim.read(sp)["cell"], n_nodes) for sp in (0, 1)]
    for _ in range(6):
        sim.step(1)
        st = sim.stats()
        assert st["abs_e_cathode"] + st["abs_e_anode"] + st["abs_i_cathode"] + st["abs_i_anode"] == 0
    for sp in (0, 1):
        after = _ge(sim.read(sp)["cell"], n_nodes)
        net = sim.flux(sp) / run.w_j0
        assert np.array_equal(net, (after - before[sp]).astype(float)), sp
        assert np.any(net != 0)


def test_equal_physical_fluxes_measure_equal_whatever_the_speed():
    # Sec. II.B: a marker represents w_j particles every time it crosses a
    # surface.  Beam A moves at 0.5 v0 (beta = 1); beam B at 20 v0 (beta =
    # 0.05) carries the same physical flux n v, n_B = n_A v_A / v_B, so with
    # density weight w_p = beta w_j its marker spacing is s_B = s_A v0 / v_A
    # (it moves at v0 on the grid).  Both must measure the same flux at a
    # node the beams cover for the whole window; counting w_p instead of w_j
    # would make B's flux 20 times smaller.
    inst = _gap(V=0.0, v_limit=4.0e4)
    xs = xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0)
    run = configs.Run(precision=64, area=1e30, w_j0=2.0)
    v0 = inst.v_limit
    dx = inst.d / inst.cells
    out = []
    for v_phys, spacing in ((0.5 * v0, dx / 40.0), (20.0 * v0, dx / 20.0)):
        n = int(round(40 * dx / spacing))
        x = 4 * dx + spacing * (np.arange(n) + 0.5)
        pop = {"cell": np.floor(x / dx).astype(np.int32), "off": x / dx - np.floor(x / dx),
               "vx": np.full(n, v_phys), "vy": np.zeros(n), "vz": np.zeros(n),
               "id": np.arange(1, n + 1, dtype=np.uint64)}
        sim = oracle.Sim(inst, run, xs, flags=oracle.FLAG_FLUX)
        sim.load(0, pop)
        sim.step(32)   # the grid speed is at most v0: 16 cells
        out.append(sim.flux(0))
        # the measured flux is w_j per crossing, not the density weight
        beta = min(1.0, v0 / v_phys)
        sc = sim.scalars()
        node = 30
        expected = run.w_j0 * (beta * v_phys) * (32 * sc["dt"]) / spacing
        assert out[-1][node] == pytest.approx(expected, abs=run.w_j0), (v_phys, out[-1][node])
    assert out[0][30] == out[1][30]


def test_townsend_electron_flux_grows_as_the_multiplication():
    # Zero-threshold constant-cross-section ionization, both electrons of an
    # ionization restarting at rest: electrons only move toward the anode,
    # so the net electron flux through the plane at x per seed is the
    # multiplication of a gap of length x, which the renewal equation of the
    # discrete process gives (Sec. III: the physical mean free path).
    sigma, V = 1e-20, 300.0
    xs = xsec.constant([(xsec.IONIZATION, sigma)], [0.0])
    inst = _gap(V=V, seed_mode=configs.SEED_CATHODE, n_seed=3000,
                capacity=configs.capacity_for(120000, 3000))
    run = configs.Run(precision=64, area=1e30, cfl=0.5)
    sim = oracle.Sim(inst, run, xs, flags=oracle.FLAG_PRODUCTS_AT_REST | oracle.FLAG_FLUX)
    sc = sim.scalars()
    anode = 0
    for _ in range(600):
        sim.step(1)
        anode += sim.stats()["abs_e_anode"]
        if sim.count(oracle.ELECTRON) == 0:
            break
    assert sim.count(oracle.ELECTRON) == 0
    flux = sim.flux(0) / run.w_j0
    # every anode absorption crossed the anode node; nothing moved down
    assert flux[inst.cells] == anode
    assert np.all(np.diff(flux) >= 0) and flux[0] == 0
    P = -math.expm1(-sc["n_g"] * sigma * sc["v0"] * sc["dt"])
    a = QE / ME * V / inst.d
    for k in (8, 24, 40, 56):
        x = k * inst.d / inst.cells
        want = _renewal_mean(P, sc["v0"] * sc["dt"], sc["v0"] ** 2 / (2 * a), x)
        sd = math.sqrt(max(want * (want - 1), 1e-9) / inst.n_seed)
        assert abs(flux[k] / inst.n_seed - want) < 4 * sd + 1e-9, (k, flux[k] / inst.n_seed, want, sd)
