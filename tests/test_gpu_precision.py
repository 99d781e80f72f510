"""Error of each FP32 stage of the HIP path against the FP64 oracle.

The push, the collision sampling and the deposit run in FP32 on the GPU; the
Poisson solve and the population totals stay in FP64 (the deposit is summed
in 64-bit fixed point).  Each stage's error is measured on its own, from one
loaded state of 9000 electrons and 4100 ions in a 64-cell gap whose space
charge is about a tenth of the applied field, so that deposit errors reach
the field.  Positions are compared in units of the gap (cells / N),
velocities relative to max(|v|, v0)."""


import numpy as np
import pytest

import oracle
import synth
from synth import configs, xsec
from parity import by_id, compare_populations

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402

CELLS = 64


def _gap():
    return configs.Instance(d=0.01, p_torr=3.0, V=300.0, cells=CELLS, gamma_se=0.0,
                            seed_mode=configs.SEED_NONE, capacity=40000)


def _loaded(xs, area=8e-9):
    e, i = synth.markers.mixed(7, 9000, 4100, CELLS)
    gpu = slpic.Sim([_gap()], configs.Run(precision=32, area=area), xs)
    ref = oracle.Sim(_gap(), configs.Run(precision=64, area=area), xs)
    for sim in (gpu, ref):
        sim.load(0, e)
        sim.load(1, i)
    return gpu, ref


def test_fp32_error_of_each_stage_against_the_fp64_oracle(xs_argon):
    errs = {}
    gpu, ref = _loaded(xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0))
    sc = gpu.scalars()
    # deposit (FP32 weights, fixed-point sums) of the same loaded markers
    rho_g, _, E_g = gpu.fields()
    rho_o, _, E_o = ref.fields()
    errs["deposit rho"] = np.abs(rho_g - rho_o).max() / np.abs(rho_o).max()
    # Poisson (FP64) on the GPU's own charge, against the oracle's solver
    _, E_p = oracle.poisson(CELLS, sc["dx"], _gap().V, rho_g)
    errs["poisson E"] = np.abs(E_g - E_p).max() / np.abs(E_p).max()
    errs["field E (deposit + Poisson)"] = np.abs(E_g - E_o).max() / np.abs(E_o).max()
    # the space charge is a sizeable part of the field
    vac = _gap().V / _gap().d
    assert np.abs(E_o + vac).max() > 0.05 * vac
    # push: collisionless steps from the same state
    for steps in (1, 20):
        gpu.step(1 if steps == 1 else 19)
        ref.step(1 if steps == 1 else 19)
        assert gpu.sync() == 0
        for sp in (0, 1):
            w = compare_populations(gpu.read(sp), ref.read(sp), 1e-5 * CELLS, 1e-5, sc["v0"],
                                    label=f"push {steps} steps species {sp}")
            errs[f"push x/d, {steps} step(s), sp {sp}"] = w["x_cells"] / CELLS
            errs[f"push v, {steps} step(s), sp {sp}"] = max(w["vx"], w["vy"], w["vz"])
    # totals (FP64 from the fixed-point deposit sums) against the FP64 sum of
    # beta w_j over the GPU's own markers
    st = gpu.stats()
    for sp, key in ((0, "w_e"), (1, "w_i")):
        p = gpu.read(sp)
        v = np.sqrt(p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2)
        beta = np.where(v > sc["v0"], sc["v0"] / np.maximum(v, 1e-300), 1.0)
        want = st["w_j"] * beta.sum()
        errs[f"total {key}"] = abs(st[key] - want) / want
    gpu.close()

    # collision sampling: one step of the argon-shaped gas from the same
    # state; outcomes that differ are decisions taken on either side of a
    # threshold within FP32 rounding
    gpu, ref = _loaded(xs_argon)
    gpu.step(1)
    ref.step(1)
    assert gpu.sync() == 0
    so = ref.stats()
    n_coll = so["elastic"] + so["excitation"] + so["ionization"] + so["cx"]
    differ = 0
    for sp in (0, 1):
        g, r = by_id(gpu.read(sp)), by_id(ref.read(sp))
        differ += len(np.setxor1d(g["id"], r["id"]))
        common, gi, ri = np.intersect1d(g["id"], r["id"], return_indices=True)
        dv = np.abs(g["vx"][gi] - r["vx"][ri]) / np.maximum(np.abs(r["vx"][ri]), sc["v0"])
        differ += int(np.sum(dv > 1e-3))   # same id, different scatter outcome
    errs["collision outcomes differing / collisions"] = differ / max(n_coll, 1)
    assert n_coll > 1000
    gpu.close()

    for k, v in errs.items():
        print(f"{k:44s} {v:.3e}")
    assert errs["deposit rho"] < 1e-5
    assert errs["poisson E"] < 1e-12
    assert errs["field E (deposit + Poisson)"] < 1e-5
    assert errs["total w_e"] < 1e-6 and errs["total w_i"] < 1e-6
    assert errs["collision outcomes differing / collisions"] < 1e-3


def test_fp32_flight_across_speed_ratios():
    """One collisionless FP32 step against the FP64 oracle for electrons from
    just above to 1000 times the speed limit, in every direction, in the
    vacuum field of a 256-cell gap: the FP32 flight's series path (markers
    above v0 all along whose relative change of v is small) and its
    iteration (the rest: slow markers, large changes, turning points) both
    run, in the same waves, and every state agrees within 1e-5."""
    cells = 256
    gap = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=cells, gamma_se=0.0,
                           seed_mode=configs.SEED_NONE, capacity=60000)
    xs = xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=0.0)
    gpu = slpic.Sim([gap], configs.Run(precision=32), xs)
    ref = oracle.Sim(gap, configs.Run(precision=64), xs)
    sc = gpu.scalars()
    v0, dt, dx = sc["v0"], sc["dt"], sc["dx"]
    rng = np.random.default_rng(11)
    n = 20000
    speed = v0 * 10.0 ** rng.uniform(-0.5, 3.0, n)
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - mu * mu)
    pop = {"cell": rng.integers(64, 192, n).astype(np.int32), "off": rng.uniform(0.0, 1.0, n),
           "vx": speed * mu, "vy": speed * st * np.cos(phi), "vz": speed * st * np.sin(phi),
           "id": np.arange(1, n + 1, dtype=np.uint64)}
    # FP32 values on both sides
    for k in ("off", "vx", "vy", "vz"):
        pop[k] = pop[k].astype(np.float32).astype(np.float64)
    e_none = {k: v[:0] for k, v in pop.items()}
    for sim in (gpu, ref):
        sim.load(0, pop)
        sim.load(1, e_none)
    # how the markers split between the two paths (vacuum field, a = qE/m)
    a = 1.602176634e-19 / 9.1093837015e-31 * gap.V / gap.d
    rt = v0 * a * dt / speed ** 2
    series = (speed > v0) & (rt < 0.2)
    print(f"v0 {v0:.3e} m/s, |a| dt {a * dt:.3e} m/s: {series.mean():.2f} of the markers "
          f"within the series' reach", flush=True)
    assert 0.2 < series.mean() < 0.9
    gpu.step(1)
    ref.step(1)
    assert gpu.sync() == 0
    w = compare_populations(gpu.read(0), ref.read(0), 1e-5 * cells, 1e-5, v0, label="electrons")
    print("flight across speed ratios:", {q: w[q] for q in ("n", "x_cells", "vx", "vy", "vz")})
    assert w["n"] == n
    gpu.close()
