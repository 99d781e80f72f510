"""The workloads at their full sizes, in the launch shape bench.py times
(the library's default: claimed runs where a launch has four tiles per
workgroup or more, five waves per SIMD), each on its evolved state after the
bench's warmup: the 64-instance Paschen sweep (2.5e7 target markers), the
256-instance bisection round (1.8e8), the 4096-cell gap with its cell sort
every 16 steps (1e7) and the 512-cell gap (1e6).

- Every instance keeps the marker balance of the events it reports, step by
  step (entering - absorbed + 2 ionizations + emissions - roulette + splits
  = leaving), with no error flags.
- Sampled instances (from the smallest to the largest by markers) are taken
  over by the FP64 oracle at the GPU's step counter and flux weight (Philox
  draws are keyed by marker id, step and channel) and both take one step:
  states within 1e-5 (positions relative to the gap), decisions with a
  margin below 1e-6 excused (at most 1 in 1000 markers), counts equal up to
  the excused markers, charge density and field within 1e-6 of their
  largest magnitude.
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

BOOK_STEPS = 8

# workload, the bench's warmup, sampled instances
CASES = {
    "sweep64": (lambda xs: configs.c4(xs.sigma_total_max(), precision=32), 200, 4),
    "bisection256": (lambda xs: configs.c5(xs.sigma_total_max(), precision=32), 100, 3),
    "gap4096_sorted": (lambda xs: configs.c3(), 2048, 1),
    "gap512": (lambda xs: configs.c2(300.0), 200, 1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_full_size_workload_sampled_against_the_oracle(case):
    make, warm, n_pick = CASES[case]
    xs = synth.argon_like()
    w = make(xs)
    n_inst = len(w.instances)
    targets = sum(i.n_target for i in w.instances)
    print(f"{case}: {n_inst} instances, {targets:.3e} target markers", flush=True)
    gpu = slpic.Sim(w.instances, w.run, xs)
    print("launch shape", gpu.launch_shape(), "claimed runs", gpu.work_distribution(), flush=True)
    gpu.step(warm)
    assert gpu.sync() == 0
    s0 = gpu.steps_done()
    gpu.step(BOOK_STEPS)
    assert gpu.sync() == 0
    total = 0
    for k in range(n_inst):
        h = gpu.history(s0, BOOK_STEPS, inst=k)
        absorbed = h["abs_e_cathode"] + h["abs_e_anode"] + h["abs_i_cathode"] + h["abs_i_anode"]
        out = h["n_in"] - absorbed + 2 * h["ionization"] + h["see"] - h["roulette"] + h["split"]
        assert np.array_equal(out, h["n_e"] + h["n_i"]), k
        assert np.array_equal(h["n_in"][1:], (h["n_e"] + h["n_i"])[:-1]), k
        assert np.all(h["err"] == 0), k
        total += int(h["n_in"][-1])
    print(f"markers entering the last step: {total:.3e}", flush=True)
    assert total > 0.3 * targets

    # the sampled instances, taken over by the oracle
    counts = [gpu.count(0, k) + gpu.count(1, k) for k in range(n_inst)]
    order = np.argsort(counts)
    picks = sorted({int(order[round(j * (n_inst - 1) / max(1, n_pick - 1))]) for j in range(n_pick)})
    run64 = dataclasses.replace(w.run, precision=64)
    refs = {}
    for k in picks:
        sc = gpu.scalars(k)
        inst = dataclasses.replace(w.instances[k], seed_mode=configs.SEED_NONE, n_seed=0)
        ref = oracle.Sim(inst, run64, xs, instance_index=k)
        ref.set_clock(int(sc["step"]), sc["w_j"])
        ref.load(0, gpu.read(0, k))
        ref.load(1, gpu.read(1, k))
        refs[k] = ref
        print(f"instance {k}: {counts[k]} markers, {w.instances[k].cells} cells, step "
              f"{int(sc['step'])}, w_j {sc['w_j']:.4g}", flush=True)
    gpu.step(1)
    assert gpu.sync() == 0
    for k in picks:
        refs[k].step(1)
        x = w.instances[k]
        v0 = gpu.scalars(k)["v0"]
        tied = 0
        for sp in (0, 1):
            n = refs[k].count(sp)
            r = compare_populations(gpu.read(sp, k), refs[k].read(sp), 1e-5 * x.cells, 1e-5,
                                    v0, tie_tol=1e-6, max_tied=max(1, n // 1000),
                                    label=f"inst {k} sp {sp}")
            tied += r["tied"]
            print(case, k, sp, {q: r[q] for q in ("n", "tied", "x_cells", "vx", "vy", "vz")},
                  flush=True)
        sg, so = gpu.stats(inst=k), refs[k].stats()
        for key in STAT_INT:
            assert abs(sg[key] - so[key]) <= tied, (k, key, sg[key], so[key], tied)
        rho_g, _, E_g = gpu.fields(inst=k)
        rho_o, _, E_o = refs[k].fields()
        assert np.allclose(rho_g, rho_o, rtol=0, atol=1e-6 * np.abs(rho_o).max()), k
        assert np.allclose(E_g, E_o, rtol=0, atol=1e-6 * np.abs(E_o).max()), k
