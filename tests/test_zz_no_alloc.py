"""slpic_create_static: a handle whose device workspace is the library's
static per-device array (no device allocation by the library or the
caller) steps exactly like an slpic_create handle of the same setup."""

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


def _gap(**kw):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=3000,
                            n_target=2500, capacity=configs.capacity_for(2500, 3000))
    for k, v in kw.items():
        setattr(inst, k, v)
    return inst


def _same_run(a, b, n_inst, steps, label):
    """Statistics rows, markers and fields of two handles bit-identical."""
    assert a.sync() == 0 and b.sync() == 0
    for k in range(n_inst):
        ha, hb = a.history(0, steps, inst=k), b.history(0, steps, inst=k)
        for f in STAT_INT + ["w_e", "w_i", "w_j", "n_in"]:
            assert np.array_equal(ha[f], hb[f]), (label, k, f)
        for sp in (0, 1):
            compare_populations(a.read(sp, k), b.read(sp, k), 0.0, 0.0,
                                a.scalars(k)["v0"], label=f"{label} inst {k} sp {sp}")
        for fa, fb in zip(a.fields(inst=k), b.fields(inst=k)):
            assert np.array_equal(fa, fb), (label, k)


def test_static_workspace_steps_like_an_allocated_one(xs_argon):
    # first call: two uneven instances, FP64, full physics with population
    # control and a cathode source
    insts = [_gap(),
             configs.Instance(d=0.02, p_torr=0.5, V=250.0, cells=130, gamma_se=0.1,
                              seed_mode=configs.SEED_CATHODE, n_seed=400, n_target=0,
                              capacity=20000)]
    run = configs.Run(precision=64)
    print("no-alloc: call 1, FP64, 2 instances, 30 steps", flush=True)
    ref = slpic.Sim(insts, run, xs_argon)
    st = slpic.Sim(insts, run, xs_argon, static_workspace=True)
    assert st.workspace is None
    # the array holds one handle at a time: a second create is refused and
    # leaves the first one working
    with pytest.raises(slpic.SlpicError) as ei:
        slpic.Sim(insts, run, xs_argon, static_workspace=True)
    assert ei.value.code == -1
    for sim in (ref, st):
        sim.set_source(3.5, inst=1)
        sim.step(30)
    _same_run(st, ref, len(insts), 30, "call 1")
    assert sum(st.stats(inst=k)["n_e"] for k in range(2)) > 0
    first_bytes = st.nbytes
    st.close()
    ref.close()

    # second call, smaller: one FP32 instance in the array the first call
    # left behind
    small = [_gap(cells=40, n_seed=700, n_target=600,
                  capacity=configs.capacity_for(600, 700), V=350.0)]
    run32 = configs.Run(precision=32)
    print("no-alloc: call 2, FP32, 1 instance, 25 steps", flush=True)
    ref = slpic.Sim(small, run32, xs_argon)
    st = slpic.Sim(small, run32, xs_argon, static_workspace=True)
    assert st.nbytes < first_bytes
    for sim in (ref, st):
        sim.step(25)
    _same_run(st, ref, 1, 25, "call 2")
    st.close()
    ref.close()


def test_static_workspace_rejects_a_setup_larger_than_the_array(xs_argon):
    big = [_gap(n_seed=1000, n_target=0, capacity=2_000_000)]
    with pytest.raises(slpic.SlpicError) as ei:
        slpic.Sim(big, configs.Run(precision=32), xs_argon, static_workspace=True)
    assert ei.value.code == -2
    # the refused create holds nothing: the array is free for the next one
    st = slpic.Sim([_gap()], configs.Run(precision=32), xs_argon, static_workspace=True)
    st.step(3)
    assert st.sync() == 0
    st.close()
