"""The C ABI library loads, exports what include/slpic.h declares, and its
host-only entry points validate their arguments (no GPU needed)."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2103_12194_amd as slpic
import synth
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slpic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slpic_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    if slpic.stale():
        slpic.build()
    return slpic.lib()


def test_library_exports_every_declared_symbol(built):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(built, n), n
    assert set(names) == set(slpic.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", slpic.LIB],
                         capture_output=True, text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\sT {n}$", out, flags=re.M), n


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(f'''
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu\\n", sizeof(slpic_config), sizeof(slpic_instance),
         sizeof(slpic_xs), sizeof(slpic_stats));
  printf("%zu %zu %zu %zu\\n", offsetof(slpic_config, T_gas),
         offsetof(slpic_instance, cells), offsetof(slpic_xs, fixed_prob_cx),
         offsetof(slpic_stats, err));
  return 0;
}}''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True,
                          check=True).stdout.split("\n")[:2]
    sizes = [int(x) for x in a.split()]
    offs = [int(x) for x in b.split()]
    assert sizes == [C.sizeof(slpic.slpic_config), C.sizeof(slpic.slpic_instance),
                     C.sizeof(slpic.slpic_xs), C.sizeof(slpic.slpic_stats)]
    assert offs == [slpic.slpic_config.T_gas.offset, slpic.slpic_instance.cells.offset,
                    slpic.slpic_xs.fixed_prob_cx.offset, slpic.slpic_stats.err.offset]


def _ws(built, insts, run, xs):
    cfg = slpic.make_config(run)
    arr = slpic.make_instances(insts)
    x = slpic._Xs(xs)
    return built.slpic_workspace_bytes(C.byref(cfg), arr, len(insts), C.byref(x.c))


def test_workspace_size_and_validation(built, xs_argon):
    w = configs.c1()
    n1 = _ws(built, w.instances, w.run, xs_argon)
    assert n1 > 0
    # bigger capacity needs more workspace; FP64 more than FP32
    big = configs.replace(w.instances[0], capacity=10 * w.instances[0].capacity)
    assert _ws(built, [big], w.run, xs_argon) > n1
    r32 = configs.Run(precision=32)
    assert _ws(built, w.instances, r32, xs_argon) < n1
    # any Philox stream below 2^32, or the batch index (negative), is valid
    for st in (-1, 0, (1 << 32) - 1):
        assert _ws(built, [configs.replace(w.instances[0], stream=st)], w.run, xs_argon) == n1
    # invalid setups report 0
    bad = [configs.replace(w.instances[0], cells=1),
           configs.replace(w.instances[0], gamma_se=1.5),
           configs.replace(w.instances[0], d=0.0),
           configs.replace(w.instances[0], capacity=5, n_seed=10),
           configs.replace(w.instances[0], stream=1 << 32)]
    for b in bad:
        assert _ws(built, [b], w.run, xs_argon) == 0
    assert _ws(built, w.instances, configs.Run(precision=16), xs_argon) == 0
    assert _ws(built, w.instances, configs.Run(cfl=1.5), xs_argon) == 0
    xs_bad = synth.argon_like()
    xs_bad.energies = xs_bad.energies.copy()
    xs_bad.energies[10] *= 1.01
    assert _ws(built, w.instances, w.run, xs_bad) == 0
    fx = synth.fixed_event([0.5, 0.4, 0.1])
    fx.fixed_prob = np.array([0.5, 0.4, 0.3])  # sums above one
    assert _ws(built, w.instances, w.run, fx) == 0


def test_create_without_a_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(slpic.SlpicError):
        slpic.Sim(configs.c1().instances, configs.c1().run, synth.argon_like())


def test_split_fraction_is_validated(built, xs_argon):
    import dataclasses
    w = configs.c1()
    for s, flags, ok in ((0.0, 0, True), (0.5, 0, True), (1.0, 0, True),
                         (1.5, 0, False), (-0.1, 0, False), (float("nan"), 0, False),
                         (0.5, slpic.FLAG_FLUX, False), (1.0, slpic.FLAG_FLUX, True)):
        run = dataclasses.replace(w.run, split_frac=s)
        cfg = slpic.make_config(run, flags)
        arr = slpic.make_instances(w.instances)
        x = slpic._Xs(xs_argon)
        n = built.slpic_workspace_bytes(C.byref(cfg), arr, 1, C.byref(x.c))
        assert (n > 0) == ok, (s, flags)
    # weights take one more value per marker slot
    r0 = dataclasses.replace(w.run, split_frac=0.0)
    r1 = dataclasses.replace(w.run, split_frac=0.5)
    n0 = _ws(built, w.instances, r0, xs_argon)
    n1 = _ws(built, w.instances, r1, xs_argon)
    assert n1 > n0


def test_partitions_of_2_gib_or_more_are_refused(built, xs_argon):
    """The kernels address a partition's marker slots by 32-bit byte offsets,
    so a setup whose partitions would reach 2 GiB is refused (size 0): at
    16 partitions that is a capacity of about 1.23e9 markers in FP32 (28
    bytes a slot) and 7.8e8 in FP64 (44 bytes).  Nothing is allocated."""
    w = configs.c1()
    for prec, ok, bad in ((32, 1.20e9, 1.26e9), (64, 7.7e8, 8.0e8)):
        run = configs.Run(precision=prec)
        good = configs.replace(w.instances[0], capacity=int(ok))
        over = configs.replace(w.instances[0], capacity=int(bad))
        assert _ws(built, [good], run, xs_argon) > int(ok) * 4 * (28 if prec == 32 else 44), prec
        assert _ws(built, [over], run, xs_argon) == 0, prec
