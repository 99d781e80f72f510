"""Plain PIC on the GPU (v_limit = +inf: beta == 1 and the PIC time step of
Sec. IV), against the oracle and against SLPIC.

Sec. II.B: with an infinite speed limit SLPIC is PIC.  Sec. IV: the PIC step
resolves the fastest electron, dt = dx / v_max with v_max = sqrt(2 e V / m_e),
while the SLPIC step resolves v0 = v_max sqrt(m_e / m_Ar), so SLPIC takes
sqrt(m_Ar / m_e) (about 270) times fewer steps (Table I).  Sec. III: the
SLPIC collision rate keeps the physical mean free path, so the Townsend
multiplication from the cathode, which fixes the breakdown condition
gamma_se (exp(alpha d) - 1) = 1, must come out the same in both.
"""

import math

import numpy as np
import pytest

import oracle
from synth import configs, xsec
from synth.constants import QE, ME, M_AR
from parity import compare_populations, STAT_INT
from test_oracle_collisions import _renewal_mean

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import paper_2103_12194_amd as slpic  # noqa: E402


def test_fp64_plain_pic_matches_oracle_step_by_step(xs_argon, steps=60):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                            v_limit=math.inf, seed_mode=configs.SEED_MAXWELL_CELL0,
                            n_seed=5000, n_target=3000,
                            capacity=configs.capacity_for(3000, 5000))
    run = configs.Run(precision=64)
    gpu = slpic.Sim([inst], run, xs_argon)
    ref = oracle.Sim(inst, run, xs_argon)
    sg = gpu.scalars()
    v_max = math.sqrt(2 * QE * inst.V / ME)
    assert sg["v0"] == math.inf
    assert sg["dt"] == pytest.approx(run.cfl * (inst.d / inst.cells) / v_max, rel=1e-15)
    for n in range(steps):
        gpu.step(1)
        ref.step(1)
        a, b = gpu.stats(), ref.stats()
        for k in STAT_INT:
            assert a[k] == b[k], (n, k, a[k], b[k])
        assert a["w_e"] == pytest.approx(b["w_e"], rel=1e-9)
    assert gpu.sync() == 0
    assert ref.stats()["n_e"] > 0
    for sp in (0, 1):
        # velocities scaled by the fastest electron speed (v0 is infinite)
        compare_populations(gpu.read(sp), ref.read(sp), 1e-12 * inst.cells, 1e-12,
                            v_max, label=f"species {sp}")
    assert np.allclose(gpu.fields()[2], ref.fields()[2], rtol=1e-11)


def _townsend_gap(v_limit, n_seed):
    return configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.0,
                            v_limit=v_limit, seed_mode=configs.SEED_CATHODE,
                            n_seed=n_seed, capacity=configs.capacity_for(40 * n_seed, n_seed))


def test_slpic_and_pic_give_the_same_townsend_multiplication():
    # Constant-cross-section ionization (zero threshold, both electrons
    # restart at rest, no secondary emission): seeds at rest at the cathode,
    # every electron followed to the anode.  One handle holds the SLPIC gap
    # and the PIC gap (instances may differ in speed limit and step).
    sigma, n_seed = 1e-20, 20000
    xs = xsec.constant([(xsec.IONIZATION, sigma)], [0.0])
    insts = [_townsend_gap(0.0, n_seed), _townsend_gap(math.inf, n_seed)]
    sim = slpic.Sim(insts, configs.Run(precision=32, area=1e30),
                    xs, flags=slpic.FLAG_PRODUCTS_AT_REST | slpic.FLAG_FLUX)
    dt_s, dt_p = sim.scalars(0)["dt"], sim.scalars(1)["dt"]
    # Table I: the SLPIC step is sqrt(m_Ar / m_e) PIC steps
    assert dt_s / dt_p == pytest.approx(math.sqrt(M_AR / ME), rel=1e-12)
    anode = np.zeros(2)
    done, chunk = 0, 256
    while done < 8192:
        sim.step(chunk)
        for k in range(2):
            anode[k] += sim.history(done, chunk, inst=k)["abs_e_anode"].sum()
        done += chunk
        if sim.count(0, 0) == 0 and sim.count(0, 1) == 0:
            break
    assert sim.sync() == 0
    assert sim.count(0, 0) == 0 and sim.count(0, 1) == 0, "electrons left"
    M = anode / n_seed
    m_cont = math.exp(sim.scalars(0)["n_g"] * sigma * insts[0].d)
    sd = math.sqrt(m_cont * (m_cont - 1) / n_seed)
    print(f"multiplication: SLPIC {M[0]:.3f}, PIC {M[1]:.3f} +- {sd:.3f} each "
          f"(continuum exp(n sigma d) = {m_cont:.3f}); {done} steps")
    assert abs(M[0] - M[1]) < 4 * math.sqrt(2) * sd
    # both discretizations sit within 15 % of the continuum value
    for m in M:
        assert m == pytest.approx(m_cont, rel=0.15)
    # flux diagnostic: electrons only move toward the anode, so the flux
    # through the anode node is the anode count and the flux through the
    # plane at x per seed is the multiplication of a gap of length x (for
    # SLPIC, the renewal equation of the discrete process)
    w_j = configs.Run().w_j0
    for k in range(2):
        f = sim.flux(0, inst=k) / w_j
        assert f[insts[k].cells] == anode[k] and f[0] == 0
        assert np.all(np.diff(f) >= 0)
    sc = sim.scalars(0)
    P = -math.expm1(-sc["n_g"] * sigma * sc["v0"] * sc["dt"])
    a = QE / ME * insts[0].V / insts[0].d
    f = sim.flux(0, inst=0) / w_j / n_seed
    for node in (16, 32, 48):
        x = node * insts[0].d / insts[0].cells
        want = _renewal_mean(P, sc["v0"] * sc["dt"], sc["v0"] ** 2 / (2 * a), x)
        sdx = math.sqrt(want * (want - 1) / n_seed)
        assert abs(f[node] - want) < 4 * sdx, (node, f[node], want)
    sim.close()
