"""Pins of the oracle's collision sampling, scatter laws and bookkeeping."""

import functools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import configs, xsec
from synth.constants import QE, ME, M_AR, KB


# ------------------------------------------------------------ cross sections
def test_table_lookup_nodes_midpoints_threshold_and_clamp(xs_argon):
    inst = configs.Instance(d=0.01, p_torr=1.0, V=300.0, cells=64,
                            seed_mode=0)
    sim = oracle.Sim(inst, configs.Run(), xs_argon)
    e, sg = xs_argon.energies, xs_argon.sigma
    for k in range(3):
        for j in (0, 7, 200, 300, 511):
            if e[j] >= xs_argon.threshold_eV[k]:
                assert sim.sigma(k, e[j]) == pytest.approx(sg[k, j], rel=1e-14)
        for j in (5, 250, 400):
            mid = 0.5 * (e[j] + e[j + 1])
            assert sim.sigma(k, mid) == pytest.approx(
                0.5 * (sg[k, j] + sg[k, j + 1]), rel=1e-12)
        assert sim.sigma(k, 1e-5) == sg[k, 0]
        assert sim.sigma(k, 5e3) == sg[k, -1]
    # channels are closed below threshold even where interpolation is not 0
    assert sim.sigma(2, 15.75) == 0.0
    assert sim.sigma(1, 11.49) == 0.0


def test_null_bound_for_constant_cross_section():
    xs = xsec.constant([(xsec.ELASTIC, 2e-20)], [0.0])
    inst = configs.Instance(d=0.01, p_torr=2.0, V=300.0, cells=64,
                            seed_mode=0)
    sc = oracle.Sim(inst, configs.Run(), xs).scalars()
    # every electron above 0.004 eV is speed-limited, so nu' = n_g sigma v0
    assert sc["nu_max_e"] == pytest.approx(sc["n_g"] * 2e-20 * sc["v0"],
                                           rel=1e-14)


# ------------------------------------------------------------ scatter laws
def _cos_samples(eps, n, seed=0):
    u = np.random.default_rng(seed).uniform(size=n)
    return np.array([oracle.vs_cos_chi(eps, x) for x in u])


@pytest.mark.parametrize("eps", [0.05, 1.0, 30.0, 500.0])
def test_vahedi_surendra_angle_density(eps):
    # differential cross section proportional to 1/(1 + eps sin^2(chi/2)):
    # pdf of mu = cos chi is eps / (2 (1 + eps (1 - mu)/2) ln(1 + eps))
    mu = _cos_samples(eps, 20000, seed=int(eps * 10))
    assert mu.min() >= -1 - 1e-12 and mu.max() <= 1 + 1e-12

    def cdf(m):
        m = np.clip(m, -1, 1)
        return 1.0 - np.log1p(eps * (1 - m) / 2) / np.log1p(eps)
    assert stats.kstest(mu, cdf).pvalue > 1e-3
    pdf_mean = stats.mstats  # noqa: F841 (placeholder to keep scipy import)
    # mean from direct numerical integration of the density
    grid = np.linspace(-1, 1, 200001)
    pdf = eps / (2 * (1 + eps * (1 - grid) / 2) * np.log1p(eps))
    want = np.trapezoid(grid * pdf, grid)
    assert mu.mean() == pytest.approx(want, abs=4 * mu.std() / np.sqrt(mu.size))


def test_isotropic_limit_of_the_angle_law():
    mu = _cos_samples(0.0, 20000)
    assert stats.kstest(mu, stats.uniform(-1, 2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("eps_av", [5.0, 40.0, 300.0])
def test_ejected_energy_lorentzian(eps_av):
    # ejected-electron spectrum proportional to 1/(1 + (e/B)^2) on [0, eps_av/2]
    B = 10.0
    u = np.random.default_rng(1).uniform(size=20000)
    e = np.array([oracle.ejected_energy(eps_av, B, x) for x in u])
    assert e.min() >= 0 and e.max() <= eps_av / 2 * (1 + 1e-12)

    def cdf(x):
        x = np.clip(x, 0, eps_av / 2)
        return np.arctan(x / B) / np.arctan(eps_av / (2 * B))
    assert stats.kstest(e, cdf).pvalue > 1e-3


def test_rotation_keeps_angle_and_spreads_azimuth():
    rng = np.random.default_rng(4)
    for v_in in ([1e6, 0, 0], [3e5, -2e5, 7e5], [0, 0, 2e6], [1, 1, 1e-9]):
        v_in = np.array(v_in, float)
        vh = v_in / np.linalg.norm(v_in)
        outs = []
        for _ in range(4000):
            uc, up = rng.uniform(size=2)
            eps1 = 7.0
            v = oracle.scatter(xsec.EXCITATION, v_in, eps1, uc, up, 0.0)
            sp = math.sqrt(2 * QE * eps1 / ME)
            assert np.linalg.norm(v) == pytest.approx(sp, rel=1e-13)
            assert v @ vh / sp == pytest.approx(1 - 2 * uc, abs=1e-12)
            outs.append(v / sp)
        outs = np.array(outs)
        # isotropic: mean direction ~ 0, second moments ~ 1/3
        assert np.all(np.abs(outs.mean(0)) < 4 / np.sqrt(len(outs)))
        np.testing.assert_allclose((outs ** 2).mean(0), 1 / 3, atol=0.03)


# ------------------------------------------------------------ full-step laws
def _gap(p=1.0, V=300.0, cells=64, v_limit=0.0, gamma=0.0, seed_mode=0,
         n_seed=0):
    return configs.Instance(d=0.01, p_torr=p, V=V, cells=cells,
                            gamma_se=gamma, v_limit=v_limit,
                            seed_mode=seed_mode, n_seed=n_seed)


def _beam(n, speed, cells, cell_lo, seed=0):
    z = np.zeros(n)
    return {"cell": np.full(n, cell_lo, np.int32), "off": z + 0.5,
            "vx": z + speed, "vy": z, "vz": z,
            "id": np.arange(1, n + 1, dtype=np.uint64) + (seed << 40)}


def test_elastic_energy_loss_matches_two_body_kinematics():
    xs = xsec.fixed_event([1.0, 0.0, 0.0])
    inst = _gap(V=0.0, v_limit=1e4)
    sim = oracle.Sim(inst, configs.Run(precision=64), xs)
    pop = _beam(3000, 2e6, 64, 30)
    sim.load(oracle.ELECTRON, pop)
    sim.step(1)
    out = sim.read(oracle.ELECTRON)
    v = np.stack([out["vx"], out["vy"], out["vz"]], 1)
    sp = np.linalg.norm(v, axis=1)
    cosx = v[:, 0] / sp
    m, M = ME, M_AR
    # exact lab-frame speed ratio after an elastic hit on a resting target
    ratio = (m * cosx + np.sqrt(M * M - m * m * (1 - cosx ** 2))) / (m + M)
    np.testing.assert_allclose(sp / 2e6, ratio, rtol=1e-8)


def test_fixed_event_channel_frequencies():
    probs = [0.2, 0.1, 0.05]
    xs = xsec.fixed_event(probs, probs_cx=0.3)
    inst = _gap(V=0.0, v_limit=1e4)
    sim = oracle.Sim(inst, configs.Run(precision=64), xs)
    n = 20000
    sim.load(oracle.ELECTRON, _beam(n, 6e6, 64, 30))
    ions = _beam(n, 100.0, 64, 30, seed=1)
    sim.load(oracle.ION, ions)
    sim.step(1)
    st = sim.stats()
    for key, p in zip(["elastic", "excitation", "ionization"], probs):
        assert abs(st[key] - n * p) < 4 * math.sqrt(n * p * (1 - p)), key
    assert abs(st["cx"] - n * 0.3) < 4 * math.sqrt(n * 0.21)
    assert st["n_e"] == n + st["ionization"]
    assert st["n_i"] == n + st["ionization"]


def test_five_channel_gas_picks_each_excitation_by_its_cross_section():
    # A 20 eV beam in a field-free gap collides once per step with
    # probability P_null; channel k is taken with probability
    # P_null n_g sigma_k(eps) min(v, v0) / nu'_max.  The three excitations
    # are told apart by the energy they leave (20 eV minus the threshold);
    # sigma_k(20 eV) comes from the tables by linear interpolation in energy.
    xs = synth.argon_five()
    n, eps = 200000, 20.0
    v = math.sqrt(2 * QE * eps / ME)
    inst = _gap(V=0.0, v_limit=1e4)
    inst.capacity = 3 * n
    sim = oracle.Sim(inst, configs.Run(precision=64, area=1e30), xs)
    sim.load(oracle.ELECTRON, _beam(n, v, 64, 30))
    sim.step(1)
    sc = sim.scalars()
    p_null = -math.expm1(-sc["nu_max_e"] * sc["dt"])
    scale = p_null * sc["n_g"] * min(v, sc["v0"]) / sc["nu_max_e"]
    sig = [np.interp(eps, xs.energies, xs.sigma[k]) for k in range(5)]
    out = sim.read(oracle.ELECTRON)
    e_out = 0.5 * ME * (out["vx"] ** 2 + out["vy"] ** 2 + out["vz"] ** 2) / QE
    for k in (1, 2, 3):
        want = n * scale * sig[k]
        got = np.count_nonzero(np.abs(e_out - (eps - xs.threshold_eV[k])) < 1e-9)
        assert abs(got - want) < 4 * math.sqrt(want), (k, got, want)
    st = sim.stats()
    for key, ks in (("elastic", [0]), ("excitation", [1, 2, 3]), ("ionization", [4])):
        want = n * scale * sum(sig[k] for k in ks)
        assert abs(st[key] - want) < 4 * math.sqrt(want), (key, st[key], want)


def _surviving_beam_fraction(v_limit, steps, speed=1e6, sigma=4e-20,
                             pic_cfl=0.02):
    xs = xsec.constant([(xsec.ELASTIC, sigma)], [0.0])
    inst = _gap(p=1.0, V=0.0, v_limit=v_limit, cells=400)
    run = configs.Run(precision=64, cfl=0.5, area=1e30)
    if not (v_limit < math.inf):
        inst.dt = pic_cfl * 0.01 / 400 / speed
    sim = oracle.Sim(inst, run, xs)
    n = 20000
    sim.load(oracle.ELECTRON, _beam(n, speed, 400, 5))
    sim.step(steps)
    out = sim.read(oracle.ELECTRON)
    # any scatter gives the marker a transverse velocity
    unscattered = np.sum((out["vy"] == 0) & (out["vz"] == 0))
    sc = sim.scalars()
    dist = steps * min(speed, sc["v0"]) * sc["dt"]
    # per-step law of null-collision sampling: (1 - e^{-nu_max dt}) nu/nu_max
    nu = sc["n_g"] * sigma * min(speed, sc["v0"])
    p_step = -math.expm1(-sc["nu_max_e"] * sc["dt"]) * nu / sc["nu_max_e"]
    return unscattered / n, dist, sc, n, p_step


@pytest.mark.parametrize("v_limit", [5e4, 2e5, math.inf])
def test_beam_keeps_physical_mean_free_path(v_limit):
    # Eq. (15): a SLPIC marker scatters with probability beta v dt / lambda,
    # so the unscattered fraction after a path x is exp(-x/lambda) whatever
    # the speed limit
    steps = 120
    frac, dist, sc, n, p_step = _surviving_beam_fraction(v_limit, steps)
    exact = (1 - p_step) ** steps
    sd = math.sqrt(exact * (1 - exact) / n)
    assert abs(frac - exact) < 4 * sd
    lam = 1.0 / (sc["n_g"] * 4e-20)
    want = math.exp(-dist / lam)
    if v_limit < math.inf:
        # speed-limited markers all sit at the bound: the discrete law is the
        # continuous one exactly
        assert exact == pytest.approx(want, rel=1e-12)
    else:
        # PIC: the law approaches exp(-x/lambda) as nu_max dt -> 0
        assert exact == pytest.approx(want, rel=2 * sc["nu_max_e"] * sc["dt"])


def _renewal_mean(P, ell, delta, d):
    """Expected anode count per electron born at rest at the cathode for the
    discrete process: flights end at x + m ell - delta, each interior end
    point ionizes with probability P, products restart at rest."""
    @functools.lru_cache(maxsize=None)
    def M(m_total, j):
        # electron at rest at position m_total*ell - j*delta
        x = m_total * ell - j * delta
        K = 0
        while x + (K + 1) * ell - delta < d:
            K += 1
        total = (1 - P) ** K
        for m in range(1, K + 1):
            total += (1 - P) ** (m - 1) * P * 2 * M(m_total + m, j + 1)
        return total
    import sys
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(100000)
    try:
        for mt in range(int(d / ell) + 2, -1, -1):
            for j in range(0, mt + 1):
                M(mt, j)
        return M(0, 0)
    finally:
        sys.setrecursionlimit(old)


def test_townsend_multiplication_constant_cross_section():
    # Test gas: one ionization channel with a constant cross section and zero
    # threshold; both electrons of an ionization restart at rest.  Continuous
    # limit (Furry process): mean anode count per seed = exp(n_g sigma d).
    sigma, d, V = 1e-20, 0.01, 300.0
    xs = xsec.constant([(xsec.IONIZATION, sigma)], [0.0])
    inst = _gap(p=1.0, V=V, cells=64, seed_mode=configs.SEED_CATHODE,
                n_seed=3000)
    run = configs.Run(precision=64, area=1e30, cfl=0.5)
    sim = oracle.Sim(inst, run, xs, flags=oracle.FLAG_PRODUCTS_AT_REST)
    sc = sim.scalars()
    anode = 0
    for _ in range(600):
        sim.step(1)
        anode += sim.stats()["abs_e_anode"]
        if sim.count(oracle.ELECTRON) == 0:
            break
    assert sim.count(oracle.ELECTRON) == 0
    mean = anode / inst.n_seed
    ng = sc["n_g"]
    P = -math.expm1(-ng * sigma * sc["v0"] * sc["dt"])
    a = QE / ME * V / d
    want = _renewal_mean(P, sc["v0"] * sc["dt"], sc["v0"] ** 2 / (2 * a), d)
    m_cont = math.exp(ng * sigma * d)
    # the discrete process converges to the Furry mean as the step shrinks
    assert want == pytest.approx(m_cont, rel=0.15)
    sd = math.sqrt(want * (want - 1) / inst.n_seed)
    assert abs(mean - want) < 4 * sd, (mean, want, sd)


def test_bookkeeping_and_population_control(xs_argon):
    w = configs.c1(precision=64)
    inst = configs.replace(w.instances[0], n_seed=4000, n_target=1500)
    sim = oracle.Sim(inst, w.run, xs_argon)
    n_prev = sim.count(0) + sim.count(1)
    wj_prev = sim.scalars()["w_j"]
    saw_roulette = saw_split = False
    for _ in range(300):
        sim.step(1)
        st = sim.stats()
        assert st["n_in"] == n_prev
        absorbed = (st["abs_e_cathode"] + st["abs_e_anode"] +
                    st["abs_i_cathode"] + st["abs_i_anode"])
        n_now = st["n_e"] + st["n_i"]
        pre = n_prev - absorbed + 2 * st["ionization"] + st["see"]
        assert n_now == pre - st["roulette"] + st["split"]
        if n_prev > 2 * inst.n_target:
            saw_roulette = True
            assert st["w_j"] == 2 * wj_prev
            assert abs(st["roulette"] - pre / 2) < 5 * math.sqrt(pre / 4)
        elif 0 < n_prev and 2 * n_prev < inst.n_target:
            saw_split = True
            assert st["w_j"] == wj_prev / 2 and st["split"] == pre
        else:
            assert st["w_j"] == wj_prev
        n_prev, wj_prev = n_now, st["w_j"]
        assert st["err"] == 0
    assert saw_roulette


def test_split_keeps_physical_population():
    xs = xsec.fixed_event([0.0, 0.0, 0.0])
    inst = _gap(V=0.0, v_limit=1e4)
    inst.n_target = 1000
    sim = oracle.Sim(inst, configs.Run(precision=64, w_j0=8.0), xs)
    pop = synth.markers.electrons(3, 100, 64, cell_lo=20, cell_hi=40)
    sim.load(oracle.ELECTRON, pop)
    w_before = None
    sim.step(1)
    st = sim.stats()
    assert st["split"] == 100 and st["n_e"] == 200 and st["w_j"] == 4.0
    ids = sim.read(0)["id"]
    assert len(np.unique(ids)) == 200
    del w_before


def test_secondary_emission_probability():
    xs = xsec.fixed_event([0.0, 0.0, 0.0])
    inst = _gap(V=300.0, gamma=0.3)
    sim = oracle.Sim(inst, configs.Run(precision=64, area=1e30), xs)
    n = 20000
    ions = _beam(n, -3.7e4, 64, 0)
    ions["off"][:] = 0.05
    sim.load(oracle.ION, ions)
    sim.step(1)
    st = sim.stats()
    assert st["abs_i_cathode"] == n
    assert abs(st["see"] - 0.3 * n) < 4 * math.sqrt(n * 0.21)
    e = sim.read(0)
    assert np.all(e["cell"] == 0) and np.all(e["off"] == 0)
    assert np.all(e["vx"] == 0) and np.all(e["id"] >> np.uint64(63) == 1)


def test_energy_dependent_secondary_emission_follows_eq17():
    # Ions released at rest at height x0 in the vacuum field reach the cathode
    # with e E x0 (plus any perpendicular energy they carry): the fraction
    # that emits must follow Eq. (17) at that energy, within binomial error,
    # and be told apart from the constant gamma_se = 0.09 path.
    xs = xsec.fixed_event([0.0, 0.0, 0.0])
    V, cells, n = 1000.0, 16, 60000
    inst = _gap(V=V, cells=cells, gamma=0.09)
    inst.capacity = 4 * n
    dx = inst.d / cells
    v_perp_2k = math.sqrt(2 * QE * 2000.0 / M_AR)
    for cell, off, vperp, extra in ((0, 0.8, 0.0, 0.0), (14, 0.4, 0.0, 0.0),
                                    (0, 0.8, v_perp_2k, 2000.0)):
        sim = oracle.Sim(inst, configs.Run(precision=64, area=1e30), xs,
                         flags=oracle.FLAG_SEE_ENERGY)
        ions = {"cell": np.full(n, cell, np.int32), "off": np.full(n, off),
                "vx": np.zeros(n), "vy": np.full(n, vperp), "vz": np.zeros(n),
                "id": np.arange(n, dtype=np.uint64) + np.uint64(1 << 40)}
        sim.load(oracle.ION, ions)
        hits = see = 0
        for _ in range(400):
            sim.step(1)
            st = sim.stats()
            hits += st["abs_i_cathode"]
            see += st["see"]
            if sim.count(oracle.ION) == 0:
                break
        assert hits == n
        eps = V * (cell + off) * dx / inst.d + extra
        g = oracle.see_yield(eps)
        sd = math.sqrt(g * (1 - g) / n)
        assert abs(see / n - g) < 4 * sd, (eps, see / n, g, sd)
        assert abs(g - 0.09) > 6 * sd, eps   # the constant yield is rejected
    # the two branches of Eq. (17) meet at 700 eV
    assert oracle.see_yield(700.0) == pytest.approx(0.09, rel=1e-15)
    assert oracle.see_yield(700.0 * (1 - 1e-12)) == pytest.approx(0.09, rel=1e-12)


def test_seeded_maxwellian_first_cell(xs_argon):
    inst = _gap(seed_mode=configs.SEED_MAXWELL_CELL0, n_seed=20000)
    sim = oracle.Sim(inst, configs.Run(kTe_seed_eV=1.0), xs_argon)
    e = sim.read(0)
    assert np.all(e["cell"] == 0)
    assert stats.kstest(e["off"], "uniform").pvalue > 1e-3
    s = math.sqrt(QE * 1.0 / ME)
    for k in ("vx", "vy", "vz"):
        assert stats.kstest(e[k] / s, "norm").pvalue > 1e-3
    np.testing.assert_array_equal(np.sort(e["id"]), np.arange(20000))


def test_charge_exchange_thermalizes_ions():
    xs = xsec.fixed_event([0.0, 0.0, 0.0], probs_cx=1.0)
    inst = _gap(V=0.0, v_limit=5e4)
    sim = oracle.Sim(inst, configs.Run(precision=64, T_gas=300.0), xs)
    n = 20000
    sim.load(oracle.ION, _beam(n, 3e4, 64, 30))
    sim.step(1)
    ions = sim.read(1)
    s = math.sqrt(KB * 300.0 / M_AR)
    for k in ("vx", "vy", "vz"):
        assert stats.kstest(ions[k] / s, "norm").pvalue > 1e-3
