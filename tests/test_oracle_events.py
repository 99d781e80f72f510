"""Pins of the oracle's ionization products, charge-exchange rate,
turning-point absorption and null-collision bound on a non-constant table.

Each test checks a full oracle step against something the oracle does not
compute itself: energy conservation per event, the analytic laws the
products are drawn from, the mean free path of Sec. III, the turning point
of the closed-form orbit, and a brute-force maximum of the collision rate.
"""

import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import configs, xsec
from synth.constants import QE, ME, M_AR, KB, gas_density

I_EV = xsec.I_IZ_EV
B_EV = 10.0


def _field_free_gap(cells=64, v_limit=1e4, d=0.01, p=1.0):
    return configs.Instance(d=d, p_torr=p, V=0.0, cells=cells, gamma_se=0.0,
                            v_limit=v_limit, seed_mode=configs.SEED_NONE,
                            capacity=1 << 20)


def _energy(v):
    return 0.5 * ME * (v["vx"] ** 2 + v["vy"] ** 2 + v["vz"] ** 2) / QE


def _vs_cdf(eps, mu):
    """P(cos chi <= mu) of the Vahedi-Surendra law at energy eps [eV] (from
    its differential cross section, proportional to 1/(1 + eps sin^2(chi/2)));
    isotropic as eps -> 0."""
    mu = np.clip(mu, -1.0, 1.0)
    out = (1.0 + mu) / 2.0
    big = eps > 1e-9
    e = eps[big]
    out[big] = 1.0 - np.log1p(e * (1.0 - mu[big]) / 2.0) / np.log1p(e)
    return out


def _ionize_beam(eps, n=20000, seed=3):
    """One step of a field-free electron beam along +x in which every
    electron ionizes (fixed-event mode): primaries, ejected electrons and
    ions, matched by the position where the event happened."""
    xs = xsec.fixed_event([0.0, 0.0, 1.0])
    sim = oracle.Sim(_field_free_gap(), configs.Run(precision=64, area=1e30,
                                                    ion_B_eV=B_EV), xs)
    rng = np.random.default_rng(seed)
    v = math.sqrt(2 * QE * eps / ME)
    beam = {"cell": rng.integers(20, 40, n).astype(np.int32),
            "off": rng.uniform(0, 1, n), "vx": np.full(n, v),
            "vy": np.zeros(n), "vz": np.zeros(n),
            "id": np.arange(1, n + 1, dtype=np.uint64)}
    sim.load(oracle.ELECTRON, beam)
    sim.step(1)
    st = sim.stats()
    assert st["ionization"] == n
    e, i = sim.read(oracle.ELECTRON), sim.read(oracle.ION)
    top = np.uint64(1) << np.uint64(63)
    prim = {k: a[(e["id"] & top) == 0] for k, a in e.items()}
    ej = {k: a[(e["id"] & top) != 0] for k, a in e.items()}
    out = []
    for pop in (prim, ej, i):
        assert pop["id"].size == n
        x = pop["cell"] + pop["off"]
        order = np.argsort(x, kind="stable")
        out.append({k: a[order] for k, a in pop.items()})
    xp, xe, xi = (p["cell"] + p["off"] for p in out)
    assert np.unique(xp).size == n
    np.testing.assert_array_equal(xp, xe)
    np.testing.assert_array_equal(xp, xi)
    return out


@pytest.mark.parametrize("eps", [30.0, 100.0, 400.0])
def test_ionization_conserves_energy_and_draws_products_from_their_laws(eps):
    prim, ej, ion = _ionize_beam(eps)
    e_sc, e_ej = _energy(prim), _energy(ej)
    avail = eps - I_EV
    # every event: the two electrons share what the ionization energy leaves
    np.testing.assert_allclose(e_sc + e_ej, avail, rtol=0, atol=1e-12 * eps)
    # the ejected electron takes the smaller share, with the Lorentzian
    # spectrum proportional to 1 / (1 + (e / B)^2) on [0, avail / 2]
    assert e_ej.max() <= avail / 2 * (1 + 1e-12) and e_ej.min() >= 0
    cdf = lambda x: np.arctan(np.clip(x, 0, avail / 2) / B_EV) / np.arctan(avail / (2 * B_EV))
    assert stats.kstest(e_ej, cdf).pvalue > 1e-3
    # each electron leaves at the Vahedi-Surendra angle of its own energy,
    # measured from the incident direction (+x): the CDF at the observed
    # cosine is uniform
    for pop, en in ((prim, e_sc), (ej, e_ej)):
        sp = np.sqrt(pop["vx"] ** 2 + pop["vy"] ** 2 + pop["vz"] ** 2)
        mu = pop["vx"] / sp
        u = _vs_cdf(en, mu)
        assert stats.kstest(u, "uniform").pvalue > 1e-3
        # azimuth about the incident direction uniform and independent of
        # the polar angle
        phi = np.arctan2(pop["vz"], pop["vy"])
        assert stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
        h, _, _ = np.histogram2d(u, phi, bins=[6, 6])
        assert stats.chi2_contingency(h)[1] > 1e-3
    # the new ion: a 300 K neutral's velocity
    s = math.sqrt(KB * 300.0 / M_AR)
    for k in ("vx", "vy", "vz"):
        assert stats.kstest(ion[k] / s, "norm").pvalue > 1e-3


def test_angles_at_the_wrong_energy_would_fail():
    # the angle test above has the power to tell the primary's own energy
    # from the incident one: at 100 eV the primary's cosines, transformed
    # with the incident energy, are far from uniform
    prim, _, _ = _ionize_beam(100.0, n=20000, seed=5)
    sp = np.sqrt(prim["vx"] ** 2 + prim["vy"] ** 2 + prim["vz"] ** 2)
    u = _vs_cdf(np.full(sp.size, 100.0), prim["vx"] / sp)
    assert stats.kstest(u, "uniform").pvalue < 1e-6


def _cx_survivors(p_torr, v_beam, v_limit, steps, dt=0.0, n=20000, sigma_cx=5e-19):
    xs = xsec.constant([(xsec.ELASTIC, 0.0)], [0.0], sigma_cx=sigma_cx)
    inst = _field_free_gap(cells=64, v_limit=v_limit, d=0.05, p=p_torr)
    inst.dt = dt
    sim = oracle.Sim(inst, configs.Run(precision=64, area=1e30), xs)
    z = np.zeros(n)
    sim.load(oracle.ION, {"cell": np.full(n, 12, np.int32), "off": z + 0.25,
                          "vx": z + v_beam, "vy": z, "vz": z,
                          "id": np.arange(1, n + 1, dtype=np.uint64)})
    sim.step(steps)
    ions = sim.read(oracle.ION)
    assert ions["id"].size == n
    # an exchange gives the ion a thermal velocity: survivors keep the beam's
    unscattered = np.sum((ions["vx"] == v_beam) & (ions["vy"] == 0) & (ions["vz"] == 0))
    sc = sim.scalars()
    sc["err"] = sim.stats()["err"]
    return unscattered / n, sc, n


def test_charge_exchange_keeps_the_physical_mean_free_path():
    # Sec. III: a marker scatters with probability beta v dt / lambda per
    # step, lambda = 1 / (n_g sigma_cx); the unscattered fraction after the
    # path x' = sum beta v dt is exp(-x' / lambda) whatever the speed limit
    sigma = 5e-19
    # (a) a speed-limited beam (v = 4 v0): each step is v0 dt of path, at
    # the null-collision bound, so the law holds exactly
    frac, sc, n = _cx_survivors(0.05, 4e4, 1e4, steps=8)
    # the rate stayed within the bound (a rate without the speed limit,
    # n_g sigma v = 4 nu'_max, would raise the error bit)
    assert sc["err"] == 0
    lam = 1.0 / (sc["n_g"] * sigma)
    want = math.exp(-8 * 1e4 * sc["dt"] / lam)
    sd = math.sqrt(want * (1 - want) / n)
    assert abs(frac - want) < 4 * sd, (frac, want, sd)
    # (b) a beam below the limit (v = v0 / 2): rate n_g sigma v, sampled
    # against the bound n_g sigma v0 with a step short enough
    # (nu_max dt = 0.01) that the finite-step law is within a tenth of the
    # statistical error of exp(-x / lambda)
    n_g = gas_density(0.05)
    dt = 0.01 / (n_g * sigma * 1e4)
    frac, sc, n = _cx_survivors(0.05, 5e3, 1e4, steps=200, dt=dt)
    assert sc["dt"] == dt
    lam = 1.0 / (sc["n_g"] * sigma)
    want = math.exp(-200 * 5e3 * dt / lam)
    sd = math.sqrt(want * (1 - want) / n)
    assert abs(frac - want) < 4 * sd, (frac, want, sd)
    assert sc["err"] == 0
    # a rate at the bound whatever the speed (n_g sigma v0) would leave
    # exp(-2 x / lambda) in case (b), far outside the bound above


@pytest.mark.parametrize("v_limit", [math.inf, 2e5])
def test_a_turning_point_beyond_an_electrode_absorbs_the_marker(v_limit):
    # Closed-form orbit: in a uniform field a marker moving against its
    # acceleration turns at x_t = x0 - vx^2 / (2 a), whatever the speed
    # limit (the limited orbit has the unlimited phase path).  A flight whose
    # turning point lies beyond an electrode is absorbed there even when it
    # ends inside the gap; one that turns just inside continues.
    V, d, cells = 300.0, 0.01, 64
    dx = d / cells
    xs = xsec.fixed_event([0.0, 0.0, 0.0])
    for species, qm, x0, sign, dt in ((oracle.ELECTRON, QE / ME, 0.5 * dx, -1.0, 1e-9),
                                      (oracle.ION, -QE / M_AR, d - 0.5 * dx, 1.0, 4e-7)):
        a = qm * V / d                  # electrons toward the anode, ions toward the cathode
        for beyond in (True, False):
            # turning point 0.2 dx outside (or inside) the electrode
            edge = 0.0 if species == oracle.ELECTRON else d
            xt = edge + (0.2 * dx if beyond else -0.2 * dx) * (-1 if species == oracle.ELECTRON else 1)
            vx = sign * math.sqrt(2 * abs(a) * abs(xt - x0))
            inst = configs.Instance(d=d, p_torr=0.0, V=V, cells=cells, gamma_se=0.0,
                                    v_limit=v_limit, dt=dt, seed_mode=configs.SEED_NONE,
                                    capacity=4096)
            sim = oracle.Sim(inst, configs.Run(precision=64, area=1e30), xs)
            c = int(x0 // dx)
            sim.load(species, {"cell": np.array([c], np.int32),
                               "off": np.array([x0 / dx - c]), "vx": np.array([vx]),
                               "vy": np.zeros(1), "vz": np.zeros(1),
                               "id": np.array([7], np.uint64)})
            sim.step(1)
            st = sim.stats()
            key = ("abs_e_cathode" if species == oracle.ELECTRON else "abs_i_anode")
            assert st[key] == (1 if beyond else 0), (species, beyond, v_limit)
            left = sim.read(species)
            if not beyond:
                # it turned inside the step and is back in the gap
                x1 = (left["cell"][0] + left["off"][0]) * dx
                assert 0.0 < x1 < d
                assert np.sign(left["vx"][0]) == -sign
                if not (v_limit < math.inf):
                    want = x0 + vx * dt + 0.5 * a * dt * dt
                    assert x1 == pytest.approx(want, rel=1e-12, abs=1e-12 * d)


def test_null_bound_covers_the_argon_table_in_pic():
    # In PIC (no speed limit) nu'(eps) = n_g sigma_T(eps) v(eps) varies over
    # the table; the bound must hold everywhere up to the cap energy and be
    # tight to the table's node spacing.  The brute-force maximum takes
    # sigma_T by linear interpolation of the tables (numpy), the channel
    # thresholds and the constant continuation above the last node.
    xs = synth.argon_like()
    V = 300.0
    inst = configs.Instance(d=0.01, p_torr=1.0, V=V, cells=64, v_limit=math.inf,
                            seed_mode=configs.SEED_NONE)
    sc = oracle.Sim(inst, configs.Run(), xs).scalars()
    ecap = max(xs.energies[-1], 2 * V + 100.0)
    e = np.geomspace(1e-3, ecap, 2_000_000)
    sig = np.zeros_like(e)
    for k in range(xs.n_chan):
        s = np.interp(e, xs.energies, xs.sigma[k])
        s[e < xs.threshold_eV[k]] = 0.0
        sig += s
    rate = sc["n_g"] * sig * np.sqrt(2 * QE * e / ME)
    brute = rate.max()
    print("nu_max", sc["nu_max_e"], "brute force", brute)
    assert sc["nu_max_e"] >= brute
    # node spacing of the 512-point grid is 2.3 % in energy (1.1 % in speed)
    assert sc["nu_max_e"] <= 1.03 * brute
    # and with a speed limit the bound is n_g max(sigma_T) min(v, v0)
    inst.v_limit = 0.0
    sc = oracle.Sim(inst, configs.Run(), xs).scalars()
    lim = np.minimum(np.sqrt(2 * QE * e / ME), sc["v0"])
    brute = (sc["n_g"] * sig * lim).max()
    assert brute <= sc["nu_max_e"] <= 1.03 * brute
