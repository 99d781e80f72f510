"""Pins of the oracle's deposit and 1D Poisson solve."""

import math

import numpy as np
import pytest

import oracle
import synth
from synth import configs
from synth.constants import EPS0, QE


def _green_phi(N, dx, V, rho):
    # discrete Green's function of -(phi[i-1] - 2 phi[i] + phi[i+1]) on
    # interior nodes with phi[0] = 0, phi[N] = V:
    # phi_i = V i/N + dx^2/eps0 sum_j G_ij rho_j, G_ij = min(i,j)(N-max(i,j))/N
    i = np.arange(N + 1)[:, None]
    j = np.arange(N + 1)[None, :]
    G = np.minimum(i, j) * (N - np.maximum(i, j)) / N
    G[:, 0] = 0
    G[:, N] = 0
    return V * np.arange(N + 1) / N + dx * dx / EPS0 * G @ rho


@pytest.mark.parametrize("N", [2, 3, 17, 64, 513])
def test_poisson_matches_green_function(N):
    rng = np.random.default_rng(N)
    dx = 0.01 / N
    rho = rng.normal(0, 1e-6, N + 1)
    phi, E = oracle.poisson(N, dx, 250.0, rho)
    want = _green_phi(N, dx, 250.0, rho)
    np.testing.assert_allclose(phi, want, rtol=1e-12, atol=1e-12 * 250)


def test_poisson_uniform_charge_is_exact_parabola():
    N, d, V, r0 = 40, 0.02, 123.0, 3.3e-7
    dx = d / N
    x = np.arange(N + 1) * dx
    phi, E = oracle.poisson(N, dx, V, np.full(N + 1, r0))
    want = V * x / d + r0 * x * (d - x) / (2 * EPS0)
    np.testing.assert_allclose(phi, want, rtol=1e-12)
    # interior E = -phi' of the parabola, exact for central differences
    Ew = -(V / d + r0 * (d - 2 * x) / (2 * EPS0))
    np.testing.assert_allclose(E[1:-1], Ew[1:-1], rtol=1e-11)


def test_empty_gap_field_is_uniform():
    phi, E = oracle.poisson(64, 0.01 / 64, 300.0, np.zeros(65))
    np.testing.assert_allclose(E, -300.0 / 0.01, rtol=1e-13)


def test_gauss_law_at_the_electrodes():
    rng = np.random.default_rng(3)
    N, dx = 50, 2e-4
    rho = rng.normal(0, 1e-6, N + 1)
    phi, E = oracle.poisson(N, dx, 10.0, rho)
    # E_N - E_0 = total charge per area / eps0, boundary nodes hold half cells
    q = (rho[1:-1].sum() + 0.5 * (rho[0] + rho[-1])) * dx
    assert E[-1] - E[0] == pytest.approx(q / EPS0, rel=1e-9)


def test_run_conserves_charge_between_markers_and_grid(xs_argon):
    w = configs.c1(precision=64)
    inst = configs.replace(w.instances[0], n_seed=3000, n_target=0)
    run = configs.Run(precision=64, w_j0=1e6)
    sim = oracle.Sim(inst, run, xs_argon)
    for _ in range(30):
        sim.step(1)
        st = sim.stats()
        rho, phi, E = sim.fields()
        dx = sim.scalars()["dx"]
        q_grid = (rho[1:-1].sum() + 0.5 * (rho[0] + rho[-1])) * dx * run.area
        q_markers = QE * (st["w_i"] - st["w_e"])
        assert q_grid == pytest.approx(q_markers, rel=1e-11,
                                       abs=1e-12 * QE * (st["w_i"] + st["w_e"]))
        assert (E[-1] - E[0]) * EPS0 * run.area == pytest.approx(
            q_markers, rel=1e-8, abs=1e-10 * QE * (st["w_i"] + st["w_e"]))


def test_deposit_linear_weights_single_marker():
    inst = configs.Instance(d=0.01, p_torr=0.0, V=0.0, cells=10,
                            v_limit=1e4, seed_mode=configs.SEED_NONE)
    run = configs.Run(precision=64, area=2.0, w_j0=5.0)
    sim = oracle.Sim(inst, run, synth.argon_like())
    # one electron at x = (3 + 0.25) dx moving at 4 v0: beta = 1/4
    pop = {"cell": np.array([3], np.int32), "off": np.array([0.25]),
           "vx": np.array([4e4]), "vy": np.array([0.0]),
           "vz": np.array([0.0]), "id": np.array([9], np.uint64)}
    sim.load(oracle.ELECTRON, pop)
    rho, phi, E = sim.fields()
    dx = 0.001
    wp = 0.25 * 5.0
    want = np.zeros(11)
    want[3] = -QE * wp * 0.75 / (2.0 * dx)
    want[4] = -QE * wp * 0.25 / (2.0 * dx)
    np.testing.assert_allclose(rho, want, rtol=1e-14)


def _long_double_field(N, dx, V, rho):
    """E of the same discrete problem solved in extended precision (x87 long
    double, 64-bit mantissa) by elimination on the tridiagonal system."""
    ld = np.longdouble
    eps0 = ld(8.8541878128e-12)
    r = np.asarray(rho, dtype=ld)
    dx, V = ld(dx), ld(V)
    b = r * dx * dx / eps0
    m = N - 1
    cp = np.zeros(m, dtype=ld)
    dp = np.zeros(m, dtype=ld)
    for k in range(m):
        den = ld(2) if k == 0 else ld(2) + cp[k - 1]
        cp[k] = ld(-1) / den
        dp[k] = (b[k + 1] + (dp[k - 1] if k else ld(0))) / den
    psi = np.zeros(N + 1, dtype=ld)
    psi[m] = dp[m - 1]
    for k in range(m - 2, -1, -1):
        psi[k + 1] = dp[k] - cp[k] * psi[k + 2]
    Ev = -V / (ld(N) * dx)
    E = np.empty(N + 1, dtype=ld)
    E[1:N] = Ev + (psi[0:N - 1] - psi[2:N + 1]) / (2 * dx)
    E[0] = Ev + (psi[0] - psi[1]) / dx - r[0] * dx / (2 * eps0)
    E[N] = Ev + (psi[N - 1] - psi[N]) / dx + r[N] * dx / (2 * eps0)
    return E


@pytest.mark.parametrize("N", [1024, 8192])
def test_field_is_accurate_to_rounding_on_long_grids(N):
    # the marker pushes see E, so on long grids it must keep FP64 accuracy:
    # within a few 1e-16 of the extended-precision solution of the same
    # problem, for a space charge that moves the field by a tenth of V/d
    assert np.finfo(np.longdouble).eps < 1e-18
    rng = np.random.default_rng(N)
    d, V = 0.01, 500.0
    dx = d / N
    rho = rng.normal(0.0, 1.0, N + 1) + 0.3 * np.sin(np.linspace(0, 7, N + 1))
    rho *= 0.1 * (V / d) * 8.8541878128e-12 / d / np.abs(rho).mean()
    _, E = oracle.poisson(N, dx, V, rho)
    ref = _long_double_field(N, dx, V, rho)
    err = float(np.abs(E - ref).max() / np.abs(ref).max())
    print(N, "relative error of E", err)
    assert err < 1e-15
