"""Expected electron multiplication of the Townsend test gas, two ways.

Test gas: one ionization channel with a constant cross section sigma above
the threshold I, both electrons of an ionization restart at rest, no other
channel, a uniform field E = V/d across the gap, electrons born at rest at
the cathode.  A(x) is the expected number of electrons that reach the anode
per electron born at rest at x; ions made per seed electron are A(0) - 1, and
with gamma_se secondary electrons per ion at the cathode a generation
multiplies by gamma (A(0) - 1) (the breakdown condition of Sec. I when it
equals 1).

continuum_multiplication: the continuous process.  An electron born at rest
at x gains e E (y - x) by y, so it cannot ionize before y = x + l_I,
l_I = I / (e E); beyond that it ionizes at n_g sigma per unit path, and the
two electrons restart at rest.  With u = d - x,
    dA/du = -c A(u) + 2 c A(u - l_I),   A(u) = 1 for u <= l_I,   c = n_g sigma,
a delay equation integrated here by the implicit trapezoid rule on a grid
whose step divides l_I.

discrete_multiplication: the same gas as the time-stepped speed-limited
method sees it.  A speed-limited electron moves exactly v0 dt per step once
faster than v0 (at every energy of interest here); from rest its first
step is shorter by delta = v0^2 / (2 a) (it starts below v0), so an electron
born at rest at x ends its steps at x + k l - delta, l = v0 dt, with energy
e E (k l - delta) (the phase path is that of unlimited motion).  At each end
point at or above the threshold it ionizes with the null-collision
probability P = 1 - exp(-n_g sigma v0 dt); it is absorbed when a step would
end at or beyond d.  Positions are then m l - j delta (j restarts along the
lineage), and A over layer j follows from layer j + 1 by a suffix sum.
"""

import math

import numpy as np

QE = 1.602176634e-19
ME = 9.1093837015e-31
M_AR = 39.948 * 1.66053906660e-27
KB = 1.380649e-23
TORR = 101325.0 / 760.0


def gas_density(p_torr, T_gas=300.0):
    return p_torr * TORR / (KB * T_gas)


def continuum_multiplication(V, d, p_torr, sigma, I, K=400, T_gas=300.0):
    """A(0) of the continuous process (grid step l_I / K)."""
    c = gas_density(p_torr, T_gas) * sigma
    lI = I * d / V
    if lI >= d:
        return 1.0
    h = lI / K
    n = int(math.floor(d / h))
    A = np.ones(n + 2)
    for i in range(K, n):
        f0 = -c * A[i] + 2 * c * A[i - K]
        A[i + 1] = (A[i] + 0.5 * h * (f0 + 2 * c * A[i + 1 - K])) / (1 + 0.5 * h * c)
    hp = d - n * h
    lag = A[n - K] + (A[n - K + 1] - A[n - K]) * hp / h
    f0 = -c * A[n] + 2 * c * A[n - K]
    return (A[n] + 0.5 * hp * (f0 + 2 * c * lag)) / (1 + 0.5 * hp * c)


def discrete_multiplication(V, d, p_torr, sigma, I, cells, cfl, T_gas=300.0):
    """A(0) of the stepped speed-limited process (speed limit sqrt(2 e V / M),
    dt = cfl dx / v0)."""
    c = gas_density(p_torr, T_gas) * sigma
    E = V / d
    a = QE / ME * E
    v0 = math.sqrt(2 * QE * V / M_AR)
    dt = cfl * (d / cells) / v0
    ell = v0 * dt
    delta = v0 * v0 / (2 * a)
    P = -math.expm1(-c * v0 * dt)
    # first step whose end point is at or above the threshold energy
    kmin = max(1, math.ceil((I / E + delta) / ell - 1e-12))
    mmax = int(d / ell) + 3
    jmax = mmax // kmin + 3
    A_next = None
    for j in range(jmax, -1, -1):
        # the last interior end point of layer j + 1
        imax = int(math.ceil((d + (j + 1) * delta) / ell)) + 1
        while imax * ell - (j + 1) * delta >= d:
            imax -= 1
        T = np.zeros(mmax + kmin + 2)
        if A_next is not None:
            for n in range(min(imax, len(T) - 2), -1, -1):
                T[n] = 2 * P * A_next[n] + (1 - P) * T[n + 1]
        A = np.empty(mmax + 1)
        for m in range(mmax + 1):
            n_opp = max(0, imax - (m + kmin) + 1)
            s = (1 - P) ** n_opp
            if A_next is not None and m + kmin <= imax:
                s += T[m + kmin]
            A[m] = s
        A_next = np.concatenate([A, np.ones(kmin + 4)])
    return float(A[0])


def breakdown_voltage(multiplication, gamma, lo, hi, xtol=1e-3):
    """Voltage at which gamma (A(0) - 1) = 1, by bisection on [lo, hi]."""
    from scipy.optimize import brentq
    return brentq(lambda V: gamma * (multiplication(V) - 1.0) - 1.0, lo, hi, xtol=xtol)
