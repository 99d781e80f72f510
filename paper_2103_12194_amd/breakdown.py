"""Breakdown classification and breakdown-voltage search (Sec. IV).

Sec. IV decides whether a gap at voltage V is above or below breakdown from
the ion population over 30 ion crossing times: it rises for V > V_b and
falls back to zero for V < V_b, and V_b is bracketed between the highest
voltage found below and the lowest found above.  Here that reading is made
quantitative:

  * the ion population is the physical ion count, the sum of the density
    weights beta w_j over ion markers (Sec. III), so population control
    (which rescales w_j) does not change it;
  * its growth rate lambda is the least-squares slope of ln(population)
    against time over [15, 30] crossing times (after the seeding transient),
    in units of 1 / crossing time; a population that dies out in the window
    has lambda = -inf;
  * an ensemble of independent replicas gives lambda's mean and standard
    error; V_b is the linear zero of the mean lambda(V) between the two
    voltages that bracket it, with its standard error by propagation;
  * a bisection round spreads n voltages over the current bracket and keeps
    the two around the zero.

All stepping is done by the library (many replicas and voltages batched as
instances of one handle); this module only reduces the statistics rows.
"""

import math

import numpy as np

QE = 1.602176634e-19
M_AR = 39.948 * 1.66053906660e-27


def crossing_time(d, V):
    """Ion crossing time of Sec. IV, sqrt(2 m_Ar d / (e E)) with E = V/d."""
    return d * math.sqrt(2.0 * M_AR / (QE * abs(V)))


def growth_rate(t, population, t_cross, window=(15.0, 30.0)):
    """Slope of ln(population) against t / t_cross over the window.

    t: times of the samples [s]; population: physical ion count at those
    times.  Returns -inf if the population reaches zero inside the window.
    """
    t = np.asarray(t, dtype=np.float64)
    pop = np.asarray(population, dtype=np.float64)
    sel = (t >= window[0] * t_cross) & (t <= window[1] * t_cross)
    if np.count_nonzero(sel) < 2:
        raise ValueError("fewer than two samples inside the fit window")
    tt, pp = t[sel] / t_cross, pop[sel]
    if np.any(pp <= 0.0):
        return -math.inf
    x = tt - tt.mean()
    return float(np.dot(x, np.log(pp)) / np.dot(x, x))


def ensemble(rates):
    """Mean and standard error of replica growth rates (-inf if any replica
    died out, which classifies the voltage as below breakdown)."""
    r = np.asarray(rates, dtype=np.float64)
    if r.size == 0:
        raise ValueError("no replicas")
    if np.any(~np.isfinite(r)):
        return -math.inf, 0.0
    se = float(r.std(ddof=1) / math.sqrt(r.size)) if r.size > 1 else math.inf
    return float(r.mean()), se


def zero_crossing(V, lam, se):
    """Breakdown voltage as the linear zero of lambda(V).

    Takes the lowest pair of neighbouring voltages (in increasing V) with
    lambda_a <= 0 < lambda_b, both finite, and returns (V_b, sigma_Vb) with
    sigma from first-order propagation of the two standard errors:
      V_b = V_a - lambda_a dV / D,  D = lambda_b - lambda_a,
      dV_b/dlambda_a = -dV lambda_b / D^2,  dV_b/dlambda_b = dV lambda_a / D^2.
    Returns None if no such pair exists.
    """
    V = np.asarray(V, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    se = np.asarray(se, dtype=np.float64)
    order = np.argsort(V)
    V, lam, se = V[order], lam[order], se[order]
    for a in range(len(V) - 1):
        b = a + 1
        la, lb = lam[a], lam[b]
        if not (math.isfinite(la) and math.isfinite(lb)):
            continue
        if la <= 0.0 < lb:
            dV = V[b] - V[a]
            D = lb - la
            Vb = V[a] - la * dV / D
            ga, gb = -dV * lb / D ** 2, dV * la / D ** 2
            return float(Vb), float(math.sqrt((ga * se[a]) ** 2 + (gb * se[b]) ** 2))
    return None


def bracket(V, above):
    """(highest voltage classified below, lowest classified above) in the
    manner of Sec. IV; either side is None if missing."""
    V = np.asarray(V, dtype=np.float64)
    above = np.asarray(above, dtype=bool)
    lo = V[~above].max() if np.any(~above) else None
    hi = V[above].min() if np.any(above) else None
    return lo, hi


def bisection_voltages(lo, hi, n):
    """n voltages spread evenly over [lo, hi] (both ends included)."""
    if n < 2 or not hi > lo:
        raise ValueError("need n >= 2 and hi > lo")
    return [lo + (hi - lo) * k / (n - 1) for k in range(n)]


def ion_population(rows):
    """Physical ion count per step from the statistics rows of one instance
    (the w_i column: sum of beta w_j over ions)."""
    return np.asarray(rows["w_i"], dtype=np.float64)


def step_and_record(sim, n_steps, chunk=2048):
    """Advance a library handle by n_steps, reading the statistics rows as it
    goes (the device keeps only the last 4096 steps).  Returns the step
    numbers and the physical ion count of every instance at every step:
    (steps[n], pop[n_inst, n])."""
    if not 0 < chunk <= 4096:
        raise ValueError("chunk must be in 1..4096")
    s0 = sim.steps_done()
    steps, pops = [], [[] for _ in range(sim.n_inst)]
    done = 0
    while done < n_steps:
        n = min(chunk, n_steps - done)
        sim.step(n)
        for k in range(sim.n_inst):
            h = sim.history(s0 + done, n, inst=k)
            pops[k].append(ion_population(h))
        steps.append(np.asarray(h["step"], dtype=np.float64))
        done += n
    return np.concatenate(steps), np.array([np.concatenate(p) for p in pops])


def instance_rates(sim, instances, steps, pops, window=(15.0, 30.0)):
    """Growth rate of every instance of a handle from step_and_record's
    output (instances: the records the handle was created from)."""
    out = []
    for k, inst in enumerate(instances):
        dt = sim.scalars(k)["dt"]
        out.append(growth_rate(steps * dt, pops[k], crossing_time(inst.d, inst.V), window))
    return np.array(out)


def paired_difference(rates_a, rates_b):
    """Mean and standard error of the replica-by-replica differences a - b of
    two ensembles run with the same replica seeds (paired samples: the
    correlation between a_k and b_k cancels in the difference).  Replicas
    that died out on both sides are left out; one that died out on one side
    only makes the difference -inf or +inf."""
    a = np.asarray(rates_a, dtype=np.float64)
    b = np.asarray(rates_b, dtype=np.float64)
    if a.shape != b.shape or a.size == 0:
        raise ValueError("paired ensembles must have the same, nonzero size")
    both = np.isneginf(a) & np.isneginf(b)
    a, b = a[~both], b[~both]
    if np.any(~np.isfinite(a)) or np.any(~np.isfinite(b)):
        return (-math.inf if np.any(np.isneginf(a)) else math.inf), 0.0
    d = a - b
    if d.size < 2:
        return float(d.mean()) if d.size else 0.0, math.inf
    return float(d.mean()), float(d.std(ddof=1) / math.sqrt(d.size))


def paired_breakdown_difference(V, rates_a, rates_b, n_boot=2000, seed=1):
    """Difference of the breakdown voltages (zero_crossing of the ensemble
    means) of two paired ensembles, with its standard error from a paired
    bootstrap: replicas are resampled with the same indices on both sides.

    V: voltages [n_v]; rates_a, rates_b: growth rates [n_v, R] with replica k
    of every voltage run from the same seeds on both sides.  Returns
    (Vb_a - Vb_b, se) or None if either side has no zero crossing."""
    ra = np.asarray(rates_a, dtype=np.float64)
    rb = np.asarray(rates_b, dtype=np.float64)
    if ra.shape != rb.shape or ra.ndim != 2 or ra.shape[0] != len(V):
        raise ValueError("rates must be [n_voltages, replicas] on both sides")

    def vb(r):
        z = zero_crossing(V, r.mean(axis=1), np.zeros(len(V)))
        return None if z is None else z[0]
    va, vb0 = vb(ra), vb(rb)
    if va is None or vb0 is None:
        return None
    rng = np.random.default_rng(seed)
    R = ra.shape[1]
    diffs = []
    for _ in range(n_boot):
        k = rng.integers(0, R, size=R)
        a, b = vb(ra[:, k]), vb(rb[:, k])
        if a is not None and b is not None:
            diffs.append(a - b)
    if len(diffs) < n_boot // 2:
        return None
    return va - vb0, float(np.std(diffs, ddof=1))
