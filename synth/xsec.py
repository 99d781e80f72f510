"""Synthetic, argon-shaped electron-neutral cross-section tables.

The paper draws its five electron-argon channels from the Biagi-v7.1 and
Phelps LXCat databases (Sec. IV).  Those tables are not available here, so
this module builds analytic stand-ins with the same qualitative shape on the
same kind of grid: a 512-point log-uniform energy grid from 0.01 eV to
1000 eV, an elastic channel with a Ramsauer minimum near 0.25 eV, one lumped
excitation channel with an 11.5 eV threshold and ionization with a 15.76 eV
threshold peaking near 3e-20 m^2 at about 100 eV.  Each shape is normalised
so that its maximum over the grid nodes equals the stated peak.

The elastic peak is 1.70e-19 m^2 so that the quarter-mean-free-path cell rule
of Sec. IV reproduces the cell counts of Table I (about 218.9 cells per
Torr cm at 300 K).

Ar+ charge exchange is a constant cross section (5e-19 m^2, a synthetic
order-of-magnitude choice, not a value from the paper, which has no ion
collisions).

Channel kinds (shared numbering; the oracle and the library each define the
same three values):
    ELASTIC = 0, EXCITATION = 1, IONIZATION = 2
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

ELASTIC, EXCITATION, IONIZATION = 0, 1, 2

E_MIN_EV = 0.01
E_MAX_EV = 1000.0
N_GRID = 512

I_IZ_EV = 15.76      # argon ionization energy
E_EX_EV = 11.5       # lumped excitation threshold
PEAK_IZ = 3.0e-20
PEAK_EX = 1.0e-20
PEAK_EL = 1.70e-19
SIGMA_CX = 5.0e-19


@dataclass
class CrossSections:
    """Tabulated electron-neutral channels plus the ion charge-exchange value.

    energies      float64[n_grid]  node energies [eV], log-uniform
    sigma         float64[n_chan, n_grid] cross sections at the nodes [m^2]
    threshold_eV  float64[n_chan]  energy below which a channel is closed
    kind          int32[n_chan]    ELASTIC / EXCITATION / IONIZATION
    sigma_cx      Ar+ on Ar charge-exchange cross section [m^2] (0 = off)
    fixed_prob    optional float64[n_chan]: if given, channel k happens with
                  this constant per-step probability instead of the
                  cross-section rate (the fixed-event test mode)
    fixed_prob_cx optional constant per-step charge-exchange probability
    """
    energies: np.ndarray
    sigma: np.ndarray
    threshold_eV: np.ndarray
    kind: np.ndarray
    sigma_cx: float = SIGMA_CX
    fixed_prob: Optional[np.ndarray] = None
    fixed_prob_cx: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n_chan(self):
        return int(self.sigma.shape[0])

    @property
    def n_grid(self):
        return int(self.sigma.shape[1])

    @property
    def e_min(self):
        return float(self.energies[0])

    @property
    def e_max(self):
        return float(self.energies[-1])

    def sigma_total_max(self):
        """Largest total cross section over the grid nodes [m^2]."""
        return float(self.sigma.sum(axis=0).max())


def log_grid(n=N_GRID, e_min=E_MIN_EV, e_max=E_MAX_EV):
    """n node energies e_j = e_min (e_max/e_min)^(j/(n-1)) in eV."""
    j = np.arange(n, dtype=np.float64)
    return e_min * np.exp(j * (np.log(e_max / e_min) / (n - 1)))


def _ionization_shape(e):
    x = e / I_IZ_EV
    out = np.zeros_like(e)
    m = x > 1.0
    out[m] = (1.0 - 1.0 / x[m]) ** 2.5 * np.log(x[m]) / x[m]
    return out


def _excitation_shape(e):
    x = e / E_EX_EV
    out = np.zeros_like(e)
    m = x > 1.0
    out[m] = (1.0 - 1.0 / x[m]) * np.log(x[m]) / x[m]
    return out


def _elastic_shape(e):
    L = np.log(e / 0.25)
    y = e / 10.0
    return (0.01 + L * L) / (1.0 + L * L) * y ** 0.4 / (1.0 + y ** 1.2)


def argon_like(n=N_GRID, sigma_cx=SIGMA_CX):
    """The three-channel synthetic argon set (elastic, excitation, ionization)."""
    e = log_grid(n)
    shapes = [_elastic_shape(e), _excitation_shape(e), _ionization_shape(e)]
    peaks = [PEAK_EL, PEAK_EX, PEAK_IZ]
    sig = np.stack([s * (p / s.max()) for s, p in zip(shapes, peaks)])
    return CrossSections(
        energies=e,
        sigma=sig,
        threshold_eV=np.array([0.0, E_EX_EV, I_IZ_EV]),
        kind=np.array([ELASTIC, EXCITATION, IONIZATION], dtype=np.int32),
        sigma_cx=float(sigma_cx),
        meta={"name": "argon_like", "peaks_m2": peaks},
    )


# three excitation channels in the place of the lumped one (the paper's
# argon set has five channels: elastic, three excitations, ionization);
# synthetic thresholds near argon's 4s, 4p and higher manifolds, with peaks
# summing to the lumped excitation's
EX3_THRESHOLDS_EV = (11.55, 13.0, 14.1)
EX3_PEAK_SHARES = (0.45, 0.35, 0.20)


def _excitation_shape_at(e, threshold):
    x = e / threshold
    out = np.zeros_like(e)
    m = x > 1.0
    out[m] = (1.0 - 1.0 / x[m]) * np.log(x[m]) / x[m]
    return out


def argon_five(n=N_GRID, sigma_cx=SIGMA_CX):
    """Five-channel synthetic argon: elastic, three excitations, ionization."""
    e = log_grid(n)
    shapes = [_elastic_shape(e)]
    peaks = [PEAK_EL]
    for thr, share in zip(EX3_THRESHOLDS_EV, EX3_PEAK_SHARES):
        shapes.append(_excitation_shape_at(e, thr))
        peaks.append(PEAK_EX * share)
    shapes.append(_ionization_shape(e))
    peaks.append(PEAK_IZ)
    sig = np.stack([s * (p / s.max()) for s, p in zip(shapes, peaks)])
    return CrossSections(
        energies=e,
        sigma=sig,
        threshold_eV=np.array([0.0, *EX3_THRESHOLDS_EV, I_IZ_EV]),
        kind=np.array([ELASTIC, EXCITATION, EXCITATION, EXCITATION, IONIZATION],
                      dtype=np.int32),
        sigma_cx=float(sigma_cx),
        meta={"name": "argon_five", "peaks_m2": peaks},
    )


def constant(sig_by_kind, thresholds, n=N_GRID, sigma_cx=0.0):
    """Energy-independent channels (closed-form test gases).

    sig_by_kind: list of (kind, sigma_m2); thresholds: list of eV values.
    """
    e = log_grid(n)
    kinds = np.array([k for k, _ in sig_by_kind], dtype=np.int32)
    sig = np.stack([np.full(n, s, dtype=np.float64) for _, s in sig_by_kind])
    return CrossSections(energies=e, sigma=sig,
                         threshold_eV=np.asarray(thresholds, dtype=np.float64),
                         kind=kinds, sigma_cx=float(sigma_cx),
                         meta={"name": "constant"})


def fixed_event(probs, probs_cx=0.0, base=None):
    """Fixed-event test mode: channel k with constant per-step probability.

    The scatter laws of each channel still apply; only the choice of event
    stops depending on energy, so every event is a function of the counter
    based random draw alone.
    """
    xs = base if base is not None else argon_like()
    p = np.asarray(probs, dtype=np.float64)
    if p.shape != (xs.n_chan,):
        raise ValueError("one probability per channel")
    if p.min() < 0 or p.sum() > 1:
        raise ValueError("probabilities must be >= 0 and sum to <= 1")
    return CrossSections(energies=xs.energies, sigma=xs.sigma,
                         threshold_eV=xs.threshold_eV, kind=xs.kind,
                         sigma_cx=xs.sigma_cx, fixed_prob=p,
                         fixed_prob_cx=float(probs_cx),
                         meta=dict(xs.meta, fixed=True))
