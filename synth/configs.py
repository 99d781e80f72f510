"""Workload parameter sets for the 1D3V argon gap.

Each workload is a list of `Instance` records (one per independent
(p, d, V) gap) plus one `Run` record of settings shared by the batch.  Values
follow the setup of Sec. IV of the paper where it fixes them (absorbing
electrodes, speed limit v0 = sqrt(2 e V / m_Ar), quarter-mean-free-path
cells) and the synthetic-workload recipe otherwise.

Seed modes (shared numbering; the oracle and the library each define them):
    SEED_NONE = 0           markers are loaded explicitly
    SEED_CATHODE = 1        n_seed electrons at x = 0 with zero velocity
                            (the paper's injection, Sec. IV)
    SEED_MAXWELL_CELL0 = 2  n_seed electrons uniform in the first cell with
                            an isotropic Maxwellian of kT_e = 1 eV
"""

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

from .constants import QE, M_AR, ME, gas_density

SEED_NONE, SEED_CATHODE, SEED_MAXWELL_CELL0 = 0, 1, 2

# Paschen's-law fit constants used only to place sweep voltages (Eq. 1 with
# the A, B and gamma_se values quoted for argon in the results section).
PASCHEN_A = 11.5     # 1/(cm Torr)
PASCHEN_B = 176.0    # V/(cm Torr)
PASCHEN_GAMMA = 0.07


@dataclass
class Instance:
    d: float                 # gap [m]
    p_torr: float            # pressure [Torr]
    V: float                 # anode potential [V] (cathode at 0)
    cells: int
    gamma_se: float = 0.07   # ion-induced secondary electron yield
    v_limit: float = 0.0     # speed limit v0 [m/s]; 0 -> sqrt(2 e V/m_Ar)
    dt: float = 0.0          # time step [s]; 0 -> cfl * dx / v0
    seed_mode: int = SEED_MAXWELL_CELL0
    n_seed: int = 0
    n_target: int = 0        # population-control target (0 = off)
    capacity: int = 0        # markers per species (0 -> derived)
    stream: int = -1         # Philox key word 1; < 0 -> the index in its batch

    def speed_limit(self):
        if self.v_limit > 0:
            return self.v_limit
        return math.sqrt(2.0 * QE * self.V / M_AR)

    def dx(self):
        return self.d / self.cells


@dataclass
class Run:
    precision: int = 32      # 32 or 64
    seed: int = 0x5EED
    T_gas: float = 300.0
    area: float = 1.0        # electrode area [m^2]
    w_j0: float = 1.0        # initial flux weight
    cfl: float = 0.5         # v0 dt / dx
    resort_period: int = 0   # cell sort every n steps (0 = never)
    ion_B_eV: float = 10.0   # ionization energy-sharing parameter
    kTe_seed_eV: float = 1.0
    split_frac: float = 0.0  # collision strategy: 0 (or 1) whole markers;
                             # in (0, 1) weight splitting (per-marker w_j)


@dataclass
class Workload:
    name: str
    run: Run
    instances: List[Instance]
    steps: int
    notes: str = ""
    extra: dict = field(default_factory=dict)


def cells_quarter_mfp(d, p_torr, sigma_max, T_gas=300.0, lo=1, hi=1 << 30):
    """Cells so that dx is a quarter of the shortest mean free path."""
    lam = 1.0 / (gas_density(p_torr, T_gas) * sigma_max)
    return int(min(max(math.ceil(4.0 * d / lam), lo), hi))


def paschen_voltage(pd_torr_cm, A=PASCHEN_A, B=PASCHEN_B, gamma=PASCHEN_GAMMA):
    """Eq. (1) breakdown estimate in volts, or None where it is singular."""
    den = math.log(A * pd_torr_cm) - math.log(math.log(1.0 + 1.0 / gamma))
    if den <= 0:
        return None
    return B * pd_torr_cm / den


def capacity_for(n_target, n_seed):
    return int(max(3 * n_target, 4 * n_seed, 4096))


def c1(precision=64):
    """Plain single instance: d=1 cm, p=1 Torr, V=300 V, 64 cells, 1e4 seeds."""
    inst = Instance(d=0.01, p_torr=1.0, V=300.0, cells=64, gamma_se=0.07,
                    seed_mode=SEED_MAXWELL_CELL0, n_seed=10000,
                    n_target=10000)
    inst.capacity = capacity_for(inst.n_target, inst.n_seed)
    return Workload("C1 d=1cm p=1Torr V=300V 64 cells 1e4 markers",
                    Run(precision=precision), [inst], steps=2000)


def c2(V=300.0, precision=32, n_markers=1_000_000):
    """Single instance near the Paschen minimum: d=2 cm, p=1 Torr, 512 cells."""
    inst = Instance(d=0.02, p_torr=1.0, V=float(V), cells=512,
                    gamma_se=0.07, seed_mode=SEED_MAXWELL_CELL0,
                    n_seed=n_markers, n_target=n_markers)
    inst.capacity = capacity_for(inst.n_target, inst.n_seed)
    return Workload(f"C2 d=2cm p=1Torr V={V:g}V 512 cells ~1e6 markers",
                    Run(precision=precision), [inst], steps=20000)


C2_VOLTAGES = [200.0 + 20.0 * k for k in range(11)]


def c3(precision=32, n_markers=10_000_000):
    """Large single instance: d=5 cm, p=10 Torr, V=1000 V, 4096 cells."""
    inst = Instance(d=0.05, p_torr=10.0, V=1000.0, cells=4096,
                    gamma_se=0.07, seed_mode=SEED_MAXWELL_CELL0,
                    n_seed=n_markers, n_target=n_markers)
    inst.capacity = capacity_for(inst.n_target, inst.n_seed)
    return Workload("C3 d=5cm p=10Torr V=1000V 4096 cells ~1e7 markers",
                    Run(precision=precision, resort_period=16), [inst],
                    steps=50000)


def c4(sigma_max, precision=32, n_inst=64, scale=1.0):
    """Batched Paschen sweep: pd log-spaced 0.1..100 Torr cm, d = 1 cm."""
    insts = []
    for i in range(n_inst):
        pd = 0.1 * 1000.0 ** (i / (n_inst - 1))
        cells = cells_quarter_mfp(0.01, pd, sigma_max, lo=128, hi=4096)
        Vp = paschen_voltage(pd) if pd >= 0.3 else None
        V = Vp if Vp is not None else 1000.0
        nt = int(round(scale * 1e4 * 200.0 ** (i / (n_inst - 1))))
        inst = Instance(d=0.01, p_torr=pd, V=V, cells=cells, gamma_se=0.07,
                        seed_mode=SEED_MAXWELL_CELL0, n_seed=nt, n_target=nt)
        inst.capacity = capacity_for(nt, nt)
        insts.append(inst)
    return Workload(f"C4 batched Paschen sweep {n_inst} instances",
                    Run(precision=precision), insts, steps=20000)


def c5(sigma_max, precision=32, n_pd=32, n_v=8, scale=1.0, v_lo=None,
       v_hi=None):
    """Batched bisection round: n_pd pd points x n_v voltages in a bracket."""
    insts = []
    for a in range(n_pd):
        pd = 0.1 * 1000.0 ** (a / (n_pd - 1))
        cells = cells_quarter_mfp(0.01, pd, sigma_max, lo=64, hi=8192)
        Vp = paschen_voltage(pd) or 1000.0
        lo = v_lo[a] if v_lo is not None else 0.5 * Vp
        hi = v_hi[a] if v_hi is not None else 2.0 * Vp
        nt = int(round(scale * min(4e6, 1e4 * 400.0 ** (a / (n_pd - 1)))))
        for b in range(n_v):
            V = lo + (hi - lo) * b / (n_v - 1)
            inst = Instance(d=0.01, p_torr=pd, V=V, cells=cells,
                            gamma_se=0.07, seed_mode=SEED_MAXWELL_CELL0,
                            n_seed=min(nt, 10000), n_target=nt)
            inst.capacity = capacity_for(nt, inst.n_seed)
            insts.append(inst)
    return Workload(f"C5 bisection round {n_pd}x{n_v}", Run(precision=precision),
                    insts, steps=0)


def scaled(w: Workload, markers_scale: float, steps: int = None) -> Workload:
    """A copy of a workload with marker counts scaled (for small test runs)."""
    insts = []
    for inst in w.instances:
        ns = max(1, int(round(inst.n_seed * markers_scale)))
        nt = int(round(inst.n_target * markers_scale)) if inst.n_target else 0
        insts.append(replace(inst, n_seed=ns, n_target=nt,
                             capacity=capacity_for(nt, ns)))
    return Workload(w.name + f" (x{markers_scale:g} markers)", w.run, insts,
                    steps if steps is not None else w.steps, w.notes)


def as_arrays(instances):
    """Column arrays of instance fields (for logging and tables)."""
    keys = ["d", "p_torr", "V", "cells", "gamma_se", "n_seed", "n_target"]
    return {k: np.array([getattr(i, k) for i in instances]) for k in keys}
