"""Oracle for the SLPIC-MCC particle step (TEST INFRASTRUCTURE ONLY).

A ctypes wrapper around `slpic_oracle.c`, a plain FP64 CPU implementation of
the speed-limited PIC step with Monte Carlo collisions.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the GPU library (`paper_2103_12194_amd`) and neither
imports the other; both take their inputs from `synth`.
"""

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "slpic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ELECTRON, ION = 0, 1
FLAG_PRODUCTS_AT_REST = 1
FLAG_SEE_ENERGY = 2
FLAG_FLUX = 4
STAT_NAMES = ["step", "n_e", "n_i", "w_e", "w_i", "w_j", "elastic",
              "excitation", "ionization", "cx", "abs_e_cathode",
              "abs_e_anode", "abs_i_cathode", "abs_i_anode", "see",
              "roulette", "split", "n_in", "err"]
NSTAT = len(STAT_NAMES)


def build(verbose=False):
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("d", C.c_double), ("p_torr", C.c_double), ("V", C.c_double),
        ("gamma_se", C.c_double), ("v_limit", C.c_double), ("dt", C.c_double),
        ("T_gas", C.c_double), ("area", C.c_double), ("w_j0", C.c_double),
        ("cfl", C.c_double), ("ion_B_eV", C.c_double),
        ("kTe_seed_eV", C.c_double), ("sigma_cx", C.c_double),
        ("fixed_prob_cx", C.c_double),
        ("n_seed", C.c_int64), ("n_target", C.c_int64),
        ("cells", C.c_int32), ("seed_mode", C.c_int32),
        ("seed", C.c_uint32), ("instance", C.c_uint32),
        ("flags", C.c_uint32), ("pad0", C.c_int32),
        ("n_chan", C.c_int32), ("n_grid", C.c_int32),
        ("energies", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
        ("threshold_eV", C.POINTER(C.c_double)),
        ("kind", C.POINTER(C.c_int32)),
        ("fixed_prob", C.POINTER(C.c_double)),
        ("split_frac", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.or_create.restype = vp
        L.or_create.argtypes = [C.POINTER(_Params)]
        L.or_destroy.argtypes = [vp]
        L.or_load.argtypes = [vp, C.c_int, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.or_step.argtypes = [vp, C.c_int]
        L.or_count.restype = C.c_int64
        L.or_count.argtypes = [vp, C.c_int]
        L.or_read.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        L.or_read_weights.argtypes = [vp, C.c_int, vp]
        L.or_fields.argtypes = [vp, vp, vp, vp]
        L.or_last_stats.argtypes = [vp, vp]
        L.or_flux.argtypes = [vp, C.c_int, vp]
        L.or_flux_reset.argtypes = [vp]
        L.or_set_source.argtypes = [vp, C.c_double]
        L.or_set_clock.argtypes = [vp, C.c_uint32, C.c_double]
        L.or_scalars.argtypes = [vp, vp]
        L.or_min_margin.restype = C.c_double
        L.or_min_margin.argtypes = [vp]
        L.or_philox4x32.argtypes = [vp, vp, vp]
        L.or_philox4x64.argtypes = [vp, vp, vp]
        L.or_beta.restype = C.c_double
        L.or_beta.argtypes = [C.c_double, C.c_double]
        L.or_sigma.restype = C.c_double
        L.or_sigma.argtypes = [vp, C.c_int, C.c_double]
        L.or_free_flight.restype = C.c_double
        L.or_free_flight.argtypes = [C.c_double] * 5 + [dp, dp]
        L.or_poisson.argtypes = [C.c_int, C.c_double, C.c_double, vp, vp, vp]
        L.or_scatter.argtypes = [C.c_int, vp, C.c_double, C.c_double,
                                 C.c_double, C.c_double, vp]
        L.or_vs_cos_chi.restype = C.c_double
        L.or_vs_cos_chi.argtypes = [C.c_double, C.c_double]
        L.or_ejected_energy.restype = C.c_double
        L.or_ejected_energy.argtypes = [C.c_double] * 3
        L.or_see_yield.restype = C.c_double
        L.or_see_yield.argtypes = [C.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- building blocks
def philox4x32(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x64(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def beta(v, v0):
    return lib().or_beta(float(v), float(v0))


def free_flight(vx, vperp, a, dt, v0):
    """Exact speed-limited flight: returns (tau, displacement, new v_x)."""
    dx = C.c_double()
    vx1 = C.c_double()
    tau = lib().or_free_flight(float(vx), float(vperp), float(a), float(dt),
                               float(v0), C.byref(dx), C.byref(vx1))
    return tau, dx.value, vx1.value


def poisson(n_cells, dx, V, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.zeros(n_cells + 1)
    E = np.zeros(n_cells + 1)
    lib().or_poisson(int(n_cells), float(dx), float(V), _ptr(rho), _ptr(phi),
                     _ptr(E))
    return phi, E


def vs_cos_chi(eps, u):
    return lib().or_vs_cos_chi(float(eps), float(u))


def ejected_energy(eps_av, B, u):
    return lib().or_ejected_energy(float(eps_av), float(B), float(u))


def see_yield(eps_ion):
    """Secondary electrons per ion at the cathode, Eq. (17)."""
    return lib().or_see_yield(float(eps_ion))


def scatter(kind, v_in, eps_out, u_chi, u_phi, vs_eps):
    v = np.ascontiguousarray(v_in, dtype=np.float64)
    out = np.zeros(3)
    lib().or_scatter(int(kind), _ptr(v), float(eps_out), float(u_chi),
                     float(u_phi), float(vs_eps), _ptr(out))
    return out


# ---------------------------------------------------------------- simulation
class Sim:
    """One gap instance stepped by the oracle.

    inst: synth.configs.Instance, run: synth.configs.Run,
    xs: synth.CrossSections, instance_index: Philox key word 1 (the
    instance's index in a batch), unless inst.stream >= 0 sets it.
    """

    def __init__(self, inst, run, xs, instance_index=0, flags=0):
        self._keep = []
        e = np.ascontiguousarray(xs.energies, dtype=np.float64)
        sg = np.ascontiguousarray(xs.sigma, dtype=np.float64)
        th = np.ascontiguousarray(xs.threshold_eV, dtype=np.float64)
        kd = np.ascontiguousarray(xs.kind, dtype=np.int32)
        self._keep += [e, sg, th, kd]
        fp = None
        if xs.fixed_prob is not None:
            fp = np.ascontiguousarray(xs.fixed_prob, dtype=np.float64)
            self._keep.append(fp)
        dp = C.POINTER(C.c_double)
        P = _Params(
            d=inst.d, p_torr=inst.p_torr, V=inst.V, gamma_se=inst.gamma_se,
            v_limit=inst.v_limit, dt=inst.dt, T_gas=run.T_gas, area=run.area,
            w_j0=run.w_j0, cfl=run.cfl, ion_B_eV=run.ion_B_eV,
            kTe_seed_eV=run.kTe_seed_eV, sigma_cx=xs.sigma_cx,
            fixed_prob_cx=xs.fixed_prob_cx, n_seed=inst.n_seed,
            n_target=inst.n_target, cells=inst.cells,
            seed_mode=inst.seed_mode, seed=run.seed & 0xFFFFFFFF,
            instance=inst.stream if getattr(inst, "stream", -1) >= 0 else instance_index,
            flags=flags, pad0=0,
            n_chan=xs.n_chan, n_grid=xs.n_grid,
            energies=e.ctypes.data_as(dp), sigma=sg.ctypes.data_as(dp),
            threshold_eV=th.ctypes.data_as(dp),
            kind=kd.ctypes.data_as(C.POINTER(C.c_int32)),
            fixed_prob=fp.ctypes.data_as(dp) if fp is not None else None,
            split_frac=float(getattr(run, "split_frac", 0.0)))
        self.cells = inst.cells
        self.h = lib().or_create(C.byref(P))
        if not self.h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def load(self, species, pop):
        n = len(pop["id"])
        cols = [np.ascontiguousarray(pop["cell"], dtype=np.int32)]
        cols += [np.ascontiguousarray(pop[k], dtype=np.float64)
                 for k in ("off", "vx", "vy", "vz")]
        cols += [np.ascontiguousarray(pop["id"], dtype=np.uint64)]
        rc = lib().or_load(self.h, species, n, *[_ptr(c) for c in cols])
        if rc:
            raise MemoryError("oracle load failed")

    def step(self, n=1):
        rc = lib().or_step(self.h, int(n))
        if rc == -1:
            raise MemoryError("oracle step failed")
        return rc

    def count(self, species):
        return int(lib().or_count(self.h, species))

    def read(self, species):
        n = self.count(species)
        out = {"cell": np.zeros(n, np.int32), "off": np.zeros(n),
               "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n),
               "id": np.zeros(n, np.uint64), "tie": np.zeros(n)}
        lib().or_read(self.h, species, *[_ptr(out[k]) for k in
                                         ("cell", "off", "vx", "vy", "vz",
                                          "id", "tie")])
        out["w"] = np.zeros(n)
        lib().or_read_weights(self.h, species, _ptr(out["w"]))
        return out

    def fields(self):
        n = self.cells + 1
        rho, phi, E = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().or_fields(self.h, _ptr(rho), _ptr(phi), _ptr(E))
        return rho, phi, E

    def flux(self, species, reset=False):
        """Time-integrated flux through each node (sum over steps of w_j
        times the net upward crossings), needs FLAG_FLUX."""
        out = np.zeros(self.cells + 1)
        lib().or_flux(self.h, species, _ptr(out))
        if reset:
            lib().or_flux_reset(self.h)
        return out

    def set_source(self, per_step):
        """Continuous cathode source: per_step markers per step at the
        initial flux weight (electrons at rest at x = 0); 0 switches it off."""
        if lib().or_set_source(self.h, float(per_step)) != 0:
            raise ValueError(f"source rate {per_step} outside [0, 2^24]")

    def set_clock(self, step, w_j):
        """Continue a run from its step counter (which keys the draws) and
        flux weight w_j; the field is re-solved from the markers present."""
        if lib().or_set_clock(self.h, int(step), float(w_j)) != 0:
            raise ValueError(f"flux weight {w_j} must be finite and positive")

    def stats(self):
        row = np.zeros(NSTAT)
        lib().or_last_stats(self.h, _ptr(row))
        return dict(zip(STAT_NAMES, row.tolist()))

    def scalars(self):
        out = np.zeros(8)
        lib().or_scalars(self.h, _ptr(out))
        keys = ["dx", "dt", "v0", "n_g", "nu_max_e", "nu_max_cx", "w_j",
                "step"]
        return dict(zip(keys, out.tolist()))

    def min_margin(self):
        return float(lib().or_min_margin(self.h))

    def sigma(self, chan, eps):
        return lib().or_sigma(self.h, int(chan), float(eps))


def run_history(inst, run, xs, steps, instance_index=0, every=1):
    """Step an instance and return the per-step statistics as arrays."""
    sim = Sim(inst, run, xs, instance_index)
    rows = []
    for n in range(steps):
        sim.step(1)
        if (n + 1) % every == 0:
            rows.append(sim.stats())
    return sim, {k: np.array([r[k] for r in rows]) for k in STAT_NAMES}


isfinite = math.isfinite
