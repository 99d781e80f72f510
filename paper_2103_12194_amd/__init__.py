"""MI355X speed-limited PIC / Monte Carlo collision particle step.

Python binding of `libslpic.so` (C ABI in include/slpic.h).  The binding only
marshals arguments: every step of the method runs in the HIP kernels of the
library.  PyTorch supplies the device workspace and the stream.  If the
library is not built, importing works but every call raises SlpicError.
"""

import ctypes as C
import math
import os

import numpy as np

from ._build import LIB, build, stale  # noqa: F401

ELECTRON, ION = 0, 1
ELASTIC, EXCITATION, IONIZATION = 0, 1, 2
SEED_NONE, SEED_CATHODE, SEED_MAXWELL_CELL0 = 0, 1, 2
FLAG_PRODUCTS_AT_REST = 1
FLAG_SEE_ENERGY = 2
FLAG_FLUX = 4
MAX_PARTITIONS = 16   # SLPIC_MAX_PARTITIONS

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "WORKSPACE_TOO_SMALL",
          -3: "CAPACITY_EXCEEDED", -4: "NONFINITE_STATE", -5: "HIP_ERROR",
          -6: "NU_BOUND_EXCEEDED", -7: "NOT_BUILT"}


class SlpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class slpic_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("seed", C.c_uint32),
                ("flags", C.c_uint32), ("resort_period", C.c_int32),
                ("T_gas", C.c_double), ("area", C.c_double),
                ("w_j0", C.c_double), ("cfl", C.c_double),
                ("ion_B_eV", C.c_double), ("kTe_seed_eV", C.c_double),
                ("split_frac", C.c_double)]


class slpic_instance(C.Structure):
    _fields_ = [("d", C.c_double), ("p_torr", C.c_double), ("V", C.c_double),
                ("gamma_se", C.c_double), ("v_limit", C.c_double),
                ("dt", C.c_double), ("cells", C.c_int32),
                ("seed_mode", C.c_int32), ("n_seed", C.c_int64),
                ("n_target", C.c_int64), ("capacity", C.c_int64),
                ("stream", C.c_int64)]


class slpic_xs(C.Structure):
    _fields_ = [("n_chan", C.c_int32), ("n_grid", C.c_int32),
                ("energies", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)),
                ("threshold_eV", C.POINTER(C.c_double)),
                ("kind", C.POINTER(C.c_int32)),
                ("fixed_prob", C.POINTER(C.c_double)),
                ("fixed_prob_cx", C.c_double), ("sigma_cx", C.c_double)]


STAT_FIELDS = ["step", "n_e", "n_i", "n_in", "w_e", "w_i", "w_j", "elastic",
               "excitation", "ionization", "cx", "abs_e_cathode",
               "abs_e_anode", "abs_i_cathode", "abs_i_anode", "see",
               "roulette", "split", "err"]


class slpic_stats(C.Structure):
    _fields_ = [(n, C.c_double if n in ("w_e", "w_i", "w_j") else C.c_int64)
                for n in STAT_FIELDS]


_lib = None
EXPORTS = ["slpic_workspace_bytes", "slpic_create", "slpic_create_static", "slpic_step", "slpic_sync",
           "slpic_use_graph", "slpic_load_markers", "slpic_count",
           "slpic_read_markers", "slpic_read_fields", "slpic_read_flux", "slpic_set_source",
           "slpic_read_stats",
           "slpic_scalars", "slpic_steps_done", "slpic_last_error",
           "slpic_destroy", "slpic_philox_device", "slpic_profile",
           "slpic_kernel_times", "slpic_partitions", "slpic_autotune",
           "slpic_grid", "slpic_sort", "slpic_read_weights", "slpic_launch_shape",
           "slpic_set_launch_shape", "slpic_set_work_distribution",
           "slpic_work_distribution"]


def lib():
    """The loaded library; raises SlpicError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise SlpicError(-7, f"{LIB} is not built (run paper_2103_12194_amd._build.build())")
        L = C.CDLL(LIB)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        P = C.POINTER
        L.slpic_workspace_bytes.restype = C.c_size_t
        L.slpic_workspace_bytes.argtypes = [P(slpic_config), P(slpic_instance), i32, P(slpic_xs)]
        L.slpic_create.argtypes = [P(slpic_config), P(slpic_instance), i32, P(slpic_xs), vp,
                                   C.c_size_t, vp, P(vp)]
        L.slpic_create_static.argtypes = [P(slpic_config), P(slpic_instance), i32, P(slpic_xs),
                                          vp, P(vp)]
        L.slpic_step.argtypes = [vp, i32]
        L.slpic_sync.argtypes = [vp]
        L.slpic_use_graph.argtypes = [vp, i32]
        L.slpic_load_markers.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp]
        L.slpic_count.argtypes = [vp, i32, i32, P(i64)]
        L.slpic_read_markers.argtypes = [vp, i32, i32, i64, P(i64), vp, vp, vp, vp, vp, vp]
        L.slpic_read_fields.argtypes = [vp, i32, vp, vp, vp]
        L.slpic_read_weights.argtypes = [vp, i32, i32, i64, P(i64), vp]
        L.slpic_read_flux.argtypes = [vp, i32, i32, vp, i32]
        L.slpic_set_source.argtypes = [vp, i32, C.c_double]
        L.slpic_read_stats.argtypes = [vp, i32, i64, i32, vp]
        L.slpic_scalars.argtypes = [vp, i32, vp]
        L.slpic_steps_done.restype = i64
        L.slpic_steps_done.argtypes = [vp]
        L.slpic_last_error.restype = C.c_char_p
        L.slpic_last_error.argtypes = [vp]
        L.slpic_destroy.argtypes = [vp]
        L.slpic_profile.argtypes = [vp, i32]
        L.slpic_autotune.argtypes = [vp, i32, P(i32)]
        L.slpic_sort.argtypes = [vp]
        L.slpic_grid.argtypes = [vp, P(i32)]
        L.slpic_launch_shape.argtypes = [vp, P(i32), P(i32)]
        L.slpic_set_launch_shape.argtypes = [vp, i32, i32]
        L.slpic_set_work_distribution.argtypes = [vp, i32]
        L.slpic_work_distribution.argtypes = [vp, P(i32)]
        L.slpic_partitions.argtypes = [vp, i32, i32, P(C.c_int32), P(i64), vp]
        L.slpic_kernel_times.argtypes = [vp, P(C.c_double), P(C.c_double), P(i64)]
        L.slpic_philox_device.argtypes = [vp, C.c_uint32, C.c_uint32, i64, vp, vp]
        _lib = L
    return _lib


def _check(rc, h=None):
    if rc != 0:
        msg = lib().slpic_last_error(h)
        raise SlpicError(rc, msg.decode() if msg else "")
    return rc


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def make_config(run, flags=0):
    return slpic_config(precision=run.precision, seed=run.seed & 0xFFFFFFFF,
                        flags=flags, resort_period=run.resort_period,
                        T_gas=run.T_gas, area=run.area, w_j0=run.w_j0,
                        cfl=run.cfl, ion_B_eV=run.ion_B_eV,
                        kTe_seed_eV=run.kTe_seed_eV,
                        split_frac=float(getattr(run, "split_frac", 0.0)))


def make_instances(insts):
    arr = (slpic_instance * len(insts))()
    for k, i in enumerate(insts):
        cap = i.capacity if i.capacity else max(4 * i.n_seed, 4096)
        arr[k] = slpic_instance(d=i.d, p_torr=i.p_torr, V=i.V,
                                gamma_se=i.gamma_se, v_limit=i.v_limit,
                                dt=i.dt, cells=i.cells, seed_mode=i.seed_mode,
                                n_seed=i.n_seed, n_target=i.n_target,
                                capacity=cap, stream=getattr(i, "stream", -1))
    return arr


class _Xs:
    """slpic_xs plus the arrays it points into."""

    def __init__(self, xs):
        dp = C.POINTER(C.c_double)
        self.e = np.ascontiguousarray(xs.energies, dtype=np.float64)
        self.s = np.ascontiguousarray(xs.sigma, dtype=np.float64)
        self.t = np.ascontiguousarray(xs.threshold_eV, dtype=np.float64)
        self.k = np.ascontiguousarray(xs.kind, dtype=np.int32)
        self.f = (np.ascontiguousarray(xs.fixed_prob, dtype=np.float64)
                  if xs.fixed_prob is not None else None)
        self.c = slpic_xs(
            n_chan=int(self.s.shape[0]), n_grid=int(self.e.shape[0]),
            energies=self.e.ctypes.data_as(dp), sigma=self.s.ctypes.data_as(dp),
            threshold_eV=self.t.ctypes.data_as(dp),
            kind=self.k.ctypes.data_as(C.POINTER(C.c_int32)),
            fixed_prob=self.f.ctypes.data_as(dp) if self.f is not None else None,
            fixed_prob_cx=float(xs.fixed_prob_cx), sigma_cx=float(xs.sigma_cx))


class Sim:
    """A batch of gap instances stepped on the current HIP device.

    insts: list of objects with the slpic_instance fields (d, p_torr, V,
    cells, gamma_se, v_limit, dt, seed_mode, n_seed, n_target, capacity);
    run: object with the slpic_config fields; xs: cross-section tables with
    energies, sigma, threshold_eV, kind, sigma_cx, fixed_prob, fixed_prob_cx.
    """

    def __init__(self, insts, run, xs, flags=0, stream=None, static_workspace=False):
        """static_workspace: take the device workspace from the library's
        per-device static array (slpic_create_static) instead of allocating
        one with torch; at most one such Sim per device at a time."""
        import torch
        if not torch.cuda.is_available():
            raise SlpicError(-5, "no HIP device")
        if not isinstance(insts, (list, tuple)):
            insts = [insts]
        self.n_inst = len(insts)
        self.cells = [int(i.cells) for i in insts]
        self.cfg = make_config(run, flags)
        self.inst = make_instances(insts)
        self.xs = _Xs(xs)
        L = lib()
        nbytes = L.slpic_workspace_bytes(C.byref(self.cfg), self.inst,
                                         self.n_inst, C.byref(self.xs.c))
        if nbytes == 0:
            raise SlpicError(-1, "invalid parameters for the workspace")
        self.nbytes = int(nbytes)
        # a stream of its own (default priority): graph capture is refused on
        # the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        if static_workspace:
            self.workspace = None
            rc = L.slpic_create_static(C.byref(self.cfg), self.inst, self.n_inst,
                                       C.byref(self.xs.c), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h))
        else:
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
            self.workspace.record_stream(self.stream)
            rc = L.slpic_create(C.byref(self.cfg), self.inst, self.n_inst,
                                C.byref(self.xs.c), C.c_void_p(self.workspace.data_ptr()),
                                self.nbytes, C.c_void_p(self.stream.cuda_stream),
                                C.byref(h))
        _check(rc, None)
        self.h = h

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "h", None):
            lib().slpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ stepping
    def step(self, n=1):
        _check(lib().slpic_step(self.h, int(n)), self.h)

    def sync(self):
        return _check(lib().slpic_sync(self.h), self.h)

    def use_graph(self, enable=True):
        _check(lib().slpic_use_graph(self.h, 1 if enable else 0), self.h)

    def autotune(self, trial_steps=4):
        """Pick the fastest particle-kernel grid by timing trial steps (they
        are real steps); returns the grid."""
        g = C.c_int()
        _check(lib().slpic_autotune(self.h, int(trial_steps), C.byref(g)), self.h)
        return int(g.value)

    def sort(self):
        """Sort every instance's markers by cell (enqueued)."""
        _check(lib().slpic_sort(self.h), self.h)

    def grid(self):
        g = C.c_int()
        _check(lib().slpic_grid(self.h, C.byref(g)), self.h)
        return int(g.value)

    def launch_shape(self):
        """(particle-kernel grid, waves per SIMD of its register budget)."""
        g, w = C.c_int(), C.c_int()
        _check(lib().slpic_launch_shape(self.h, C.byref(g), C.byref(w)), self.h)
        return g.value, w.value

    def set_launch_shape(self, grid, waves_per_simd):
        _check(lib().slpic_set_launch_shape(self.h, int(grid), int(waves_per_simd)), self.h)

    def work_distribution(self):
        """1: workgroups claim runs of tiles; 0: equal contiguous shares."""
        d = C.c_int()
        _check(lib().slpic_work_distribution(self.h, C.byref(d)), self.h)
        return d.value

    def set_work_distribution(self, claimed):
        _check(lib().slpic_set_work_distribution(self.h, int(claimed)), self.h)

    def profile(self, enable=True):
        """Record per-kernel HIP events around the following steps."""
        _check(lib().slpic_profile(self.h, 1 if enable else 0), self.h)

    def kernel_times(self):
        """(particle-kernel ms, tail-kernel ms, steps) since profile(True)."""
        g, t, n = C.c_double(), C.c_double(), C.c_int64()
        _check(lib().slpic_kernel_times(self.h, C.byref(g), C.byref(t),
                                        C.byref(n)), self.h)
        return g.value, t.value, int(n.value)

    def steps_done(self):
        return int(lib().slpic_steps_done(self.h))

    # ------------------------------------------------------------ markers
    def load(self, species, pop, inst=0):
        n = len(pop["id"])
        cols = [np.ascontiguousarray(pop["cell"], dtype=np.int32)]
        cols += [np.ascontiguousarray(pop[k], dtype=np.float64)
                 for k in ("off", "vx", "vy", "vz")]
        cols += [np.ascontiguousarray(pop["id"], dtype=np.uint64)]
        _check(lib().slpic_load_markers(self.h, inst, species, n,
                                        *[_p(c) for c in cols]), self.h)

    def count(self, species, inst=0):
        n = C.c_int64()
        _check(lib().slpic_count(self.h, inst, species, C.byref(n)), self.h)
        return int(n.value)

    def partitions(self, species, inst=0):
        """(occupancy of each output partition, slots per partition)."""
        parts, cap = C.c_int32(), C.c_int64()
        out = np.zeros(MAX_PARTITIONS, np.uint32)
        _check(lib().slpic_partitions(self.h, inst, species, C.byref(parts),
                                      C.byref(cap), _p(out)), self.h)
        return out[:parts.value].copy(), int(cap.value)

    def read(self, species, inst=0):
        n = self.count(species, inst)
        out = {"cell": np.zeros(n, np.int32), "off": np.zeros(n),
               "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n),
               "id": np.zeros(n, np.uint64)}
        got = C.c_int64()
        _check(lib().slpic_read_markers(
            self.h, inst, species, n, C.byref(got),
            *[_p(out[k]) for k in ("cell", "off", "vx", "vy", "vz", "id")]),
            self.h)
        if 0.0 < self.cfg.split_frac < 1.0:
            # flux weights (units of w_j), in the same order
            out["w"] = np.zeros(n)
            _check(lib().slpic_read_weights(self.h, inst, species, n, C.byref(got),
                                            _p(out["w"])), self.h)
        return out

    def fields(self, inst=0):
        n = self.cells[inst] + 1
        rho, phi, E = np.zeros(n), np.zeros(n), np.zeros(n)
        _check(lib().slpic_read_fields(self.h, inst, _p(rho), _p(phi), _p(E)),
               self.h)
        return rho, phi, E

    def set_source(self, per_step, inst=0):
        """Continuous cathode source of one instance: per_step markers per
        step at the initial flux weight (electrons at rest at x = 0), from
        the next step on; 0 switches it off."""
        _check(lib().slpic_set_source(self.h, inst, float(per_step)), self.h)

    def flux(self, species, inst=0, reset=False):
        """Time-integrated flux through each node since create or the last
        reset (w_j times net upward crossings per step; needs FLAG_FLUX)."""
        out = np.zeros(self.cells[inst] + 1)
        _check(lib().slpic_read_flux(self.h, inst, species, _p(out), 1 if reset else 0),
               self.h)
        return out

    def stats(self, first_step=None, n=1, inst=0):
        """Statistics rows (dicts) for steps first_step+1 .. first_step+n;
        default: the last step."""
        if first_step is None:
            first_step = self.steps_done() - n
        rows = (slpic_stats * n)()
        _check(lib().slpic_read_stats(self.h, inst, int(first_step), n, rows),
               self.h)
        out = [{f: getattr(r, f) for f in STAT_FIELDS} for r in rows]
        return out[0] if n == 1 else out

    def history(self, first_step, n, inst=0):
        rows = self.stats(first_step, n, inst) if n > 1 else [self.stats(first_step, 1, inst)]
        return {f: np.array([r[f] for r in rows]) for f in STAT_FIELDS}

    def scalars(self, inst=0):
        out = np.zeros(8)
        _check(lib().slpic_scalars(self.h, inst, _p(out)), self.h)
        keys = ["dx", "dt", "v0", "n_g", "nu_max_e", "nu_max_cx", "w_j", "step"]
        return dict(zip(keys, out.tolist()))


def philox_device(ctr, key0, key1):
    """Philox4x32-10 evaluated by the library's device code (test hook)."""
    import torch
    c = torch.as_tensor(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32),
                        device="cuda").contiguous()
    n = c.numel() // 4
    out = torch.empty_like(c)
    s = torch.cuda.current_stream()
    rc = lib().slpic_philox_device(C.c_void_p(c.data_ptr()), key0 & 0xFFFFFFFF,
                                   key1 & 0xFFFFFFFF, n, C.c_void_p(out.data_ptr()),
                                   C.c_void_p(s.cuda_stream))
    _check(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).reshape(-1, 4)


def inf():
    return math.inf
