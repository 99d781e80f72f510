"""Seeded marker populations for parity tests.

A population is a dict of column arrays in the structure-of-arrays layout
both implementations load:

    cell  int32    index of the cell holding the marker (x = (cell+off) dx)
    off   float64  offset within the cell in [0, 1)
    vx, vy, vz  float64  true velocity components [m/s]
    id    uint64   unique marker id

Every float value is rounded to the nearest float32 so that an FP32 store of
the population is exact and both sides start from bit-identical states.
Ids are unique; the generator draws them with numpy's seeded PCG64 stream
(these are inputs, not the method's own random draws).
"""

import numpy as np

from .constants import QE, ME, M_AR, KB


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _unique_ids(rng, n, top_bit=True):
    ids = rng.integers(0, 2 ** 62, size=n, dtype=np.uint64)
    ids = np.unique(ids)
    while ids.size < n:
        more = rng.integers(0, 2 ** 62, size=n - ids.size, dtype=np.uint64)
        ids = np.unique(np.concatenate([ids, more]))
    ids = rng.permutation(ids[:n])
    if top_bit:
        ids = ids | np.uint64(1 << 63)
    return ids.astype(np.uint64)


def _isotropic(rng, n):
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([mu, s * np.cos(ph), s * np.sin(ph)])


def _place(rng, n, cells, cell_lo=0, cell_hi=None):
    hi = cells if cell_hi is None else cell_hi
    cell = rng.integers(cell_lo, hi, size=n).astype(np.int32)
    off = _f32(rng.uniform(0.0, 1.0, n))
    off = np.where(off >= 1.0, np.nextafter(np.float32(1), np.float32(0)),
                   off).astype(np.float64)
    return cell, off


def electrons(seed, n, cells, e_lo=0.005, e_hi=300.0, cell_lo=0,
              cell_hi=None, ids=None, beam_frac=0.3):
    """Electrons with log-uniform energies, isotropic or +x beam directions."""
    rng = np.random.default_rng([seed, 1])
    cell, off = _place(rng, n, cells, cell_lo, cell_hi)
    eps = np.exp(rng.uniform(np.log(e_lo), np.log(e_hi), n))
    speed = np.sqrt(2.0 * QE * eps / ME)
    d = _isotropic(rng, n)
    beam = rng.uniform(size=n) < beam_frac
    d[:, beam] = np.array([1.0, 0.0, 0.0])[:, None] * 0.98 + d[:, beam] * 0.02
    d /= np.linalg.norm(d, axis=0)
    v = d * speed
    if ids is None:
        ids = _unique_ids(rng, n)
    return {"cell": cell, "off": off, "vx": _f32(v[0]), "vy": _f32(v[1]),
            "vz": _f32(v[2]), "id": np.asarray(ids, dtype=np.uint64)}


def ions(seed, n, cells, T_gas=300.0, e_beam_hi=200.0, cell_lo=0,
         cell_hi=None, ids=None, beam_frac=0.5):
    """Ar+ ions: thermal, plus a fraction moving toward the cathode."""
    rng = np.random.default_rng([seed, 2])
    cell, off = _place(rng, n, cells, cell_lo, cell_hi)
    sig = np.sqrt(KB * T_gas / M_AR)
    v = rng.normal(0.0, sig, size=(3, n))
    beam = rng.uniform(size=n) < beam_frac
    eb = rng.uniform(0.0, e_beam_hi, size=n)
    v[0, beam] -= np.sqrt(2.0 * QE * eb[beam] / M_AR)
    if ids is None:
        ids = _unique_ids(rng, n)
    return {"cell": cell, "off": off, "vx": _f32(v[0]), "vy": _f32(v[1]),
            "vz": _f32(v[2]), "id": np.asarray(ids, dtype=np.uint64)}


def mixed(seed, n_e, n_i, cells, **kw):
    """Electron and ion populations with disjoint ids."""
    rng = np.random.default_rng([seed, 3])
    ids = _unique_ids(rng, n_e + n_i)
    return (electrons(seed, n_e, cells, ids=ids[:n_e], **kw),
            ions(seed, n_i, cells, ids=ids[n_e:]))


def empty():
    z = np.zeros(0)
    return {"cell": np.zeros(0, np.int32), "off": z, "vx": z, "vy": z,
            "vz": z, "id": np.zeros(0, np.uint64)}
