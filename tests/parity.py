"""Helpers to compare the HIP path with the oracle marker by marker."""

import numpy as np


def by_id(pop):
    order = np.argsort(pop["id"], kind="stable")
    return {k: v[order] for k, v in pop.items()}


def speed(p):
    return np.sqrt(p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2)


def compare_populations(gpu, ref, tol_x_cells, tol_v, v_scale, tie_tol=None,
                        label="", max_tied=None, tol_w=None):
    """Compare two populations keyed by id.

    Without tie_tol the id sets must be identical.  With tie_tol, oracle
    markers whose decision margin along their history is below tie_tol (a
    float decision that FP32 rounding can turn the other way: the relative
    gap of a collision-channel or emission test, a wall distance in cells,
    the gap between the two smallest velocity components that picks the
    scattering frame) are excused: they may be missing on the GPU side (and
    GPU-only ids are allowed up to the same number) and their states are not
    compared; everything else must match.  max_tied bounds the number of
    excused markers.  Positions (cell + offset) must agree within tol_x_cells
    cells, velocity components within tol_v * max(|v_ref|, v_scale).
    Returns a dict of the worst errors and the number of excused markers.
    """
    g, r = by_id(gpu), by_id(ref)
    gid, rid = g["id"], r["id"]
    if tie_tol is None:
        assert gid.shape == rid.shape and np.array_equal(gid, rid), (
            f"{label}: id sets differ ({len(gid)} vs {len(rid)}, "
            f"{len(np.setxor1d(gid, rid))} differ)")
        gi = np.arange(len(gid))
        ri = np.arange(len(rid))
    else:
        common, gi, ri = np.intersect1d(gid, rid, return_indices=True)
        missing = np.setdiff1d(rid, gid)
        extra = np.setdiff1d(gid, rid)
        tie = r["tie"]
        tied = rid[tie < tie_tol]
        if max_tied is not None:
            assert len(tied) <= max_tied, (
                f"{label}: {len(tied)} markers excused, more than {max_tied}")
        assert np.all(np.isin(missing, tied)), (
            f"{label}: {np.sum(~np.isin(missing, tied))} untied oracle markers "
            f"missing on the GPU")
        assert len(extra) <= max(len(tied), 0), (
            f"{label}: {len(extra)} GPU-only markers, {len(tied)} tied")
        keep = tie[ri] >= tie_tol
        gi, ri = gi[keep], ri[keep]
    xg = g["cell"][gi] + g["off"][gi]
    xr = r["cell"][ri] + r["off"][ri]
    ex = np.abs(xg - xr)
    worst = {"x_cells": float(ex.max()) if ex.size else 0.0, "n": int(len(gi)),
             "tied": 0 if tie_tol is None else int(np.count_nonzero(r["tie"] < tie_tol))}
    assert np.all(ex <= tol_x_cells), (
        f"{label}: position error {ex.max():.3e} cells > {tol_x_cells:.1e}")
    scale = np.maximum(speed({k: r[k][ri] for k in ("vx", "vy", "vz")}), v_scale)
    per_marker = np.zeros(len(ri))
    for k in ("vx", "vy", "vz"):
        ev = np.abs(g[k][gi] - r[k][ri]) / scale
        per_marker = np.maximum(per_marker, ev)
        worst[k] = float(ev.max()) if ev.size else 0.0
        if not np.all(ev <= tol_v):
            w = int(np.argmax(ev))
            a, b = gi[w], ri[w]
            detail = {"id": hex(int(r["id"][b])),
                      "ref": [float(r[q][b]) for q in ("cell", "off", "vx", "vy", "vz")],
                      "gpu": [float(g[q][a]) for q in ("cell", "off", "vx", "vy", "vz")],
                      "tie": float(r["tie"][b]) if "tie" in r else None,
                      "n_bad": int(np.sum(ev > tol_v))}
            raise AssertionError(f"{label}: {k} error {ev.max():.3e} > {tol_v:.1e} {detail}")
    worst["v_errors"] = per_marker
    if tol_w is not None:
        # flux weights (weight splitting), relative
        ew = np.abs(g["w"][gi] - r["w"][ri]) / r["w"][ri]
        worst["w"] = float(ew.max()) if ew.size else 0.0
        assert np.all(ew <= tol_w), f"{label}: weight error {ew.max():.3e} > {tol_w:.1e}"
    return worst


STAT_INT = ["n_e", "n_i", "elastic", "excitation", "ionization", "cx",
            "abs_e_cathode", "abs_e_anode", "abs_i_cathode", "abs_i_anode",
            "see", "roulette", "split"]
