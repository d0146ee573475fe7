"""Parity rule between the HIP caster and the FP64 oracle.

For every ray the oracle gives the closest (t, id), the second best (t2, id2)
on another triangle, and flags marking where single and double precision may
legitimately differ.  The rule:

  * Unflagged rays: hit/miss and triangle id identical, |d - t| <= tol(t),
    tol = 1e-5 t, the stated criterion.
  * GRAZING_INCIDENCE only (|cos incidence| < 0.05 for the hit triangle):
    same id; tol widened to max(1e-5, 5e-7 / |cos|) t.  The FP32 distance is
    h * rcp(d . n): the direction from rounded tables (<= 1.9e-7), the rounded
    unit normal (<= 6e-8) and the three-term dot product (<= 1.2e-7) give an
    absolute error of at most about 3.7e-7 in d . n, i.e. a relative error of
    3.7e-7 / |cos| in t, plus about 3e-7 from the reciprocal and the plane
    distance.  Below |cos| = 0.05 that bound exceeds 1e-5, and 5e-7 / |cos|
    covers it with a quarter to spare.  The widened tolerance is the oracle's
    distance band (`dist_band` in the oracle).
  * GRAZING / NEAR_TIE / RANGE_EDGE rays are counted, and the GPU answer must
    still be a legitimate one:
      - the oracle's id at a matching distance; or
      - a miss, only if the oracle's hit grazes (within 1e-6 rad of its
        boundary) or its distance band holds a range limit, and so does the
        second best, if there is one; or
      - another triangle k that the ray reaches in FP64 (a face hit, or within
        1e-6 rad of k's boundary), at k's FP64 distance, inside the range
        limits up to k's band, and not behind the oracle's hit beyond the two
        bands -- unless the oracle's hit grazes, in which case k may be the
        second best (or lie behind it if the second best grazes too).

Besides pass/fail, the report carries how many rays took the widened
tolerance and the largest relative distance error seen, both plain and
scaled by |cos incidence|, so that the margin of the widened tolerance is
measured, not assumed.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

GRAZE = math.sin(1e-6)
REL = 1e-5
WIDE = 5e-7          # widened tolerance: WIDE / |cos| relative, below |cos| = WIDE / REL
MAX_KEYS = ("max_rel_err", "max_rel_err_x_cos")


def band(cos_inc: float | None) -> float:
    """Relative distance tolerance for a hit at incidence cosine cos_inc."""
    if cos_inc is None or not math.isfinite(cos_inc):
        return REL
    return max(REL, WIDE / max(abs(cos_inc), 1e-300))


def dist_tol(t: float, cos_inc: float | None) -> float:
    return band(cos_inc) * t


def _near_limit(t: float, b: float, dmin: float, dmax: float) -> bool:
    return abs(t - dmin) <= b * dmin or abs(t - dmax) <= b * dmax


def _grazes(p: dict) -> bool:
    return abs(p["margin"]) <= GRAZE or p["degenerate"]


def check(sensor: dict, vertices, indices, orc: dict, gpu_dist: np.ndarray,
          gpu_tri: np.ndarray) -> dict:
    """Compare GPU results (already gathered at orc['rays']) with oracle output."""
    rays = orc["rays"]
    n = rays.shape[0]
    dmin = float(np.float32(sensor.get("range_min", 0.05)))
    dmax = float(np.float32(sensor.get("range_max", 1000.0)))
    bad_clean, bad_flag = [], []
    counts = {"rays": n, "flagged": 0, "grazing": 0, "near_tie": 0, "range_edge": 0,
              "grazing_incidence": 0, "flagged_differ": 0, "hits": 0, "widened": 0,
              "max_rel_err": 0.0, "max_rel_err_x_cos": 0.0}

    def pair(g, k):
        return O.pair(sensor, vertices, indices, g, k)

    def note_err(d_g, t, ci):
        rel = abs(d_g - t) / t
        counts["max_rel_err"] = max(counts["max_rel_err"], rel)
        if ci is not None and abs(ci) < WIDE / REL:
            counts["widened"] += 1
            counts["max_rel_err_x_cos"] = max(counts["max_rel_err_x_cos"], rel * abs(ci))

    for i in range(n):
        g = int(rays[i])
        fl = int(orc["flags"][i])
        k_o = int(orc["tri"][i])
        t_o = float(orc["t"][i])
        k_g = int(gpu_tri[i])
        d_g = float(gpu_dist[i])
        if k_o != O.MISS:
            counts["hits"] += 1
        if fl & O.GRAZING_INCIDENCE:
            counts["grazing_incidence"] += 1
        hard = fl & (O.GRAZING | O.NEAR_TIE | O.RANGE_EDGE)
        if fl & O.GRAZING:
            counts["grazing"] += 1
        if fl & O.NEAR_TIE:
            counts["near_tie"] += 1
        if fl & O.RANGE_EDGE:
            counts["range_edge"] += 1
        if not hard:
            ok = k_g == k_o
            if ok and k_o != O.MISS:
                ci = pair(g, k_o)["cos_inc"] if fl & O.GRAZING_INCIDENCE else None
                ok = abs(d_g - t_o) <= dist_tol(t_o, ci)
                note_err(d_g, t_o, ci)
            if ok and k_o == O.MISS:
                ok = math.isinf(d_g)
            if not ok:
                bad_clean.append((g, k_o, t_o, k_g, d_g, fl))
            continue
        counts["flagged"] += 1
        pb = pair(g, k_o) if k_o != O.MISS else None
        if k_g == k_o:
            if k_o == O.MISS:
                if math.isinf(d_g):
                    continue
            elif abs(d_g - t_o) <= dist_tol(t_o, pb["cos_inc"]):
                note_err(d_g, t_o, pb["cos_inc"])
                continue
            bad_flag.append((g, k_o, t_o, k_g, d_g, fl, "same id, distance off"))
            continue
        counts["flagged_differ"] += 1
        best_grazes = pb is not None and _grazes(pb)
        b_o = band(pb["cos_inc"]) if pb is not None else REL
        if k_g == O.MISS:
            # every in-range hit the ray has must be uncertain: the best, and
            # the second best behind it (a clean second best would be hit)
            ok = pb is not None and (best_grazes or _near_limit(t_o, b_o, dmin, dmax))
            k2 = int(orc["tri2"][i])
            if ok and k2 != O.MISS:
                p2 = pair(g, k2)
                ok = _grazes(p2) or _near_limit(float(orc["t2"][i]), band(p2["cos_inc"]),
                                                 dmin, dmax)
            if ok:
                continue
            bad_flag.append((g, k_o, t_o, k_g, d_g, fl, "gpu miss"))
            continue
        pk = pair(g, k_g)
        reach = pk["hit"] or _grazes(pk)
        t_k = pk["t"] if pk["hit"] else pk["plane_t"]
        b_k = band(pk["cos_inc"])
        dist_ok = math.isfinite(t_k) and abs(d_g - t_k) <= b_k * abs(t_k)
        range_ok = math.isfinite(t_k) and dmin * (1 - b_k) <= t_k <= dmax * (1 + b_k)
        order_ok = k_o == O.MISS or t_k <= t_o * (1 + max(b_o, b_k))
        if not order_ok and best_grazes:
            k2 = int(orc["tri2"][i])
            t2 = float(orc["t2"][i])
            if k2 == O.MISS or k2 == k_g:
                order_ok = True
            else:
                p2 = pair(g, k2)
                order_ok = t_k <= t2 * (1 + max(band(p2["cos_inc"]), b_k)) or _grazes(p2)
        if reach and dist_ok and range_ok and order_ok:
            continue
        bad_flag.append((g, k_o, t_o, k_g, d_g, fl,
                         f"reach={reach} dist={dist_ok} range={range_ok} order={order_ok}"))
    counts["clean_mismatch"] = len(bad_clean)
    counts["flagged_unacceptable"] = len(bad_flag)
    return {"counts": counts, "bad_clean": bad_clean, "bad_flag": bad_flag}


def merge(total: dict, counts: dict) -> dict:
    """Accumulate one report's counts into `total` (sums, and maxima for the error keys)."""
    for k, x in counts.items():
        if k in MAX_KEYS:
            total[k] = max(total.get(k, 0.0), x)
        else:
            total[k] = total.get(k, 0) + x
    return total


def assert_parity(rep: dict, label: str = ""):
    c = rep["counts"]
    msg = f"{label} {c} first clean mismatches {rep['bad_clean'][:5]} flagged {rep['bad_flag'][:5]}"
    assert c["clean_mismatch"] == 0 and c["flagged_unacceptable"] == 0, msg


def hit_match(orc: dict, gpu_dist: np.ndarray, tol_m: float = 1e-3) -> np.ndarray:
    """Per ray: the GPU answer matches the oracle's hit distance within
    `tol_m` metres, or both miss (the hit-distance criterion of the paper's
    accuracy section, 1 mm absolute)."""
    t = orc["t"]
    d = np.asarray(gpu_dist, np.float64)
    both_miss = np.isinf(t) & np.isinf(d)
    fin = np.isfinite(t) & np.isfinite(d)
    close = np.zeros_like(fin)
    close[fin] = np.abs(d[fin] - t[fin]) <= tol_m
    return both_miss | close


def sort_keys(dist: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """The 64-bit closest-hit keys (order-preserving distance bits above the
    triangle id) of distances >= 0 (or +inf) and ids, as uint64."""
    b = np.asarray(dist, np.float32).view(np.uint32).astype(np.uint64) | np.uint64(0x80000000)
    return (b << np.uint64(32)) | np.asarray(tri, np.uint32).astype(np.uint64)
