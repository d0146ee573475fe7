"""Parity rule between the HIP caster and the FP64 oracle.

For every ray the oracle gives the closest (t, id) and flags marking where
FP32 and FP64 may legitimately differ.  The rule:
  * unflagged rays: hit/miss and triangle id identical, |d - t| <= 1e-5 t;
  * GRAZING_INCIDENCE only: same id, distance tolerance widened to
    max(1e-5, 5e-7 / |cos incidence|) relative (the FP32 direction error is
    amplified by 1 / |cos| along the ray);
  * GRAZING / NEAR_TIE / RANGE_EDGE: counted; the GPU answer must still be a
    legitimate one: the oracle's id with a matching distance, a miss only if
    the oracle's hit itself grazes (or sits on a range edge), or another
    triangle that the ray reaches or grazes in FP64 at the GPU's distance and
    that is not farther than the oracle's hit unless that hit grazes.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

GRAZE = math.sin(2e-6)
REL = 1e-5


def dist_tol(t: float, cos_inc: float | None) -> float:
    rel = REL
    if cos_inc is not None and abs(cos_inc) < 0.05:
        rel = max(REL, 5e-7 / max(abs(cos_inc), 1e-12))
    return rel * t


def check(sensor: dict, vertices, indices, orc: dict, gpu_dist: np.ndarray,
          gpu_tri: np.ndarray) -> dict:
    """Compare GPU results (already gathered at orc['rays']) with oracle output."""
    rays = orc["rays"]
    n = rays.shape[0]
    bad_clean, bad_flag = [], []
    counts = {"rays": n, "flagged": 0, "grazing": 0, "near_tie": 0, "range_edge": 0,
              "grazing_incidence": 0, "flagged_differ": 0, "hits": 0}
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
                ci = None
                if fl & O.GRAZING_INCIDENCE:
                    ci = O.pair(sensor, vertices, indices, g, k_o)["cos_inc"]
                ok = abs(d_g - t_o) <= dist_tol(t_o, ci)
            if ok and k_o == O.MISS:
                ok = math.isinf(d_g)
            if not ok:
                bad_clean.append((g, k_o, t_o, k_g, d_g, fl))
            continue
        counts["flagged"] += 1
        if k_g == k_o:
            if k_o == O.MISS or abs(d_g - t_o) <= dist_tol(t_o, O.pair(sensor, vertices, indices, g, k_o)["cos_inc"]):
                continue
        counts["flagged_differ"] += 1
        best_grazes = False
        if k_o != O.MISS:
            pb = O.pair(sensor, vertices, indices, g, k_o)
            best_grazes = abs(pb["margin"]) <= GRAZE or pb["degenerate"]
        if k_g == O.MISS:
            if best_grazes or (fl & O.RANGE_EDGE):
                continue
            bad_flag.append((g, k_o, t_o, k_g, d_g, fl, "gpu miss"))
            continue
        pk = O.pair(sensor, vertices, indices, g, k_g)
        reach = pk["hit"] or abs(pk["margin"]) <= GRAZE or pk["degenerate"]
        t_k = pk["t"] if pk["hit"] else pk["plane_t"]
        dist_ok = t_k == t_k and abs(d_g - t_k) <= dist_tol(abs(t_k), pk["cos_inc"])
        order_ok = (k_o == O.MISS or t_k <= t_o * (1 + REL) + 1e-6 or best_grazes
                    or (fl & (O.NEAR_TIE | O.RANGE_EDGE)))
        if reach and dist_ok and order_ok:
            continue
        bad_flag.append((g, k_o, t_o, k_g, d_g, fl, f"reach={reach} dist={dist_ok} order={order_ok}"))
    counts["clean_mismatch"] = len(bad_clean)
    counts["flagged_unacceptable"] = len(bad_flag)
    return {"counts": counts, "bad_clean": bad_clean, "bad_flag": bad_flag}


def assert_parity(rep: dict, label: str = ""):
    c = rep["counts"]
    msg = f"{label} {c} first clean mismatches {rep['bad_clean'][:5]} flagged {rep['bad_flag'][:5]}"
    assert c["clean_mismatch"] == 0 and c["flagged_unacceptable"] == 0, msg
