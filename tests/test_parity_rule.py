"""The parity rule itself, on planted GPU answers (CPU only).

Each case plants a wrong (or a legitimately different) answer for one ray and
checks that the rule rejects (or accepts) it.  The geometry is a sensor at the
origin whose ray 2 points along +x, and square-ish walls across that ray."""
import numpy as np

from oracle import oracle as O
from paper_2605_10457_amd import synth
from tests import parity


def _setup(rmax=10.0):
    s = synth.sensor((0.0, 0.0, 0.0), 0.0, np.array([0.0], np.float32), 4, 360.0, 0.05, rmax)
    return s, np.array([2], np.uint32)


def _walls(*xs, half=1.0):
    v = []
    for x in xs:
        v += [[x, -half, -half], [x, half, -half], [x, 0, half]]
    return np.array(v, np.float32), np.arange(3 * len(xs), dtype=np.uint32).reshape(-1, 3)


def _rule(s, v, f, r, d, t):
    orc = O.cast(s, v, f, rays=r)
    rep = parity.check(s, v, f, orc, np.array([d], np.float32), np.array([t], np.uint32))
    return rep["counts"]["clean_mismatch"] + rep["counts"]["flagged_unacceptable"] == 0


def test_hidden_range_max_triangle_does_not_excuse_a_miss():
    s, r = _setup(10.0)
    v, f = _walls(5.0, 10.0)
    assert _rule(s, v, f, r, 5.0, 0)
    assert not _rule(s, v, f, r, np.inf, O.MISS), "a miss behind a clean 5 m hit"
    assert not _rule(s, v, f, r, 10.0, 1), "the hidden 10 m triangle"


def test_near_tie_excuses_only_the_tied_pair():
    s, r = _setup(20.0)
    x2 = float(np.float32(5.0 * (1 + 5e-6)))
    v, f = _walls(5.0, x2, 8.0)
    orc = O.cast(s, v, f, rays=r)
    assert orc["flags"][0] & O.NEAR_TIE
    assert _rule(s, v, f, r, 5.0, 0)
    assert _rule(s, v, f, r, x2, 1), "the other triangle of the tie"
    assert not _rule(s, v, f, r, 8.0, 2), "a third triangle behind the tie"
    assert not _rule(s, v, f, r, np.inf, O.MISS), "a miss"


def test_range_edge_best_hit_may_be_missed():
    s, r = _setup(10.0)
    v, f = _walls(10.0)
    assert _rule(s, v, f, r, np.inf, O.MISS)
    assert _rule(s, v, f, r, 10.0, 0)
    # but not a triangle beyond the range limit
    v2, f2 = _walls(10.0, 12.0)
    assert not _rule(s, v2, f2, r, 12.0, 1)


def test_out_of_range_hit_just_past_the_limit_is_accepted():
    s, r = _setup(10.0)
    v, f = _walls(10.00003)
    assert _rule(s, v, f, r, np.inf, O.MISS)
    assert _rule(s, v, f, r, 10.00003, 0)
    assert not _rule(s, v, f, r, 10.2, 0), "distance off"


def test_clean_distance_tolerance():
    s, r = _setup(20.0)
    v, f = _walls(5.0)
    assert _rule(s, v, f, r, 5.0 * (1 + 0.9e-5), 0)
    assert not _rule(s, v, f, r, 5.0 * (1 + 2e-5), 0)
    assert not _rule(s, v, f, r, 5.0, 1)


def test_grazing_best_allows_the_second_best_only():
    s, r = _setup(20.0)
    # the ray runs along the shared vertical edge y = 0 of two triangles at
    # x = 5 ... the triangle on y >= 0 is hit exactly on its edge
    v = np.array([[5, 0, -1], [5, 2, -1], [5, 0, 1],
                  [7, -1, -1], [7, 1, -1], [7, 0, 1],
                  [9, -1, -1], [9, 1, -1], [9, 0, 1]], np.float32)
    f = np.arange(9, dtype=np.uint32).reshape(-1, 3)
    orc = O.cast(s, v, f, rays=r)
    assert orc["tri"][0] == 0 and orc["flags"][0] & O.GRAZING
    assert _rule(s, v, f, r, 5.0, 0)
    assert _rule(s, v, f, r, 7.0, 1), "the second best behind a grazed edge"
    assert not _rule(s, v, f, r, 9.0, 2), "the third behind a clean second best"
    assert not _rule(s, v, f, r, np.inf, O.MISS), "a miss with a clean second best"
    # with nothing behind the grazed edge, a miss is legitimate
    assert _rule(s, v[:3], f[:1], r, np.inf, O.MISS)


def test_report_carries_error_statistics():
    s, r = _setup(20.0)
    v, f = _walls(5.0)
    orc = O.cast(s, v, f, rays=r)
    rep = parity.check(s, v, f, orc, np.array([5.0 * (1 + 3e-6)], np.float32),
                       np.array([0], np.uint32))
    c = rep["counts"]
    assert 2e-6 < c["max_rel_err"] < 4e-6 and c["widened"] == 0
    tot = parity.merge({}, c)
    tot = parity.merge(tot, dict(c, max_rel_err=1e-6))
    assert tot["max_rel_err"] == c["max_rel_err"] and tot["rays"] == 2
