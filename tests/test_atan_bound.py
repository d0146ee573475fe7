"""CPU check of the bounds pass's FP32 atan2 (``atan2_bounded`` and ``atan_unit`` in
grca_kernels.hip): its error bound of 5e-7 rad feeds the azimuth margin of the
conservative candidate spans (section 3.3's angular bounding of a triangle).
The sphere tests' elevation (``atan2_right`` with ``atan_unit_coarse``) is
checked against its own bound of 2e-6 rad, inside their 3e-5 rad margin.

The coefficients are read from the kernel source, and the FP32 evaluation is
replayed step by step in numpy (each fmaf rounded once, the hardware
reciprocal taken as correctly rounded and then perturbed by +-1 ulp)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2605_10457_amd", "csrc", "grca_kernels.hip")
BOUND = 5e-7


def _body(name):
    txt = open(SRC).read()
    body = txt[txt.index("__device__ inline float %s(" % name):]
    return body[:body.index("\n}\n")]


def _coefficients(fn="atan_unit"):
    poly = _body(fn)
    first = re.search(r"float p = (-?[0-9.e-]+)f;", poly).group(1)
    rest = re.findall(r"p = fmaf\(p, u, (-?[0-9.e-]+)f\);", poly)
    consts = re.findall(r"r = (\d\.\d+)f - r;", _body("atan2_bounded"))
    return [np.float32(first)] + [np.float32(c) for c in rest], [np.float32(c) for c in consts]


def _f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def _atan2(y, x, coef, consts, rcp_ulps):
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    rc = _f32(1.0 / mx.astype(np.float64))
    rc = _f32(rc.astype(np.float64) * (1.0 + rcp_ulps * 2.0 ** -23))
    t = _f32(mn.astype(np.float64) * rc)
    u = _f32(t.astype(np.float64) * t)
    p = np.full_like(u, coef[0])
    for c in coef[1:]:
        p = _f32(p.astype(np.float64) * u + np.float64(c))  # fmaf: one rounding
    r = _f32(p.astype(np.float64) * t)
    half_pi, pi = consts
    r = np.where(ay > ax, _f32(np.float64(half_pi) - r), r)
    r = np.where(x < 0, _f32(np.float64(pi) - r), r)
    return np.where(y < 0, -r, r)


def test_coefficients_found():
    coef, consts = _coefficients()
    assert len(coef) == 8 and len(consts) == 2
    assert abs(float(consts[0]) - np.pi / 2) < 1e-7 and abs(float(consts[1]) - np.pi) < 2e-7
    # atan(t) = t - t^3/3 + ...: the leading terms are the Taylor ones, nearly
    assert abs(float(coef[-1]) - 1.0) < 1e-5 and abs(float(coef[-2]) + 1.0 / 3.0) < 1e-3


def test_atan2_error_bound():
    coef, consts = _coefficients()
    rng = np.random.default_rng(1234)
    th = np.concatenate([rng.uniform(-np.pi, np.pi, 2_000_000),
                         np.arange(-8, 9) * (np.pi / 8),                    # axes, octant edges
                         np.arange(-8, 9) * (np.pi / 8) + 1e-6,
                         np.arange(-8, 9) * (np.pi / 8) - 1e-6])
    rad = 10.0 ** rng.uniform(-3, 4, th.size)
    x = _f32(rad * np.cos(th))
    y = _f32(rad * np.sin(th))
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    for ulps in (-1.0, 0.0, 1.0):
        got = _atan2(y, x, coef, consts, ulps).astype(np.float64)
        err = np.abs(got - ref)
        err = np.minimum(err, 2 * np.pi - err)  # +-pi are the same direction
        assert err.max() <= BOUND, (ulps, err.max())


COARSE_BOUND = 2e-6


def test_right_half_plane_variant():
    # atan2_right (elevations of the sphere tests: x >= 0) takes
    # atan2_bounded's steps with the coarse polynomial and without the x < 0
    # reflection; check that the source still says so, then replay it
    body = _body("atan2_right")
    quarter = re.findall(r"r = (\d\.\d+)f - r;", _body("atan2_bounded"))[0]
    assert "atan_unit_coarse(" in body and "__builtin_amdgcn_rcpf(mx)" in body
    assert re.findall(r"r = (\d\.\d+)f - r;", body) == [quarter]
    assert "x < 0.0f" not in body
    coef, consts = _coefficients("atan_unit_coarse")
    assert len(coef) == 6
    rng = np.random.default_rng(4321)
    th = np.concatenate([rng.uniform(-np.pi / 2, np.pi / 2, 1_000_000),
                         np.arange(-4, 5) * (np.pi / 8), np.arange(-4, 5) * (np.pi / 8) + 1e-6])
    rad = 10.0 ** rng.uniform(-3, 4, th.size)
    x = _f32(np.abs(rad * np.cos(th)))
    y = _f32(rad * np.sin(th))
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    for ulps in (-1.0, 0.0, 1.0):
        got = _atan2(y, x, coef, consts, ulps).astype(np.float64)
        err = np.abs(got - ref).max()
        assert err <= COARSE_BOUND, (ulps, err)
    # a planted error: the bound is tight enough to see a dropped term
    worse = list(coef[:-2]) + [coef[-1]]
    got = _atan2(y, x, worse, consts, 0.0).astype(np.float64)
    assert np.abs(got - ref).max() > COARSE_BOUND
