"""ctypes wrapper for the FP64 brute-force oracle (``grca_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the HIP path and imports nothing from the product package.

Every function here passes numpy arrays straight to the C library; the
arithmetic (ray directions per section 3.1 Eq. ray_dir, two-sided
Moller-Trumbore, lexicographic (t, id) closest hit, pose formulas) lives in
``grca_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GRAZING = 1
NEAR_TIE = 2
RANGE_EDGE = 4
GRAZING_INCIDENCE = 8
MISS = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, no -ffast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
             "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OracleSensor(ctypes.Structure):
    _fields_ = [
        ("origin", ctypes.c_float * 3),
        ("forward", ctypes.c_float * 3),
        ("right", ctypes.c_float * 3),
        ("up", ctypes.c_float * 3),
        ("num_channels", ctypes.c_uint32),
        ("rays_per_channel", ctypes.c_uint32),
        ("channel_elevation_rad", ctypes.POINTER(ctypes.c_float)),
        ("fov_rad", ctypes.c_float),
        ("range_min", ctypes.c_float),
        ("range_max", ctypes.c_float),
        ("flags", ctypes.c_uint32),
        ("azimuth_offset_rad", ctypes.POINTER(ctypes.c_float)),
        ("ray_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("channel_elevation_offset_rad", ctypes.POINTER(ctypes.c_float)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_cast.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_uint64, ctypes.c_int,
                                    P, P, P, P, P]
        lib.oracle_cast.restype = ctypes.c_int
        lib.oracle_pair.argtypes = [P, P, P, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.oracle_pair.restype = None
        lib.oracle_ray_direction.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.oracle_ray_direction.restype = None
        lib.oracle_pose_rigid.argtypes = [P, ctypes.c_uint64, P, P]
        lib.oracle_pose_rigid.restype = None
        lib.oracle_pose_deform.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_float,
                                           ctypes.c_float, ctypes.c_double, P]
        lib.oracle_pose_deform.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class _Sensor:
    """Holds the ctypes struct and keeps the elevation array alive."""

    def __init__(self, sensor: dict):
        self.elev = _f32(sensor["elevation"])
        s = OracleSensor()
        for name in ("origin", "forward", "right", "up"):
            v = _f32(sensor[name]).reshape(3)
            getattr(s, name)[:] = [float(x) for x in v]
        s.num_channels = int(self.elev.shape[0])
        s.rays_per_channel = int(sensor["rays_per_channel"])
        s.channel_elevation_rad = self.elev.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        s.fov_rad = float(np.float32(sensor["fov"]))
        s.range_min = float(np.float32(sensor.get("range_min", 0.05)))
        s.range_max = float(np.float32(sensor.get("range_max", 1000.0)))
        s.flags = int(sensor.get("oracle_flags", 0))
        self.az_off = None
        self.mask = None
        if sensor.get("azimuth_offset") is not None:
            self.az_off = _f32(sensor["azimuth_offset"])
            s.azimuth_offset_rad = self.az_off.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        if sensor.get("ray_mask") is not None:
            self.mask = np.ascontiguousarray(sensor["ray_mask"], np.uint8).reshape(-1)
            s.ray_mask = self.mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.el_off = None
        if sensor.get("elevation_offset") is not None:
            self.el_off = _f32(sensor["elevation_offset"])
            s.channel_elevation_offset_rad = self.el_off.ctypes.data_as(
                ctypes.POINTER(ctypes.c_float))
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


def cast(sensor: dict, vertices: np.ndarray, indices: np.ndarray, rays=None,
         nthreads: int | None = None) -> dict:
    """Brute-force closest hit of the listed rays (global ids C*chi + R) of one sensor.

    Returns dict with t (float64, inf on miss), tri (uint32, MISS on miss),
    flags (uint32), t2/tri2 (second best on another triangle) and threads.
    """
    lib = _load()
    S = _Sensor(sensor)
    xyz = _f32(vertices).reshape(-1, 3)
    idx = np.ascontiguousarray(indices, dtype=np.uint32).reshape(-1, 3)
    n_all = S.s.num_channels * S.s.rays_per_channel
    if rays is None:
        rays = np.arange(n_all, dtype=np.uint32)
    rays = np.ascontiguousarray(rays, dtype=np.uint32)
    if rays.size and int(rays.max()) >= n_all:
        raise ValueError("ray id out of range")
    n = rays.shape[0]
    out_t = np.empty(n, np.float64)
    out_tri = np.empty(n, np.uint32)
    out_flags = np.empty(n, np.uint32)
    out_t2 = np.empty(n, np.float64)
    out_tri2 = np.empty(n, np.uint32)
    if nthreads is None:
        nthreads = max(1, min(len(os.sched_getaffinity(0)), 64))
    used = lib.oracle_cast(S.ref, _ptr(xyz), _ptr(idx), idx.shape[0], _ptr(rays), n, nthreads,
                           _ptr(out_t), _ptr(out_tri), _ptr(out_flags), _ptr(out_t2),
                           _ptr(out_tri2))
    return {"t": out_t, "tri": out_tri, "flags": out_flags, "t2": out_t2, "tri2": out_tri2,
            "rays": rays, "threads": used}


def pair(sensor: dict, vertices: np.ndarray, indices: np.ndarray, g: int, k: int) -> dict:
    """FP64 evaluation of ray g against triangle k (see ``oracle_pair``)."""
    lib = _load()
    S = _Sensor(sensor)
    xyz = _f32(vertices).reshape(-1, 3)
    idx = np.ascontiguousarray(indices, dtype=np.uint32).reshape(-1, 3)
    out = np.zeros(6, np.float64)
    lib.oracle_pair(S.ref, _ptr(xyz), _ptr(idx), int(g), int(k), _ptr(out))
    return {"hit": bool(out[0]), "t": out[1], "margin": out[2], "plane_t": out[3],
            "cos_inc": out[4], "degenerate": bool(out[5])}


def ray_direction(sensor: dict, C: int, R: int) -> np.ndarray:
    lib = _load()
    S = _Sensor(sensor)
    d = np.zeros(3, np.float64)
    lib.oracle_ray_direction(S.ref, int(C), int(R), _ptr(d))
    return d


def pose_rigid(rest_xyz: np.ndarray, M: np.ndarray) -> np.ndarray:
    lib = _load()
    rest = _f32(rest_xyz).reshape(-1, 3)
    M = _f32(M).reshape(3, 4)
    out = np.empty_like(rest)
    lib.oracle_pose_rigid(_ptr(rest), rest.shape[0], _ptr(M), _ptr(out))
    return out


def pose_deform(rest_xyz, normal_xyz, phase, amplitude: float, omega: float,
                time: float) -> np.ndarray:
    lib = _load()
    rest = _f32(rest_xyz).reshape(-1, 3)
    nrm = _f32(normal_xyz).reshape(-1, 3)
    ph = _f32(phase).reshape(-1)
    out = np.empty_like(rest)
    lib.oracle_pose_deform(_ptr(rest), _ptr(nrm), _ptr(ph), rest.shape[0],
                           float(np.float32(amplitude)), float(np.float32(omega)),
                           float(time), _ptr(out))
    return out
