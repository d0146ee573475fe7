"""Thin ctypes binding of libgrca.so (the C ABI of include/grca.h).

Functions carry the C names (``grca_create``, ``grca_scene_update``,
``grca_cast`` ...) and only marshal arguments: numpy arrays become host
pointers, torch tensors (or anything with ``data_ptr()``) device pointers.
Every step of a cast runs in the library's HIP kernels; there is no Python or
CPU fallback: loading fails loudly when the library has not been built.

``Context`` wraps a context handle with the same calls as methods.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrca.so")

GRCA_OK = 0
GRCA_ERR_INVALID_ARG = 1
GRCA_ERR_OUT_OF_MEMORY = 2
GRCA_ERR_DEVICE = 3
GRCA_ERR_CAPACITY = 4
GRCA_ERR_NOT_FOUND = 5
GRCA_MISS_TRI = 0xFFFFFFFF
GRCA_MEM_HOST = 0
GRCA_MEM_DEVICE = 1
GRCA_UPDATE_VERTICES_ONLY = 2
GRCA_CULL_BACKFACE = 4
GRCA_CAST_ALL_PAIRS = 8
GRCA_LOSSY_AREA = 16
GRCA_LOSSY_CSPAN = 32
GRCA_LOSSY_RSPAN = 64
GRCA_NOALLOC_SCRATCH_BYTES = 64 << 20
GRCA_NOALLOC_MAX_SENSORS = 64
GRCA_NOALLOC_MIN_QUEUE_BYTES = 2 << 20

_STATUS = {1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "CAPACITY", 5: "NOT_FOUND"}


class GrcaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"GRCA_ERR_{_STATUS.get(status, status)}: {msg}")
        self.status = status


class SensorDesc(ctypes.Structure):
    _fields_ = [
        ("scene_id", ctypes.c_uint32),
        ("origin", ctypes.c_float * 3),
        ("forward", ctypes.c_float * 3),
        ("right", ctypes.c_float * 3),
        ("up", ctypes.c_float * 3),
        ("num_channels", ctypes.c_uint32),
        ("channel_elevation_rad", ctypes.POINTER(ctypes.c_float)),
        ("rays_per_channel", ctypes.c_uint32),
        ("fov_rad", ctypes.c_float),
        ("range_min", ctypes.c_float),
        ("range_max", ctypes.c_float),
        ("azimuth_offset_rad", ctypes.POINTER(ctypes.c_float)),
        ("ray_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("channel_elevation_offset_rad", ctypes.POINTER(ctypes.c_float)),
    ]


class DeformGroup(ctypes.Structure):
    _fields_ = [("vertex_start", ctypes.c_uint32), ("vertex_count", ctypes.c_uint32),
                ("amplitude", ctypes.c_float), ("omega", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_uint64), ("pairs_tested", ctypes.c_uint64),
                ("rect_items", ctypes.c_uint64), ("large_records", ctypes.c_uint64),
                ("row_items", ctypes.c_uint64), ("rtic", ctypes.c_uint64),
                ("recasts", ctypes.c_uint32), ("overflowed", ctypes.c_uint32),
                ("pairs_evaluated", ctypes.c_uint64), ("sphere_tests", ctypes.c_uint64),
                ("atomics", ctypes.c_uint64)]


class Options(ctypes.Structure):
    _fields_ = [("small_channels", ctypes.c_uint32), ("small_rays", ctypes.c_uint32),
                ("row_chunk", ctypes.c_uint32), ("bounds_block", ctypes.c_uint32),
                ("persist_waves_cu", ctypes.c_uint32), ("group_cull", ctypes.c_uint32),
                ("inline_max", ctypes.c_uint32),
                ("isect_ticket", ctypes.c_uint32), ("eps_area", ctypes.c_float),
                ("item_capacity", ctypes.c_uint64),
                ("large_capacity", ctypes.c_uint64)]


_lib = None


def load() -> ctypes.CDLL:
    """Open libgrca.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run paper_2605_10457_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "grca_create": ([ctypes.c_int, ctypes.POINTER(P)], ctypes.c_int),
        "grca_destroy": ([P], None),
        "grca_last_error": ([P], ctypes.c_char_p),
        "grca_scene_update": ([P, U32, P, U32, P, U32, U32, P], ctypes.c_int),
        "grca_scene_release": ([P, U32], ctypes.c_int),
        "grca_scene_download": ([P, U32, P, P], ctypes.c_int),
        "grca_scene_set_rigid": ([P, U32, U32, P, P, P], ctypes.c_int),
        "grca_scene_set_deform": ([P, U32, U32, P, P, P, P], ctypes.c_int),
        "grca_scene_pose": ([P, U32, P, ctypes.c_double, U32, P], ctypes.c_int),
        "grca_sensor_config": ([P, U32, ctypes.POINTER(SensorDesc)], ctypes.c_int),
        "grca_sensor_release": ([P, U32], ctypes.c_int),
        "grca_cast": ([P, P, U32, P, P, U32, P], ctypes.c_int),
        "grca_synchronize": ([P, P], ctypes.c_int),
        "grca_last_stats": ([P, ctypes.POINTER(Stats)], ctypes.c_int),
        "grca_get_options": ([P, ctypes.POINTER(Options)], ctypes.c_int),
        "grca_set_options": ([P, ctypes.POINTER(Options)], ctypes.c_int),
        "grca_frame_create": ([P, U32, P, U32, P, P, ctypes.POINTER(P)], ctypes.c_int),
        "grca_frame_launch": ([P, P, ctypes.c_double, P], ctypes.c_int),
        "grca_frame_synchronize": ([P, P], ctypes.c_int),
        "grca_frame_destroy": ([P], None),
        "grca_frame_profile": ([P, P, ctypes.c_double, P, P], ctypes.c_int),
        "grca_workspace_create": ([P, U64, U64, ctypes.POINTER(P), ctypes.POINTER(U64)],
                                  ctypes.c_int),
        "grca_workspace_destroy": ([P], None),
        "grca_cast_ws": ([P, P, P, U32, P, P, P], ctypes.c_int),
        "grca_workspace_synchronize": ([P, P, P], ctypes.c_int),
        "grca_workspace_stats": ([P, P, ctypes.POINTER(Stats)], ctypes.c_int),
        "grca_cast_noalloc": ([P, P, U32, P, P, U32, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return [
        "grca_create", "grca_destroy", "grca_last_error", "grca_scene_update",
        "grca_scene_release", "grca_scene_download", "grca_scene_set_rigid", "grca_scene_set_deform", "grca_scene_pose",
        "grca_sensor_config", "grca_sensor_release", "grca_cast", "grca_synchronize",
        "grca_last_stats", "grca_get_options", "grca_set_options", "grca_frame_create",
        "grca_frame_launch", "grca_frame_synchronize", "grca_frame_destroy",
        "grca_frame_profile",
        "grca_workspace_create", "grca_workspace_destroy", "grca_cast_ws",
        "grca_workspace_synchronize", "grca_workspace_stats", "grca_cast_noalloc",
    ]


# ---------------------------------------------------------------- marshalling
def _is_device(a) -> bool:
    return hasattr(a, "data_ptr") and not isinstance(a, np.ndarray)


def _ptr(a):
    if a is None:
        return None
    if _is_device(a):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        return None
    s = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(s))


def _check(ctx, rc):
    if rc != GRCA_OK:
        msg = load().grca_last_error(ctx).decode() if ctx else ""
        raise GrcaError(rc, msg)


# ---------------------------------------------------------------- C-named calls
def grca_create(device: int = 0):
    h = ctypes.c_void_p()
    rc = load().grca_create(int(device), ctypes.byref(h))
    if rc != GRCA_OK:
        raise GrcaError(rc, f"grca_create({device}) failed")
    return h


def grca_destroy(ctx):
    load().grca_destroy(ctx)


def grca_scene_update(ctx, scene_id, vertices, indices, flags=0, stream=None):
    dev = _is_device(vertices)
    if not dev:
        vertices = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
        if indices is not None:
            indices = np.ascontiguousarray(indices, np.uint32).reshape(-1, 3)
    else:
        flags |= GRCA_MEM_DEVICE
    nv = int(vertices.shape[0]) if not dev else int(vertices.numel() // 3)
    nt = 0 if indices is None else (int(indices.shape[0]) if not dev else int(indices.numel() // 3))
    _check(ctx, load().grca_scene_update(ctx, scene_id, _ptr(vertices), nv, _ptr(indices), nt,
                                         flags, _stream(stream)))


def grca_scene_download(ctx, scene_id, num_vertices: int, stream=None) -> np.ndarray:
    out = np.empty((int(num_vertices), 3), np.float32)
    _check(ctx, load().grca_scene_download(ctx, scene_id, _ptr(out), _stream(stream)))
    return out


def grca_scene_release(ctx, scene_id):
    _check(ctx, load().grca_scene_release(ctx, scene_id))


def grca_scene_set_rigid(ctx, scene_id, vertex_start, vertex_count, stream=None):
    st = np.ascontiguousarray(vertex_start, np.uint32)
    ct = np.ascontiguousarray(vertex_count, np.uint32)
    _check(ctx, load().grca_scene_set_rigid(ctx, scene_id, st.shape[0], _ptr(st), _ptr(ct),
                                            _stream(stream)))


def grca_scene_set_deform(ctx, scene_id, groups, normals, phases, stream=None):
    arr = (DeformGroup * max(1, len(groups)))()
    for i, g in enumerate(groups):
        arr[i] = DeformGroup(int(g[0]), int(g[1]), float(g[2]), float(g[3]))
    nrm = np.ascontiguousarray(normals, np.float32).reshape(-1, 3)
    ph = np.ascontiguousarray(phases, np.float32).reshape(-1)
    _check(ctx, load().grca_scene_set_deform(ctx, scene_id, len(groups),
                                             ctypes.cast(arr, ctypes.c_void_p), _ptr(nrm),
                                             _ptr(ph), _stream(stream)))


def grca_scene_pose(ctx, scene_id, matrices, time_s: float, stream=None):
    flags = 0
    if matrices is not None and not _is_device(matrices):
        matrices = np.ascontiguousarray(matrices, np.float32).reshape(-1, 12)
    elif matrices is not None:
        flags |= GRCA_MEM_DEVICE
    _check(ctx, load().grca_scene_pose(ctx, scene_id, _ptr(matrices), float(time_s), flags,
                                       _stream(stream)))


def make_sensor_desc(sensor: dict, scene_id: int):
    """ctypes descriptor from a sensor dict (keys as produced by ``synth.sensor``)."""
    elev = np.ascontiguousarray(sensor["elevation"], np.float32)
    d = SensorDesc()
    d.scene_id = int(scene_id)
    for name in ("origin", "forward", "right", "up"):
        getattr(d, name)[:] = [float(x) for x in np.asarray(sensor[name], np.float32).reshape(3)]
    d.num_channels = int(elev.shape[0])
    d.channel_elevation_rad = elev.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    d.rays_per_channel = int(sensor["rays_per_channel"])
    d.fov_rad = float(np.float32(sensor["fov"]))
    d.range_min = float(np.float32(sensor.get("range_min", 0.05)))
    d.range_max = float(np.float32(sensor.get("range_max", 1000.0)))
    keep = [elev]
    if sensor.get("azimuth_offset") is not None:
        off = np.ascontiguousarray(sensor["azimuth_offset"], np.float32)
        d.azimuth_offset_rad = off.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        keep.append(off)
    if sensor.get("ray_mask") is not None:
        m = np.ascontiguousarray(sensor["ray_mask"], np.uint8).reshape(-1)
        d.ray_mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        keep.append(m)
    if sensor.get("elevation_offset") is not None:
        eo = np.ascontiguousarray(sensor["elevation_offset"], np.float32)
        d.channel_elevation_offset_rad = eo.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        keep.append(eo)
    return d, keep


def grca_sensor_config(ctx, sensor_id, sensor: dict, scene_id: int):
    d, elev = make_sensor_desc(sensor, scene_id)
    _check(ctx, load().grca_sensor_config(ctx, sensor_id, ctypes.byref(d)))
    del elev


def grca_sensor_release(ctx, sensor_id):
    _check(ctx, load().grca_sensor_release(ctx, sensor_id))


def grca_cast(ctx, sensor_ids, out_distance, out_tri, flags=0, stream=None):
    ids = np.ascontiguousarray(sensor_ids, np.uint32).reshape(-1)
    if (out_distance is not None and _is_device(out_distance)) or (
            out_tri is not None and _is_device(out_tri)):
        flags |= GRCA_MEM_DEVICE
    _check(ctx, load().grca_cast(ctx, _ptr(ids), ids.shape[0], _ptr(out_distance), _ptr(out_tri),
                                 flags, _stream(stream)))


def grca_cast_noalloc(ctx, sensor_ids, out_distance, out_tri, flags=0, stream=None):
    """grca_cast into device outputs with no allocation (fixed static scratch)."""
    ids = np.ascontiguousarray(sensor_ids, np.uint32).reshape(-1)
    _check(ctx, load().grca_cast_noalloc(ctx, _ptr(ids), ids.shape[0], _ptr(out_distance),
                                         _ptr(out_tri), flags | GRCA_MEM_DEVICE,
                                         _stream(stream)))


def grca_synchronize(ctx, stream=None):
    _check(ctx, load().grca_synchronize(ctx, _stream(stream)))


def grca_last_stats(ctx) -> dict:
    s = Stats()
    _check(ctx, load().grca_last_stats(ctx, ctypes.byref(s)))
    return {f: int(getattr(s, f)) for f, _ in Stats._fields_}


def grca_get_options(ctx) -> dict:
    o = Options()
    _check(ctx, load().grca_get_options(ctx, ctypes.byref(o)))
    return {f: (float(getattr(o, f)) if t is ctypes.c_float else int(getattr(o, f)))
            for f, t in Options._fields_}


def grca_set_options(ctx, **kw):
    cur = grca_get_options(ctx)
    cur.update(kw)
    types = dict(Options._fields_)
    o = Options(**{k: (float(v) if types[k] is ctypes.c_float else int(v))
                   for k, v in cur.items()})
    _check(ctx, load().grca_set_options(ctx, ctypes.byref(o)))


def grca_frame_create(ctx, scene_id, sensor_ids, out_distance_dev, out_tri_dev):
    ids = np.ascontiguousarray(sensor_ids, np.uint32).reshape(-1)
    h = ctypes.c_void_p()
    _check(ctx, load().grca_frame_create(ctx, scene_id, _ptr(ids), ids.shape[0],
                                         _ptr(out_distance_dev), _ptr(out_tri_dev),
                                         ctypes.byref(h)))
    return h


def grca_frame_launch(ctx, frame, matrices, time_s, stream=None):
    if matrices is not None:
        matrices = np.ascontiguousarray(matrices, np.float32).reshape(-1, 12)
    _check(ctx, load().grca_frame_launch(frame, _ptr(matrices), float(time_s), _stream(stream)))


def grca_frame_synchronize(ctx, frame, stream=None):
    _check(ctx, load().grca_frame_synchronize(frame, _stream(stream)))


def grca_frame_destroy(frame):
    load().grca_frame_destroy(frame)


STAGES = ("pose", "init", "bounds", "expand", "isect", "resolve")


def grca_frame_profile(ctx, frame, matrices, time_s, stream=None) -> dict:
    """Run one frame stage by stage with events between stages; per-stage ms."""
    if matrices is not None:
        matrices = np.ascontiguousarray(matrices, np.float32).reshape(-1, 12)
    ms = np.zeros(6, np.float32)
    _check(ctx, load().grca_frame_profile(frame, _ptr(matrices), float(time_s), _stream(stream),
                                          _ptr(ms)))
    return dict(zip(STAGES, (float(x) for x in ms)))


def grca_workspace_create(ctx, max_rays, item_capacity):
    h = ctypes.c_void_p()
    nbytes = ctypes.c_uint64()
    _check(ctx, load().grca_workspace_create(ctx, int(max_rays), int(item_capacity),
                                             ctypes.byref(h), ctypes.byref(nbytes)))
    return h, int(nbytes.value)


def grca_workspace_destroy(ws):
    load().grca_workspace_destroy(ws)


def grca_cast_ws(ctx, ws, sensor_ids, out_distance_dev, out_tri_dev, stream=None):
    ids = np.ascontiguousarray(sensor_ids, np.uint32).reshape(-1)
    _check(ctx, load().grca_cast_ws(ctx, ws, _ptr(ids), ids.shape[0], _ptr(out_distance_dev),
                                    _ptr(out_tri_dev), _stream(stream)))


def grca_workspace_synchronize(ctx, ws, stream=None):
    _check(ctx, load().grca_workspace_synchronize(ctx, ws, _stream(stream)))


def grca_workspace_stats(ctx, ws) -> dict:
    s = Stats()
    _check(ctx, load().grca_workspace_stats(ctx, ws, ctypes.byref(s)))
    return {f: int(getattr(s, f)) for f, _ in Stats._fields_}


# ---------------------------------------------------------------- object wrapper
class Context:
    """Owns one grca context; methods mirror the C calls without the prefix."""

    def __init__(self, device: int = 0):
        self.h = grca_create(device)

    def close(self):
        if self.h:
            grca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scene_update(self, scene_id, vertices, indices, flags=0, stream=None):
        grca_scene_update(self.h, scene_id, vertices, indices, flags, stream)

    def scene_download(self, scene_id, num_vertices, stream=None):
        return grca_scene_download(self.h, scene_id, num_vertices, stream)

    def scene_release(self, scene_id):
        grca_scene_release(self.h, scene_id)

    def scene_set_rigid(self, scene_id, starts, counts, stream=None):
        grca_scene_set_rigid(self.h, scene_id, starts, counts, stream)

    def scene_set_deform(self, scene_id, groups, normals, phases, stream=None):
        grca_scene_set_deform(self.h, scene_id, groups, normals, phases, stream)

    def scene_pose(self, scene_id, matrices, time_s, stream=None):
        grca_scene_pose(self.h, scene_id, matrices, time_s, stream)

    def sensor_config(self, sensor_id, sensor: dict, scene_id: int):
        grca_sensor_config(self.h, sensor_id, sensor, scene_id)

    def sensor_release(self, sensor_id):
        grca_sensor_release(self.h, sensor_id)

    def cast(self, sensor_ids, out_distance=None, out_tri=None, flags=0, stream=None):
        grca_cast(self.h, sensor_ids, out_distance, out_tri, flags, stream)

    def cast_host(self, sensor_ids, n_rays: int, flags=0):
        d = np.empty(n_rays, np.float32)
        t = np.empty(n_rays, np.uint32)
        grca_cast(self.h, sensor_ids, d, t, flags)
        return d, t

    def cast_noalloc(self, sensor_ids, out_distance=None, out_tri=None, flags=0, stream=None):
        grca_cast_noalloc(self.h, sensor_ids, out_distance, out_tri, flags, stream)

    def synchronize(self, stream=None):
        grca_synchronize(self.h, stream)

    def last_stats(self):
        return grca_last_stats(self.h)

    def get_options(self):
        return grca_get_options(self.h)

    def set_options(self, **kw):
        grca_set_options(self.h, **kw)


def load_workload(ctx: Context, wl, scene_id: int = 0, first_sensor_id: int = 0,
                  frame: int | None = 0, stream=None) -> list[int]:
    """Upload a ``synth.Workload``: scene, dynamic declarations, sensors; pose at `frame`."""
    sc = wl.scene
    ctx.scene_update(scene_id, sc.vertices, sc.indices, stream=stream)
    if sc.rigid is not None:
        ctx.scene_set_rigid(scene_id, sc.rigid.vertex_start, sc.rigid.vertex_count, stream)
    if sc.deform:
        ctx.scene_set_deform(scene_id, [(g.vertex_start, g.vertex_count, g.amplitude, g.omega)
                                        for g in sc.deform], sc.deform_normals, sc.deform_phase,
                             stream)
    ids = []
    for k, s in enumerate(wl.sensors):
        ctx.sensor_config(first_sensor_id + k, s, scene_id)
        ids.append(first_sensor_id + k)
    if frame is not None and (sc.rigid is not None or sc.deform):
        from . import synth
        mats = sc.instance_matrices(frame) if sc.rigid is not None else None
        ctx.scene_pose(scene_id, mats, synth.deform_time(frame), stream)
    return ids
