"""Seeded synthetic LiDAR workloads: scenes, sensor rigs and motion streams.

This module only *constructs inputs*: vertex and index buffers, sensor
descriptors, instance pose matrices and deformation parameters.  It holds none
of the casting arithmetic and none of the pose application (that is done by
the library on the GPU, and independently by the oracle on the CPU), so both
sides can consume the same inputs without sharing any method code.

Shapes follow the paper's workloads (section 5 "Benchmarks": full-sphere
128x4096 LiDARs, range 0.05-1000 m, up to eight origins, ~22M triangles of
which ~9M dynamic, per-axis instance scale in [0.001, 30] with "full instant"
random pose every frame, 100 Hz simulation clock).  The paper's meshes are not
available; these scenes stand in for them.

Conventions: metres, right-handed world, z up.  A sensor with yaw psi has
forward f = (cos psi, sin psi, 0), up u = (0, 0, 1) and right r = f x u, so
ray azimuth grows clockwise seen from above (section 3.1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 260510457
SIM_HZ = 100.0

# --------------------------------------------------------------------------
# primitive meshes (unit size, outward CCW winding)
# --------------------------------------------------------------------------
_ICO_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere with 20 * 4**level faces (float64 vertices, uint32 faces)."""
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        es = np.sort(e, axis=1)
        uniq, inv = np.unique(es, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = v[uniq[:, 0]] + v[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid], axis=0)
        nf = f.shape[0]
        m01 = base + inv[0:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:3 * nf]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], 1),
            np.stack([f[:, 1], m12, m01], 1),
            np.stack([f[:, 2], m20, m12], 1),
            np.stack([m01, m12, m20], 1)], axis=0)
    out = (v, f.astype(np.uint32))
    _ICO_CACHE[level] = out
    return out


def unit_box() -> tuple[np.ndarray, np.ndarray]:
    """Axis-aligned box [-0.5, 0.5]^3, 8 vertices, 12 outward-wound triangles."""
    v = np.array([[x, y, z] for z in (-0.5, 0.5) for y in (-0.5, 0.5) for x in (-0.5, 0.5)],
                 np.float64)
    # vertex id = x + 2y + 4z (each in {0, 1})
    f = np.array([
        [0, 2, 1], [1, 2, 3],      # z = -0.5 (normal -z)
        [4, 5, 6], [5, 7, 6],      # z = +0.5
        [0, 1, 4], [1, 5, 4],      # y = -0.5
        [2, 6, 3], [3, 6, 7],      # y = +0.5
        [0, 4, 2], [2, 4, 6],      # x = -0.5
        [1, 3, 5], [3, 7, 5],      # x = +0.5
    ], np.uint32)
    return v, f


def grid(nx: int, ny: int, sx: float, sy: float, x0: float, y0: float):
    """Flat grid in the z = 0 plane: (nx+1)(ny+1) vertices, 2*nx*ny triangles.

    Vertex (i, j) sits at (x0 + i*sx/nx, y0 + j*sy/ny); its id is j*(nx+1)+i.
    Cell (i, j) is split on its (i, j)->(i+1, j+1) diagonal into triangles
    2*(j*nx+i) (lower-right) and 2*(j*nx+i)+1 (upper-left), both wound
    counter-clockwise seen from +z.
    """
    xs = x0 + np.arange(nx + 1, dtype=np.float64) * (sx / nx)
    ys = y0 + np.arange(ny + 1, dtype=np.float64) * (sy / ny)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    v = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    i = np.arange(nx, dtype=np.int64)
    j = np.arange(ny, dtype=np.int64)
    I, J = np.meshgrid(i, j, indexing="xy")
    a = (J * (nx + 1) + I).ravel()
    b = a + 1
    c = a + (nx + 1) + 1
    d = a + (nx + 1)
    f = np.empty((2 * nx * ny, 3), np.int64)
    f[0::2] = np.stack([a, b, c], 1)
    f[1::2] = np.stack([a, c, d], 1)
    return v, f.astype(np.uint32)


# --------------------------------------------------------------------------
# scene assembly
# --------------------------------------------------------------------------
@dataclasses.dataclass
class RigidSet:
    """Dynamic rigid instances: rest geometry in instance-local coordinates."""
    vertex_start: np.ndarray   # uint32 [n_inst]
    vertex_count: np.ndarray   # uint32 [n_inst]
    kind: str                  # "jitter" (config 2) or "instant" (configs 3-5)
    base: np.ndarray           # float64 [n_inst, 5]: x, y, z, yaw, size (jitter kind)
    half_extent: np.ndarray    # float64 [n_inst, 3]: rest half-extent (for placement)
    seed: int


@dataclasses.dataclass
class DeformGroup:
    vertex_start: int
    vertex_count: int
    amplitude: float
    omega: float


@dataclasses.dataclass
class Scene:
    vertices: np.ndarray       # float32 [n_v, 3]  (dynamic ranges hold rest positions)
    indices: np.ndarray        # uint32  [n_tri, 3]
    rigid: RigidSet | None = None
    deform: list[DeformGroup] = dataclasses.field(default_factory=list)
    deform_normals: np.ndarray | None = None  # float32 [sum counts, 3]
    deform_phase: np.ndarray | None = None    # float32 [sum counts]
    n_dynamic_tris: int = 0
    ground: dict | None = None                # grid description, for closed-form checks

    @property
    def num_triangles(self) -> int:
        return int(self.indices.shape[0])

    @property
    def num_vertices(self) -> int:
        return int(self.vertices.shape[0])

    def instance_matrices(self, frame: int) -> np.ndarray:
        """Row-major 3x4 FP32 pose matrices of the rigid instances at `frame`."""
        return rigid_matrices(self.rigid, frame, getattr(self, "_sensor_xy", None))


class _Builder:
    def __init__(self):
        self.v: list[np.ndarray] = []
        self.f: list[np.ndarray] = []
        self.nv = 0
        self.nt = 0

    def add(self, v: np.ndarray, f: np.ndarray) -> tuple[int, int]:
        vs, ts = self.nv, self.nt
        self.v.append(np.asarray(v, np.float64))
        self.f.append(np.asarray(f, np.int64) + self.nv)
        self.nv += v.shape[0]
        self.nt += f.shape[0]
        return vs, ts

    def build(self) -> tuple[np.ndarray, np.ndarray]:
        v = np.concatenate(self.v, 0).astype(np.float32)
        f = np.concatenate(self.f, 0).astype(np.uint32)
        return v, f


def _far_from(sensors_xyz: np.ndarray, c: np.ndarray, half: np.ndarray, gap: float = 1.0) -> bool:
    """True if the axis-aligned box (c +- half) keeps `gap` metres from every sensor."""
    if sensors_xyz is None or len(sensors_xyz) == 0:
        return True
    d = np.maximum(np.abs(sensors_xyz - c) - half, 0.0)
    return bool(np.all(np.linalg.norm(d, axis=1) > gap))


def _ground(b: _Builder, size: float, cells: int, rng: np.random.Generator) -> dict:
    """Ground grid centred on the origin, shifted by a seeded sub-cell offset so
    that no sensor sits exactly above a grid vertex or edge."""
    c = size / cells
    off = rng.uniform(0.2, 0.8, 2) * c
    x0, y0 = -size / 2 + off[0], -size / 2 + off[1]
    v, f = grid(cells, cells, size, size, x0, y0)
    vs, ts = b.add(v, f)
    return {"x0": x0, "y0": y0, "cell": c, "n": cells, "tri_start": ts, "vert_start": vs}


def _place(rng, lo, hi, half, sensors_xyz, tries=1000):
    for _ in range(tries):
        cxy = rng.uniform(lo, hi, 2)
        c = np.array([cxy[0], cxy[1], half[2]])
        if _far_from(sensors_xyz, c, half):
            return c
    raise RuntimeError("placement failed")


def _add_box(b, rng, size_lo, size_hi, lo, hi, sensors_xyz):
    bv, bf = unit_box()
    s = rng.uniform(size_lo, size_hi, 3)
    c = _place(rng, lo, hi, s / 2, sensors_xyz)
    return b.add(bv * s + c, bf)


def _add_sphere(b, rng, level, r, lo, hi, sensors_xyz):
    sv, sf = icosphere(level)
    c = _place(rng, lo, hi, np.array([r, r, r]), sensors_xyz)
    return b.add(sv * r + c, sf)


# --------------------------------------------------------------------------
# sensors
# --------------------------------------------------------------------------
def sensor(origin, yaw: float, channels, rays: int, fov_deg: float = 360.0,
           range_min: float = 0.05, range_max: float = 1000.0) -> dict:
    """Sensor descriptor; `channels` is the ascending elevation table in radians."""
    f = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    u = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, u)
    return {
        "origin": np.asarray(origin, np.float32).reshape(3),
        "forward": f.astype(np.float32),
        "right": r.astype(np.float32),
        "up": u.astype(np.float32),
        "elevation": np.asarray(channels, np.float32),
        "rays_per_channel": int(rays),
        "fov": np.float32(2 * math.pi if fov_deg >= 360.0 else math.radians(fov_deg)),
        "range_min": np.float32(range_min),
        "range_max": np.float32(range_max),
    }


def elevations_uniform(lo_deg: float, hi_deg: float, n: int) -> np.ndarray:
    """Inclusive uniform grid lo..hi (configs with a stated elevation band)."""
    if n == 1:
        return np.array([math.radians(lo_deg)], np.float32)
    return np.radians(lo_deg + (hi_deg - lo_deg) * np.arange(n) / (n - 1)).astype(np.float32)


def elevations_full_sphere(n: int) -> np.ndarray:
    """Centred full-vertical grid of section 3.1: phi_j = (j - floor(n/2)) * pi/n."""
    return ((np.arange(n) - n // 2) * (math.pi / n)).astype(np.float32)


def ring_rig(shapes, radius=20.0, seed=0, fov_mode=None, full_sphere=True):
    """Sensors on a ring at azimuth 2*pi*k/n, z ~ U[1.5, 2.5]; 180-degree sensors face outward.

    `shapes` is a list of (channels, rays, fov_deg)."""
    rng = np.random.default_rng(seed)
    n = len(shapes)
    out = []
    for k, (g, x, fov) in enumerate(shapes):
        a = 2 * math.pi * k / n
        z = rng.uniform(1.5, 2.5)
        o = [radius * math.cos(a), radius * math.sin(a), z]
        yaw = a if fov < 360.0 else rng.uniform(0, 2 * math.pi)
        elev = elevations_full_sphere(g) if full_sphere else elevations_uniform(-25, 15, g)
        out.append(sensor(o, yaw, elev, x, fov))
    return out


# --------------------------------------------------------------------------
# motion (inputs of the pose step)
# --------------------------------------------------------------------------
def _yaw_scale_matrix(t, yaw, scale):
    c, s = math.cos(yaw), math.sin(yaw)
    R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    M = np.zeros((3, 4))
    M[:, :3] = R * np.asarray(scale)[None, :]
    M[:, 3] = t
    return M


def rigid_matrices(rs: RigidSet, frame: int, sensors_xy=None) -> np.ndarray:
    """Per-instance pose matrices for `frame` from the seeded motion stream."""
    n = rs.vertex_start.shape[0]
    rng = np.random.default_rng([rs.seed, int(frame)])
    out = np.empty((n, 3, 4), np.float64)
    if rs.kind == "jitter":
        # translation uniform in a disc of radius 1 m, yaw U[-5, 5] degrees
        rr = np.sqrt(rng.uniform(0, 1, n))
        aa = rng.uniform(0, 2 * math.pi, n)
        dyaw = np.radians(rng.uniform(-5, 5, n))
        for i in range(n):
            x, y, z, yaw, size = rs.base[i]
            t = np.array([x + rr[i] * math.cos(aa[i]), y + rr[i] * math.sin(aa[i]), z])
            out[i] = _yaw_scale_matrix(t, yaw + dyaw[i], (size, size, size))
    else:
        # "full instant": position U[-L, L]^2, yaw U[0, 2 pi), per-axis scale
        # log-uniform [0.001, 30]; the instance rests on the ground.
        L = float(rs.base[0, 0]) if rs.base.size else 500.0
        for i in range(n):
            for _ in range(1000):
                sc = np.exp(rng.uniform(math.log(0.001), math.log(30.0), 3))
                yaw = rng.uniform(0, 2 * math.pi)
                xy = rng.uniform(-L, L, 2)
                he = rs.half_extent[i] * sc
                rad = float(np.linalg.norm(he[:2]))
                c = np.array([xy[0], xy[1], he[2]])
                if sensors_xy is None or _far_from(sensors_xy, c, np.array([rad, rad, he[2]])):
                    break
            out[i] = _yaw_scale_matrix(c, yaw, sc)
    return out.reshape(n, 12).astype(np.float32)


def deform_time(frame: int) -> float:
    return frame / SIM_HZ


# --------------------------------------------------------------------------
# the workload configurations
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    sensors: list
    oracle_rays_per_sensor: int | None  # None = all rays


def _sensor_xyz(sensors):
    return np.array([s["origin"] for s in sensors], np.float64)


def config1(seed_extra: int = 0) -> Workload:
    """~19.6k static triangles, one 32x512 sensor at (0, 0, 1.8), -15..+15 deg."""
    rng = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 1 + seed_extra).spawn(4)[0])
    sens = [sensor([0.0, 0.0, 1.8], 0.0, elevations_uniform(-15, 15, 32), 512)]
    sxyz = _sensor_xyz(sens)
    b = _Builder()
    g = _ground(b, 100.0, 50, rng)
    for _ in range(150):
        _add_box(b, rng, 0.5, 4.0, -50, 50, sxyz)
    for _ in range(40):
        _add_sphere(b, rng, 2, rng.uniform(0.5, 3.0), -50, 50, sxyz)
    v, f = b.build()
    return Workload("config1", Scene(v, f, ground=g), sens, None)


def _jitter_rigid_scene(rng, b, n_ico3, n_ico4, n_box, area, sxyz, seed):
    """Rigid meshes of config 2: rest geometry centred at the origin; the base
    pose (position, yaw, size) is drawn here and jittered every frame."""
    starts, counts, base, half = [], [], [], []
    kinds = [3] * n_ico3 + [4] * n_ico4 + [-1] * n_box
    order = rng.permutation(len(kinds))
    for k in order:
        lvl = kinds[k]
        size = rng.uniform(0.5, 5.0)
        if lvl < 0:
            v, f = unit_box()
            v = v * size
            he = np.array([size / 2] * 3)
        else:
            v, f = icosphere(lvl)
            v = v * (size / 2)
            he = np.array([size / 2] * 3)
        rad = float(np.linalg.norm(he[:2])) + 1.0
        c = _place(rng, -area, area, np.array([rad, rad, he[2]]), sxyz)
        vs, _ = b.add(v, f)
        starts.append(vs)
        counts.append(v.shape[0])
        base.append([c[0], c[1], he[2], rng.uniform(0, 2 * math.pi), 1.0])
        half.append(he)
    return RigidSet(np.array(starts, np.uint32), np.array(counts, np.uint32), "jitter",
                    np.array(base), np.array(half), seed)


def config2(seed_extra: int = 0) -> Workload:
    """~1M triangles, one 128x4096 sensor (-25..+15 deg), 2,500 rigid meshes
    jittered every frame (translation <= 1 m, yaw <= 5 deg)."""
    ss = np.random.SeedSequence(BASE_SEED + 2 + seed_extra).spawn(4)
    rng = np.random.default_rng(ss[0])
    sens = [sensor([0.0, 0.0, 1.8], 0.0, elevations_uniform(-25, 15, 128), 4096)]
    sxyz = _sensor_xyz(sens)
    b = _Builder()
    g = _ground(b, 400.0, 316, rng)
    n_static_t = b.nt
    rs = _jitter_rigid_scene(rng, b, 500, 25, 1975, 200.0, sxyz, int(ss[1].generate_state(1)[0]))
    v, f = b.build()
    sc = Scene(v, f, rigid=rs, ground=g, n_dynamic_tris=int(f.shape[0] - n_static_t))
    sc._sensor_xy = sxyz
    return Workload("config2", sc, sens, 5243)


def _sheets(b, rng, n, cells, w, h, rmin, rmax, amp, omega):
    """Vertical deformable sheets (w x h metres, cells x cells) facing a random yaw."""
    groups, normals, phases = [], [], []
    for _ in range(n):
        gv, gf = grid(cells, cells, w, h, -w / 2, 0.0)
        yaw = rng.uniform(0, 2 * math.pi)
        dist = rng.uniform(rmin, rmax)
        ang = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(yaw), math.sin(yaw)
        # sheet plane spanned by (c, s, 0) and z; normal (-s, c, 0)
        x = gv[:, 0]
        y = gv[:, 1]
        world = np.stack([dist * math.cos(ang) + x * c, dist * math.sin(ang) + x * s, y + 0.5], 1)
        vs, _ = b.add(world, gf)
        nrm = np.tile(np.array([[-s, c, 0.0]]), (gv.shape[0], 1))
        groups.append(DeformGroup(vs, gv.shape[0], amp, omega))
        normals.append(nrm)
        phases.append(rng.uniform(0, 2 * math.pi, gv.shape[0]))
    return groups, np.concatenate(normals).astype(np.float32), np.concatenate(phases).astype(np.float32)


def config3(seed_extra: int = 0, scale: float = 1.0) -> Workload:
    """8 ring sensors of uneven shape; 3.0M static + 2.0M deformable triangles."""
    ss = np.random.SeedSequence(BASE_SEED + 3 + seed_extra).spawn(4)
    rng = np.random.default_rng(ss[0])
    shapes = [(128, 4096, 360.0)] * 4 + [(64, 2048, 360.0)] * 2 + [(128, 4096, 180.0)] * 2
    sens = ring_rig(shapes, seed=int(ss[2].generate_state(1)[0]))
    sxyz = _sensor_xyz(sens)
    b = _Builder()
    cells = max(2, int(round(750 * math.sqrt(scale))))
    g = _ground(b, 500.0, cells, rng)
    for _ in range(int(1000 * scale)):
        _add_sphere(b, rng, 3, rng.uniform(0.5, 5.0), -250, 250, sxyz)
    for _ in range(int(100 * scale)):
        _add_sphere(b, rng, 4, rng.uniform(0.5, 5.0), -250, 250, sxyz)
    for _ in range(int(6916 * scale)):
        _add_box(b, rng, 0.5, 10.0, -250, 250, sxyz)
    n_static = b.nt
    sheet_cells = max(2, int(round(354 * math.sqrt(scale))))
    groups, nrm, ph = _sheets(b, rng, 8, sheet_cells, 30.0, 15.0, 20.0, 150.0, 0.1, 2 * math.pi)
    v, f = b.build()
    sc = Scene(v, f, deform=groups, deform_normals=nrm, deform_phase=ph, ground=g,
               n_dynamic_tris=int(f.shape[0] - n_static))
    return Workload("config3", sc, sens, 256)


def _props_log_area(b, rng, n_tris, sxyz, area=500.0, rmax=60.0):
    """Icosphere props (levels 2..7) whose triangle areas are log-uniform on
    [1e-4, 10] m^2 when counted per triangle: each decade gets an equal share
    of the triangle budget."""
    decades = [(-4, -3), (-3, -2), (-2, -1), (-1, 0), (0, 1)]
    per = n_tris // len(decades)
    total = 0
    for lo, hi in decades:
        got = 0
        while got < per:
            a = 10 ** rng.uniform(lo, hi)
            levels = [L for L in range(2, 8)
                      if math.sqrt(a * 20 * 4 ** L / (4 * math.pi)) <= rmax
                      and 20 * 4 ** L <= max(per - got, 320)]
            if not levels:
                levels = [2]
            L = int(rng.choice(levels))
            r = math.sqrt(a * 20 * 4 ** L / (4 * math.pi))
            _add_sphere(b, rng, L, r, -area, area, sxyz)
            got += 20 * 4 ** L
        total += got
    return total


def config4(seed_extra: int = 0, range_max: float = 1000.0, scale: float = 1.0) -> Workload:
    """8 ring sensors 128x4096 (4 x 360, 4 x 180 deg), ~22M triangles (~9M dynamic)."""
    ss = np.random.SeedSequence(BASE_SEED + 4 + seed_extra).spawn(4)
    rng = np.random.default_rng(ss[0])
    shapes = [(128, 4096, 360.0)] * 4 + [(128, 4096, 180.0)] * 4
    sens = ring_rig(shapes, seed=int(ss[2].generate_state(1)[0]))
    for s in sens:
        s["range_max"] = np.float32(range_max)
    sxyz = _sensor_xyz(sens)
    b = _Builder()
    cells = max(2, int(round(1000 * math.sqrt(scale))))
    g = _ground(b, 1000.0, cells, rng)
    _props_log_area(b, rng, int(11_000_000 * scale), sxyz)
    n_static = b.nt
    # 20 rigid vehicle proxies: icosphere level 7 squashed to 4.57 x 2.28 x 1.08 m
    lvl = 7 if scale >= 0.5 else 4
    iv, if_ = icosphere(lvl)
    he = np.array([4.57 / 2, 2.28 / 2, 1.08 / 2])
    starts, counts = [], []
    for _ in range(20):
        vs, _ = b.add(iv * he, if_)
        starts.append(vs)
        counts.append(iv.shape[0])
    rs = RigidSet(np.array(starts, np.uint32), np.array(counts, np.uint32), "instant",
                  np.full((20, 5), 500.0), np.tile(he, (20, 1)), int(ss[1].generate_state(1)[0]))
    gcells = max(2, int(round(350 * math.sqrt(scale))))
    groups, nrm, ph = _sheets(b, rng, 10, gcells, 30.0, 15.0, 20.0, 150.0, 0.1, 2 * math.pi)
    v, f = b.build()
    sc = Scene(v, f, rigid=rs, deform=groups, deform_normals=nrm, deform_phase=ph, ground=g,
               n_dynamic_tris=int(f.shape[0] - n_static))
    sc._sensor_xy = sxyz
    return Workload("config4", sc, sens, 128)


def colocated_rig(origins, heads: int = 4, channels: int = 128, rays: int = 4096,
                  range_max: float = 1000.0):
    """Rigs of co-located heads: at each origin, `heads` sensors with yaws
    2*pi*j/heads, each covering 360/heads degrees, on the same full-vertical
    channel grid (several oriented LiDARs sharing one origin)."""
    out = []
    for o in origins:
        a0 = math.atan2(float(o[1]), float(o[0]))
        for j in range(heads):
            yaw = a0 + 2 * math.pi * j / heads
            out.append(sensor(o, yaw, elevations_full_sphere(channels), rays, 360.0 / heads,
                              range_max=range_max))
    return out


def oriented_heads(origin, n: int, channels: int = 128, rays: int = 4096,
                   range_max: float = 1000.0, tilt_deg: float = 20.0):
    """n full-turn heads sharing one origin, independently oriented: head k
    turned by 2*pi*k/n about the vertical and, for odd k, its spin axis tilted
    by tilt_deg towards its forward direction; full-vertical channel grid."""
    out = []
    for k in range(n):
        yaw = 2 * math.pi * k / n
        tau = math.radians(tilt_deg) if k % 2 else 0.0
        f = np.array([math.cos(yaw) * math.cos(tau), math.sin(yaw) * math.cos(tau),
                      math.sin(tau)])
        u = np.array([-math.cos(yaw) * math.sin(tau), -math.sin(yaw) * math.sin(tau),
                      math.cos(tau)])
        s = sensor(origin, yaw, elevations_full_sphere(channels), rays, 360.0,
                   range_max=range_max)
        s["forward"] = f.astype(np.float32)
        s["up"] = u.astype(np.float32)
        s["right"] = np.cross(f, u).astype(np.float32)
        out.append(s)
    return out


def distributed_heads(origins, channels: int = 128, rays: int = 4096,
                      range_max: float = 1000.0):
    """One upright full-turn head at each origin (yaw towards the origin's
    azimuth), full-vertical channel grid: the distributed counterpart of
    oriented_heads."""
    return [sensor(o, math.atan2(float(o[1]), float(o[0])), elevations_full_sphere(channels),
                   rays, 360.0, range_max=range_max) for o in origins]


def config4_colocated(seed_extra: int = 0, range_max: float = 1000.0,
                      scale: float = 1.0) -> Workload:
    """Config 4's scene seen by 2 rigs of 4 co-located 90-degree heads of 128x4096
    rays (the same 4.19M rays per frame), at the ring origins of config 4's
    sensors 0 and 4."""
    base = config4(seed_extra, range_max, scale)
    origins = [base.sensors[0]["origin"], base.sensors[4]["origin"]]
    sens = colocated_rig(origins, range_max=range_max)
    return Workload("config4_colocated", base.scene, sens, base.oracle_rays_per_sensor)


def client_workload(client: int, seed_extra: int = 0, tri_scale: float = 1.0) -> Workload:
    """One serving client: its own scene of 0.5-4M triangles (30-50% dynamic)
    built with config 3's recipe scaled, and 1-4 sensors drawn from
    {128x4096, 64x2048, 32x1024} x {360, 180} deg."""
    ss = np.random.SeedSequence([BASE_SEED + 5 + seed_extra, client]).spawn(4)
    rng = np.random.default_rng(ss[0])
    tau = rng.uniform(0.5e6, 4e6) * tri_scale
    dyn = rng.uniform(0.3, 0.5)
    n_s = int(rng.integers(1, 5))
    shapes = []
    for _ in range(n_s):
        g, x = [(128, 4096), (64, 2048), (32, 1024)][int(rng.integers(0, 3))]
        shapes.append((g, x, [360.0, 180.0][int(rng.integers(0, 2))]))
    sens = ring_rig(shapes, seed=int(ss[2].generate_state(1)[0]))
    sxyz = _sensor_xyz(sens)
    b = _Builder()
    static_t = tau * (1 - dyn)
    cells = max(2, int(math.sqrt(static_t * 0.4 / 2)))
    g = _ground(b, 500.0, cells, rng)
    while b.nt < static_t:
        if rng.uniform() < 0.3:
            _add_sphere(b, rng, 3, rng.uniform(0.5, 5.0), -250, 250, sxyz)
        else:
            _add_box(b, rng, 0.5, 10.0, -250, 250, sxyz)
    n_static = b.nt
    sheet_cells = max(2, int(math.sqrt(tau * dyn / 8 / 2)))
    groups, nrm, ph = _sheets(b, rng, 8, sheet_cells, 30.0, 15.0, 20.0, 150.0, 0.1, 2 * math.pi)
    v, f = b.build()
    sc = Scene(v, f, deform=groups, deform_normals=nrm, deform_phase=ph, ground=g,
               n_dynamic_tris=int(f.shape[0] - n_static))
    return Workload(f"client{client}", sc, sens, 64)


def small_random_scene(seed: int, n_tris: int = 64, spread: float = 6.0):
    """Tiny adversarial scene for property tests: random triangles around the
    origin, some huge, some tiny, some edge-on, some through the seam."""
    rng = np.random.default_rng(seed)
    v = []
    for _ in range(n_tris):
        kind = rng.integers(0, 4)
        c = rng.uniform(-spread, spread, 3)
        if kind == 0:      # ordinary
            tri = c + rng.normal(0, 1.0, (3, 3))
        elif kind == 1:    # tiny
            tri = c + rng.normal(0, 1e-3, (3, 3))
        elif kind == 2:    # huge, around the sensor
            tri = rng.normal(0, spread * 3, (3, 3))
        else:              # thin sliver
            a = c + rng.normal(0, 1.0, 3)
            bb = c + rng.normal(0, 1.0, 3)
            tri = np.stack([a, bb, a + (bb - a) * 0.5 + rng.normal(0, 1e-2, 3)])
        v.append(tri)
    v = np.concatenate(v).astype(np.float32)
    f = np.arange(v.shape[0], dtype=np.uint32).reshape(-1, 3)
    return v, f


def degenerate_scene():
    """Exact-degenerate inputs for parity tests, on a 10 x 10 m ground grid of
    1 m cells with a vertex at the origin and no sub-cell offset:
      * full-sphere sensors (nadir channel at -90 deg) exactly above a grid
        vertex, above a cell diagonal and above a cell boundary edge;
      * zero-area triangles: one repeated vertex three times, one with a
        repeated index, one with collinear vertices;
      * a vertical triangle whose plane contains the first sensor's origin;
      * a small wall in front of the first sensor straddling its range_min
        (0.5 m): the rays near its centre meet it closer than range_min;
      * an exactly duplicated triangle (same vertices, two ids).
    Returns (vertices, indices, sensors, (smaller id, larger id) of the duplicate)."""
    b = _Builder()
    gv, gf = grid(10, 10, 10.0, 10.0, -5.0, -5.0)
    b.add(gv, gf)
    extra = [
        np.array([[2.0, 1.0, 0.8]] * 3),                              # one point
        np.array([[2.5, -1.0, 0.5], [2.5, -1.5, 1.5], [2.5, -1.5, 1.5]]),  # repeated vertex
        np.array([[-2.0, 2.0, 0.3], [-2.0, 3.0, 1.3], [-2.0, 2.5, 0.8]]),  # collinear
        np.array([[2.0, 0.0, 0.5], [4.0, 0.0, 0.5], [3.0, 0.0, 3.0]]),   # plane y = 0 through o
        np.array([[0.4, -0.6, 1.0], [0.4, 0.6, 1.0], [0.4, 0.0, 2.1]]),  # straddles range_min
        np.array([[-3.0, -1.0, 0.2], [-3.0, 1.0, 0.2], [-3.0, 0.0, 2.5]]),  # duplicated wall
    ]
    for tri in extra:
        b.add(tri, np.array([[0, 1, 2]], np.uint32))
    v, f = b.build()
    # repeated index: the same stored vertex used twice
    f[b.nt - 5] = [f[b.nt - 5][0], f[b.nt - 5][1], f[b.nt - 5][1]]
    dup_v = v[f[b.nt - 1]]
    v = np.concatenate([v, dup_v]).astype(np.float32)
    n0 = v.shape[0] - 3
    f = np.concatenate([f, np.array([[n0, n0 + 1, n0 + 2]], np.uint32)]).astype(np.uint32)
    dup = (f.shape[0] - 2, f.shape[0] - 1)
    el = elevations_full_sphere(24)
    sensors = [sensor([0.0, 0.0, 1.5], 0.0, el, 96, 360.0, range_min=0.5, range_max=30.0),
               sensor([0.5, 0.5, 1.2], 0.7, el, 96, 360.0, range_max=30.0),
               sensor([0.5, 0.0, 2.0], -1.1, el, 96, 180.0, range_max=30.0)]
    return v, f, sensors, dup
