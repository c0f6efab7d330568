"""Seeded synthetic scenes, trajectories and depth frames.

This package generates inputs only.  Both the oracle (``oracle/``)
and the GPU library consume its output; it holds no part of the mapping
method itself (no TSDF, ESDF or alignment arithmetic).

Workloads (sizes follow the synthetic stand-ins for the paper's datasets):

* ``tiny``  -- 20 frames 160x120 (fx = fy = 120, cx = 80, cy = 60) of a
  4 x 4 x 3 m room with 5 spheres, camera on a 1 m circle at 1.2 m height
  looking at the room centre, additive noise sigma = 5 mm, range 5 m.
* ``room``  -- 300 frames 640x480 (fx = fy = 525, cx = 319.5, cy = 239.5) of
  an 8 x 6 x 3 m room with 20 boxes and 20 spheres, Catmull-Rom camera path
  at 1 cm/frame, noise sigma = 0.0012 z^2, 10 % invalid pixels, range 5 m.
* ``mav``   -- an outdoor scene of 120 x 80 x 20 m (heightfield rubble plus
  building boxes with wall openings), 640x480 frames with fx = fy = 380,
  range 10 m, noise sigma = 0.002 z^2.

Random scene layouts come from ``numpy.random.default_rng(seed)`` (PCG64);
per-pixel noise comes from Philox4x32-10 keyed by (seed, frame, pixel) in
``render.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "render.c")
_LIB = os.path.join(_HERE, "_render.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the renderer with gcc (host C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.sg_render.restype = None
        lib.sg_render.argtypes = [
            ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
            dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint32, ctypes.c_uint32, fp,
        ]
        lib.sg_philox4x32_10.restype = None
        lib.sg_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.sg_pixel_draws.restype = None
        lib.sg_pixel_draws.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.sg_render_outdoor.restype = None
        lib.sg_render_outdoor.argtypes = [
            dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, i32p, i32p,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
            ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, fp,
        ]
        lib.sg_hfield_eval.restype = ctypes.c_double
        lib.sg_hfield_eval.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key (for tests)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.sg_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def pixel_draws(seed, frame, pixel):
    """(standard normal, uniform) drawn for one pixel of one frame."""
    lib = _load()
    out = np.zeros(2, np.float64)
    lib.sg_pixel_draws(seed, frame, pixel, _dp(out))
    return float(out[0]), float(out[1])


# ------------------------------------------------------------------ geometry

def look_at(pos, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """T_world_cam (4x4, float64) for a camera at ``pos`` looking at ``target``.

    Camera axes: x right, y down, z forward."""
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    return pose_from_forward(pos, f, up)


def pose_from_forward(pos, forward, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    x = x / np.linalg.norm(x)
    y = np.cross(f, x)
    T = np.eye(4)
    T[:3, 0] = x
    T[:3, 1] = y
    T[:3, 2] = f
    T[:3, 3] = pos
    return T


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1.0, 0], [-s, 0, c]])


def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0, 0], [0, c, -s], [0, s, c]])


# ------------------------------------------------------------------- scenes

@dataclass
class Camera:
    H: int
    W: int
    fx: float
    fy: float
    cx: float
    cy: float
    max_range: float
    noise_model: int = 0      # 0 none, 1 additive sigma = noise_a, 2 sigma = noise_a * z^2
    noise_a: float = 0.0
    invalid_frac: float = 0.0

    @property
    def K(self):
        return np.array([self.fx, self.fy, self.cx, self.cy], np.float32)


@dataclass
class Scene:
    room: np.ndarray | None = None                     # (6,) interior box lo, hi
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    hfield: np.ndarray | None = None                   # (ny, nx) heights
    hf_origin: tuple = (0.0, 0.0)
    hf_step: float = 1.0
    hf_slope: float = 0.0

    def sdf(self, p: np.ndarray) -> np.ndarray:
        """Signed distance to the nearest surface (positive in free space) for
        rooms with spheres and boxes; heightfields give the vertical gap, an
        upper bound."""
        p = np.atleast_2d(np.asarray(p, np.float64))
        d = np.full(len(p), np.inf)
        if self.room is not None:
            lo, hi = self.room[:3], self.room[3:]
            d = np.minimum(d, np.min(np.concatenate([p - lo, hi - p], axis=1), axis=1))
        for s in self.spheres:
            d = np.minimum(d, np.linalg.norm(p - s[:3], axis=1) - s[3])
        for b in self.boxes:
            lo, hi = b[:3], b[3:]
            q = np.maximum(lo - p, p - hi)
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
            inside = np.minimum(np.max(q, axis=1), 0.0)
            d = np.minimum(d, outside + inside)
        if self.hfield is not None:
            lib = _load()
            hf = np.ascontiguousarray(self.hfield, np.float64)
            ny, nx = hf.shape
            hz = np.array([lib.sg_hfield_eval(_dp(hf), nx, ny, self.hf_origin[0], self.hf_origin[1],
                                              self.hf_step, float(x), float(y)) for x, y in p[:, :2]])
            d = np.minimum(d, p[:, 2] - hz)
        return d


def render(scene: Scene, cam: Camera, T_world_cam: np.ndarray, seed: int, frame: int) -> np.ndarray:
    """Render one float32 depth frame (H x W, metres, 0 = invalid)."""
    if isinstance(scene, OutdoorScene):
        return scene.render(cam, T_world_cam, seed, frame)
    lib = _load()
    out = np.zeros((cam.H, cam.W), np.float32)
    room = np.ascontiguousarray(scene.room if scene.room is not None else np.zeros(6), np.float64)
    sph = np.ascontiguousarray(scene.spheres.reshape(-1), np.float64)
    box = np.ascontiguousarray(scene.boxes.reshape(-1), np.float64)
    if sph.size == 0:
        sph = np.zeros(4)
    if box.size == 0:
        box = np.zeros(6)
    T = np.ascontiguousarray(T_world_cam, np.float64).reshape(16)
    if scene.hfield is not None:
        hf = np.ascontiguousarray(scene.hfield, np.float64)
        hf_ptr, ny, nx = _dp(hf), hf.shape[0], hf.shape[1]
    else:
        hf = None
        hf_ptr, ny, nx = ctypes.POINTER(ctypes.c_double)(), 0, 0
    lib.sg_render(int(scene.room is not None), _dp(room), len(scene.spheres), _dp(sph),
                  len(scene.boxes), _dp(box), hf_ptr, nx, ny, float(scene.hf_origin[0]),
                  float(scene.hf_origin[1]), float(scene.hf_step), float(scene.hf_slope),
                  cam.H, cam.W, cam.fx, cam.fy, cam.cx, cam.cy, _dp(T), cam.max_range,
                  cam.noise_model, cam.noise_a, cam.invalid_frac, seed & 0xFFFFFFFF,
                  frame & 0xFFFFFFFF, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    del hf
    return out


@dataclass
class OutdoorScene:
    """Heightfield ground (bilinear on a grid of spacing hs) plus solid boxes
    (building walls), with a coarse 2-D cell list for the boxes."""
    hfield: np.ndarray            # (ny, nx)
    hs: float
    origin: tuple
    boxes: np.ndarray             # (n, 6)
    cell: float = 5.0
    buildings: list = field(default_factory=list)   # (lo, hi) footprints with base and height

    def __post_init__(self):
        x0, y0 = self.origin
        ny, nx = self.hfield.shape
        self.ncx = int(math.ceil((nx - 1) * self.hs / self.cell))
        self.ncy = int(math.ceil((ny - 1) * self.hs / self.cell))
        lists = [[] for _ in range(self.ncx * self.ncy)]
        for i, b in enumerate(self.boxes):
            cx0 = max(0, int((b[0] - x0) // self.cell)); cx1 = min(self.ncx - 1, int((b[3] - x0) // self.cell))
            cy0 = max(0, int((b[1] - y0) // self.cell)); cy1 = min(self.ncy - 1, int((b[4] - y0) // self.cell))
            for cy in range(cy0, cy1 + 1):
                for cx in range(cx0, cx1 + 1):
                    lists[cy * self.ncx + cx].append(i)
        self._start = np.zeros(len(lists) + 1, np.int32)
        self._start[1:] = np.cumsum([len(l) for l in lists])
        self._items = np.array([i for l in lists for i in l] or [0], np.int32)
        self._hf = np.ascontiguousarray(self.hfield, np.float64)
        self._box = np.ascontiguousarray(self.boxes.reshape(-1) if len(self.boxes) else np.zeros(6), np.float64)

    def height(self, x, y):
        lib = _load()
        ny, nx = self._hf.shape
        return lib.sg_hfield_eval(_dp(self._hf), nx, ny, self.origin[0], self.origin[1], self.hs, float(x), float(y))

    def render(self, cam, T_world_cam, seed, frame):
        lib = _load()
        out = np.zeros((cam.H, cam.W), np.float32)
        T = np.ascontiguousarray(T_world_cam, np.float64).reshape(16)
        ny, nx = self._hf.shape
        i32 = ctypes.POINTER(ctypes.c_int32)
        lib.sg_render_outdoor(_dp(self._hf), nx, ny, self.origin[0], self.origin[1], self.hs, _dp(self._box),
                              self._start.ctypes.data_as(i32), self._items.ctypes.data_as(i32), self.ncx, self.ncy,
                              self.origin[0], self.origin[1], self.cell, cam.H, cam.W, cam.fx, cam.fy, cam.cx, cam.cy,
                              _dp(T), cam.max_range, cam.noise_model, cam.noise_a, cam.invalid_frac,
                              seed & 0xFFFFFFFF, frame & 0xFFFFFFFF,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        return out


@dataclass
class Workload:
    name: str
    scene: Scene
    cam: Camera
    poses: np.ndarray          # (F, 4, 4) T_world_cam, float64
    seed: int
    voxel_size: float
    trunc_vox: int = 4
    d_max: float = 2.0
    submap_every: int = 0      # 0: a single submap

    @property
    def n_frames(self):
        return len(self.poses)

    def frame(self, f: int) -> np.ndarray:
        return render(self.scene, self.cam, self.poses[f], self.seed, f)

    def frames(self, start: int = 0, stop: int | None = None) -> np.ndarray:
        stop = self.n_frames if stop is None else stop
        return np.stack([self.frame(f) for f in range(start, stop)])


def _dist_to_circle(p, radius, height):
    rho = math.hypot(p[0], p[1])
    return math.hypot(rho - radius, p[2] - height)


def tiny(seed: int = 1, n_frames: int = 20, noise: bool = True) -> Workload:
    """4 x 4 x 3 m room, 5 spheres, 20 frames of 160x120 on a 1 m circle."""
    rng = np.random.default_rng(seed)
    lo = np.array([-2.0, -2.0, 0.0])
    hi = np.array([2.0, 2.0, 3.0])
    spheres = []
    while len(spheres) < 5:
        r = rng.uniform(0.2, 0.5)
        c = rng.uniform(lo + r + 0.05, hi - r - 0.05)
        if _dist_to_circle(c, 1.0, 1.2) < r + 0.3:
            continue
        if any(np.linalg.norm(c - s[:3]) < r + s[3] for s in spheres):
            continue
        spheres.append(np.array([c[0], c[1], c[2], r]))
    scene = Scene(room=np.concatenate([lo, hi]), spheres=np.array(spheres))
    cam = Camera(H=120, W=160, fx=120.0, fy=120.0, cx=80.0, cy=60.0, max_range=5.0,
                 noise_model=1 if noise else 0, noise_a=0.005)
    poses = []
    for k in range(n_frames):
        th = 2.0 * math.pi * k / n_frames
        poses.append(look_at([math.cos(th), math.sin(th), 1.2], [0.0, 0.0, 1.2]))
    return Workload("tiny", scene, cam, np.array(poses), seed, voxel_size=0.05, d_max=2.0)


def _catmull_rom(pts: np.ndarray, samples_per_seg: int = 2000) -> np.ndarray:
    """Uniform Catmull-Rom curve through every point (end points repeated)."""
    P = np.concatenate([pts[:1], pts, pts[-1:]], axis=0)
    out = []
    t = np.linspace(0.0, 1.0, samples_per_seg, endpoint=False)[:, None]
    for i in range(1, len(P) - 2):
        p0, p1, p2, p3 = P[i - 1], P[i], P[i + 1], P[i + 2]
        c = 0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                   + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3)
        out.append(c)
    out.append(P[-2][None])
    return np.concatenate(out, axis=0)


def _resample_arclength(curve: np.ndarray, step: float, n: int) -> tuple[np.ndarray, np.ndarray]:
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    want = step * np.arange(n)
    if want[-1] > s[-1]:
        raise ValueError("curve too short for the requested frames")
    pos = np.stack([np.interp(want, s, curve[:, k]) for k in range(3)], axis=1)
    # tangent from a finite difference along the curve
    eps = 1e-3
    pos2 = np.stack([np.interp(np.minimum(want + eps, s[-1]), s, curve[:, k]) for k in range(3)], axis=1)
    pos1 = np.stack([np.interp(np.maximum(want - eps, 0.0), s, curve[:, k]) for k in range(3)], axis=1)
    return pos, pos2 - pos1


def _box_point_dist(b, p):
    q = np.maximum(b[:3] - p, p - b[3:])
    return float(np.linalg.norm(np.maximum(q, 0.0)) + min(np.max(q), 0.0))


def room(seed: int = 2, n_frames: int = 300, noise: bool = True) -> Workload:
    """8 x 6 x 3 m room, 20 boxes + 20 spheres, 300 frames 640x480."""
    rng = np.random.default_rng(seed)
    lo = np.array([0.0, 0.0, 0.0])
    hi = np.array([8.0, 6.0, 3.0])
    # camera path: 6 waypoints ~0.8 m apart inside the central region
    while True:
        wp = [np.array([rng.uniform(2.5, 5.5), rng.uniform(2.0, 4.0), rng.uniform(1.0, 2.0)])]
        head = rng.uniform(-math.pi, math.pi)
        ok = True
        for _ in range(5):
            head += rng.uniform(-0.7, 0.7)
            nxt = wp[-1] + 0.8 * np.array([math.cos(head), math.sin(head), 0.0])
            nxt[2] = rng.uniform(1.0, 2.0)
            if np.any(nxt[:2] < 1.2) or nxt[0] > 6.8 or nxt[1] > 4.8:
                ok = False
                break
            wp.append(nxt)
        if ok:
            break
    curve = _catmull_rom(np.array(wp))
    pos, tan = _resample_arclength(curve, 0.01, n_frames)
    ph_y, ph_p = rng.uniform(0, 2 * math.pi, size=2)
    s = 0.01 * np.arange(n_frames)
    poses = []
    for k in range(n_frames):
        yaw = math.atan2(tan[k, 1], tan[k, 0]) + math.radians(15.0) * math.sin(2 * math.pi * s[k] / 2.0 + ph_y)
        pitch = math.radians(10.0) * math.sin(2 * math.pi * s[k] / 1.5 + ph_p)
        fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        poses.append(pose_from_forward(pos[k], fwd))
    path = pos

    boxes, spheres = [], []

    def clear_of_path(dist_fn):
        return all(dist_fn(p) >= 0.5 for p in path[::5])

    while len(boxes) < 20:
        side = rng.uniform(0.2, 1.0, size=3)
        c = rng.uniform(lo[:2] + side[:2] / 2 + 0.05, hi[:2] - side[:2] / 2 - 0.05)
        z0 = 0.0 if rng.uniform() < 0.5 else rng.uniform(0.3, 2.5 - side[2])
        b = np.array([c[0] - side[0] / 2, c[1] - side[1] / 2, z0,
                      c[0] + side[0] / 2, c[1] + side[1] / 2, z0 + side[2]])
        if any(np.all(b[:3] < o[3:] + 0.05) and np.all(o[:3] < b[3:] + 0.05) for o in boxes):
            continue
        if not clear_of_path(lambda p: _box_point_dist(b, p)):
            continue
        boxes.append(b)
    while len(spheres) < 20:
        r = rng.uniform(0.1, 0.5)
        c = rng.uniform(lo + r + 0.05, hi - r - 0.05)
        if any(np.linalg.norm(c - o[:3]) < r + o[3] + 0.05 for o in spheres):
            continue
        if any(_box_point_dist(b, c) < r + 0.05 for b in boxes):
            continue
        if not clear_of_path(lambda p: np.linalg.norm(p - c) - r):
            continue
        spheres.append(np.array([c[0], c[1], c[2], r]))
    scene = Scene(room=np.concatenate([lo, hi]), spheres=np.array(spheres), boxes=np.array(boxes))
    cam = Camera(H=480, W=640, fx=525.0, fy=525.0, cx=319.5, cy=239.5, max_range=5.0,
                 noise_model=2 if noise else 0, noise_a=0.0012, invalid_frac=0.1 if noise else 0.0)
    return Workload("room", scene, cam, np.array(poses), seed, voxel_size=0.05, d_max=2.0)


def wall_scene(z0: float, H: int = 12, W: int = 16, f: float = 12.0) -> tuple[Scene, Camera]:
    """A camera at the origin of a large box looking at a fronto-parallel wall
    at depth ``z0`` (no noise).  Used by closed-form checks."""
    scene = Scene(room=np.array([-50.0, -50.0, -50.0, 50.0, 50.0, z0]))
    cam = Camera(H=H, W=W, fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0, max_range=10.0)
    return scene, cam


# ------------------------------------------------------------ outdoor (MAV)

def _value_noise(rng, nx, ny, hs, spacing):
    """Value noise on the sample grid: uniform lattice values every `spacing`
    metres, smoothstep-bilinear in between."""
    gx = np.arange(nx) * hs / spacing
    gy = np.arange(ny) * hs / spacing
    lat = rng.uniform(-1.0, 1.0, size=(int(gy[-1]) + 2, int(gx[-1]) + 2))
    ix, iy = np.floor(gx).astype(int), np.floor(gy).astype(int)
    fx, fy = gx - ix, gy - iy
    sx, sy = fx * fx * (3 - 2 * fx), fy * fy * (3 - 2 * fy)
    a = lat[iy][:, ix] * (1 - sx) + lat[iy][:, ix + 1] * sx
    b = lat[iy + 1][:, ix] * (1 - sx) + lat[iy + 1][:, ix + 1] * sx
    return a * (1 - sy[:, None]) + b * sy[:, None]


def _wall_boxes(lo, hi, axis, door_c, door_w, door_h, z0):
    """A wall box [lo, hi] with a door opening centred at door_c along `axis`
    (0: wall runs along x, 1: along y), split into left, right and lintel."""
    out = []
    a0, a1 = lo[axis], hi[axis]
    d0, d1 = door_c - door_w / 2, door_c + door_w / 2
    for s0, s1 in ((a0, d0), (d1, a1)):
        if s1 - s0 > 1e-6:
            l, h = lo.copy(), hi.copy()
            l[axis], h[axis] = s0, s1
            out.append(np.concatenate([l, h]))
    l, h = lo.copy(), hi.copy()
    l[axis], h[axis] = d0, d1
    l[2] = z0 + door_h
    if h[2] > l[2]:
        out.append(np.concatenate([l, h]))
    return out


def mav(seed: int = 3, n_frames: int = 3000, path_length: float = 400.0, noise: bool = True,
        scale: float = 1.0) -> Workload:
    """Outdoor 120 x 80 x 20 m scene: rubble heightfield (4 octaves of value
    noise, 0.5 m samples) plus 15-30 buildings with 0.3 m walls and door
    openings; a seeded spline at 2-8 m above ground that passes through one
    building; 640x480 frames, fx = fy = 380, range 10 m, sigma = 0.002 z^2.
    scale < 1 renders the same views with fewer pixels (same field of view:
    W, H, fx, fy scaled, pixel-centre principal point)."""
    rng = np.random.default_rng(seed)
    hs, X, Y = 0.5, 120.0, 80.0
    nx, ny = int(X / hs) + 1, int(Y / hs) + 1
    h = np.zeros((ny, nx))
    for spacing, amp in ((8.0, 1.4), (4.0, 0.8), (2.0, 0.5), (1.0, 0.3)):
        h += amp * _value_noise(rng, nx, ny, hs, spacing)
    h -= h.min()
    xs, ys = np.arange(nx) * hs, np.arange(ny) * hs
    boxes, foot = [], []
    n_b = int(rng.integers(15, 31))
    corridor = None  # (x0, x1, y0, y1): kept free for the passage through building 0
    tries = 0
    while len(foot) < n_b and tries < 4000:
        tries += 1
        w, l, ht = rng.uniform(7, 12), rng.uniform(7, 10), rng.uniform(3, 6)
        if not foot:
            c = rng.uniform([35, 25], [X - 35, Y - 25])
        else:
            c = rng.uniform([12, 12], [X - 12, Y - 12])
        lo = np.array([c[0] - w / 2, c[1] - l / 2])
        hi = np.array([c[0] + w / 2, c[1] + l / 2])
        if any(np.all(lo < f[1] + 4) and np.all(f[0] < hi + 4) for f in foot):
            continue
        if corridor is not None and lo[0] < corridor[1] and corridor[0] < hi[0] and lo[1] < corridor[3] \
                and corridor[2] < hi[1]:
            continue
        mx = (xs >= lo[0] - 1) & (xs <= hi[0] + 1)
        my = (ys >= lo[1] - 1) & (ys <= hi[1] + 1)
        base = float(h[np.ix_(my, mx)].mean())
        h[np.ix_(my, mx)] = base
        if not foot:
            cyc = (lo[1] + hi[1]) / 2
            corridor = (lo[0] - 25, hi[0] + 25, cyc - 5, cyc + 5)
            cx_ = (xs >= corridor[0]) & (xs <= corridor[1])
            cy_ = (ys >= corridor[2]) & (ys <= corridor[3])
            h[np.ix_(cy_, cx_)] = np.minimum(h[np.ix_(cy_, cx_)], base)
        foot.append((lo, hi, base, ht))
    for k, (lo, hi, base, ht) in enumerate(foot):
        t, z0, z1 = 0.3, base - 0.5, base + ht
        dw, dh = 3.0, 3.5
        # walls at y = lo/hi (running along x) and x = lo/hi (running along y); the
        # first building gets doors facing each other on its x walls
        cy = (lo[1] + hi[1]) / 2 if k == 0 else rng.uniform(lo[1] + 2, hi[1] - 2)
        walls = [
            (np.array([lo[0], lo[1], z0]), np.array([hi[0], lo[1] + t, z1]), 0, rng.uniform(lo[0] + 2, hi[0] - 2)),
            (np.array([lo[0], hi[1] - t, z0]), np.array([hi[0], hi[1], z1]), 0, rng.uniform(lo[0] + 2, hi[0] - 2)),
            (np.array([lo[0], lo[1], z0]), np.array([lo[0] + t, hi[1], z1]), 1, cy),
            (np.array([hi[0] - t, lo[1], z0]), np.array([hi[0], hi[1], z1]), 1, cy),
        ]
        for wlo, whi, axis, dc in walls:
            boxes.extend(_wall_boxes(wlo, whi, axis, dc, dw, dh, base))
        boxes.append(np.array([lo[0], lo[1], z1 - t, hi[0], hi[1], z1]))
    scene = OutdoorScene(hfield=h, hs=hs, origin=(0.0, 0.0), boxes=np.array(boxes), buildings=foot)

    def inside_building(p, margin=0.6):
        for lo, hi, base, ht in foot:
            if lo[0] - margin < p[0] < hi[0] + margin and lo[1] - margin < p[1] < hi[1] + margin \
                    and p[2] < base + ht + margin:
                return True
        return False

    # path: cruise waypoints (2-5 m above ground, 1.5 m above roofs within 10 m)
    # and a passage through building 0 from door to door along +x
    lo0, hi0, base0, _ = foot[0]
    cy0 = (lo0[1] + hi0[1]) / 2
    zin = base0 + 1.75
    passage = [np.array([x, cy0, zin]) for x in (lo0[0] - 20, lo0[0] - 8, lo0[0] - 1, (lo0[0] + hi0[0]) / 2,
                                                  hi0[0] + 1, hi0[0] + 8, hi0[0] + 20)]

    def cruise(p):
        z = scene.height(p[0], p[1]) + rng.uniform(2.0, 5.0)
        for lo, hi, base, ht in foot:
            dx = max(lo[0] - p[0], 0.0, p[0] - hi[0])
            dy = max(lo[1] - p[1], 0.0, p[1] - hi[1])
            if math.hypot(dx, dy) < 10.0:
                z = max(z, base + ht + 1.5)
        return np.array([p[0], p[1], z])

    for attempt in range(1000):
        n_before = int(rng.integers(3, 7))
        n_after = 10 - n_before
        seq = []
        cur = passage[0].copy()
        for _ in range(n_before):
            ang = rng.uniform(-math.pi, math.pi)
            cur = cur + rng.uniform(25, 45) * np.array([math.cos(ang), math.sin(ang), 0.0])
            cur[0] = min(max(cur[0], 8.0), X - 8.0)
            cur[1] = min(max(cur[1], 8.0), Y - 8.0)
            seq.append(cruise(cur))
        pts = seq[::-1] + passage
        cur = passage[-1].copy()
        for _ in range(n_after):
            ang = rng.uniform(-math.pi, math.pi)
            cur = cur + rng.uniform(25, 45) * np.array([math.cos(ang), math.sin(ang), 0.0])
            cur[0] = min(max(cur[0], 8.0), X - 8.0)
            cur[1] = min(max(cur[1], 8.0), Y - 8.0)
            pts.append(cruise(cur))
        pts = np.array(pts)
        curve = _catmull_rom(pts, samples_per_seg=400)
        seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
        if seg.sum() < path_length:
            continue
        ok = True
        for q in curve[::20]:
            if q[2] < scene.height(q[0], q[1]) + 1.0:
                ok = False
                break
            in_corr = corridor[0] < q[0] < corridor[1] and abs(q[1] - cy0) < 1.4
            if not in_corr and inside_building(q):
                ok = False
                break
        if ok:
            break
    else:
        raise RuntimeError("no collision-free path found")
    pos, tan = _resample_arclength(curve, path_length / n_frames, n_frames)
    poses = []
    for k in range(n_frames):
        yaw = math.atan2(tan[k, 1], tan[k, 0])
        inside = lo0[0] - 2 < pos[k, 0] < hi0[0] + 2 and abs(pos[k, 1] - cy0) < 2
        pitch = 0.0 if inside else math.radians(-30.0)
        fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        poses.append(pose_from_forward(pos[k], fwd))
    Wd, Hd = int(round(640 * scale)), int(round(480 * scale))
    cam = Camera(H=Hd, W=Wd, fx=380.0 * scale, fy=380.0 * scale, cx=(Wd - 1) / 2.0, cy=(Hd - 1) / 2.0,
                 max_range=10.0, noise_model=2 if noise else 0, noise_a=0.002)
    return Workload("mav", scene, cam, np.array(poses), seed, voxel_size=0.10, d_max=3.0, submap_every=100)


def gravity_aligned(T: np.ndarray) -> np.ndarray:
    """Pose with the same position and yaw as T and no roll or pitch (the
    camera's forward axis projected on the ground plane)."""
    f = T[:3, 2]
    yaw = math.atan2(f[1], f[0])
    G = np.eye(4)
    G[:3, :3] = rot_z(yaw)
    G[:3, 3] = T[:3, 3]
    return G


def _fmix64(k: np.ndarray) -> np.ndarray:
    """MurmurHash3's 64-bit finaliser (Appleby): a bijection of uint64."""
    k = k.copy()
    s = np.uint64(33)
    k ^= k >> s
    k *= np.uint64(0xFF51AFD7ED558CCD)
    k ^= k >> s
    k *= np.uint64(0xC4CEB9FE1A85EC53)
    k ^= k >> s
    return k


def hash_keys(n: int, seed: int = 7) -> np.ndarray:
    """n distinct pseudo-random uint64 keys, none equal to all ones (the empty
    slot of a table): a bijection of n consecutive counters from a seeded
    random start, so distinct by construction."""
    start = np.random.default_rng(seed).integers(0, 2 ** 63, dtype=np.uint64)
    ctr = np.arange(n + 1, dtype=np.uint64)
    ctr += start
    k = _fmix64(ctr)
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    bad = np.flatnonzero(k[:n] == full)
    if len(bad):
        k[bad] = k[n]  # the spare counter (all ones appears at most once)
    return k[:n]
