"""Seeded synthetic scenes, trajectories and depth frames.

This package generates inputs only.  Both the reference checker (``oracle/``)
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
