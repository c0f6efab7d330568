"""covox oracle -- TEST INFRASTRUCTURE ONLY.

A thin ctypes wrapper around ``covox_oracle.c`` (and, in ``pgo.py``, the
submap pose-graph optimisation in numpy): a plain, slow CPU
implementation of projective TSDF integration, the exact truncated ESDF and
the correspondence-free ESDF alignment (Hoss and De Cristoforis, coVoxSLAM,
arXiv 2410.21149: Sec. III-C, III-D, III-E, III-F, Eq. 1).  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it;
the GPU library never imports or links it, and it imports nothing from the
GPU library.

Build flags: gcc -O2 -ffp-contract=off (no FMA contraction, no fast-math), so
that the binary32 mode follows the pinned operation order; -fopenmp for the
loops over independent items (set_threads), whose results do not depend on
the thread count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "covox_oracle.c")
_SRC_NET = os.path.join(_HERE, "covox_net.c")
_LIB = os.path.join(_HERE, "_covox_oracle.so")
_lib = None

OK, EINVAL, EDEGENERATE, NOT_CONVERGED = 0, -1, -5, 1


def build(force: bool = False) -> str:
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in (_SRC, _SRC_NET))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, _SRC_NET, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("vs", ctypes.c_double), ("trunc_vox", ctypes.c_int), ("max_range", ctypes.c_double),
                ("d_max", ctypes.c_double), ("w_reg", ctypes.c_double), ("fp64", ctypes.c_int),
                ("fp16", ctypes.c_int), ("max_iter", ctypes.c_int), ("n_min", ctypes.c_int),
                ("tol_rho", ctypes.c_double), ("tol_theta", ctypes.c_double), ("align_dof", ctypes.c_int),
                ("weight_mode", ctypes.c_int), ("integrator", ctypes.c_int), ("ray_carve", ctypes.c_int),
                ("esdf_mode", ctypes.c_int), ("align_solver", ctypes.c_int)]


class _Conv(ctypes.Structure):
    _fields_ = [("cin", ctypes.c_int), ("cout", ctypes.c_int), ("din", ctypes.c_int), ("dout", ctypes.c_int),
                ("stride", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_submap_create.restype = _vp
        L.orc_submap_create.argtypes = [ctypes.POINTER(_Params), _dp]
        L.orc_set_solver.restype = None
        L.orc_set_solver.argtypes = [_vp, ctypes.POINTER(_Params)]
        L.orc_submap_destroy.restype = None
        L.orc_submap_destroy.argtypes = [_vp]
        L.orc_integrate.restype = ctypes.c_int
        L.orc_integrate.argtypes = [_vp, _fp, ctypes.c_int, ctypes.c_int, _fp, _dp, _i64p]
        L.orc_update_esdf.restype = ctypes.c_int
        L.orc_update_esdf.argtypes = [_vp]
        L.orc_n_blocks.restype = ctypes.c_int64
        L.orc_n_blocks.argtypes = [_vp]
        L.orc_export.restype = None
        L.orc_export.argtypes = [_vp, _u64p, _dp, _dp, _dp, _i32p]
        L.orc_import.restype = ctypes.c_int
        L.orc_import.argtypes = [_vp, ctypes.c_int64, _u64p, _dp, _dp]
        L.orc_iso_points.restype = ctypes.c_int64
        L.orc_iso_points.argtypes = [_vp, _vp, ctypes.c_int64]
        L.orc_normal_eq.restype = None
        L.orc_normal_eq.argtypes = [_vp, _vp, ctypes.c_int64, _dp, _dp]
        L.orc_align_points.restype = ctypes.c_int
        L.orc_align_points.argtypes = [_vp, _vp, ctypes.c_int64, _dp, _dp, _dp, _i64p]
        L.orc_align_multistart.restype = ctypes.c_int
        L.orc_align_multistart.argtypes = [_vp, _vp, ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _i64p,
                                           ctypes.POINTER(ctypes.c_int), _dp]
        L.orc_se3_exp.restype = None
        L.orc_se3_exp.argtypes = [_dp, _dp]
        L.orc_solve6.restype = ctypes.c_int
        L.orc_solve6.argtypes = [_dp, _dp]
        L.orc_solve6_damped.restype = ctypes.c_int
        L.orc_solve6_damped.argtypes = [_dp, ctypes.c_double, _dp]
        L.orc_solve_xyz_yaw_damped.restype = ctypes.c_int
        L.orc_solve_xyz_yaw_damped.argtypes = [_dp, ctypes.c_double, _dp]
        L.orc_hash_insert.restype = None
        L.orc_hash_insert.argtypes = [_u64p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int64, _u64p, ctypes.c_int64,
                                      ctypes.c_uint32, _i64p, _i64p]
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_f2h.restype = ctypes.c_uint16
        L.orc_f2h.argtypes = [ctypes.c_float]
        L.orc_h2f.restype = ctypes.c_float
        L.orc_h2f.argtypes = [ctypes.c_uint16]
        L.orc_net_num_params.restype = ctypes.c_int64
        L.orc_net_num_params.argtypes = [ctypes.POINTER(_Conv), ctypes.c_int, ctypes.c_int]
        L.orc_net_forward.restype = ctypes.c_int
        L.orc_net_forward.argtypes = [ctypes.POINTER(_Conv), ctypes.c_int, ctypes.c_int, _fp, _fp, ctypes.c_int,
                                      ctypes.c_int, _dp]
        L.orc_net_loss_grad.restype = ctypes.c_int
        L.orc_net_loss_grad.argtypes = [ctypes.POINTER(_Conv), ctypes.c_int, ctypes.c_int, _fp, _fp, _fp, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_summary.restype = ctypes.c_int
        L.orc_summary.argtypes = [_vp, ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.orc_bf16_round.restype = ctypes.c_float
        L.orc_bf16_round.argtypes = [ctypes.c_float]
        L.orc_esdf_wavefront.restype = ctypes.c_int
        L.orc_esdf_wavefront.argtypes = [_vp, _i64p]
        L.orc_ray_walk32.restype = ctypes.c_int64
        L.orc_ray_walk32.argtypes = [_fp, _fp, ctypes.c_float, ctypes.c_float, ctypes.c_float, _i64p, ctypes.c_int64]
        L.orc_ray_walk32_fragile.restype = ctypes.c_int64
        L.orc_ray_walk32_fragile.argtypes = [_fp, _fp, ctypes.c_float, ctypes.c_float, ctypes.c_float, _i64p,
                                             ctypes.c_int64, _i64p, ctypes.c_int64, _i64p]
        L.orc_fragile_voxels.restype = ctypes.c_int64
        L.orc_fragile_voxels.argtypes = [_vp, _i64p, ctypes.c_int64]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_pose_cam_sub.restype = None
        L.orc_pose_cam_sub.argtypes = [_dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (n < 1: all cores); returns
    the count in use.  Results do not depend on it."""
    return int(_load().orc_set_threads(int(n)))


def _mat(T):
    return np.ascontiguousarray(np.asarray(T, np.float64).reshape(16))


class Params:
    """Map and solver parameters (metres)."""

    def __init__(self, vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, w_reg=2.0, fp64=False, fp16=False,
                 max_iter=30, n_min=100, tol_rho=1e-7, tol_theta=1e-8, align_dof=6, weight_mode=0, integrator=0,
                 ray_carve=True, esdf_mode=0, align_solver=0):
        self.vs, self.trunc_vox, self.max_range, self.d_max = vs, trunc_vox, max_range, d_max
        self.w_reg, self.fp64, self.fp16, self.max_iter, self.n_min = w_reg, fp64, fp16, max_iter, n_min
        self.tol_rho, self.tol_theta, self.align_dof, self.weight_mode = tol_rho, tol_theta, align_dof, weight_mode
        self.integrator, self.ray_carve = integrator, ray_carve  # 0: projection mapping, 1: raycasting
        self.esdf_mode = esdf_mode  # 0: exact EDT, 1: incremental wavefront
        self.align_solver = align_solver  # 0: Gauss-Newton, 1: Levenberg-Marquardt

    def _c(self):
        return _Params(self.vs, self.trunc_vox, self.max_range, self.d_max, self.w_reg, int(self.fp64),
                       int(self.fp16), self.max_iter, self.n_min, self.tol_rho, self.tol_theta, int(self.align_dof),
                       int(self.weight_mode), int(self.integrator), int(bool(self.ray_carve)), int(self.esdf_mode),
                       int(self.align_solver))


class Submap:
    """A submap of 8^3-voxel blocks with TSDF (D, W) and ESDF (phi) state."""

    def __init__(self, params: Params, T_world_submap=None):
        self.params = params
        L = _load()
        T = _mat(np.eye(4) if T_world_submap is None else T_world_submap)
        self._cp = params._c()
        self._h = L.orc_submap_create(ctypes.byref(self._cp), _p(T, _dp))

    def set_solver(self, params: Params):
        """Takes the alignment solver's parameters (max_iter, n_min, tol_rho,
        tol_theta, align_dof, align_solver) from params; the map is kept."""
        cp = params._c()
        _load().orc_set_solver(self._h, ctypes.byref(cp))
        for k in ("max_iter", "n_min", "tol_rho", "tol_theta", "align_dof", "align_solver"):
            setattr(self.params, k, getattr(params, k))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_submap_destroy(h)
            self._h = None

    @property
    def n_blocks(self) -> int:
        return int(_load().orc_n_blocks(self._h))

    def integrate(self, depth, K, T_world_cam):
        d = np.ascontiguousarray(depth, np.float32)
        k = np.ascontiguousarray(K, np.float32)
        st = np.zeros(4, np.int64)
        rc = _load().orc_integrate(self._h, _p(d, _fp), d.shape[0], d.shape[1], _p(k, _fp),
                                   _p(_mat(T_world_cam), _dp), _p(st, _i64p))
        if rc != OK:
            raise ValueError("oracle integrate: status %d" % rc)
        # n_valid: valid voxels (projection) or contributions (raycasting);
        # n_voxels: voxels updated
        return {"n_new": int(st[0]), "n_touched": int(st[1]), "n_valid": int(st[2]), "n_voxels": int(st[3])}

    def update_esdf(self):
        _load().orc_update_esdf(self._h)

    def fragile_voxels(self) -> np.ndarray:
        """Voxels (n, 3), with repeats, next to the fragile steps of every
        raycast walk so far: where another faithful rounding of the crossing
        parameters could visit a different voxel (see ray_walk32)."""
        L = _load()
        n = int(L.orc_fragile_voxels(self._h, None, 0))
        out = np.zeros((max(n, 1), 3), np.int64)
        L.orc_fragile_voxels(self._h, _p(out, _i64p), n)
        return out[:n]

    def esdf_wavefront(self) -> dict:
        """One incremental (wavefront) ESDF update; returns its round count,
        block-rounds processed and blocks queued first."""
        st = np.zeros(3, np.int64)
        _load().orc_esdf_wavefront(self._h, _p(st, _i64p))
        return {"rounds": int(st[0]), "block_rounds": int(st[1]), "dirty": int(st[2])}

    def export(self) -> dict:
        n = self.n_blocks
        keys = np.zeros(n, np.uint64)
        D = np.zeros(n * 512, np.float64)
        W = np.zeros(n * 512, np.float64)
        phi = np.zeros(n * 512, np.float64)
        ksq = np.zeros(n * 512, np.int32)
        _load().orc_export(self._h, _p(keys, _u64p), _p(D, _dp), _p(W, _dp), _p(phi, _dp), _p(ksq, _i32p))
        return {"keys": keys, "D": D.reshape(n, 512), "W": W.reshape(n, 512),
                "phi": phi.reshape(n, 512), "ksq": ksq.reshape(n, 512)}

    def import_blocks(self, keys, D, W):
        keys = np.ascontiguousarray(keys, np.uint64)
        D = np.ascontiguousarray(D, np.float64).reshape(-1)
        W = np.ascontiguousarray(W, np.float64).reshape(-1)
        _load().orc_import(self._h, len(keys), _p(keys, _u64p), _p(D, _dp), _p(W, _dp))

    def iso_points(self) -> np.ndarray:
        L = _load()
        n = int(L.orc_iso_points(self._h, None, 0))
        dt = np.float64 if self.params.fp64 else np.float32
        out = np.zeros((max(n, 1), 3), dt)
        L.orc_iso_points(self._h, out.ctypes.data_as(_vp), n)
        return out[:n]


def _pts(A: Submap, pts):
    dt = np.float64 if A.params.fp64 else np.float32
    return np.ascontiguousarray(np.asarray(pts, dt).reshape(-1, 3))


def normal_eq(A: Submap, pts, T):
    """(H 6x6, b 6, c, n) at pose T (points of B in B coordinates)."""
    p = _pts(A, pts)
    out = np.zeros(29)
    _load().orc_normal_eq(A._h, p.ctypes.data_as(_vp), len(p), _p(_mat(T), _dp), _p(out, _dp))
    H = np.zeros((6, 6))
    m = 0
    for a in range(6):
        for b in range(a, 6):
            H[a, b] = H[b, a] = out[m]
            m += 1
    return H, out[21:27].copy(), float(out[27]), int(out[28]), out


def align(A: Submap, pts, T_init):
    p = _pts(A, pts)
    T = np.zeros(16)
    cost = np.zeros(1)
    info = np.zeros(3, np.int64)
    st = _load().orc_align_points(A._h, p.ctypes.data_as(_vp), len(p), _p(_mat(T_init), _dp), _p(T, _dp),
                                  _p(cost, _dp), _p(info, _i64p))
    return {"T": T.reshape(4, 4), "cost": float(cost[0]), "status": int(st), "iters": int(info[0]),
            "n": int(info[1]), "solves": int(info[2])}


def align_multistart(A: Submap, pts, T_init, n_starts=8):
    p = _pts(A, pts)
    T = np.zeros(16)
    cost = np.zeros(1)
    info = np.zeros(3, np.int64)
    best = ctypes.c_int(-1)
    starts = np.zeros(16 * n_starts)
    st = _load().orc_align_multistart(A._h, p.ctypes.data_as(_vp), len(p), _p(_mat(T_init), _dp), n_starts,
                                      _p(T, _dp), _p(cost, _dp), _p(info, _i64p), ctypes.byref(best),
                                      _p(starts, _dp))
    return {"T": T.reshape(4, 4), "cost": float(cost[0]), "status": int(st), "iters": int(info[0]),
            "n": int(info[1]), "solves": int(info[2]), "best": best.value,
            "starts": starts.reshape(n_starts, 4, 4)}


def ray_walk32(o, u, s0, s1, vs, fragile=False):
    """Voxel indices (n, 3) crossed by the binary32 ray segment o + s u,
    s in [s0, s1], in walk order (Amanatides-Woo with correctly rounded
    crossing parameters).  With fragile=True also the voxels (m, 3) that
    another faithful rounding of the crossing parameters could visit
    instead: returns (walk, fragile_voxels)."""
    o = np.ascontiguousarray(o, np.float32)
    u = np.ascontiguousarray(u, np.float32)
    s0, s1, vs = np.float32(s0), np.float32(s1), np.float32(vs)
    cap = 3 * int(np.ceil(np.float32(s1 - s0) / vs)) + 6
    out = np.zeros((cap, 3), np.int64)
    if not fragile:
        n = _load().orc_ray_walk32(_p(o, _fp), _p(u, _fp), s0, s1, vs, _p(out, _i64p), cap)
        return out[:n]
    fr = np.zeros((7 * cap, 3), np.int64)
    nf = np.zeros(1, np.int64)
    n = _load().orc_ray_walk32_fragile(_p(o, _fp), _p(u, _fp), s0, s1, vs, _p(out, _i64p), cap, _p(fr, _i64p),
                                       7 * cap, _p(nf, _i64p))
    return out[:n], fr[:int(nf[0])]


def se3_exp(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, np.float64)
    E = np.zeros(16)
    _load().orc_se3_exp(_p(x, _dp), _p(E, _dp))
    return E.reshape(4, 4)


def solve6(ne29, mu=None):
    """The step x of H x = -b, or of (H + mu diag(H)) x = -b when mu is given
    (Levenberg-Marquardt); None when the matrix is not positive definite."""
    ne = np.ascontiguousarray(ne29, np.float64)
    x = np.zeros(6)
    if mu is None:
        rc = _load().orc_solve6(_p(ne, _dp), _p(x, _dp))
    else:
        rc = _load().orc_solve6_damped(_p(ne, _dp), float(mu), _p(x, _dp))
    return (x if rc == 0 else None)


def solve_xyz_yaw(ne29, mu=0.0):
    """The 4-DoF step (rho, 0, 0, theta_z) with damping mu."""
    ne = np.ascontiguousarray(ne29, np.float64)
    x = np.zeros(6)
    rc = _load().orc_solve_xyz_yaw_damped(_p(ne, _dp), float(mu), _p(x, _dp))
    return (x if rc == 0 else None)


def mix64(k: int) -> int:
    return int(_load().orc_mix64(ctypes.c_uint64(k & 0xFFFFFFFFFFFFFFFF)))


def f2h(x: float) -> int:
    return int(_load().orc_f2h(ctypes.c_float(x)))


def h2f(h: int) -> float:
    return float(_load().orc_h2f(ctypes.c_uint16(h)))


def pose_cam_sub(T_world_cam, T_world_sub) -> np.ndarray:
    out = np.zeros(16)
    _load().orc_pose_cam_sub(_p(_mat(T_world_cam), _dp), _p(_mat(T_world_sub), _dp), _p(out, _dp))
    return out.reshape(4, 4)


def pack_key(bx, by, bz) -> np.ndarray:
    """Packed block key ((bx + 2^20) << 42) | ((by + 2^20) << 21) | (bz + 2^20)."""
    off = np.int64(1 << 20)
    bx, by, bz = (np.asarray(v, np.int64) + off for v in (bx, by, bz))
    return ((bx.astype(np.uint64) << np.uint64(42)) | (by.astype(np.uint64) << np.uint64(21))
            | bz.astype(np.uint64))


def unpack_key(k) -> np.ndarray:
    k = np.asarray(k, np.uint64)
    m = np.uint64(0x1FFFFF)
    off = 1 << 20
    return np.stack([((k >> np.uint64(42)) & m).astype(np.int64) - off,
                     ((k >> np.uint64(21)) & m).astype(np.int64) - off,
                     (k & m).astype(np.int64) - off], axis=-1)


def voxel_coords(keys) -> np.ndarray:
    """(n, 512, 3) integer voxel indices of every voxel of the given blocks."""
    b = unpack_key(keys)
    l = np.arange(512)
    off = np.stack([l & 7, (l >> 3) & 7, l >> 6], axis=1)
    return 8 * b[:, None, :] + off[None, :, :]


def home_bucket(keys, table_cap: int) -> np.ndarray:
    return np.array([mix64(int(k)) & (table_cap - 1) for k in np.asarray(keys, np.uint64)], np.int64)


class HashTable:
    """Open-addressing table with linear probing (Sec. III-B; the stress test
    of Sec. IV): keys inserted one after another, sequentially."""

    EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)

    def __init__(self, capacity: int):
        if capacity < 2 or capacity & (capacity - 1):
            raise ValueError("capacity must be a power of two >= 2")
        self.keys = np.full(capacity, self.EMPTY, np.uint64)
        self.vals = np.zeros(capacity, np.uint32)
        self.stats = np.zeros(3, np.int64)  # max probe, probe sum, failed inserts

    def insert(self, keys, val_base: int = 0) -> np.ndarray:
        """Inserts keys in order; returns each key's probe length (-1: table full)."""
        k = np.ascontiguousarray(keys, np.uint64)
        probe = np.zeros(len(k), np.int64)
        _load().orc_hash_insert(_p(self.keys, _u64p), self.vals.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                len(self.keys), _p(k, _u64p), len(k), int(val_base) & 0xFFFFFFFF, _p(probe, _i64p),
                                _p(self.stats, _i64p))
        return probe

    def occupied(self) -> np.ndarray:
        return self.keys != self.EMPTY


# ------------------------------------------------------------ learned proposal

#: The proposal network's layers (cin, cout, din, dout, stride); 64 features.
NET_LAYERS = [(4, 16, 32, 32, 1), (16, 32, 32, 16, 2), (32, 64, 16, 8, 2), (64, 64, 8, 4, 2)]
NET_FEAT = 64


def _conv_array(layers):
    arr = (_Conv * len(layers))()
    for i, (ci, co, di, do, st) in enumerate(layers):
        arr[i] = _Conv(ci, co, di, do, st)
    return arr


def net_num_params(layers=NET_LAYERS, feat=NET_FEAT) -> int:
    return int(_load().orc_net_num_params(_conv_array(layers), len(layers), feat))


def net_forward(params, x, layers=NET_LAYERS, feat=NET_FEAT, bf16=True) -> np.ndarray:
    """Outputs (n, 5) of the network for inputs x (n, D, D, D, cin) NDHWC."""
    p = np.ascontiguousarray(params, np.float32)
    xx = np.ascontiguousarray(x, np.float32)
    n = xx.shape[0]
    out = np.zeros((n, 5))
    _load().orc_net_forward(_conv_array(layers), len(layers), feat, _p(p, _fp), _p(xx, _fp), n, int(bf16), _p(out, _dp))
    return out


def net_loss_grad(params, x, y, trans_scale, layers=NET_LAYERS, feat=NET_FEAT, bf16=True):
    """(loss, gradient) of the proposal loss, by backpropagation."""
    p = np.ascontiguousarray(params, np.float32)
    xx = np.ascontiguousarray(x, np.float32)
    yy = np.ascontiguousarray(y, np.float32)
    n = xx.shape[0]
    g = np.zeros(len(p))
    loss = np.zeros(1)
    _load().orc_net_loss_grad(_conv_array(layers), len(layers), feat, _p(p, _fp), _p(xx, _fp), _p(yy, _fp), n,
                              int(bf16), float(trans_scale), _p(g, _dp), _p(loss, _dp))
    return float(loss[0]), g


def summary(s: Submap, T_submap_grid, cell) -> np.ndarray:
    """(32^3, 2) coarse ESDF summary (clamped phi / d_max, mask), binary64."""
    out = np.zeros((32768, 2))
    _load().orc_summary(s._h, s.params.vs, s.params.d_max, _p(_mat(T_submap_grid), _dp), float(cell), _p(out, _dp))
    return out


def bf16_round(x: float) -> float:
    return float(_load().orc_bf16_round(ctypes.c_float(x)))
