"""Python binding of libcovox.so (include/covox.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch provides device memory
(depth frames are torch CUDA/HIP tensors) and the stream the library
enqueues its work on.  If the library has not been built this module raises
at import time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import weakref
import math
import os

import numpy as np
import torch  # loads the HIP runtime the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcovox.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcovox.so is not built: run __graft_entry__.build() (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EPOOL_FULL, ETABLE_FULL, EHIP, EDEGENERATE, NOT_CONVERGED = 0, -1, -2, -3, -4, -5, 1
FP32, FP16 = 0, 1
WEIGHT_CONSTANT, WEIGHT_INV_DEPTH2 = 0, 1
PROJECTIVE, RAYCAST = 0, 1
ESDF_EXACT, ESDF_WAVEFRONT = 0, 1
GAUSS_NEWTON, LEVENBERG_MARQUARDT = 0, 1
NET_NOALLOC_MAX_PAIRS = 8  # COVOX_NET_NOALLOC_MAX_PAIRS
KERNELS = ["probe", "scan", "integrate", "esdf_page", "esdf_sites", "edt_x", "edt_y", "edt_z", "iso", "align",
           "summary", "net", "ray_mark", "ray_accum", "ray_apply", "pgo", "wavefront", "hash"]


class CovoxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_lib.covox_status_string(code).decode(), msg))
        self.code = code


class covox_params(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_double), ("trunc_vox", ctypes.c_int32), ("max_range", ctypes.c_double),
                ("d_max", ctypes.c_double), ("w_reg", ctypes.c_double), ("block_capacity", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("n_min", ctypes.c_int32),
                ("tol_rho", ctypes.c_double), ("tol_theta", ctypes.c_double), ("align_dof", ctypes.c_int32),
                ("weight_mode", ctypes.c_int32), ("integrator", ctypes.c_int32), ("ray_carve", ctypes.c_int32),
                ("esdf_mode", ctypes.c_int32), ("align_solver", ctypes.c_int32)]


class covox_align_stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_used", ctypes.c_int64), ("iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("best_start", ctypes.c_int32), ("solves", ctypes.c_int32)]


class covox_pair(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("T_init_A_B", ctypes.c_double * 16)]


class covox_submap_info(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("block_capacity", ctypes.c_int64), ("table_capacity", ctypes.c_int64),
                ("n_updates", ctypes.c_int64), ("bbox_min", ctypes.c_int32 * 3), ("bbox_max", ctypes.c_int32 * 3),
                ("precision", ctypes.c_int32), ("status", ctypes.c_int32)]


class covox_train_cfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("trans_scale", ctypes.c_double), ("cell", ctypes.c_double), ("trans_xy", ctypes.c_double),
                ("trans_z", ctypes.c_double), ("yaw", ctypes.c_double), ("tilt", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class covox_tuning(ctypes.Structure):
    _fields_ = [("edt_y_env_min_cols", ctypes.c_int64), ("edt_z_env_min_cols", ctypes.c_int64),
                ("align_threads", ctypes.c_int64), ("align_points_per_step", ctypes.c_int64),
                ("edt_pipe_max_workgroups", ctypes.c_int64), ("edt_col_seg", ctypes.c_int64),
                ("esdf_full_recompute", ctypes.c_int64), ("mapping_xcd_order", ctypes.c_int64)]


class covox_pose_factor(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2),
                ("z", ctypes.c_double * 4), ("sigma", ctypes.c_double * 4)]


class covox_pgo_cfg(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("cg_max_iter", ctypes.c_int32), ("sigma_reg", ctypes.c_double),
                ("lambda0", ctypes.c_double), ("tol_step", ctypes.c_double), ("cg_tol", ctypes.c_double)]


class covox_pgo_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("accepted", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("cg_iterations", ctypes.c_int32), ("cost_init", ctypes.c_double), ("cost_final", ctypes.c_double)]


class covox_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(KERNELS)), ("launches", ctypes.c_int64 * len(KERNELS))]


class covox_summary_req(ctypes.Structure):
    _fields_ = [("s", ctypes.c_void_p), ("T_submap_grid", ctypes.c_double * 16), ("cell", ctypes.c_double),
                ("out_dev", ctypes.c_void_p), ("channel", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp, _dp, _fp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
_sig = {
    "covox_default_params": (None, [ctypes.POINTER(covox_params)]),
    "covox_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(covox_params)]),
    "covox_destroy": (None, [_vp]),
    "covox_set_stream": (ctypes.c_int, [_vp, _vp]),
    "covox_set_params": (ctypes.c_int, [_vp, ctypes.POINTER(covox_params)]),
    "covox_sync": (ctypes.c_int, [_vp]),
    "covox_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "covox_last_error": (ctypes.c_char_p, [_vp]),
    "covox_submap_create": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(_vp)]),
    "covox_submap_destroy": (None, [_vp]),
    "covox_submap_reset": (ctypes.c_int, [_vp, _vp]),
    "covox_integrate_depth": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _fp, _dp]),
    "covox_integrate_depth_batch": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   _fp, _dp]),
    "covox_update_esdf": (ctypes.c_int, [_vp, _vp]),
    "covox_update_esdf_batch": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int32]),
    "covox_map_sequence": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _fp, _dp,
                                          ctypes.c_int32]),
    "covox_align_submaps": (ctypes.c_int, [_vp, _vp, _vp, _dp, _dp, _dp, ctypes.POINTER(covox_align_stats)]),
    "covox_align_multistart": (ctypes.c_int, [_vp, _vp, _vp, _dp, ctypes.c_int32, _dp, _dp,
                                              ctypes.POINTER(covox_align_stats)]),
    "covox_align_batch": (ctypes.c_int, [_vp, ctypes.POINTER(covox_pair), ctypes.c_int32, ctypes.c_int32, _dp, _dp,
                                         ctypes.POINTER(covox_align_stats)]),
    "covox_align_prepare": (ctypes.c_int, [_vp, ctypes.POINTER(covox_pair), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(_vp)]),
    "covox_align_launch": (ctypes.c_int, [_vp, _vp]),
    "covox_align_collect": (ctypes.c_int, [_vp, _vp, _dp, _dp, ctypes.POINTER(covox_align_stats)]),
    "covox_align_set_destroy": (None, [_vp]),
    "covox_submap_info_get": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(covox_submap_info)]),
    "covox_export_blocks": (ctypes.c_int64, [_vp, _vp, _vp, _vp, _fp, _fp, _fp, ctypes.c_int64]),
    "covox_export_points": (ctypes.c_int64, [_vp, _vp, _fp, ctypes.c_int64]),
    "covox_normal_equations": (ctypes.c_int, [_vp, _vp, _vp, _dp, _dp]),
    "covox_summaries": (ctypes.c_int, [_vp, ctypes.POINTER(covox_summary_req), ctypes.c_int32]),
    "covox_net_create": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "covox_net_destroy": (None, [_vp]),
    "covox_net_num_params": (ctypes.c_int64, [_vp]),
    "covox_net_get_params": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
    "covox_net_set_params": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
    "covox_net_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp]),
    "covox_net_forward_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp]),
    "covox_net_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _fp]),
    "covox_net_gradients": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, _fp, _fp]),
    "covox_align_learned": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(covox_pair), ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _dp, _dp,
                                           ctypes.POINTER(covox_align_stats)]),
    "covox_propose": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(covox_pair), ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int32, _dp]),
    "covox_train_proposal": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(covox_train_cfg), ctypes.POINTER(covox_pair),
                                            ctypes.c_int32, _fp]),
    "covox_graph_begin": (ctypes.c_int, [_vp]),
    "covox_graph_end": (ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    "covox_graph_launch": (ctypes.c_int, [_vp]),
    "covox_graph_destroy": (None, [_vp]),
    "covox_default_tuning": (None, [ctypes.POINTER(covox_tuning)]),
    "covox_tuning_get": (ctypes.c_int, [_vp, ctypes.POINTER(covox_tuning)]),
    "covox_tuning_set": (ctypes.c_int, [_vp, ctypes.POINTER(covox_tuning)]),
    "covox_autotune_esdf": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(covox_tuning)]),
    "covox_autotune_align": (ctypes.c_int, [_vp, ctypes.POINTER(covox_pair), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(covox_tuning)]),
    "covox_default_pgo_cfg": (None, [ctypes.POINTER(covox_pgo_cfg)]),
    "covox_pgo_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int32, _dp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_int32, ctypes.POINTER(covox_pose_factor), ctypes.c_int32,
                                       ctypes.POINTER(covox_pgo_cfg), ctypes.POINTER(covox_pgo_stats)]),
    "covox_hash_insert": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int64, _vp, ctypes.c_int64,
                                         ctypes.c_uint32, _vp]),
    "covox_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "covox_timing_get": (ctypes.c_int, [_vp, ctypes.POINTER(covox_timing)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _mat(T) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(T, np.float64).reshape(16))


def _p(a, t):
    return a.ctypes.data_as(t)


def default_params(**kw) -> covox_params:
    p = covox_params()
    _lib.covox_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = FP16 if v.lower() in ("fp16", "half") else FP32
        setattr(p, k, v)
    return p


class Submap:
    def __init__(self, ctx: "Context", handle):
        self.ctx, self.handle = ctx, handle

    def destroy(self):
        if self.handle:
            _lib.covox_submap_destroy(self.handle)
            self.handle = None


class Context:
    """A covox context bound to the current device and a torch stream."""

    def __init__(self, params: covox_params | None = None, stream: torch.cuda.Stream | None = None, **kw):
        self.params = params if params is not None else default_params(**kw)
        h = _vp()
        rc = _lib.covox_create(ctypes.byref(h), ctypes.byref(self.params))
        if rc != OK:
            raise CovoxError(rc, "covox_create")
        self.handle = h
        self.set_stream(stream if stream is not None else torch.cuda.current_stream())
        self._subs = []
        self._nets = weakref.WeakSet()

    # -- plumbing
    def _check(self, rc, what, ok=(OK,)):
        if rc not in ok:
            raise CovoxError(rc, "%s: %s" % (what, _lib.covox_last_error(self.handle).decode()))
        return rc

    def set_params(self, **kw):
        """Changes non-storage parameters (w_reg, max_iter, n_min, tol_rho,
        tol_theta, align_dof, weight_mode, integrator, ray_carve, esdf_mode,
        align_solver)."""
        p = covox_params.from_buffer_copy(self.params)
        for k, v in kw.items():
            setattr(p, k, v)
        self._check(_lib.covox_set_params(self.handle, ctypes.byref(p)), "set_params")
        self.params = p

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        self._check(_lib.covox_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)), "set_stream")

    def close(self):
        if getattr(self, "handle", None):
            for g in getattr(self, "_graphs", []):
                g.close()
            for s in self._subs:
                s.handle = None
            for n in list(getattr(self, "_nets", ())):
                n.close()
            _lib.covox_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        self._check(_lib.covox_sync(self.handle), "sync")

    # -- submaps
    def submap_create(self, T_world_submap=None) -> Submap:
        T = _mat(np.eye(4) if T_world_submap is None else T_world_submap)
        h = _vp()
        self._check(_lib.covox_submap_create(self.handle, _p(T, _dp), ctypes.byref(h)), "submap_create")
        s = Submap(self, h)
        self._subs.append(s)
        return s

    def submap_reset(self, s: Submap):
        self._check(_lib.covox_submap_reset(self.handle, s.handle), "submap_reset")

    def submap_info(self, s: Submap) -> dict:
        info = covox_submap_info()
        self._check(_lib.covox_submap_info_get(self.handle, s.handle, ctypes.byref(info)), "submap_info")
        return {"n_blocks": info.n_blocks, "block_capacity": info.block_capacity,
                "table_capacity": info.table_capacity, "n_updates": info.n_updates,
                "bbox_min": tuple(info.bbox_min), "bbox_max": tuple(info.bbox_max), "precision": info.precision,
                "status": info.status}

    # -- hot path
    @staticmethod
    def _depth_ptr(depth: torch.Tensor, ndim: int):
        if not (isinstance(depth, torch.Tensor) and depth.is_cuda and depth.dtype == torch.float32
                and depth.dim() == ndim and depth.is_contiguous()):
            raise ValueError("depth must be a contiguous float32 device tensor with %d dims" % ndim)
        return ctypes.c_void_p(depth.data_ptr())

    def integrate_depth(self, s: Submap, depth: torch.Tensor, K, T_world_cam):
        k = np.ascontiguousarray(K, np.float32)
        T = _mat(T_world_cam)
        H, W = depth.shape
        return self._check(_lib.covox_integrate_depth(self.handle, s.handle, self._depth_ptr(depth, 2), H, W,
                                                      _p(k, _fp), _p(T, _dp)), "integrate_depth")

    def integrate_depth_batch(self, s: Submap, depths: torch.Tensor, K, T_world_cam):
        k = np.ascontiguousarray(K, np.float32)
        T = np.ascontiguousarray(np.asarray(T_world_cam, np.float64).reshape(-1, 16))
        F, H, W = depths.shape
        assert len(T) == F
        return self._check(_lib.covox_integrate_depth_batch(self.handle, s.handle, self._depth_ptr(depths, 3), F, H,
                                                            W, _p(k, _fp), _p(T, _dp)), "integrate_depth_batch")

    def map_sequence(self, s: Submap, depths: torch.Tensor, K, T_world_cam, esdf_every=1):
        k = np.ascontiguousarray(K, np.float32)
        T = np.ascontiguousarray(np.asarray(T_world_cam, np.float64).reshape(-1, 16))
        F, H, W = depths.shape
        assert len(T) == F
        return self._check(_lib.covox_map_sequence(self.handle, s.handle, self._depth_ptr(depths, 3), F, H, W,
                                                   _p(k, _fp), _p(T, _dp), esdf_every), "map_sequence")

    def update_esdf_batch(self, subs):
        arr = (_vp * max(len(subs), 1))(*[s.handle for s in subs])
        return self._check(_lib.covox_update_esdf_batch(self.handle, arr, len(subs)), "update_esdf_batch")

    def update_esdf(self, s: Submap):
        return self._check(_lib.covox_update_esdf(self.handle, s.handle), "update_esdf")

    def align_submaps(self, A: Submap, B: Submap, T_init):
        T0 = _mat(T_init)
        T = np.zeros(16)
        cost = ctypes.c_double()
        st = covox_align_stats()
        rc = _lib.covox_align_submaps(self.handle, A.handle, B.handle, _p(T0, _dp), _p(T, _dp), ctypes.byref(cost),
                                      ctypes.byref(st))
        self._check(rc, "align_submaps", ok=(OK, NOT_CONVERGED, EDEGENERATE))
        return T.reshape(4, 4), cost.value, _stats(st)

    def align_multistart(self, A: Submap, B: Submap, T_init, n_starts=8):
        T0 = _mat(T_init)
        T = np.zeros(16)
        cost = ctypes.c_double()
        st = covox_align_stats()
        rc = _lib.covox_align_multistart(self.handle, A.handle, B.handle, _p(T0, _dp), n_starts, _p(T, _dp),
                                         ctypes.byref(cost), ctypes.byref(st))
        self._check(rc, "align_multistart", ok=(OK, NOT_CONVERGED, EDEGENERATE))
        return T.reshape(4, 4), cost.value, _stats(st)

    def align_batch(self, pairs, n_starts=1):
        n = len(pairs)
        arr = (covox_pair * max(n, 1))()
        for i, (A, B, T0) in enumerate(pairs):
            arr[i].A = A.handle
            arr[i].B = B.handle
            arr[i].T_init_A_B[:] = list(_mat(T0))
        T = np.zeros(16 * max(n, 1))
        cost = np.zeros(max(n, 1))
        st = (covox_align_stats * max(n, 1))()
        self._check(_lib.covox_align_batch(self.handle, arr, n, n_starts, _p(T, _dp), _p(cost, _dp), st),
                    "align_batch")
        return T.reshape(-1, 4, 4)[:n], cost[:n], [_stats(st[i]) for i in range(n)]

    def align_prepare(self, pairs, n_starts=1) -> "AlignSet":
        """The problems of align_batch(pairs, n_starts) on the device, for
        repeated or graph-captured launches (AlignSet.launch / collect)."""
        n = len(pairs)
        arr = (covox_pair * max(n, 1))()
        for i, (A, B, T0) in enumerate(pairs):
            arr[i].A = A.handle
            arr[i].B = B.handle
            arr[i].T_init_A_B[:] = list(_mat(T0))
        h = _vp()
        self._check(_lib.covox_align_prepare(self.handle, arr, n, n_starts, ctypes.byref(h)), "align_prepare")
        return AlignSet(self, h, n)

    def normal_equations(self, A: Submap, B: Submap, T) -> np.ndarray:
        out = np.zeros(29)
        Tm = _mat(T)
        self._check(_lib.covox_normal_equations(self.handle, A.handle, B.handle, _p(Tm, _dp), _p(out, _dp)),
                    "normal_equations")
        return out

    # -- pose graph (Eq. 1)
    def pgo_solve(self, subs, x0, reg_pairs, factors, **cfg):
        """Submap pose-graph optimisation.  subs: submaps; x0: (n, 4) poses
        (t, yaw) of their T_world_submap estimates (x0[0] is held fixed);
        reg_pairs: (i, j) pairs (ESDF of i, registration points of j);
        factors: dicts with i, j, z (4), sigma (4); cfg: max_iter,
        cg_max_iter, sigma_reg, lambda0, tol_step, cg_tol.  Returns the
        poses and a stats dict."""
        c = covox_pgo_cfg()
        _lib.covox_default_pgo_cfg(ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        n = len(subs)
        hs = (_vp * n)(*[sm.handle for sm in subs])
        x = np.ascontiguousarray(np.asarray(x0, np.float64).reshape(n, 4)).copy()
        rp = np.ascontiguousarray(np.asarray(reg_pairs, np.int32).reshape(-1, 2))
        fa = (covox_pose_factor * max(len(factors), 1))()
        for k, f in enumerate(factors):
            fa[k].i, fa[k].j = int(f["i"]), int(f["j"])
            for a in range(4):
                fa[k].z[a] = float(f["z"][a])
                fa[k].sigma[a] = float(f["sigma"][a])
        st = covox_pgo_stats()
        self._check(_lib.covox_pgo_solve(self.handle, hs, n, _p(x, _dp), rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         len(rp), fa, len(factors), ctypes.byref(c), ctypes.byref(st)), "pgo_solve")
        return x, {"iterations": st.iterations, "accepted": st.accepted, "converged": bool(st.converged),
                   "cg_iterations": st.cg_iterations, "cost_init": st.cost_init, "cost_final": st.cost_final}

    # -- hash-table stress test (Sec. IV)
    def hash_insert(self, table_keys, table_vals, n_present, keys, stats, val_base=0):
        """Inserts the device keys (int64 or uint64 tensor, distinct, absent,
        none equal to all ones) into the caller's table (table_keys:
        capacity 64-bit slots, empty = all ones; table_vals: capacity 32-bit
        slots).  stats: int64 device tensor of 3, raised by the call (max
        probe, probe sum, failures).  Asynchronous on the context stream."""
        def dev(t, bits, what):
            if not (t.is_cuda and t.is_contiguous() and t.element_size() * 8 == bits and not t.is_floating_point()):
                raise ValueError("%s must be a contiguous %d-bit integer device tensor" % (what, bits))
            return ctypes.c_void_p(t.data_ptr())
        if table_vals.numel() != table_keys.numel():
            raise ValueError("table_vals must have one slot per table_keys slot")
        if stats.dtype != torch.int64 or stats.numel() < 3:
            raise ValueError("stats must be an int64 device tensor of at least 3 entries")
        n = keys.numel()
        return self._check(_lib.covox_hash_insert(self.handle, dev(table_keys, 64, "table_keys"),
                                                  dev(table_vals, 32, "table_vals"), table_keys.numel(), int(n_present),
                                                  dev(keys, 64, "keys") if n else None, n, int(val_base) & 0xFFFFFFFF,
                                                  dev(stats, 64, "stats")), "hash_insert")

    # -- learned proposal
    def summaries(self, reqs):
        """reqs: list of (submap, T_submap_grid, cell, out tensor (32^3 x 4 floats, device), channel)."""
        arr = (covox_summary_req * max(len(reqs), 1))()
        for i, (sm, T, cell, out, ch) in enumerate(reqs):
            if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() == 32768 * 4):
                raise ValueError("summary output must be a contiguous float32 device tensor of 32^3 x 4")
            arr[i].s = sm.handle
            arr[i].T_submap_grid[:] = list(_mat(T))
            arr[i].cell = cell
            arr[i].out_dev = out.data_ptr()
            arr[i].channel = ch
        self._check(_lib.covox_summaries(self.handle, arr, len(reqs)), "summaries")

    def align_learned(self, net: "Net", pairs, cell, cost_thr, n_starts=8, n_rot=1):
        n = len(pairs)
        arr = self._pairs(pairs)
        T = np.zeros(16 * max(n, 1))
        cost = np.zeros(max(n, 1))
        st = (covox_align_stats * max(n, 1))()
        self._check(_lib.covox_align_learned(self.handle, net.handle, arr, n, cell, cost_thr, n_rot, n_starts,
                                             _p(T, _dp), _p(cost, _dp), st), "align_learned")
        return T.reshape(-1, 4, 4)[:n], cost[:n], [_stats(st[i]) for i in range(n)]

    def propose(self, net: "Net", pairs, cell, n_rot=1):
        """The network's proposals for (A, B, T_init) pairs: n x 4 x 4, or
        n x n_rot x 4 x 4 with the prior also turned by 2 pi k / n_rot about
        the summary grid centre."""
        arr = self._pairs(pairs)
        n = len(pairs)
        T = np.zeros(16 * n_rot * max(n, 1))
        self._check(_lib.covox_propose(self.handle, net.handle, arr, n, cell, n_rot, _p(T, _dp)), "propose")
        T = T.reshape(-1, n_rot, 4, 4)[:n]
        return T[:, 0] if n_rot == 1 else T

    def train_proposal(self, net: "Net", pairs, steps, batch=64, lr=1e-3, trans_scale=3.0, cell=1.0, trans_xy=3.0,
                       trans_z=0.5, yaw=math.pi, tilt=math.radians(2.0), seed=5):
        """Trains `net` on re-framings of (A, B, T_gt) pairs; returns the
        per-step losses."""
        cfg = covox_train_cfg(steps, batch, lr, trans_scale, cell, trans_xy, trans_z, yaw, tilt, seed)
        arr = self._pairs(pairs)
        losses = np.zeros(max(steps, 1), np.float32)
        self._check(_lib.covox_train_proposal(self.handle, net.handle, ctypes.byref(cfg), arr, len(pairs),
                                              _p(losses, _fp)), "train_proposal")
        return losses[:steps]

    @staticmethod
    def _pairs(pairs):
        arr = (covox_pair * max(len(pairs), 1))()
        for i, (A, B, T0) in enumerate(pairs):
            arr[i].A = A.handle
            arr[i].B = B.handle
            arr[i].T_init_A_B[:] = list(_mat(T0))
        return arr

    # -- inspection
    def export_blocks(self, s: Submap) -> dict:
        n = self.submap_info(s)["n_blocks"]
        keys = np.zeros(max(n, 1), np.uint64)
        home = np.zeros(max(n, 1), np.uint32)
        D = np.zeros((max(n, 1), 512), np.float32)
        W = np.zeros((max(n, 1), 512), np.float32)
        phi = np.zeros((max(n, 1), 512), np.float32)
        got = _lib.covox_export_blocks(self.handle, s.handle, keys.ctypes.data_as(_vp), home.ctypes.data_as(_vp),
                                       _p(D, _fp), _p(W, _fp), _p(phi, _fp), n)
        if got < 0:
            self._check(int(got), "export_blocks")
        return {"keys": keys[:got], "home": home[:got], "D": D[:got], "W": W[:got], "phi": phi[:got]}

    def export_points(self, B: Submap) -> np.ndarray:
        n = _lib.covox_export_points(self.handle, B.handle, None, 0)
        if n < 0:
            self._check(int(n), "export_points")
        pts = np.zeros((max(n, 1), 3), np.float32)
        _lib.covox_export_points(self.handle, B.handle, _p(pts, _fp), n)
        return pts[:n]

    # -- graphs
    def graph_begin(self):
        """Starts capturing this context's asynchronous calls (see Graph)."""
        self._check(_lib.covox_graph_begin(self.handle), "graph_begin")

    def graph_end(self) -> "Graph":
        h = _vp()
        self._check(_lib.covox_graph_end(self.handle, ctypes.byref(h)), "graph_end")
        g = Graph(self, h)
        if not hasattr(self, "_graphs"):
            self._graphs = []
        self._graphs.append(g)
        return g

    # -- tuning
    @staticmethod
    def _tuning_dict(t) -> dict:
        return {"edt_y_env_min_cols": t.edt_y_env_min_cols, "edt_z_env_min_cols": t.edt_z_env_min_cols,
                "align_threads": t.align_threads, "align_points_per_step": t.align_points_per_step,
                "edt_pipe_max_workgroups": t.edt_pipe_max_workgroups, "edt_col_seg": t.edt_col_seg,
                "esdf_full_recompute": t.esdf_full_recompute, "mapping_xcd_order": t.mapping_xcd_order}

    def tuning(self) -> dict:
        t = covox_tuning()
        self._check(_lib.covox_tuning_get(self.handle, ctypes.byref(t)), "tuning_get")
        return self._tuning_dict(t)

    def set_tuning(self, edt_y_env_min_cols=None, edt_z_env_min_cols=None, align_threads=None,
                   align_points_per_step=None, edt_pipe_max_workgroups=None, edt_col_seg=None,
                   esdf_full_recompute=None, mapping_xcd_order=None):
        t = covox_tuning()
        self._check(_lib.covox_tuning_get(self.handle, ctypes.byref(t)), "tuning_get")
        if edt_y_env_min_cols is not None:
            t.edt_y_env_min_cols = edt_y_env_min_cols
        if edt_z_env_min_cols is not None:
            t.edt_z_env_min_cols = edt_z_env_min_cols
        if align_threads is not None:
            t.align_threads = align_threads
        if align_points_per_step is not None:
            t.align_points_per_step = align_points_per_step
        if edt_pipe_max_workgroups is not None:
            t.edt_pipe_max_workgroups = edt_pipe_max_workgroups
        if edt_col_seg is not None:
            t.edt_col_seg = edt_col_seg
        if esdf_full_recompute is not None:
            t.esdf_full_recompute = int(esdf_full_recompute)
        if mapping_xcd_order is not None:
            t.mapping_xcd_order = int(mapping_xcd_order)
        self._check(_lib.covox_tuning_set(self.handle, ctypes.byref(t)), "tuning_set")

    def autotune_esdf(self, subs) -> dict:
        arr = (_vp * max(len(subs), 1))(*[s.handle for s in subs])
        t = covox_tuning()
        self._check(_lib.covox_autotune_esdf(self.handle, arr, len(subs), ctypes.byref(t)), "autotune_esdf")
        return self._tuning_dict(t)

    def autotune_align(self, pairs, n_starts=8) -> dict:
        t = covox_tuning()
        self._check(_lib.covox_autotune_align(self.handle, self._pairs(pairs), len(pairs), n_starts, ctypes.byref(t)),
                    "autotune_align")
        return self._tuning_dict(t)

    # -- timing
    def timing_enable(self, kinds=None):
        """Time the given kernel kinds (names from KERNELS; None = all, [] = off)."""
        mask = -1 if kinds is None else sum(1 << KERNELS.index(k) for k in kinds)
        self._check(_lib.covox_timing_enable(self.handle, mask), "timing_enable")

    def timing_get(self) -> dict:
        t = covox_timing()
        self._check(_lib.covox_timing_get(self.handle, ctypes.byref(t)), "timing_get")
        return {k: (t.ms[i], t.launches[i]) for i, k in enumerate(KERNELS)}


class Graph:
    """A captured sequence of calls, replayed by launch()."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    def launch(self):
        self.ctx._check(_lib.covox_graph_launch(self.handle), "graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            _lib.covox_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AlignSet:
    """Alignment problems prepared on the device: launch() enqueues the
    alignment (also inside a graph capture), collect() returns what
    align_batch returns."""

    def __init__(self, ctx: Context, handle, n: int):
        self.ctx = ctx
        self.handle = handle
        self.n = n

    def launch(self):
        self.ctx._check(_lib.covox_align_launch(self.ctx.handle, self.handle), "align_launch")

    def collect(self):
        n = self.n
        T = np.zeros(16 * n)
        cost = np.zeros(n)
        st = (covox_align_stats * n)()
        self.ctx._check(_lib.covox_align_collect(self.ctx.handle, self.handle, _p(T, _dp), _p(cost, _dp), st),
                        "align_collect")
        return T.reshape(-1, 4, 4), cost, [_stats(st[i]) for i in range(n)]

    def close(self):
        if getattr(self, "handle", None):
            _lib.covox_align_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stats(st: covox_align_stats) -> dict:
    return {"n_points": st.n_points, "n_used": st.n_used, "iterations": st.iterations, "status": st.status,
            "best_start": st.best_start, "solves": st.solves}


class Net:
    """The pose-proposal network of a context (weights on the device)."""

    def __init__(self, ctx: Context, seed: int = 1):
        self.ctx = ctx
        h = _vp()
        ctx._check(_lib.covox_net_create(ctx.handle, seed, ctypes.byref(h)), "net_create")
        self.handle = h
        ctx._nets.add(self)

    def close(self):
        if getattr(self, "handle", None):
            _lib.covox_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(_lib.covox_net_num_params(self.handle))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, np.float32)
        self.ctx._check(_lib.covox_net_get_params(self.handle, _p(out, _fp), len(out)), "net_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self.ctx._check(_lib.covox_net_set_params(self.handle, _p(p, _fp), len(p)), "net_set_params")

    @staticmethod
    def _x(x: torch.Tensor):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 5 and x.shape[1:] == (32, 32, 32, 4)):
            raise ValueError("network input must be a contiguous float32 device tensor (n, 32, 32, 32, 4)")
        return ctypes.c_void_p(x.data_ptr())

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        out = torch.empty((x.shape[0], 5), dtype=torch.float32, device=x.device)
        self.ctx._check(_lib.covox_net_forward(self.handle, self._x(x), x.shape[0], ctypes.c_void_p(out.data_ptr())),
                        "net_forward")
        return out

    def forward_noalloc(self, x: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """covox_net_forward_noalloc: the forward pass into the caller's
        `out` (n x 5 float32 on the device), n <= NET_NOALLOC_MAX_PAIRS,
        with no device allocation by the library."""
        self.ctx._check(_lib.covox_net_forward_noalloc(self.handle, self._x(x), x.shape[0],
                                                       ctypes.c_void_p(out.data_ptr())), "net_forward_noalloc")
        return out

    def train_step(self, x: torch.Tensor, y: torch.Tensor, lr: float, trans_scale: float = 3.0, want_loss=True):
        loss = ctypes.c_float(0.0)
        yy = y.contiguous()
        self.ctx._check(_lib.covox_net_train_step(self.handle, self._x(x), ctypes.c_void_p(yy.data_ptr()), x.shape[0],
                                                  lr, trans_scale, ctypes.byref(loss) if want_loss else None),
                        "net_train_step")
        return loss.value

    def gradients(self, x: torch.Tensor, y: torch.Tensor, trans_scale: float = 3.0):
        g = np.zeros(self.num_params, np.float32)
        loss = ctypes.c_float(0.0)
        yy = y.contiguous()
        self.ctx._check(_lib.covox_net_gradients(self.handle, self._x(x), ctypes.c_void_p(yy.data_ptr()), x.shape[0],
                                                 trans_scale, _p(g, _fp), ctypes.byref(loss)), "net_gradients")
        return loss.value, g
