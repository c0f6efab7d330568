"""The oracle's parallel loops (frustum-box validity, per-voxel updates, EDT
lines, final values) give bit-identical results for any thread count: every
item writes its own outputs and the per-thread lists are joined in the
sequential order."""
import numpy as np

import oracle as orc
import scenegen as sg


def _run(threads, w, n, **kw):
    orc.set_threads(threads)
    s = orc.Submap(orc.Params(vs=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max, **kw))
    for f in range(n):
        s.integrate(w.frame(f), w.cam.K, w.poses[f])
    s.update_esdf()
    return s.export()


def test_thread_count_does_not_change_results():
    w = sg.tiny(n_frames=4)
    try:
        for kw in ({}, {"fp64": True}, {"fp16": True}, {"weight_mode": 1}):
            a = _run(1, w, 4, **kw)
            b = _run(0, w, 4, **kw)
            c = _run(3, w, 4, **kw)
            for k in ("keys", "D", "W", "phi", "ksq"):
                assert np.array_equal(a[k], b[k], equal_nan=True), (kw, k)
                assert np.array_equal(a[k], c[k], equal_nan=True), (kw, k)
    finally:
        orc.set_threads(1)


def test_thread_count_room_frames():
    w = sg.room(n_frames=2)
    try:
        a = _run(1, w, 2)
        b = _run(0, w, 2)
    finally:
        orc.set_threads(1)
    for k in ("keys", "D", "W", "phi", "ksq"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
