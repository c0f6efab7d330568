"""GPU tests of covox_map_sequence with an ESDF update after every chunk of
frames: the update of one chunk runs on a second stream while the next
chunk is integrated.  The final TSDF, block table and ESDF equal bit for bit
those of the same calls issued one after another (integrate, then update),
for projection mapping, raycasting and FP16 storage; a captured sequence
replays to the same result; and the tiny room's ESDF still equals the
oracle's."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_21149_amd as cv
    return cv


def _same(a, b):
    for k in ("keys", "D", "W"):
        assert np.array_equal(a[k], b[k]), k
    pa, pb = a["phi"], b["phi"]
    assert np.array_equal(np.isnan(pa), np.isnan(pb))
    m = ~np.isnan(pa)
    assert np.array_equal(pa[m], pb[m])


def _in_order(ctx, s, dev, K, poses, every):
    """The calls map_sequence stands for, one after another on one stream."""
    F = dev.shape[0]
    for f0 in range(0, F, every):
        f1 = min(F, f0 + every)
        if f1 - f0 == 1:
            ctx.integrate_depth(s, dev[f0], K, poses[f0])
        else:
            ctx.integrate_depth_batch(s, dev[f0:f1], K, poses[f0:f1])
        ctx.update_esdf(s)


@pytest.fixture(scope="module")
def room90():
    """The first 90 frames of the room workload."""
    w = sg.room()
    return w, w.frames(0, 90)


CASES = [
    ("room", dict(), 1),
    ("room", dict(), 4),
    ("room", dict(precision="FP16"), 1),
    ("room", dict(integrator="RAYCAST"), 1),
    ("tiny", dict(integrator="RAYCAST", ray_carve=0), 3),
]


@pytest.mark.parametrize("scene,kw,every", CASES)
def test_pipelined_sequence_equals_calls_in_order(cv, room90, scene, kw, every):
    import torch
    if scene == "room":
        w, fr = room90
        poses = w.poses[:90]
        base = dict(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                    block_capacity=16384)
    else:
        w = sg.tiny()
        fr = w.frames()
        poses = w.poses
        base = dict(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)
    base.update({k: getattr(cv, v) if isinstance(v, str) else v for k, v in kw.items()})
    dev = torch.from_numpy(fr).cuda()
    print("case", scene, kw, every, flush=True)
    a = cv.Context(**base)
    sa = a.submap_create()
    a.map_sequence(sa, dev, w.cam.K, poses, esdf_every=every)
    got = a.export_blocks(sa)
    info_a = a.submap_info(sa)
    b = cv.Context(**base)
    sb = b.submap_create()
    _in_order(b, sb, dev, w.cam.K, poses, every)
    want = b.export_blocks(sb)
    info_b = b.submap_info(sb)
    _same(got, want)
    assert info_a["n_blocks"] == info_b["n_blocks"] and info_a["n_updates"] == info_b["n_updates"]
    # the same context again from a reset (the second stream now exists)
    a.submap_reset(sa)
    a.map_sequence(sa, dev, w.cam.K, poses, esdf_every=every)
    _same(a.export_blocks(sa), want)
    a.close()
    b.close()


@pytest.mark.parametrize("cap", [0, 3, 512])
def test_pass_grid_cap_does_not_change_the_result(cv, cap):
    """The EDT passes cover their work with a grid stride, so the workgroup
    cap of the pipelined passes (tuning edt_pipe_max_workgroups; 0 = none)
    leaves the result unchanged."""
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames()).cuda()
    base = dict(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)
    a = cv.Context(**base)
    a.set_tuning(edt_pipe_max_workgroups=cap)
    assert a.tuning()["edt_pipe_max_workgroups"] == cap
    sa = a.submap_create()
    a.map_sequence(sa, dev, w.cam.K, w.poses, esdf_every=1)
    b = cv.Context(**base)
    sb = b.submap_create()
    _in_order(b, sb, dev, w.cam.K, w.poses, 1)
    _same(a.export_blocks(sa), b.export_blocks(sb))
    with pytest.raises(cv.CovoxError):
        a.set_tuning(edt_pipe_max_workgroups=-1)
    a.close()
    b.close()


@pytest.mark.parametrize("capacity", [16384, 1 << 21])
def test_captured_pipelined_sequence_replays_to_the_calls_in_order(cv, room90, capacity):
    """A captured pipelined sequence replays to the calls in order.  At 2^21
    blocks the host's bound never reaches the capacity, so every frame of the
    capture takes the fused probe update (existing blocks updated in the
    probe); at 16384 the bound passes the capacity within a few frames and
    the capture falls back to the separate update."""
    import torch
    w, fr = room90
    dev = torch.from_numpy(fr[:60]).cuda()
    base = dict(voxel_size=w.voxel_size, trunc_vox=4, max_range=w.cam.max_range, d_max=w.d_max,
                block_capacity=capacity)
    b = cv.Context(**base)
    sb = b.submap_create()
    _in_order(b, sb, dev, w.cam.K, w.poses[:60], 1)
    want = b.export_blocks(sb)
    b.close()
    ctx = cv.Context(**base)
    s = ctx.submap_create()
    ctx.map_sequence(s, dev, w.cam.K, w.poses[:60], esdf_every=1)  # eager first: pipelined capture
    _same(ctx.export_blocks(s), want)
    ctx.graph_begin()
    ctx.submap_reset(s)
    ctx.map_sequence(s, dev, w.cam.K, w.poses[:60], esdf_every=1)
    g = ctx.graph_end()
    for rep in range(3):
        g.launch()
        ctx.sync()
        _same(ctx.export_blocks(s), want)
        ctx.update_esdf(s)  # eager work between the replays
        _same(ctx.export_blocks(s), want)
    g.close()
    ctx.close()


def test_pipelined_tiny_room_matches_the_oracle(cv):
    import torch
    w = sg.tiny()
    fr = w.frames()
    ctx = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)
    s = ctx.submap_create()
    ctx.map_sequence(s, torch.from_numpy(fr).cuda(), w.cam.K, w.poses, esdf_every=1)
    g = ctx.export_blocks(s)
    r = orc.Submap(orc.Params())
    for f in range(w.n_frames):
        r.integrate(fr[f], w.cam.K, w.poses[f])
    r.update_esdf()
    e = r.export()
    assert np.array_equal(g["keys"], e["keys"])
    ge, ee = g["phi"].astype(np.float64), e["phi"]
    assert np.array_equal(np.isnan(ge), np.isnan(ee))
    m = ~np.isnan(ee)
    assert np.abs(ge[m] - ee[m]).max() <= 1e-4  # the bar of the ESDF parity tests
    ctx.close()
