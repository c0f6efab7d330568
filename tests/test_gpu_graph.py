"""GPU tests of graph capture (covox_graph_*): a captured mapping sequence
(reset, frame batches, ESDF updates) replayed several times, with eager
calls and synchronisations between the replays, gives bit for bit the
eager result every time; replays read the current contents of the captured
depth buffer; the capture rules are enforced."""
import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_21149_amd as cv
    return cv


def _ctx(cv, **kw):
    base = dict(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)
    base.update(kw)
    return cv.Context(**base)


def _same(a, b):
    for k in ("keys", "D", "W"):
        assert np.array_equal(a[k], b[k]), k
    pa, pb = a["phi"], b["phi"]
    assert np.array_equal(np.isnan(pa), np.isnan(pb))
    m = ~np.isnan(pa)
    assert np.array_equal(pa[m], pb[m])


@pytest.mark.parametrize("esdf_every", [1, 5])
def test_graph_replays_equal_eager_mapping(cv, esdf_every):
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames()).cuda()
    ref_ctx = _ctx(cv)
    r = ref_ctx.submap_create()
    ref_ctx.map_sequence(r, dev, w.cam.K, w.poses, esdf_every=esdf_every)
    want = ref_ctx.export_blocks(r)
    ref_ctx.close()

    ctx = _ctx(cv)
    s = ctx.submap_create()
    ctx.graph_begin()
    ctx.submap_reset(s)
    ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=esdf_every)
    g = ctx.graph_end()
    assert ctx.submap_info(s)["n_blocks"] == 0  # nothing ran during capture
    for rep in range(3):
        g.launch()
        ctx.sync()
        _same(ctx.export_blocks(s), want)
        # eager work between replays: the ESDF is current, alignment runs
        T, cost, st = ctx.align_submaps(s, s, np.eye(4))
        assert st["status"] == cv.OK and np.max(np.abs(T - np.eye(4))) < 1e-6
        ctx.update_esdf(s)
        _same(ctx.export_blocks(s), want)
    g.close()
    ctx.close()


def test_graph_replay_reads_current_depth_contents(cv):
    import torch
    w = sg.tiny()
    fr = w.frames()
    buf = torch.from_numpy(fr[:10].copy()).cuda()
    ctx = _ctx(cv)
    s = ctx.submap_create()
    ctx.graph_begin()
    ctx.submap_reset(s)
    ctx.integrate_depth_batch(s, buf, w.cam.K, w.poses[:10])
    ctx.update_esdf(s)
    g = ctx.graph_end()
    for src in (fr[:10], fr[10:20][::-1].copy(), fr[:10]):
        buf.copy_(torch.from_numpy(np.ascontiguousarray(src)).cuda())
        g.launch()
        got = ctx.export_blocks(s)
        e = _ctx(cv)
        r = e.submap_create()
        e.integrate_depth_batch(r, torch.from_numpy(np.ascontiguousarray(src)).cuda(), w.cam.K, w.poses[:10])
        e.update_esdf(r)
        _same(got, e.export_blocks(r))
        e.close()
    g.close()
    ctx.close()


def test_capture_rules(cv):
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames(0, 4)).cuda()
    ctx = _ctx(cv)
    s = ctx.submap_create()
    # integration without a reset inside the graph is refused at the end
    ctx.graph_begin()
    ctx.integrate_depth(s, dev[0], w.cam.K, w.poses[0])
    with pytest.raises(cv.CovoxError):
        ctx.graph_end()
    assert ctx.submap_info(s)["n_blocks"] == 0
    # synchronous calls are refused while capturing
    ctx.graph_begin()
    with pytest.raises(cv.CovoxError):
        ctx.align_submaps(s, s, np.eye(4))
    with pytest.raises(cv.CovoxError):
        ctx.export_blocks(s)
    g = ctx.graph_end()
    g.launch()
    g.close()
    # an ESDF-only graph refuses a submap that has grown since the capture
    ctx.integrate_depth_batch(s, dev[:2], w.cam.K, w.poses[:2])
    ctx.graph_begin()
    ctx.update_esdf(s)
    g = ctx.graph_end()
    g.launch()
    ctx.sync()
    T = np.array(w.poses[2], np.float64).copy()
    T[:3, 3] += [3.0, 0.0, 0.0]  # a frame whose frustum reaches new blocks
    ctx.integrate_depth(s, dev[2], w.cam.K, T)
    with pytest.raises(cv.CovoxError):
        g.launch()
    g.close()
    ctx.close()


def test_graph_replays_raycast_mapping(cv):
    """Raycast integration captured with ESDF updates: every replay equals
    the eager run (keys and weights bit for bit; D within 1e-6 m, as the
    per-voxel sums come from atomics in any order)."""
    import torch
    w = sg.tiny(n_frames=10)
    dev = torch.from_numpy(w.frames()).cuda()
    ref_ctx = _ctx(cv, integrator=cv.RAYCAST)
    r = ref_ctx.submap_create()
    ref_ctx.map_sequence(r, dev, w.cam.K, w.poses, esdf_every=3)
    want = ref_ctx.export_blocks(r)
    ref_ctx.close()

    ctx = _ctx(cv, integrator=cv.RAYCAST)
    s = ctx.submap_create()
    ctx.graph_begin()
    ctx.submap_reset(s)
    ctx.map_sequence(s, dev, w.cam.K, w.poses, esdf_every=3)
    g = ctx.graph_end()
    for rep in range(3):
        g.launch()
        ctx.sync()
        got = ctx.export_blocks(s)
        assert np.array_equal(got["keys"], want["keys"]) and np.array_equal(got["W"], want["W"])
        assert np.abs(got["D"].astype(np.float64) - want["D"]).max() <= 1e-6
        ctx.integrate_depth(s, dev[0], w.cam.K, w.poses[0])  # eager work between replays
        ctx.sync()
    g.close()
    ctx.close()
