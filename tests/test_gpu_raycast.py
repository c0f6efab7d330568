"""GPU parity of raycast integration (Sec. III-C raycasting, Sec. III-D
count / allocate / merge) through the C ABI against the oracle on the same
seeded frames.

The oracle's grid walk solves each boundary crossing with one correctly
rounded division; the kernel multiplies by a reciprocal rounded once per
ray.  Both are faithful to 2^-22 relative, so their walks can differ only at
steps the oracle records as fragile (two crossing parameters, or the
nearest one and the segment end, within 2^-21 relative): the voxels such a
step could enter are excluded from the exact comparison, counted and
reported.  The bar:
  - blocks: the key sets agree except for blocks whose every observed voxel
    is fragile; buffer order agrees on the common keys of blocks that hold no
    fragile voxel (bit for bit when no block holds one), home buckets bit for
    bit;
  - voxels outside the fragile set: observed sets equal, W within 1e-6
    relative and D within 1e-6 m (the per-voxel sums are binary64 in both,
    formed in another order on the GPU, so at least 99.9 % agree bit for
    bit);
  - fragile voxels: differences counted and printed, with no bound of their
    own.  Both roundings are faithful there, and their number follows the
    geometry: the tiny workload's camera centres lie on voxel boundary planes
    and whole rows of its rays run inside such planes, so every voxel those
    rays cross is fragile (the oracle records more fragile voxel entries
    than there are observed voxels on that workload).
"""
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


def _ctx(cv, **kw):
    base = dict(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192, integrator=cv.RAYCAST)
    base.update(kw)
    return cv.Context(**base)


def _orc(**kw):
    base = dict(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, integrator=1)
    base.update(kw)
    return orc.Submap(orc.Params(**base))


def _voxel_index(keys):
    """(key, in-block index) -> flat index into the (n, 512) arrays."""
    return {int(k): i for i, k in enumerate(keys)}


def _fragile_flat(ref, keys):
    """Flat indices (into the blocks `keys`) of the oracle's fragile voxels,
    and the block keys they fall in."""
    fr = ref.fragile_voxels()
    if len(fr) == 0:
        return np.zeros(0, np.int64), set()
    b = fr >> 3
    bk = orc.pack_key(b[:, 0], b[:, 1], b[:, 2])
    lin = (fr[:, 0] & 7) + 8 * (fr[:, 1] & 7) + 64 * (fr[:, 2] & 7)
    pos = _voxel_index(keys)
    flat = [pos[int(k)] * 512 + int(l) for k, l in zip(bk, lin) if int(k) in pos]
    return np.unique(np.array(flat, np.int64)), {int(k) for k in bk}


def _compare(g, r, ref, tcap):
    gk, rk = g["keys"], r["keys"]
    gpos, rpos = _voxel_index(gk), _voxel_index(rk)
    common = [int(k) for k in rk if int(k) in gpos]
    # key sets: any block on one side only holds fragile voxels alone
    frag_r, frag_blocks = _fragile_flat(ref, rk)
    only = (set(gpos) ^ set(rpos))
    assert only <= frag_blocks, "blocks differ away from fragile walk steps"
    for k in only:
        side = g if k in gpos else r
        i = (gpos if k in gpos else rpos)[k]
        obs = np.nonzero(side["W"][i] > 0)[0]
        b = np.array(orc.unpack_key(np.array([k], np.uint64))).reshape(3)
        vox = 8 * b + np.stack([obs & 7, (obs >> 3) & 7, obs >> 6], axis=1)
        fr = {tuple(v) for v in ref.fragile_voxels()}
        assert all(tuple(v) in fr for v in vox), "a one-sided block holds a voxel no fragile step explains"
    # buffer order on the common keys of blocks without a fragile voxel (a
    # block that a fragile step touches may be allocated a frame earlier on
    # one side); home buckets
    strict_keys = [k for k in common if k not in frag_blocks]
    assert [int(k) for k in gk if int(k) in rpos and int(k) not in frag_blocks] == strict_keys, "buffer order differs"
    if not only and not frag_blocks:
        assert np.array_equal(gk, rk)
    assert np.array_equal(g["home"].astype(np.int64), orc.home_bucket(gk, tcap))
    # voxels of the common blocks, in the oracle's block order
    gi = np.array([gpos[k] for k in common], np.int64)
    ri = np.array([rpos[k] for k in common], np.int64)
    W, Wr = g["W"][gi].astype(np.float64).reshape(-1), r["W"][ri].reshape(-1)
    D, Dr = g["D"][gi].astype(np.float64).reshape(-1), r["D"][ri].reshape(-1)
    fragile = np.zeros(len(common) * 512, bool)
    rmap = {int(x): j for j, x in enumerate(ri)}
    for f in frag_r:
        j = rmap.get(int(f) // 512)
        if j is not None:
            fragile[j * 512 + int(f) % 512] = True
    obs_r, obs_g = Wr > 0, W > 0
    strict = ~fragile
    assert np.array_equal(obs_g[strict], obs_r[strict]), "observed sets differ away from fragile steps"
    m = strict & obs_r
    dW = np.abs(W - Wr)[m] / Wr[m]
    dD = np.abs(D - Dr)[m]
    assert dW.max(initial=0) <= 1e-6, dW.max()
    assert dD.max(initial=0) <= 1e-6, dD.max()
    n = int(obs_r.sum())
    assert np.count_nonzero(dW) <= 1e-3 * n and np.count_nonzero(dD) <= 1e-3 * n
    fm = fragile & (obs_r | obs_g)
    n_frag_diff = int(np.count_nonzero((W != Wr)[fm] | (np.abs(D - Dr)[fm] > 1e-6)))
    assert n_frag_diff <= int(fm.sum())
    return {"d_differ": int(np.count_nonzero(dD)), "observed": n, "fragile": int(fragile.sum()),
            "fragile_differ": n_frag_diff, "one_sided_blocks": len(only),
            "order_checked_blocks": len(strict_keys), "common_blocks": len(common)}


@pytest.mark.parametrize("carve", [1, 0])
def test_tiny_raycast_parity(cv, carve):
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv, ray_carve=carve)
    s = ctx.submap_create()
    ref = _orc(ray_carve=bool(carve))
    tcap = ctx.submap_info(s)["table_capacity"]
    n_vox = 0
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        n_vox += ref.integrate(fr[f], w.cam.K, w.poses[f])["n_voxels"]
        if f in (0, 1, 7, w.n_frames - 1):
            c = _compare(ctx.export_blocks(s), ref.export(), ref, tcap)
            print("frame %d: %s" % (f, c))
    # the contribution count: a crossing that ties with the segment end adds
    # or drops the last voxel of a ray, and every such fragile step records
    # at least one fragile voxel
    n_gpu = ctx.submap_info(s)["n_updates"]
    print("contributions: gpu %d, oracle %d" % (n_gpu, n_vox))
    assert abs(n_gpu - n_vox) <= len(ref.fragile_voxels())
    ctx.close()


def test_raycast_inverse_depth_weights(cv):
    import torch
    w = sg.tiny(n_frames=8)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv, weight_mode=cv.WEIGHT_INV_DEPTH2)
    s = ctx.submap_create()
    ref = _orc(weight_mode=1)
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    g = ctx.export_blocks(s)
    _compare(g, ref.export(), ref, ctx.submap_info(s)["table_capacity"])
    assert not np.all(g["W"] == np.round(g["W"]))
    ctx.close()


def test_room_frames_raycast_parity(cv):
    """Two 640 x 480 frames of the room benchmark sequence (23 M ray-voxel
    contributions each)."""
    import torch
    w = sg.room(n_frames=2)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv, block_capacity=16384)
    s = ctx.submap_create()
    ref = _orc()
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    c = _compare(ctx.export_blocks(s), ref.export(), ref, ctx.submap_info(s)["table_capacity"])
    print("room: %s" % c)
    ctx.close()


def test_batch_calls_match_per_frame_calls(cv):
    """integrate_depth_batch and map_sequence run the same frames in order."""
    import torch
    w = sg.tiny(n_frames=10)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv)
    a, b = ctx.submap_create(), ctx.submap_create()
    ref = _orc()
    for f in range(w.n_frames):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    ctx.integrate_depth_batch(b, dev, w.cam.K, w.poses)
    tcap = ctx.submap_info(a)["table_capacity"]
    r = ref.export()
    ga, gb = ctx.export_blocks(a), ctx.export_blocks(b)
    _compare(ga, r, ref, tcap)
    for k in ("keys", "D", "W"):
        assert np.array_equal(ga[k], gb[k]), k  # the same kernels in the same order
    ctx.close()


def test_capacity_failure_drops_the_frame_only(cv):
    """A frame that would overflow the pool is dropped whole (EPOOL_FULL);
    the next frame that fits integrates as if the dropped one never came."""
    import torch
    w = sg.tiny()
    fr = w.frames()
    # the capacity from the GPU's own count (a fragile step can allocate a
    # block on one side only)
    probe = _ctx(cv)
    ps = probe.submap_create()
    probe.integrate_depth(ps, torch.from_numpy(fr[0]).cuda(), w.cam.K, w.poses[0])
    cap = probe.submap_info(ps)["n_blocks"] + 2
    probe.close()
    ctx = _ctx(cv, block_capacity=cap)
    s = ctx.submap_create()
    ref = _orc()
    ctx.integrate_depth(s, torch.from_numpy(fr[0]).cuda(), w.cam.K, w.poses[0])
    ref.integrate(fr[0], w.cam.K, w.poses[0])
    with pytest.raises(cv.CovoxError):
        ctx.integrate_depth(s, torch.from_numpy(fr[10]).cuda(), w.cam.K, w.poses[10])
    ctx.integrate_depth(s, torch.from_numpy(fr[0]).cuda(), w.cam.K, w.poses[0])
    ref.integrate(fr[0], w.cam.K, w.poses[0])
    _compare(ctx.export_blocks(s), ref.export(), ref, ctx.submap_info(s)["table_capacity"])
    ctx.close()


def test_esdf_of_a_raycast_map(cv):
    """The ESDF of the raycast TSDF equals the oracle's ESDF of the same D
    and W (imported), so the rest of the path runs unchanged on it."""
    import torch
    w = sg.tiny(n_frames=10)
    dev = torch.from_numpy(w.frames()).cuda()
    ctx = _ctx(cv)
    s = ctx.submap_create()
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
    ctx.update_esdf(s)
    g = ctx.export_blocks(s)
    ref = _orc()
    ref.import_blocks(g["keys"], g["D"], g["W"])
    ref.update_esdf()
    r = ref.export()
    m = ~np.isnan(r["phi"])
    assert np.array_equal(np.isnan(g["phi"]), ~m)
    assert np.abs(g["phi"][m] - r["phi"][m]).max(initial=0) <= 1e-4
    ctx.close()


def test_raycast_parameter_checks(cv):
    with pytest.raises(cv.CovoxError):
        _ctx(cv, precision=cv.FP16)
    ctx = cv.Context(voxel_size=0.05, block_capacity=4096)
    ctx.set_params(integrator=cv.RAYCAST)
    s = ctx.submap_create()
    import torch
    with pytest.raises(cv.CovoxError):  # rays far too long for these intrinsics
        ctx.integrate_depth(s, torch.ones((12, 16), device="cuda"), np.array([1e-4, 1e-4, 7.5, 5.5], np.float32),
                            np.eye(4))
    assert ctx.submap_info(s)["n_blocks"] == 0
    ctx.close()
