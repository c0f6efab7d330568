"""GPU parity of the incremental (wavefront) ESDF (Sec. III-E) through the
C ABI against the oracle's wavefront on the same frames and the same update
schedule: phi bit for bit after every update (the propagation is integer
and its rounds are synchronous, so it does not depend on scheduling), in
binary32 and binary16 storage, across resets, in the mapping loop, and as
the field of an alignment."""
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
    base = dict(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192,
                esdf_mode=cv.ESDF_WAVEFRONT)
    base.update(kw)
    return cv.Context(**base)


def _phi_equal(g, r):
    gp, rp = g["phi"].astype(np.float64), r["phi"]
    assert np.array_equal(g["keys"], r["keys"])
    assert np.array_equal(np.isnan(gp), np.isnan(rp)), "unobserved sets differ"
    m = ~np.isnan(rp)
    d = np.abs(gp[m] - rp[m])
    assert d.max(initial=0) == 0.0, (int(np.count_nonzero(d)), d.max())


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_incremental_updates_match_oracle(cv, precision):
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    fp16 = precision == "fp16"
    ctx = _ctx(cv, precision=cv.FP16 if fp16 else cv.FP32)
    s = ctx.submap_create()
    ref = orc.Submap(orc.Params(fp16=fp16, esdf_mode=1))
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
        if f % 3 == 2 or f == w.n_frames - 1:
            ctx.update_esdf(s)
            st = ref.esdf_wavefront()
            _phi_equal(ctx.export_blocks(s), ref.export())
    assert st["block_rounds"] > 0
    ctx.close()


def test_reset_and_mapping_loop(cv):
    """After a reset the state starts over; map_sequence with updates every
    four frames equals the same calls one by one."""
    import torch
    w = sg.tiny(n_frames=12)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv)
    a, b = ctx.submap_create(), ctx.submap_create()
    for f in range(6):  # history to be discarded
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
    ctx.update_esdf(a)
    ctx.submap_reset(a)
    ref = orc.Submap(orc.Params(esdf_mode=1))
    for f in range(w.n_frames):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
        if f % 4 == 3:
            ctx.update_esdf(a)
            ref.esdf_wavefront()
    ctx.map_sequence(b, dev, w.cam.K, w.poses, esdf_every=4)
    r = ref.export()
    _phi_equal(ctx.export_blocks(a), r)
    _phi_equal(ctx.export_blocks(b), r)
    ctx.close()


def test_room_frames_match_oracle(cv):
    """Forty frames of the 640 x 480 room, updates every ten frames."""
    import torch
    w = sg.room(n_frames=40)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv, block_capacity=16384)
    s = ctx.submap_create()
    ref = orc.Submap(orc.Params(esdf_mode=1))
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
        if f % 10 == 9:
            ctx.update_esdf(s)
            ref.esdf_wavefront()
    _phi_equal(ctx.export_blocks(s), ref.export())
    ctx.close()


def test_alignment_on_a_wavefront_field(cv):
    """The alignment samples the wavefront field like the exact one: pose
    parity with the oracle aligning against its own wavefront field."""
    import math
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    ctx = _ctx(cv)
    A, B = ctx.submap_create(), ctx.submap_create()
    rA, rB = orc.Submap(orc.Params(esdf_mode=1)), orc.Submap(orc.Params(esdf_mode=1))
    for f in range(20):
        for _ in range(2):
            ctx.integrate_depth(A if f < 10 else B, dev[f], w.cam.K, w.poses[f])
            (rA if f < 10 else rB).integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(A)
    ctx.update_esdf(B)
    rA.update_esdf()
    rB.update_esdf()
    T0 = orc.se3_exp(np.array([0.03, -0.02, 0.01, 0.02, -0.01, 0.03]))
    Tg, cg, st = ctx.align_submaps(A, B, T0)
    r = orc.align(rA, rB.iso_points(), T0)
    assert st["iterations"] == r["iters"] and st["n_used"] == r["n"]
    dt = np.linalg.norm(Tg[:3, 3] - r["T"][:3, 3])
    c = (np.trace(Tg[:3, :3] @ r["T"][:3, :3].T) - 1) / 2
    assert dt <= 1e-6 and math.acos(max(-1.0, min(1.0, c))) <= 1e-6
    ctx.close()
