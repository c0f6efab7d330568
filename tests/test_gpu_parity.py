"""GPU parity: the HIP library (through the C ABI) against the reference
oracle on the same seeded inputs.

Bars: allocated block set, buffer indices and home buckets bit-exact; TSDF D
and W within 1e-4 m (binary32 storage; bit-exact expected, same pinned
operation order); ESDF phi within 1e-4 m with identical unobserved sets;
poses within 1e-6 (translation in m, rotation angle in rad)."""
import math
import tempfile

import numpy as np
import pytest

import oracle as orc
import scenegen as sg

pytestmark = pytest.mark.gpu

TOL = 1e-4


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


def _oracle_params(**kw):
    base = dict(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0)
    base.update(kw)
    return orc.Params(**base)


def _compare_blocks(g, r, table_cap, fp16=False):
    assert np.array_equal(g["keys"], r["keys"]), "block keys / buffer order differ"
    assert np.array_equal(g["home"].astype(np.int64), orc.home_bucket(r["keys"], table_cap)), "home buckets differ"
    dD = np.abs(g["D"].astype(np.float64) - r["D"])
    dW = np.abs(g["W"].astype(np.float64) - r["W"])
    assert dD.max(initial=0) <= TOL and dW.max(initial=0) <= TOL
    return int(np.count_nonzero(dD)), int(np.count_nonzero(dW))


def _compare_phi(g, r):
    gp, rp = g["phi"].astype(np.float64), r["phi"]
    assert np.array_equal(np.isnan(gp), np.isnan(rp)), "unobserved sets differ"
    m = ~np.isnan(rp)
    d = np.abs(gp[m] - rp[m])
    assert d.max(initial=0) <= TOL, d.max()
    return int(np.count_nonzero(d))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_tiny_integration_and_esdf_parity(cv, precision):
    import torch
    w = sg.tiny()
    fr = w.frames()
    fp16 = precision == "fp16"
    ctx = _ctx(cv, precision=cv.FP16 if fp16 else cv.FP32)
    s = ctx.submap_create()
    ref = orc.Submap(_oracle_params(fp16=fp16))
    dev = torch.from_numpy(fr).cuda()
    tcap = ctx.submap_info(s)["table_capacity"]
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
        if f in (0, 1, 7, 19):
            nd, nw = _compare_blocks(ctx.export_blocks(s), ref.export(), tcap, fp16)
            assert nd == 0 and nw == 0, "expected bit-exact TSDF (frame %d)" % f
    ctx.update_esdf(s)
    ref.update_esdf()
    assert _compare_phi(ctx.export_blocks(s), ref.export()) == 0
    ctx.close()


def test_room_full_sequence_parity(cv):
    """The 300-frame 640x480 room sequence (the benchmark workload),
    integrated with an ESDF update after every frame as the benchmark does;
    full comparison at the end and at frame 40."""
    import torch
    w = sg.room()
    ctx = _ctx(cv, block_capacity=16384)
    s = ctx.submap_create()
    ref = orc.Submap(_oracle_params())
    tcap = ctx.submap_info(s)["table_capacity"]
    for f0 in range(0, w.n_frames, 50):
        fr = w.frames(f0, min(f0 + 50, w.n_frames))
        dev = torch.from_numpy(fr).cuda()
        for k in range(len(fr)):
            ctx.integrate_depth(s, dev[k], w.cam.K, w.poses[f0 + k])
            ctx.update_esdf(s)
            ref.integrate(fr[k], w.cam.K, w.poses[f0 + k])
            if f0 + k == 40:
                ref.update_esdf()
                g = ctx.export_blocks(s)
                r = ref.export()
                assert _compare_blocks(g, r, tcap) == (0, 0)
                assert _compare_phi(g, r) == 0
    ref.update_esdf()
    g, r = ctx.export_blocks(s), ref.export()
    assert _compare_blocks(g, r, tcap) == (0, 0)
    assert _compare_phi(g, r) == 0
    assert len(g["keys"]) > 1000
    ctx.close()


def test_determinism_two_runs(cv):
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames()).cuda()
    outs = []
    for _ in range(2):
        ctx = _ctx(cv)
        s = ctx.submap_create()
        for f in range(w.n_frames):
            ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ctx.update_esdf(s)
        outs.append(ctx.export_blocks(s))
        ctx.close()
    for k in ("keys", "home", "D", "W"):
        assert np.array_equal(outs[0][k], outs[1][k])
    assert np.array_equal(outs[0]["phi"], outs[1]["phi"], equal_nan=True)


def test_batch_integration_equals_sequential(cv):
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames()).cuda()
    ctx = _ctx(cv)
    a = ctx.submap_create()
    b = ctx.submap_create()
    for f in range(w.n_frames):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
    ctx.integrate_depth_batch(b, dev, w.cam.K, w.poses)
    ea, eb = ctx.export_blocks(a), ctx.export_blocks(b)
    for k in ("keys", "home", "D", "W"):
        assert np.array_equal(ea[k], eb[k])
    ctx.close()


@pytest.mark.parametrize("precision,xcd", [("fp32", 0), ("fp16", 0), ("fp32", 1)])
def test_batched_integration_matches_oracle_and_single_frames(cv, precision, xcd):
    """Frame batches (one probe, one scan and one update launch per batch)
    against per-frame calls and the oracle: blocks in (first frame, key)
    order, D and W bit for bit, also in binary16 storage where every frame's
    result is rounded to the stored precision, and with the XCD work order
    of the depth-gathering kernels."""
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    fp16 = precision == "fp16"
    ctx = _ctx(cv, precision=cv.FP16 if fp16 else cv.FP32)
    ctx.set_tuning(mapping_xcd_order=xcd)
    a, b = ctx.submap_create(), ctx.submap_create()
    for f in range(w.n_frames):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
    # uneven batches: 7, 1, 12 frames
    ctx.integrate_depth_batch(b, dev[:7], w.cam.K, w.poses[:7])
    ctx.integrate_depth_batch(b, dev[7:8], w.cam.K, w.poses[7:8])
    ctx.integrate_depth_batch(b, dev[8:], w.cam.K, w.poses[8:])
    ea, eb = ctx.export_blocks(a), ctx.export_blocks(b)
    for k in ("keys", "home", "D", "W"):
        assert np.array_equal(ea[k], eb[k]), k
    assert ctx.submap_info(a)["n_updates"] == ctx.submap_info(b)["n_updates"]
    ref = orc.Submap(_oracle_params(fp16=fp16))
    for f in range(w.n_frames):
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    nd, nw = _compare_blocks(eb, ref.export(), ctx.submap_info(b)["table_capacity"], fp16)
    assert nd == 0 and nw == 0
    ctx.close()


def test_batch_stops_at_the_frame_that_overflows(cv):
    """A batch whose k-th frame needs more blocks than remain commits frames
    0..k-1 exactly as single calls would, drops the rest and reports
    EPOOL_FULL."""
    import torch
    w = sg.tiny()
    fr = w.frames(0, 12)
    dev = torch.from_numpy(fr).cuda()
    ref = orc.Submap(_oracle_params())
    n_after = []
    for f in range(12):
        ref.integrate(fr[f], w.cam.K, w.poses[f])
        n_after.append(len(ref.export()["keys"]))
    k = next(i for i in range(12) if n_after[i] > n_after[0])  # first frame that allocates more
    cap = n_after[k] - 1
    ctx = _ctx(cv, block_capacity=cap)
    a, b = ctx.submap_create(), ctx.submap_create()
    for f in range(k):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
    with pytest.raises(cv.CovoxError) as e:
        ctx.integrate_depth_batch(b, dev, w.cam.K, w.poses[:12])
    assert e.value.code == cv.EPOOL_FULL
    ea, eb = ctx.export_blocks(a), ctx.export_blocks(b)
    for key in ("keys", "D", "W"):
        assert np.array_equal(ea[key], eb[key]), key
    ctx.close()


def test_empty_and_invalid_frames(cv):
    import torch
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    ctx = _ctx(cv)
    s = ctx.submap_create()
    for v in (0.0, float("nan"), 5.5, -1.0):
        ctx.integrate_depth(s, torch.full((12, 16), v, device="cuda"), K, np.eye(4))
    assert ctx.submap_info(s)["n_blocks"] == 0
    ctx.update_esdf(s)  # an empty submap is a no-op
    with pytest.raises(cv.CovoxError):
        ctx.integrate_depth(s, torch.zeros((12, 16), device="cuda"), np.array([0, 1, 1, 1], np.float32), np.eye(4))
    bad = np.eye(4)
    bad[0, 0] = 2.0
    with pytest.raises(cv.CovoxError):
        ctx.integrate_depth(s, torch.zeros((12, 16), device="cuda"), K, bad)
    ctx.close()


def test_pool_full_leaves_submap_unchanged(cv):
    """A frame that needs more blocks than remain is dropped whole and the
    call reports EPOOL_FULL; a frame that fits still integrates."""
    import torch
    w = sg.tiny()
    fr = w.frames(0, 3)
    dev = torch.from_numpy(fr).cuda()
    ref = orc.Submap(_oracle_params())
    st0 = ref.integrate(fr[0], w.cam.K, w.poses[0])
    cap = st0["n_new"] + 5
    ctx = _ctx(cv, block_capacity=cap)
    s = ctx.submap_create()
    ctx.integrate_depth(s, dev[0], w.cam.K, w.poses[0])
    before = ctx.export_blocks(s)
    with pytest.raises(cv.CovoxError) as e:
        ctx.integrate_depth(s, torch.from_numpy(w.frame(10)).cuda(), w.cam.K, w.poses[10])
    assert e.value.code == cv.EPOOL_FULL
    after = ctx.export_blocks(s)
    for k in ("keys", "D", "W"):
        assert np.array_equal(before[k], after[k])
    ctx.integrate_depth(s, dev[0], w.cam.K, w.poses[0])  # re-observing fits
    assert ctx.submap_info(s)["n_blocks"] == len(before["keys"])
    ctx.close()


# ------------------------------------------------------------------ align

def _pair_from_tiny(cv, ctx):
    """A: frames 0-9, B: frames 10-19 of the tiny room, both in the world
    frame, so the true transform is the identity."""
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    A, B = ctx.submap_create(), ctx.submap_create()
    rA, rB = orc.Submap(_oracle_params()), orc.Submap(_oracle_params())
    for f in range(20):
        for _ in range(2):  # each frame twice: weights >= 2 for registration points
            ctx.integrate_depth(A if f < 10 else B, dev[f], w.cam.K, w.poses[f])
            (rA if f < 10 else rB).integrate(fr[f], w.cam.K, w.poses[f])
    for f in range(20):  # overlap: both submaps also see a few frames of the other half
        if f % 5 == 0:
            ctx.integrate_depth(B if f < 10 else A, dev[f], w.cam.K, w.poses[f])
            (rB if f < 10 else rA).integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(A)
    ctx.update_esdf(B)
    rA.update_esdf()
    rB.update_esdf()
    return A, B, rA, rB


def _pose_err(T1, T2):
    dt = np.linalg.norm(T1[:3, 3] - T2[:3, 3])
    c = (np.trace(T1[:3, :3] @ T2[:3, :3].T) - 1) / 2
    return dt, math.acos(max(-1.0, min(1.0, c)))


def test_registration_points_and_normal_equations_parity(cv):
    ctx = _ctx(cv)
    A, B, rA, rB = _pair_from_tiny(cv, ctx)
    pg = ctx.export_points(B)
    pr = rB.iso_points()
    assert pg.shape == pr.shape and len(pg) > 1000
    assert np.array_equal(pg, pr), "registration points differ"
    T = orc.se3_exp(np.array([0.01, -0.02, 0.005, 0.01, 0.02, -0.015]))
    ne_g = ctx.normal_equations(A, B, T)
    ne_r = orc.normal_eq(rA, pr, T)[4]
    assert ne_g[28] == ne_r[28]  # identical residual set
    assert np.allclose(ne_g, ne_r, rtol=1e-12, atol=1e-9)
    ctx.close()


def test_alignment_pose_parity_and_recovery(cv):
    ctx = _ctx(cv)
    A, B, rA, rB = _pair_from_tiny(cv, ctx)
    pts = rB.iso_points()
    for xi in ([0.03, -0.02, 0.01, 0.02, -0.01, 0.03], [-0.05, 0.04, 0.0, 0.0, 0.0, 0.08]):
        T0 = orc.se3_exp(np.array(xi))
        Tg, cg, st = ctx.align_submaps(A, B, T0)
        r = orc.align(rA, pts, T0)
        assert st["status"] == r["status"] and st["iterations"] == r["iters"] and st["n_used"] == r["n"]
        dt, dr = _pose_err(Tg, r["T"])
        assert dt <= 1e-6 and dr <= 1e-6, (dt, dr)
        assert abs(cg - r["cost"]) <= 1e-9 + 1e-9 * r["cost"]
        et, er = _pose_err(Tg, np.eye(4))
        assert et < 0.01 and er < math.radians(0.1), (et, er)
    ctx.close()


def test_multistart_and_batch_match_single_calls(cv):
    ctx = _ctx(cv)
    A, B, rA, rB = _pair_from_tiny(cv, ctx)
    pts = rB.iso_points()
    T0 = orc.se3_exp(np.array([0.02, 0.01, -0.01, 0.0, 0.0, 0.5]))
    Tm, cm, sm = ctx.align_multistart(A, B, T0, 8)
    rm = orc.align_multistart(rA, pts, T0, 8)
    assert sm["best_start"] == rm["best"]
    dt, dr = _pose_err(Tm, rm["T"])
    assert dt <= 1e-6 and dr <= 1e-6
    pairs = [(A, B, T0), (A, B, orc.se3_exp(np.array([0.01, 0, 0, 0, 0, 0.01])))]
    Tb, cb, sb = ctx.align_batch(pairs, n_starts=8)
    assert np.array_equal(Tb[0], Tm) and cb[0] == cm
    T1, c1, s1 = ctx.align_submaps(A, B, pairs[1][2])
    Tb1, cb1, _ = ctx.align_batch(pairs[1:], n_starts=1)
    assert np.array_equal(Tb1[0], T1) and cb1[0] == c1
    ctx.close()


def test_alignment_workgroup_sizes_agree_with_oracle(cv):
    """256 and 512 lanes per problem (tuning.align_threads) reduce the FP64
    sums in different orders: every setting meets the pose bar against the
    oracle; 1 or 2 points per step give identical results; the autotuner
    keeps one of the settings."""
    ctx = _ctx(cv)
    A, B, rA, rB = _pair_from_tiny(cv, ctx)
    pts = rB.iso_points()
    T0 = orc.se3_exp(np.array([0.03, -0.02, 0.01, 0.02, -0.01, 0.03]))
    r = orc.align(rA, pts, T0)
    for lanes in (256, 512):
        got = []
        for per_step in (1, 2):
            ctx.set_tuning(align_threads=lanes, align_points_per_step=per_step)
            Tg, cg, st = ctx.align_submaps(A, B, T0)
            assert st["status"] == r["status"] and st["n_used"] == r["n"]
            dt, dr = _pose_err(Tg, r["T"])
            assert dt <= 1e-6 and dr <= 1e-6, (lanes, dt, dr)
            got.append((Tg, cg))
        # points per step change nothing, bit for bit
        assert np.array_equal(got[0][0], got[1][0]) and got[0][1] == got[1][1]
    with pytest.raises(cv.CovoxError):
        ctx.set_tuning(align_threads=300)
    t = ctx.autotune_align([(A, B, T0), (B, A, np.linalg.inv(T0))], n_starts=8)
    assert t["align_threads"] in (256, 512) and t["align_points_per_step"] in (1, 2)
    ctx.close()


def test_alignment_needs_current_esdf_and_enough_points(cv):
    import torch
    ctx = _ctx(cv)
    A, B, rA, rB = _pair_from_tiny(cv, ctx)
    w = sg.tiny()
    ctx.integrate_depth(A, torch.from_numpy(w.frame(3)).cuda(), w.cam.K, w.poses[3])
    with pytest.raises(cv.CovoxError):
        ctx.align_submaps(A, B, np.eye(4))
    ctx.update_esdf(A)
    empty = ctx.submap_create()
    T, c, st = ctx.align_submaps(A, empty, np.eye(4))
    assert st["status"] == cv.EDEGENERATE and st["iterations"] == 0
    ctx.close()


@pytest.mark.parametrize("mode", ["window", "envelope"])
@pytest.mark.parametrize("workload", ["tiny", "room40"])
def test_esdf_modes_parity(cv, mode, workload, monkeypatch):
    """Both pass shapes of the ESDF (voxel-parallel windowed search and
    per-line lower envelopes) give the oracle's phi."""
    import torch
    monkeypatch.setenv("COVOX_EDT_MODE", mode)
    w = sg.tiny() if workload == "tiny" else sg.room(n_frames=40)
    fr = w.frames()
    ctx = _ctx(cv, block_capacity=16384)
    s = ctx.submap_create()
    ref = orc.Submap(_oracle_params())
    dev = torch.from_numpy(fr).cuda()
    for f in range(w.n_frames):
        ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(s)
    ref.update_esdf()
    assert _compare_phi(ctx.export_blocks(s), ref.export()) == 0
    ctx.close()


def test_mixed_pass_shapes_and_autotune_leave_phi_unchanged(cv):
    """Every combination of y and z pass shapes (chosen through the tuning
    thresholds) and the autotuner's own runs give the same phi, bit for bit,
    as the oracle; the autotuner returns valid thresholds."""
    import torch
    w = sg.room(n_frames=30)
    fr = w.frames()
    ctx = _ctx(cv, block_capacity=16384)
    s = ctx.submap_create()
    ref = orc.Submap(_oracle_params())
    dev = torch.from_numpy(fr).cuda()
    ctx.integrate_depth_batch(s, dev, w.cam.K, w.poses)
    for f in range(w.n_frames):
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    ref.update_esdf()
    want = ref.export()
    big = 2 ** 62
    for y_thr, z_thr in ((0, 0), (0, big), (big, 0), (big, big)):
        ctx.set_tuning(y_thr, z_thr)
        ctx.update_esdf(s)
        assert _compare_phi(ctx.export_blocks(s), want) == 0, (y_thr, z_thr)
    t = ctx.autotune_esdf([s])
    assert t["edt_y_env_min_cols"] >= 0 and t["edt_z_env_min_cols"] >= 0
    assert ctx.tuning() == t
    assert _compare_phi(ctx.export_blocks(s), want) == 0
    ctx.update_esdf(s)
    assert _compare_phi(ctx.export_blocks(s), want) == 0
    ctx.close()


@pytest.mark.parametrize("workload", ["tiny", "room40", "outdoor"])
def test_column_passes_parity(cv, workload):
    """The column passes (x fused into y, segments of S blocks staged with
    their halos) give the oracle's phi bit for bit at every segment length,
    including 1 (all halo), lengths that do not divide the box and lengths
    above the clamp; the batched form over several submaps equals the
    per-submap updates."""
    import torch
    if workload == "outdoor":
        w = sg.mav(n_frames=300)
        params = dict(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=32768)
        oparams = orc.Params(vs=0.1, trunc_vox=4, max_range=10.0, d_max=3.0)
        starts, nf = (0, 100, 200), 30
    else:
        w = sg.tiny() if workload == "tiny" else sg.room(n_frames=40)
        params = dict(block_capacity=16384)
        oparams = _oracle_params()
        starts, nf = (0,), w.n_frames
    ctx = _ctx(cv, **params)
    subs, want = [], []
    for k, f0 in enumerate(starts):
        T = sg.gravity_aligned(w.poses[f0]) if workload == "outdoor" else np.eye(4)
        fr = w.frames(f0, f0 + nf)
        s = ctx.submap_create(T)
        ctx.integrate_depth_batch(s, torch.from_numpy(fr).cuda(), w.cam.K, w.poses[f0:f0 + nf])
        subs.append(s)
        r = orc.Submap(oparams, T)
        for f in range(nf):
            r.integrate(fr[f], w.cam.K, w.poses[f0 + f])
        r.update_esdf()
        want.append(r.export())
    for seg in (1, 2, 3, 8, 64):
        ctx.set_tuning(edt_col_seg=seg)
        for s, r in zip(subs, want):
            ctx.update_esdf(s)
            assert _compare_phi(ctx.export_blocks(s), r) == 0, seg
        if len(subs) > 1:
            ctx.update_esdf_batch(subs[::-1])
            for s, r in zip(subs, want):
                assert _compare_phi(ctx.export_blocks(s), r) == 0, ("batch", seg)
    ctx.close()


@pytest.mark.parametrize("R", [5, 56])
def test_esdf_radius_extremes_parity(cv, R):
    """The exact ESDF at the smallest halo (R = 5 voxels: one halo block) and
    the largest radius the passes support (R = 56: seven halo blocks, the
    site window's full 128 bits, squared candidates up to 2 R^2 = 6272), in
    every pass shape: voxel-parallel windows, per-line envelopes and column
    passes.  phi must equal the oracle's bit for bit."""
    import torch
    w = sg.tiny()
    fr = w.frames()
    d_max = R * 0.05
    ctx = _ctx(cv, d_max=d_max)
    s = ctx.submap_create()
    ctx.integrate_depth_batch(s, torch.from_numpy(fr).cuda(), w.cam.K, w.poses)
    ref = orc.Submap(_oracle_params(d_max=d_max))
    for f in range(w.n_frames):
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    ref.update_esdf()
    want = ref.export()
    big = 2 ** 62
    shapes = {"windows": dict(edt_col_seg=0, edt_y_env_min_cols=big, edt_z_env_min_cols=big),
              "envelopes": dict(edt_col_seg=0, edt_y_env_min_cols=0, edt_z_env_min_cols=0),
              "columns": dict(edt_col_seg=2, edt_y_env_min_cols=big, edt_z_env_min_cols=big)}
    for name, tuning in shapes.items():
        ctx.set_tuning(esdf_full_recompute=1, **tuning)
        ctx.update_esdf(s)
        assert _compare_phi(ctx.export_blocks(s), want) == 0, name
    ctx.close()


def test_outdoor_submap_parity_and_batched_esdf(cv):
    """An outdoor submap at the large-scale configuration (0.1 m voxels,
    10 m range, ESDF to 3 m) against the oracle, and the batched ESDF of
    several submaps equal to per-submap updates."""
    import torch
    w = sg.mav(n_frames=600)
    params = dict(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=32768)
    ctx = _ctx(cv, **params)
    subs, refs = [], []
    for k in range(3):
        T = sg.gravity_aligned(w.poses[200 * k])
        fr = w.frames(200 * k, 200 * k + 40)
        s = ctx.submap_create(T)
        ctx.map_sequence(s, torch.from_numpy(fr).cuda(), w.cam.K, w.poses[200 * k:200 * k + 40], esdf_every=0)
        subs.append(s)
        if k == 0:
            r = orc.Submap(orc.Params(vs=0.1, trunc_vox=4, max_range=10.0, d_max=3.0), T)
            for f in range(40):
                r.integrate(fr[f], w.cam.K, w.poses[f])
            r.update_esdf()
            refs.append(r)
    g0 = ctx.export_blocks(subs[0])
    tcap = ctx.submap_info(subs[0])["table_capacity"]
    assert _compare_blocks(g0, refs[0].export(), tcap) == (0, 0)
    assert _compare_phi(g0, refs[0].export()) == 0
    for s in subs:
        ctx.update_esdf(s)
    singles = [ctx.export_blocks(s)["phi"] for s in subs]
    ctx.update_esdf_batch(subs[::-1])
    for s, ph in zip(subs, singles):
        assert np.array_equal(ctx.export_blocks(s)["phi"], ph, equal_nan=True)
    ctx.close()


def test_outdoor_alignment_and_summary_parity(cv):
    """Two overlapping outdoor submaps (0.1 m voxels, 10 m range, noise
    0.002 z^2) at full frame size: registration points bit-exact, alignment
    from perturbed priors within the pose bar of the oracle (same status,
    iterations and residual count), and the proposal's 1 m summaries against
    the oracle's binary64 ones."""
    import torch
    w = sg.mav(n_frames=80)
    K = w.cam.K
    params = dict(voxel_size=0.1, trunc_vox=4, max_range=10.0, d_max=3.0, block_capacity=16384)
    ctx = _ctx(cv, **params)
    fr = w.frames(0, 70)
    dev = torch.from_numpy(fr).cuda()
    spans = [(0, 40), (30, 70)]
    gs, rs, Ts = [], [], []
    for a, b in spans:
        T = sg.gravity_aligned(w.poses[a])
        s = ctx.submap_create(T)
        ctx.map_sequence(s, dev[a:b], K, w.poses[a:b], esdf_every=0)
        r = orc.Submap(orc.Params(vs=0.1, trunc_vox=4, max_range=10.0, d_max=3.0), T)
        for f in range(a, b):
            r.integrate(fr[f], K, w.poses[f])
        r.update_esdf()
        gs.append(s)
        rs.append(r)
        Ts.append(T)
    pts = rs[1].iso_points()
    assert np.array_equal(ctx.export_points(gs[1]), pts) and len(pts) > 1000
    T_gt = np.linalg.inv(Ts[0]) @ Ts[1]
    rng = np.random.default_rng(12)
    for _ in range(3):
        xi = np.concatenate([rng.uniform(-0.3, 0.3, 3), [0.0, 0.0, rng.uniform(-0.1, 0.1)]])
        T0 = T_gt @ orc.se3_exp(xi)
        Tg, cg, st = ctx.align_submaps(gs[0], gs[1], T0)
        r = orc.align(rs[0], pts, T0)
        assert st["status"] == r["status"] and st["iterations"] == r["iters"] and st["n_used"] == r["n"]
        dt, dr = _pose_err(Tg, r["T"])
        assert dt <= 1e-6 and dr <= 1e-6, (dt, dr)
    # summaries of A on the proposal grid (1 m cells) and of B through T_gt
    c = ctx.export_points(gs[0]).astype(np.float64).mean(axis=0)
    G = np.eye(4)
    G[:3, 3] = c
    for sm, rsub, T in ((gs[0], rs[0], G), (gs[1], rs[1], np.linalg.inv(T_gt) @ G)):
        out = torch.zeros((32768, 4), dtype=torch.float32, device="cuda")
        ctx.summaries([(sm, T, 1.0, out, 0)])
        g = out.cpu().numpy().astype(np.float64)
        want = orc.summary(rsub, T, 1.0)
        both = (g[:, 1] == 1) & (want[:, 1] == 1)
        assert both.sum() > 300  # a 40-frame submap covers several hundred 1 m cells
        assert np.mean(g[:, 1] != want[:, 1]) < 1e-3  # masks: only cells at voxel-centre planes may differ
        assert np.abs(g[both, 0] - want[both, 0]).max() <= 2e-5
    ctx.close()


def test_frustum_outside_the_key_range_is_rejected(cv):
    """A camera whose frustum leaves the addressable block range (2^20
    blocks per axis) is refused before any launch; the submap is unchanged."""
    import torch
    w = sg.tiny()
    ctx = _ctx(cv)
    s = ctx.submap_create()
    T = np.array(w.poses[0], np.float64).copy()
    T[0, 3] = 0.05 * 8 * (2 ** 20)  # beyond the last block along x
    with pytest.raises(cv.CovoxError) as e:
        ctx.integrate_depth(s, torch.from_numpy(w.frame(0)).cuda(), w.cam.K, T)
    assert e.value.code == cv.EINVAL
    assert ctx.submap_info(s)["n_blocks"] == 0
    ctx.close()


def test_precision_statement_fp16_fp32_vs_fp64(cv):
    """Error of the binary32 and binary16 storage paths against the binary64
    oracle on 60 room frames: max / RMS of |D - D64|, |W - W64| and
    |phi - phi64| over voxels with equal weights, and the number of
    voxel-frame validity decisions that differ from binary64 (pixel-edge and
    truncation ties; they appear as weight differences).  A frame can also
    pick a neighbouring pixel at a rounding tie without changing W, so the
    bounds are on RMS and the 99.9th percentile: binary32 within 1e-4 m;
    binary16 RMS within 5e-4 m and 99.9 % within 2e-3 m (a half-ulp of a
    value in [0.125, 0.25) is 6.1e-5 m, compounded over the stored
    roundings); weights are exact integers below 2048 in binary16."""
    import json
    import os
    import torch
    w = sg.room(n_frames=60)
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    r64 = orc.Submap(_oracle_params(fp64=True))
    for f in range(w.n_frames):
        r64.integrate(fr[f], w.cam.K, w.poses[f])
    r64.update_esdf()
    e64 = r64.export()
    tab64 = {int(k): i for i, k in enumerate(e64["keys"])}
    report = {"workload": "room, first 60 frames 640x480, 5 cm voxels, ESDF 2 m"}
    for name, prec in (("fp32", cv.FP32), ("fp16", cv.FP16)):
        ctx = _ctx(cv, block_capacity=16384, precision=prec)
        s = ctx.submap_create()
        for f in range(w.n_frames):
            ctx.integrate_depth(s, dev[f], w.cam.K, w.poses[f])
        ctx.update_esdf(s)
        g = ctx.export_blocks(s)
        rows = np.array([tab64.get(int(k), -1) for k in g["keys"]])
        both = rows >= 0
        D, W, P = g["D"][both].astype(np.float64), g["W"][both].astype(np.float64), g["phi"][both].astype(np.float64)
        D64, W64, P64 = e64["D"][rows[both]], e64["W"][rows[both]], e64["phi"][rows[both]]
        # voxel-frame validity decisions that differ from binary64 show up as
        # weight differences; compare values where the weights agree
        same = (W > 0) & (W64 > 0) & (W == W64)
        flips = int(np.abs(W - W64).sum())
        m = same & ~np.isnan(P) & ~np.isnan(P64)
        dD, dP = np.abs(D - D64)[same], np.abs(P - P64)[m]
        # phi outside the band is vs sqrt(k), k the squared distance to the
        # nearest site: it can differ from binary64 beyond the binary32
        # rounding of sqrt and scale only within R voxels of a voxel whose
        # site or band membership (or observed state) differs
        vs, R = 0.05, 40
        tau_b = 4 * vs * (1 - 2.0 ** -10)
        Df, Wf, Pf = D.ravel(), W.ravel(), P.ravel()
        D64f, W64f, P64f = D64.ravel(), W64.ravel(), P64.ravel()
        obs, obs64 = Wf > 0, W64f > 0
        site = obs & (np.abs(Df) <= vs)
        site64 = obs64 & (np.abs(D64f) <= vs)
        band = obs & (np.abs(Df) < tau_b)
        band64 = obs64 & (np.abs(D64f) < tau_b)
        flip = (site != site64) | (band != band64) | (obs != obs64)
        bk = orc.unpack_key(g["keys"][both]).reshape(-1, 3)
        lidx = np.arange(512)
        vox = (8 * bk[:, None, :] + np.stack([lidx & 7, (lidx >> 3) & 7, lidx >> 6], axis=1)[None]).reshape(-1, 3)
        out = m.ravel() & ~band & ~band64 & ~flip
        from scipy.ndimage import distance_transform_edt
        lo = vox.min(axis=0)
        grid = np.ones(vox.max(axis=0) - lo + 1, bool)  # False at the flips
        fv = vox[flip] - lo
        grid[fv[:, 0], fv[:, 1], fv[:, 2]] = False
        rel = vox - lo
        if len(fv):  # distance to the nearest flip, in voxels
            far = distance_transform_edt(grid)[rel[:, 0], rel[:, 1], rel[:, 2]] > R
        else:
            far = np.ones(len(vox), bool)
        dPo = np.abs(Pf - P64f)[out & far]
        assert dPo.max(initial=0) <= 5e-7, dPo.max()  # two binary32 ulps at 2 m
        report[name + "_flips"] = {"site_flips": int(np.count_nonzero(site != site64)),
                                   "band_flips": int(np.count_nonzero(band != band64)),
                                   "phi_far_from_flips_max": float(dPo.max(initial=0)),
                                   "phi_near_flips_max": float(np.abs(Pf - P64f)[out & ~far].max(initial=0))}
        report[name] = {"blocks_gpu": int(len(g["keys"])), "blocks_fp64": int(len(e64["keys"])),
                        "blocks_only_gpu": int(np.count_nonzero(~both)), "validity_flips": flips,
                        "voxels_compared": int(same.sum()),
                        "D_max": float(dD.max()), "D_rms": float(np.sqrt((dD ** 2).mean())),
                        "D_p999": float(np.quantile(dD, 0.999)),
                        "phi_max": float(dP.max()), "phi_rms": float(np.sqrt((dP ** 2).mean())),
                        "phi_over_1e-4": int(np.count_nonzero(dP > 1e-4))}
        ctx.close()
    out = os.environ.get("COVOX_REPORT_DIR", tempfile.gettempdir())  # where the statement is written
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "precision_report.json"), "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(report))
    # a frame may pick a neighbouring pixel at a rounding tie without changing
    # W, so the maximum is not a precision measure; bound RMS and 99.9 %
    assert report["fp32"]["D_rms"] <= 1e-4 and report["fp32"]["D_p999"] <= 1e-4
    assert report["fp16"]["D_rms"] <= 5e-4 and report["fp16"]["D_p999"] <= 2e-3
    assert report["fp32"]["validity_flips"] <= 1e-3 * report["fp32"]["voxels_compared"]
