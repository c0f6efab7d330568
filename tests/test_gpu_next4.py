"""GPU parity of the sensor-dependent observation weights (w = 1 / d^2) and
of the 4-DoF alignment (translation and yaw), through the C ABI against
the oracle on the same seeded inputs: D and W bit for bit (per-frame calls
and frame batches, binary32 and binary16 storage), phi within 1e-4 m, poses
within 1e-6, and the 4-DoF update keeping the gravity row of the rotation
bit for bit."""
import math

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


def _pose_err(T1, T2):
    dt = np.linalg.norm(T1[:3, 3] - T2[:3, 3])
    c = (np.trace(T1[:3, :3] @ T2[:3, :3].T) - 1) / 2
    return dt, math.acos(max(-1.0, min(1.0, c)))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_inverse_depth_weights_parity(cv, precision):
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    fp16 = precision == "fp16"
    ctx = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192,
                     precision=cv.FP16 if fp16 else cv.FP32, weight_mode=cv.WEIGHT_INV_DEPTH2)
    a, b = ctx.submap_create(), ctx.submap_create()
    for f in range(w.n_frames):
        ctx.integrate_depth(a, dev[f], w.cam.K, w.poses[f])
    ctx.integrate_depth_batch(b, dev, w.cam.K, w.poses)
    ref = orc.Submap(orc.Params(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, fp16=fp16, weight_mode=1))
    for f in range(w.n_frames):
        ref.integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(a)
    ref.update_esdf()
    r = ref.export()
    ea, eb = ctx.export_blocks(a), ctx.export_blocks(b)
    for e in (ea, eb):
        assert np.array_equal(e["keys"], r["keys"])
        assert np.array_equal(e["D"], r["D"].astype(np.float32))
        assert np.array_equal(e["W"], r["W"].astype(np.float32))
    W = ea["W"][ea["W"] > 0]
    assert W.min() < 0.5 and not np.all(W == np.round(W))  # weights 1 / d^2, not counts
    m = ~np.isnan(r["phi"])
    assert np.array_equal(np.isnan(ea["phi"]), ~m)
    assert np.abs(ea["phi"][m] - r["phi"][m]).max() <= 1e-4
    ctx.close()


def _tiny_pair(cv, ctx, params):
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    A, B = ctx.submap_create(), ctx.submap_create()
    rA, rB = orc.Submap(params), orc.Submap(params)
    for f in range(20):
        for _ in range(2):
            ctx.integrate_depth(A if f < 10 else B, dev[f], w.cam.K, w.poses[f])
            (rA if f < 10 else rB).integrate(fr[f], w.cam.K, w.poses[f])
    for f in range(20):
        if f % 5 == 0:
            ctx.integrate_depth(B if f < 10 else A, dev[f], w.cam.K, w.poses[f])
            (rB if f < 10 else rA).integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(A)
    ctx.update_esdf(B)
    rA.update_esdf()
    rB.update_esdf()
    return A, B, rA, rB


def test_four_dof_alignment_parity(cv):
    ctx = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192, align_dof=4)
    A, B, rA, rB = _tiny_pair(cv, ctx, orc.Params(align_dof=4))
    pts = rB.iso_points()
    tilt = orc.se3_exp(np.array([0.0, 0.0, 0.0, 0.004, -0.003, 0.0]))
    for xi in ([0.03, -0.02, 0.01, 0.0, 0.0, 0.03], [-0.05, 0.04, 0.0, 0.0, 0.0, 0.08]):
        T0 = orc.se3_exp(np.array(xi)) @ tilt
        Tg, cg, st = ctx.align_submaps(A, B, T0)
        r = orc.align(rA, pts, T0)
        assert st["status"] == r["status"] and st["iterations"] == r["iters"] and st["n_used"] == r["n"]
        dt, dr = _pose_err(Tg, r["T"])
        assert dt <= 1e-6 and dr <= 1e-6, (dt, dr)
        assert np.array_equal(Tg[2, :3], T0[2, :3])  # gravity row untouched
    T0 = orc.se3_exp(np.array([0.02, 0.01, -0.01, 0.0, 0.0, 0.5]))
    Tm, cm, sm = ctx.align_multistart(A, B, T0, 8)
    rm = orc.align_multistart(rA, pts, T0, 8)
    assert sm["best_start"] == rm["best"]
    dt, dr = _pose_err(Tm, rm["T"])
    assert dt <= 1e-6 and dr <= 1e-6
    # switching the same context back to 6 DoF gives the 6-DoF result
    ctx.set_params(align_dof=6)
    T6, c6, s6 = ctx.align_submaps(A, B, T0)
    rA6 = orc.Submap(orc.Params())
    e = rA.export()
    rA6.import_blocks(e["keys"], e["D"], e["W"])
    rA6.update_esdf()
    r6 = orc.align(rA6, pts, T0)
    dt, dr = _pose_err(T6, r6["T"])
    assert s6["iterations"] == r6["iters"] and dt <= 1e-6 and dr <= 1e-6
    with pytest.raises(cv.CovoxError):
        ctx.set_params(voxel_size=0.1)
    ctx.close()
