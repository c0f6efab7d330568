"""Pins of the oracle's Levenberg-Marquardt alignment mode (the trust-region
least squares Sec. III-F names for the backend, applied to one submap pair;
gain-ratio damping of Madsen, Nielsen and Tingleff).

Checked against: numpy's linear solver for the damped step; exact recovery
of a lattice-symmetric transform (every residual vanishes at the truth); the
Gauss-Newton minimum from the same starts (both methods minimise the same
cost); the method's own invariants: a taken step lowers the mean cost, a
rejected one leaves pose and cost unchanged, so the cost never rises as the
solve cap grows; the 4-DoF step keeps the gravity row of the rotation."""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg
from test_oracle_align import lattice_transform, tiny_export  # noqa: F401  (fixture)


def _packed(H, b):
    ne = np.zeros(29)
    m = 0
    for i in range(6):
        for j in range(i, 6):
            ne[m] = H[i, j]
            m += 1
    ne[21:27] = b
    return ne


@pytest.mark.parametrize("mu", [0.0, 1e-4, 0.5, 10.0])
def test_damped_step_against_numpy(mu):
    rng = np.random.default_rng(3)
    A = rng.normal(size=(6, 6))
    H = A @ A.T + 0.1 * np.eye(6)
    b = rng.normal(size=6)
    ne = _packed(H, b)
    Hd = H + mu * np.diag(np.diag(H))
    assert np.allclose(orc.solve6(ne, mu), np.linalg.solve(Hd, -b), rtol=1e-11, atol=1e-12)
    sel = [0, 1, 2, 5]
    H4 = H[np.ix_(sel, sel)]
    x4 = np.linalg.solve(H4 + mu * np.diag(np.diag(H4)), -b[sel])
    d = orc.solve_xyz_yaw(ne, mu)
    assert np.allclose(d[sel], x4, rtol=1e-11, atol=1e-12) and d[3] == 0.0 and d[4] == 0.0
    # a large damping shrinks the step towards the scaled gradient step
    if mu == 10.0:
        g = -b / ((1 + mu) * np.diag(H))
        assert np.linalg.norm(orc.solve6(ne, mu) - g) < 0.5 * np.linalg.norm(g)


def _maps(exp, k90, shift, solver, **kw):
    A = orc.Submap(orc.Params(align_solver=solver, **kw))
    A.import_blocks(exp["keys"], exp["D"], exp["W"])
    A.update_esdf()
    keys, Db, Wb, T_BA = lattice_transform(exp, k90, shift)
    B = orc.Submap(orc.Params(**kw))
    B.import_blocks(keys, Db, Wb)
    return A, B.iso_points(), np.linalg.inv(T_BA)


def _err(T, T_true):
    et = np.linalg.norm(T[:3, 3] - T_true[:3, 3])
    c = (np.trace(T[:3, :3] @ T_true[:3, :3].T) - 1) / 2
    return et, math.acos(max(-1.0, min(1.0, c)))


def _about_centroid(T, pts, yaw, shift=(0.0, 0.0, 0.0)):
    pbar = pts.astype(np.float64).mean(axis=0)
    P = np.eye(4); P[:3, 3] = pbar
    Pm = np.eye(4); Pm[:3, 3] = -pbar
    Rz = np.eye(4); Rz[:3, :3] = sg.rot_z(math.radians(yaw))
    S = np.eye(4); S[:3, 3] = shift
    return S @ T @ P @ Rz @ Pm


@pytest.mark.parametrize("fp64", [False, True])
def test_lm_recovers_a_lattice_symmetric_transform(tiny_export, fp64):  # noqa: F811
    A, pts, T_true = _maps(tiny_export, 1, (13, -7, 5), 1, fp64=fp64)
    dT = orc.se3_exp(np.array([0.02, -0.015, 0.01, 0.01, -0.008, 0.02]))
    r = orc.align(A, pts, dT @ T_true)
    assert r["status"] == orc.OK and r["iters"] > 0
    et, er = _err(r["T"], T_true)
    bound = 1e-9 if fp64 else 1e-6
    assert et < bound and er < bound, (et, er)
    # started at the truth, the first step is below the tolerances: no step taken
    r0 = orc.align(A, pts, T_true)
    assert r0["status"] == orc.OK and r0["iters"] == 0 and np.array_equal(r0["T"], T_true)


def test_lm_reaches_the_gauss_newton_minimum(tiny_export):  # noqa: F811
    A_lm, pts, T_true = _maps(tiny_export, 1, (13, -7, 5), 1)
    A_gn, _, _ = _maps(tiny_export, 1, (13, -7, 5), 0)
    for yaw, tr in ((0, 0.1), (10, 0.0), (20, 0.3), (40, 0.1)):
        T0 = _about_centroid(T_true, pts, yaw, (tr, -tr, tr / 2))
        g = orc.align(A_gn, pts, T0)
        m = orc.align(A_lm, pts, T0)
        assert g["status"] == orc.OK and m["status"] == orc.OK
        et, er = _err(m["T"], g["T"])
        assert et < 1e-6 and er < 1e-6, (yaw, et, er)
        assert _err(m["T"], T_true)[0] < 1e-6
        # the damping fades on a well-conditioned bowl: no more steps than Gauss-Newton
        assert m["iters"] <= g["iters"], (yaw, m["iters"], g["iters"])


def test_lm_cost_never_rises_and_a_rejected_step_changes_nothing(tiny_pair):
    """From a 150-degree start on two different scans the solve meets
    rejected steps on its way to a local minimum.  Growing the solve cap one
    at a time replays the same path: each extra solve either takes a step
    (the mean cost falls) or rejects it (pose and cost stay bit for bit)."""
    A, _, pts, kw = tiny_pair
    T0 = _about_centroid(np.eye(4), pts, 150)
    prev = None
    rejected = taken = 0
    for cap in range(0, 61):
        A.set_solver(orc.Params(align_solver=1, max_iter=cap, **kw))
        r = orc.align(A, pts, T0)
        assert r["solves"] <= cap
        if cap == 0:
            assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 0 and np.array_equal(r["T"], T0)
        else:
            if r["status"] == orc.OK:
                break
            if r["iters"] == prev["iters"]:
                rejected += 1
                assert np.array_equal(r["T"], prev["T"]) and r["cost"] == prev["cost"]
            else:
                taken += 1
                assert r["iters"] == prev["iters"] + 1 and r["cost"] < prev["cost"]
        prev = r
    assert rejected >= 5 and taken >= 5, (rejected, taken)


def test_lm_degenerate_when_too_few_points(tiny_export):  # noqa: F811
    A = orc.Submap(orc.Params(align_solver=1))
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    pts = A.iso_points()[:50]
    r = orc.align(A, pts, np.eye(4))
    assert r["status"] == orc.EDEGENERATE and r["iters"] == 0
    assert np.array_equal(r["T"], np.eye(4))


def test_lm_four_dof_keeps_gravity_and_meets_gauss_newton(tiny_export):  # noqa: F811
    A_lm, pts, T_true = _maps(tiny_export, 1, (13, -7, 5), 1, align_dof=4)
    A_gn, _, _ = _maps(tiny_export, 1, (13, -7, 5), 0, align_dof=4)
    T0 = _about_centroid(T_true, pts, 15, (0.05, -0.04, 0.02))
    m = orc.align(A_lm, pts, T0)
    g = orc.align(A_gn, pts, T0)
    assert m["status"] == orc.OK and g["status"] == orc.OK
    assert np.array_equal(m["T"][2, :3], T0[2, :3])
    et, er = _err(m["T"], g["T"])
    assert et < 1e-6 and er < 1e-6
    assert _err(m["T"], T_true)[0] < 1e-6


@pytest.fixture(scope="module")
def tiny_pair():
    """A: frames 0-9 of the tiny room (each twice) and every fifth frame of
    10-19; B the other way round; the true transform is the identity and the
    residuals do not vanish there (two different scans)."""
    w = sg.tiny()
    fr = w.frames()
    kw = dict(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0)
    A, B = orc.Submap(orc.Params(**kw)), orc.Submap(orc.Params(**kw))
    for f in range(20):
        for _ in range(2):
            (A if f < 10 else B).integrate(fr[f], w.cam.K, w.poses[f])
    for f in range(0, 20, 5):
        (B if f < 10 else A).integrate(fr[f], w.cam.K, w.poses[f])
    A.update_esdf()
    B.update_esdf()
    e = A.export()
    A64 = orc.Submap(orc.Params(fp64=True, **kw))  # the same TSDF, binary64 ESDF and residuals
    A64.import_blocks(e["keys"], e["D"], e["W"])
    A64.update_esdf()
    return A, A64, B.iso_points(), kw


def _box_radius(keys, vs):
    b = orc.unpack_key(keys).reshape(-1, 3).astype(np.float64)
    lo, hi = 8 * vs * b.min(axis=0), 8 * vs * (b.max(axis=0) + 1)
    return float(np.linalg.norm(np.maximum(np.abs(lo), np.abs(hi))))


def test_lm_noise_floor(tiny_pair):
    """Starts near the optimum of two different scans: binary32 residuals
    leave the cost uncertain by rounding noise, and the solve ends converged
    (the predicted decrease within 2^-19 Q sqrt(c)) inside the solve cap.
    Checked against (a) the cost's actual binary32 rounding error, from the
    binary64 residuals of the same TSDF at the same pose, which the floor's
    bound covers; (b) the binary64 solve (floor 2^-48 Q sqrt(c)) from the same
    start, whose pose it meets to a small fraction of a voxel; (c) solves >=
    steps taken, and Gauss-Newton's solves equal to its updates."""
    A, A64, pts, kw = tiny_pair
    Q = _box_radius(A.export()["keys"], float(np.float32(kw["vs"])))
    for xi in ([0.03, -0.02, 0.01, 0.02, -0.01, 0.03], [-0.05, 0.04, 0.0, 0.0, 0.0, 0.08],
               [0.02, 0.01, -0.01, 0.0, 0.0, 0.5]):
        T0 = orc.se3_exp(np.array(xi))
        A.set_solver(orc.Params(align_solver=1, max_iter=60, **kw))
        A64.set_solver(orc.Params(align_solver=1, fp64=True, max_iter=100, **kw))
        r, r64 = orc.align(A, pts, T0), orc.align(A64, pts, T0)
        assert r["status"] == orc.OK and r64["status"] == orc.OK, (xi, r["status"], r64["status"])
        assert r["iters"] <= r["solves"] < 60
        c32 = orc.normal_eq(A, pts, r["T"])[4]
        c64 = orc.normal_eq(A64, pts, r["T"])[4]
        assert c32[28] == c64[28]
        assert abs(c32[27] - c64[27]) <= 2.0 ** -19 * Q * math.sqrt(c32[27]), (c32[27], c64[27])
        et, er = _err(r["T"], r64["T"])
        assert et < 1e-4 and er < 1e-4, (xi, et, er)
        A.set_solver(orc.Params(align_solver=0, **kw))
        g = orc.align(A, pts, T0)
        assert g["solves"] == g["iters"]
