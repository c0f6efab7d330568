"""Pins of the oracle's 4-DoF alignment (translation and yaw, Sec. III-F:
submap poses in R^3 x SO(2)) and sensor-dependent observation weights
(Sec. III-C: weights following the sensor's performance curve; here
w = 1 / d^2)."""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg
from test_oracle_align import lattice_transform, tiny_export  # noqa: F401  (fixture)


def _pair(tiny_export, params, k90, shift):
    A = orc.Submap(params)
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    keys, Db, Wb, T_BA = lattice_transform(tiny_export, k90, shift)
    B = orc.Submap(params)
    B.import_blocks(keys, Db, Wb)
    return A, B.iso_points(), np.linalg.inv(T_BA)


def _yaw_shift(yaw, t):
    T = np.eye(4)
    T[:3, :3] = sg.rot_z(yaw)
    T[:3, 3] = t
    return T


@pytest.mark.parametrize("fp64", [False, True])
def test_four_dof_recovers_a_lattice_transform(tiny_export, fp64):
    A, pts, T_true = _pair(tiny_export, orc.Params(fp64=fp64, align_dof=4), 1, (13, -7, 5))
    T0 = _yaw_shift(0.02, [0.02, -0.015, 0.01]) @ T_true
    r = orc.align(A, pts, T0)
    assert r["status"] == orc.OK
    err_t = np.linalg.norm(r["T"][:3, 3] - T_true[:3, 3])
    R_err = r["T"][:3, :3] @ T_true[:3, :3].T
    err_r = math.acos(min(1.0, (np.trace(R_err) - 1) / 2))
    bound = 1e-9 if fp64 else 1e-6
    assert err_t < bound and err_r < bound, (err_t, err_r)


def test_four_dof_keeps_the_gravity_row(tiny_export):
    """Exp((rho, 0, 0, theta_z)) has third rotation row (0, 0, 1), so every
    4-DoF update leaves the third row of R, the gravity direction, bit for
    bit as in the prior, even when the prior has roll and pitch."""
    A, pts, T_true = _pair(tiny_export, orc.Params(align_dof=4), 1, (13, -7, 5))
    tilt = np.eye(4)
    tilt[:3, :3] = sg.rot_x(0.01) @ sg.rot_y(-0.008)
    T0 = _yaw_shift(0.03, [0.02, 0.01, -0.01]) @ T_true @ tilt
    r = orc.align(A, pts, T0)
    assert r["iters"] > 0
    assert np.array_equal(r["T"][2, :3], T0[2, :3])


def test_one_four_dof_step_solves_the_restricted_system(tiny_export):
    """One iteration: the step is the solution of rows and columns
    (rho_x, rho_y, rho_z, theta_z) of the 6-DoF normal equations."""
    A, pts, T_true = _pair(tiny_export, orc.Params(align_dof=4, max_iter=1), 1, (13, -7, 5))
    T0 = _yaw_shift(0.03, [0.03, -0.02, 0.015]) @ T_true
    H, b, c, n, _ = orc.normal_eq(A, pts, T0)
    sel = [0, 1, 2, 5]
    x = np.linalg.solve(H[np.ix_(sel, sel)], -b[sel])
    xi = np.zeros(6)
    xi[sel] = x
    want = orc.se3_exp(xi) @ T0
    r = orc.align(A, pts, T0)
    assert r["iters"] == 1
    assert np.allclose(r["T"], want, rtol=0, atol=1e-12)


def _flat_depth(Z, H=12, W=16):
    return np.full((H, W), Z, np.float32)


@pytest.mark.parametrize("fp64", [False, True])
def test_inverse_square_weights_give_the_weighted_mean(fp64):
    """Two constant-depth frames (Z1, Z2) from one camera looking along +z:
    every voxel valid in both holds D = (t1 / Z1^2 + t2 / Z2^2) / (1 / Z1^2 +
    1 / Z2^2) with t = min(Z - z, tau), and W = 1 / Z1^2 + 1 / Z2^2; with
    constant weights D is the plain mean and W = 2."""
    K = np.array([10.0, 10.0, 7.5, 5.5], np.float32)
    T = np.eye(4)
    Z1, Z2 = float(np.float32(1.03)), float(np.float32(1.61))  # the depth images are binary32
    for mode in (0, 1):
        s = orc.Submap(orc.Params(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, fp64=fp64, weight_mode=mode))
        s.integrate(_flat_depth(Z1), K, T)
        s.integrate(_flat_depth(Z2), K, T)
        e = s.export()
        W = np.asarray(e["W"]).reshape(-1)
        D = np.asarray(e["D"]).reshape(-1)
        c = orc.voxel_coords(e["keys"]).reshape(-1, 3)
        z = (c[:, 2] + 0.5) * 0.05
        tau = 0.2
        both = W > (1.5 if mode == 0 else 0.0)
        if mode == 1:
            w1, w2 = 1 / Z1 ** 2, 1 / Z2 ** 2
            both = np.abs(W - (w1 + w2)) < 1e-6 * (w1 + w2)
        assert both.sum() > 50
        t1 = np.minimum(Z1 - z[both], tau)
        t2 = np.minimum(Z2 - z[both], tau)
        if mode == 0:
            want_D, want_W = (t1 + t2) / 2, 2.0
        else:
            want_D, want_W = (t1 * w1 + t2 * w2) / (w1 + w2), w1 + w2
        tol = 1e-12 if fp64 else 2e-6
        assert np.allclose(D[both], want_D, rtol=0, atol=tol)
        assert np.allclose(W[both], want_W, rtol=tol, atol=0)
