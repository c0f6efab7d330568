"""Pins of the oracle's correspondence-free ESDF alignment (paper Sec. I and
Sec. III-F, Eq. 1 registration term; registration points chosen by weight;
least squares with residuals and Jacobians).

Checked against: the matrix exponential of the twist (scipy), numpy's
linear solver, central finite differences of the cost, exact recovery of a
lattice-symmetric transform (B is A re-indexed by a 90-degree yaw and an
integer voxel shift, so every residual vanishes at the true pose), closed
forms for isosurface points of a plane and a sphere."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as orc
import scenegen as sg


def _hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0.0]])


@pytest.mark.parametrize("xi", [
    [0.1, -0.2, 0.3, 0.0, 0.0, 0.0],
    [0.1, -0.2, 0.3, 0.4, -0.5, 0.6],
    [1e-3, 2e-3, -1e-3, 1e-5, -2e-5, 3e-6],
    [0.0, 0.0, 0.0, 0.0, 0.0, 2.9],
    [0.5, 0.5, 0.5, 1e-9, 0.0, 0.0],
])
def test_se3_exp_matches_matrix_exponential(xi):
    xi = np.array(xi)
    X = np.zeros((4, 4))
    X[:3, :3] = _hat(xi[3:])
    X[:3, 3] = xi[:3]
    assert np.allclose(orc.se3_exp(xi), scipy.linalg.expm(X), atol=1e-14, rtol=0)


def test_se3_exp_branch_continuity():
    for th in [9.9e-5, 1.0001e-4]:
        xi = np.array([0.3, -0.2, 0.1, th / math.sqrt(3), th / math.sqrt(3), th / math.sqrt(3)])
        X = np.zeros((4, 4))
        X[:3, :3] = _hat(xi[3:])
        X[:3, 3] = xi[:3]
        assert np.allclose(orc.se3_exp(xi), scipy.linalg.expm(X), atol=1e-15, rtol=0)


def test_solve6_against_numpy():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(6, 6))
    H = A @ A.T + 0.1 * np.eye(6)
    b = rng.normal(size=6)
    ne = np.zeros(29)
    m = 0
    for i in range(6):
        for j in range(i, 6):
            ne[m] = H[i, j]
            m += 1
    ne[21:27] = b
    x = orc.solve6(ne)
    assert np.allclose(x, np.linalg.solve(H, -b), rtol=1e-12, atol=1e-12)
    ne[0] = -1.0
    assert orc.solve6(ne) is None


def _smooth_field(params, nb=4):
    """Blocks [0, nb)^3 with D a smooth function inside the band everywhere
    (so phi = D) and W = 3."""
    keys, Ds, Ws = [], [], []
    l = np.arange(512)
    off = np.stack([l & 7, (l >> 3) & 7, l >> 6], axis=1)
    for bx in range(nb):
        for by in range(nb):
            for bz in range(nb):
                keys.append(orc.pack_key(bx, by, bz))
                c = (8 * np.array([bx, by, bz]) + off + 0.5) * params.vs
                Ds.append(0.1 * np.sin(3.1 * c[:, 0] + 0.4) * np.cos(2.3 * c[:, 1] - 0.2) + 0.05 * c[:, 2] - 0.04)
                Ws.append(np.full(512, 3.0))
    s = orc.Submap(params)
    s.import_blocks(np.array(keys, np.uint64), np.stack(Ds), np.stack(Ws))
    s.update_esdf()
    return s


def test_jacobian_matches_central_differences():
    """d c / d xi_k = 2 r J_k = 2 b_k for a single point, with c = r^2
    evaluated at Exp(+-eps e_k) T (left perturbation), binary64 mode."""
    params = orc.Params(vs=0.05, fp64=True)
    A = _smooth_field(params)
    T = orc.se3_exp(np.array([0.01, -0.02, 0.015, 0.02, -0.01, 0.03]))
    rng = np.random.default_rng(5)
    tested = 0
    for _ in range(40):
        p = rng.uniform(0.4, 1.2, size=3)
        q = T[:3, :3] @ p + T[:3, 3]
        frac = q / 0.05 - 0.5 - np.floor(q / 0.05 - 0.5)
        if np.any(frac < 0.1) or np.any(frac > 0.9):
            continue
        H, b, c, n, _ = orc.normal_eq(A, p[None], T)
        assert n == 1
        assert np.allclose(H, np.outer(b, b) / c, rtol=1e-9, atol=1e-12)
        eps = 1e-6
        for k in range(6):
            e = np.zeros(6)
            e[k] = eps
            cp = orc.normal_eq(A, p[None], orc.se3_exp(e) @ T)[2]
            cm = orc.normal_eq(A, p[None], orc.se3_exp(-e) @ T)[2]
            fd = (cp - cm) / (2 * eps)
            assert abs(fd - 2 * b[k]) <= 1e-6 * max(1.0, abs(2 * b[k])), (k, fd, 2 * b[k])
        tested += 1
    assert tested >= 5


def _tiny_field():
    w = sg.tiny()
    s = orc.Submap(orc.Params())
    for f in range(w.n_frames):
        s.integrate(w.frame(f), w.cam.K, w.poses[f])
    return s.export()


@pytest.fixture(scope="module")
def tiny_export():
    return _tiny_field()


def lattice_transform(exp, k90, shift):
    """Re-index A's voxels by a k * 90 degree yaw and an integer voxel shift.
    Returns B's (keys, D, W) and T_BA, which maps A coordinates to B
    coordinates: x_B = Rz(k pi / 2) x_A + shift * vs, i.e. voxel centres map
    onto voxel centres."""
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    D = exp["D"].reshape(-1)
    W = exp["W"].reshape(-1)
    m = W > 0
    c = coords[m] + 0.5
    Rk = np.round(sg.rot_z(k90 * math.pi / 2)).astype(np.int64)
    cb = (c @ Rk.T.astype(np.float64)) - 0.5 + np.array(shift)
    ib = np.round(cb).astype(np.int64)
    bk = np.floor_divide(ib, 8)
    keys = np.unique(orc.pack_key(bk[:, 0], bk[:, 1], bk[:, 2]))
    pos = {int(k): j for j, k in enumerate(keys)}
    Db = np.zeros((len(keys), 512))
    Wb = np.zeros((len(keys), 512))
    kk = orc.pack_key(bk[:, 0], bk[:, 1], bk[:, 2])
    lin = (ib[:, 0] & 7) + 8 * (ib[:, 1] & 7) + 64 * (ib[:, 2] & 7)
    rows = np.array([pos[int(k)] for k in kk])
    Db[rows, lin] = D[m]
    Wb[rows, lin] = W[m]
    T_BA = np.eye(4)
    T_BA[:3, :3] = Rk
    T_BA[:3, 3] = np.array(shift) * 0.05
    return keys, Db, Wb, T_BA


@pytest.mark.parametrize("fp64", [False, True])
def test_lattice_symmetric_residuals_vanish_and_pose_is_recovered(tiny_export, fp64):
    params = orc.Params(fp64=fp64)
    A = orc.Submap(params)
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    keys, Db, Wb, T_BA = lattice_transform(tiny_export, 1, (13, -7, 5))
    B = orc.Submap(params)
    B.import_blocks(keys, Db, Wb)
    pts = B.iso_points()
    assert len(pts) > 5000
    T_true = np.linalg.inv(T_BA)
    H, b, c, n, _ = orc.normal_eq(A, pts, T_true)
    assert n > 0.9 * len(pts)
    assert c / n < (1e-28 if fp64 else 1e-12)
    assert np.all(np.linalg.eigvalsh(H) > -1e-9 * np.abs(H).max())
    dT = orc.se3_exp(np.array([0.02, -0.015, 0.01, 0.01, -0.008, 0.02]))
    r = orc.align(A, pts, dT @ T_true)
    assert r["status"] == orc.OK
    err_t = np.linalg.norm(r["T"][:3, 3] - T_true[:3, 3])
    R_err = r["T"][:3, :3] @ T_true[:3, :3].T
    err_r = math.acos(min(1.0, (np.trace(R_err) - 1) / 2))
    bound = 1e-9 if fp64 else 1e-6
    assert err_t < bound and err_r < bound, (err_t, err_r)


def test_identity_pair_has_zero_cost(tiny_export):
    A = orc.Submap(orc.Params())
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    pts = A.iso_points()
    H, b, c, n, _ = orc.normal_eq(A, pts, np.eye(4))
    assert n > 0.9 * len(pts) and c / n < 1e-12


def test_multistart_recovers_a_quarter_turn(tiny_export):
    """Starting 90 degrees off in yaw about the points' centroid, one of the
    eight starts lands on the truth and has the least cost."""
    params = orc.Params()
    A = orc.Submap(params)
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    keys, Db, Wb, T_BA = lattice_transform(tiny_export, 3, (4, 9, -2))
    B = orc.Submap(params)
    B.import_blocks(keys, Db, Wb)
    pts = B.iso_points()
    T_true = np.linalg.inv(T_BA)
    pbar = pts.astype(np.float64).mean(axis=0)
    P = np.eye(4); P[:3, 3] = pbar
    Pm = np.eye(4); Pm[:3, 3] = -pbar
    Rz = np.eye(4); Rz[:3, :3] = sg.rot_z(math.pi / 2)
    T_init = T_true @ P @ Rz @ Pm  # start k = 6 (3 pi / 2) undoes this
    single = orc.align(A, pts, T_init)
    assert np.linalg.norm(single["T"][:3, 3] - T_true[:3, 3]) > 0.01
    r = orc.align_multistart(A, pts, T_init, 8)
    assert r["best"] in (5, 6, 7)  # starts within 45 degrees of the truth
    assert np.linalg.norm(r["T"][:3, 3] - T_true[:3, 3]) < 1e-6


def test_degenerate_when_too_few_points(tiny_export):
    A = orc.Submap(orc.Params())
    A.import_blocks(tiny_export["keys"], tiny_export["D"], tiny_export["W"])
    A.update_esdf()
    pts = A.iso_points()[:50]
    r = orc.align(A, pts, np.eye(4))
    assert r["status"] == orc.EDEGENERATE and r["iters"] == 0
    assert np.array_equal(r["T"], np.eye(4))


def test_iso_points_of_a_plane():
    """Integrating a constant-depth frame twice from the identity pose gives
    a linear D along z near the plane; its zero crossings sit at z0."""
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    s = orc.Submap(orc.Params())
    z0 = 0.8731
    for _ in range(2):
        s.integrate(np.full((12, 16), z0, np.float32), K, np.eye(4))
    pts = s.iso_points()
    assert len(pts) > 50
    assert np.all(np.abs(pts[:, 2] - z0) < 1e-6)


def test_iso_points_of_a_sphere():
    scene = sg.Scene(spheres=np.array([[0.0, 0.0, 2.0, 0.6]]))
    cam = sg.Camera(H=120, W=160, fx=120.0, fy=120.0, cx=80.0, cy=60.0, max_range=5.0)
    s = orc.Submap(orc.Params())
    for k in range(5):
        T = sg.look_at([0.2 * math.cos(k), 0.2 * math.sin(k) - 1e-3, 0.0], [0.0, 0.0, 2.0], up=(0, -1, 0))
        s.integrate(sg.render(scene, cam, T, 0, k), cam.K, T)
    pts = s.iso_points().astype(np.float64)
    e = np.abs(np.linalg.norm(pts - np.array([0, 0, 2.0]), axis=1) - 0.6)
    assert len(pts) > 500
    assert np.median(e) < 0.01 and e.max() < 0.05
