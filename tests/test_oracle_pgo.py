"""Pins of the oracle's submap pose-graph optimisation (Eq. 1, Sec. III-F
backend): factor Jacobians and the registration chain rule against finite
differences, an exact odometry chain recovered, a translation-only graph
against the linear least-squares solution, and registration pulling a
perturbed submap back onto its neighbour."""
import math

import numpy as np
import pytest

import oracle as orc
from oracle import pgo
import scenegen as sg


def test_factor_jacobians_match_finite_differences():
    rng = np.random.default_rng(1)
    for _ in range(20):
        xi = np.r_[rng.normal(size=3), rng.uniform(-2, 2)]
        xj = np.r_[rng.normal(size=3), rng.uniform(-2, 2)]
        z = np.r_[rng.normal(size=3), rng.uniform(-1, 1)]
        if abs(pgo.wrap(xj[3] - xi[3] - z[3])) > 2.5:
            continue  # keep away from the wrap
        e, Ji, Jj = pgo.factor_residual(xi, xj, z)
        h = 1e-6
        for k in range(4):
            d = np.zeros(4)
            d[k] = h
            fi = (pgo.factor_residual(xi + d, xj, z)[0] - pgo.factor_residual(xi - d, xj, z)[0]) / (2 * h)
            fj = (pgo.factor_residual(xi, xj + d, z)[0] - pgo.factor_residual(xi, xj - d, z)[0]) / (2 * h)
            assert np.allclose(fi, Ji[:, k], atol=1e-8) and np.allclose(fj, Jj[:, k], atol=1e-8)


def test_pose_to_twist_is_the_first_order_left_perturbation():
    """T(x + dx) = Exp(M dx) T(x) + O(|dx|^2)."""
    rng = np.random.default_rng(2)
    x = np.r_[rng.normal(size=3) * 3, 0.7]
    M = pgo.pose_to_twist(x[:3])
    for k in range(4):
        dx = np.zeros(4)
        dx[k] = 1e-6
        lhs = (pgo.pose_matrix(x + dx) - pgo.pose_matrix(x - dx)) / 2e-6
        rhs = (orc.se3_exp(M @ dx) @ pgo.pose_matrix(x) - orc.se3_exp(-M @ dx) @ pgo.pose_matrix(x)) / 2e-6
        assert np.allclose(lhs, rhs, atol=1e-7)


def _chain(N, seed, drift_t=0.3, drift_psi=0.05):
    rng = np.random.default_rng(seed)
    x_true = np.zeros((N, 4))
    for k in range(1, N):
        step = np.r_[rng.uniform(1, 2), rng.uniform(-0.5, 0.5), rng.uniform(-0.1, 0.1), rng.uniform(-0.4, 0.4)]
        R = pgo.rz(x_true[k - 1, 3])
        x_true[k, :3] = x_true[k - 1, :3] + R @ step[:3]
        x_true[k, 3] = x_true[k - 1, 3] + step[3]
    x0 = x_true.copy()
    x0[1:, :3] += rng.normal(scale=drift_t, size=(N - 1, 3))
    x0[1:, 3] += rng.normal(scale=drift_psi, size=N - 1)
    return x_true, x0


def _rel(xi, xj):
    Tij = np.linalg.inv(pgo.pose_matrix(xi)) @ pgo.pose_matrix(xj)
    return np.r_[Tij[:3, 3], math.atan2(Tij[1, 0], Tij[0, 0])]


def test_exact_odometry_chain_is_recovered():
    x_true, x0 = _chain(7, 3)
    facs = [dict(i=k, j=k + 1, z=_rel(x_true[k], x_true[k + 1]), sigma=[0.1, 0.1, 0.1, 0.02]) for k in range(6)]
    x, st = pgo.solve([], [], x0, [], facs, max_iter=50, tol_step=1e-12)
    assert st["cost_final"] < 1e-20
    d = x - x_true
    d[:, 3] = [pgo.wrap(a) for a in d[:, 3]]
    assert np.abs(d).max() < 1e-9


def test_translation_graph_is_linear_least_squares():
    """With every yaw held at zero (yaw measurements 0 with sigma 1e-6 rad)
    the translation errors are linear in t: e = t_j - t_i - z_t, so the
    optimum is the weighted linear least-squares solution (submap 0 fixed at
    the origin)."""
    rng = np.random.default_rng(4)
    N = 6
    edges = [(k, k + 1) for k in range(N - 1)] + [(0, 3), (1, 5), (2, 4)]
    sig = {e: rng.uniform(0.05, 0.3) for e in edges}
    z = {e: np.r_[rng.normal(size=3), 0.0] for e in edges}
    facs = [dict(i=i, j=j, z=z[(i, j)], sigma=[sig[(i, j)]] * 3 + [1e-6]) for (i, j) in edges]
    x, _ = pgo.solve([], [], np.zeros((N, 4)), [], facs, max_iter=50, tol_step=1e-13)
    A = np.zeros((3 * len(edges), 3 * (N - 1)))
    b = np.zeros(3 * len(edges))
    for r, (i, j) in enumerate(edges):
        w = 1.0 / sig[(i, j)]
        for a in range(3):
            if j > 0:
                A[3 * r + a, 3 * (j - 1) + a] += w
            if i > 0:
                A[3 * r + a, 3 * (i - 1) + a] -= w
            b[3 * r + a] = w * z[(i, j)][a]
    t = np.linalg.lstsq(A, b, rcond=None)[0].reshape(-1, 3)
    assert np.abs(x[1:, :3] - t).max() < 1e-8
    assert np.abs(x[:, 3]).max() < 1e-9


def _tiny_pair(fp64):
    """Submaps A (frames 0-9) and B (frames 10-19, each frame twice, a few
    shared) of the tiny room, both with the world frame as submap frame, so
    the true relative pose is the identity."""
    w = sg.tiny()
    fr = w.frames()
    p = orc.Params(fp64=fp64)
    A, B = orc.Submap(p), orc.Submap(p)
    for f in range(20):
        for _ in range(2):
            (A if f < 10 else B).integrate(fr[f], w.cam.K, w.poses[f])
    for f in range(0, 20, 5):
        (B if f < 10 else A).integrate(fr[f], w.cam.K, w.poses[f])
    A.update_esdf()
    B.update_esdf()
    return [A, B], [A.iso_points(), B.iso_points()]


def test_registration_gradient_matches_finite_differences():
    """g and the cost of a registration term (binary64 oracle) against
    central differences of F over the pose of the free submap."""
    subs, pts = _tiny_pair(fp64=True)
    x = np.array([[0.0, 0.0, 0.0, 0.0], [0.02, -0.015, 0.01, 0.01]])
    F, g, H = pgo.linearize(subs, pts, x, [(0, 1), (1, 0)], [], 0.05)
    h = 1e-6
    fd = np.zeros(4)
    for k in range(4):
        xp, xm = x.copy(), x.copy()
        xp[1, k] += h
        xm[1, k] -= h
        fd[k] = (pgo.linearize(subs, pts, xp, [(0, 1), (1, 0)], [], 0.05)[0]
                 - pgo.linearize(subs, pts, xm, [(0, 1), (1, 0)], [], 0.05)[0]) / (2 * h)
    # F = sum r^2 / sigma^2, so dF/dx = 2 g
    assert np.allclose(fd, 2 * g, rtol=2e-3, atol=1e-3 * np.abs(2 * g).max())
    assert np.all(np.linalg.eigvalsh(H) > 0)


def test_registration_pulls_a_perturbed_submap_back():
    """Two submaps whose true relative pose is the identity, B started 4 cm
    and 1.5 deg off with a weak odometry factor at the wrong pose: the
    optimum lies within 1 cm and 0.1 deg of the truth."""
    subs, pts = _tiny_pair(fp64=False)
    x0 = np.array([[0.0, 0.0, 0.0, 0.0], [0.03, -0.02, 0.015, math.radians(1.5)]])
    fac = [dict(i=0, j=1, z=x0[1], sigma=[1.0, 1.0, 1.0, 1.0])]
    x, st = pgo.solve(subs, pts, x0, [(0, 1), (1, 0)], fac, sigma_reg=0.05, max_iter=30)
    assert st["accepted"] > 0 and st["cost_final"] < st["cost_init"]
    assert np.linalg.norm(x[1, :3]) < 0.01 and abs(math.degrees(x[1, 3])) < 0.1, x[1]
