"""Submap pose-graph optimisation -- TEST INFRASTRUCTURE ONLY (part of the
oracle; used by the tests and nothing else).

Eq. (1) of the paper (Sec. III-F, Backend): the submap poses minimise the sum
of the registration errors of overlapping submaps and of the odometry and
loop-closure errors, solved by Levenberg-Marquardt.  Plain binary64 numpy,
dense normal equations, a Cholesky solve.

Readings (the paper defers the formulation to Voxgraph):
  pose of submap i: x_i = (t_x, t_y, t_z, psi), T_i = [Rz(psi) t; 0 1]
      (R^3 x SO(2): gravity is known); submap 0 is held fixed;
  registration term (i, j): the alignment residuals r = phi_i(T_i^-1 T_j p)
      over the registration points p of submap j, weight 1 / sigma_reg^2;
      its Gauss-Newton blocks come from the 6x6 normal equations of the
      relative pose T_ij = T_i^-1 T_j under the left perturbation
      T_ij <- Exp(xi) T_ij, chained to x_i and x_j;
  odometry / loop term (i, j) with measured z = (z_t, z_psi) of T_i^-1 T_j:
      e_t = Rz(-z_psi) (Rz(-psi_i) (t_j - t_i) - z_t),
      e_psi = wrap(psi_j - psi_i - z_psi), weights 1 / sigma^2;
  F(x) = sum_reg c_ij / sigma_reg^2 + sum_fac e^T Omega e (c = sum r^2);
  LM step: (H + mu diag(H)) delta = -g with H = J^T W J, g = J^T W r; the
      step is taken when the gain ratio (F - F_new) / (-(2 delta.g +
      delta.H.delta)) is positive, and mu follows the update of Madsen,
      Nielsen and Tingleff (Methods for non-linear least squares problems,
      2004): mu *= max(1/3, 1 - (2 rho - 1)^3) after a taken step, else
      mu *= nu, nu *= 2; the iteration stops when max |delta| < tol_step.
"""
from __future__ import annotations

import math

import numpy as np

from . import normal_eq


def rz(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def pose_matrix(x) -> np.ndarray:
    """T = [Rz(psi) t; 0 1] of x = (t_x, t_y, t_z, psi)."""
    T = np.eye(4)
    T[:3, :3] = rz(float(x[3]))
    T[:3, 3] = x[:3]
    return T


def _inv(T):
    R, t = T[:3, :3], T[:3, 3]
    O = np.eye(4)
    O[:3, :3] = R.T
    O[:3, 3] = -R.T @ t
    return O


def _hat(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def adjoint(T) -> np.ndarray:
    """Ad_T for xi = (rho, theta): Exp(Ad_T xi) = T Exp(xi) T^-1."""
    R, t = T[:3, :3], T[:3, 3]
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[:3, 3:] = _hat(t) @ R
    A[3:, 3:] = R
    return A


def pose_to_twist(t) -> np.ndarray:
    """M (6x4): the left perturbation xi = M dx that moves T(x) to T(x + dx)
    to first order: rho = dt - dpsi z x t, theta = dpsi z."""
    M = np.zeros((6, 4))
    M[:3, :3] = np.eye(3)
    M[0, 3], M[1, 3] = t[1], -t[0]
    M[5, 3] = 1.0
    return M


def _ne_to_hb(ne):
    H = np.zeros((6, 6))
    k = 0
    for r in range(6):
        for c in range(r, 6):
            H[r, c] = H[c, r] = ne[k]
            k += 1
    return H, np.array(ne[21:27]), float(ne[27]), int(ne[28])


def wrap(a: float) -> float:
    """Angle in (-pi, pi]."""
    a = math.fmod(a + math.pi, 2.0 * math.pi)
    if a <= 0.0:
        a += 2.0 * math.pi
    return a - math.pi


def factor_residual(xi, xj, z):
    """4-DoF relative-pose error of a factor and its Jacobians (4x4 each)."""
    Q = rz(-float(z[3])) @ rz(-float(xi[3]))
    d = np.asarray(xj[:3], float) - np.asarray(xi[:3], float)
    e = np.zeros(4)
    e[:3] = Q @ d - rz(-float(z[3])) @ np.asarray(z[:3], float)
    e[3] = wrap(float(xj[3]) - float(xi[3]) - float(z[3]))
    Jj = np.zeros((4, 4))
    Ji = np.zeros((4, 4))
    Jj[:3, :3] = Q
    Ji[:3, :3] = -Q
    Ji[:3, 3] = -Q @ (_hat([0.0, 0.0, 1.0]) @ d)
    Jj[3, 3] = 1.0
    Ji[3, 3] = -1.0
    return e, Ji, Jj


def linearize(subs, pts, x, reg_pairs, factors, sigma_reg):
    """F(x), g = J^T W r and H = J^T W J over the free poses 1..N-1 (dense).
    subs: oracle submaps, pts: their registration points, x: (N, 4),
    reg_pairs: (i, j) with the field of i and the points of j, factors:
    dicts with i, j, z (4), sigma (4)."""
    N = len(x)
    n = 4 * (N - 1)
    H = np.zeros((n, n))
    g = np.zeros(n)
    F = 0.0
    w_reg = 1.0 / sigma_reg ** 2

    for (i, j) in reg_pairs:
        Ti, Tj = pose_matrix(x[i]), pose_matrix(x[j])
        Tij = _inv(Ti) @ Tj
        H6, b6, c, _ = _ne_to_hb(normal_eq(subs[i], pts[j], Tij)[4])
        Ad = adjoint(_inv(Ti))
        A = {j: Ad @ pose_to_twist(x[j][:3]), i: -Ad @ pose_to_twist(x[i][:3])}
        F += w_reg * c
        for a in (i, j):
            if a == 0:
                continue
            ra = slice(4 * (a - 1), 4 * a)
            g[ra] += w_reg * (A[a].T @ b6)
            for b in (i, j):
                if b == 0:
                    continue
                H[ra, 4 * (b - 1):4 * b] += w_reg * (A[a].T @ H6 @ A[b])
    for f in factors:
        i, j = f["i"], f["j"]
        e, Ji, Jj = factor_residual(x[i], x[j], f["z"])
        Om = np.diag(1.0 / np.asarray(f["sigma"], float) ** 2)
        F += float(e @ Om @ e)
        J = {i: Ji, j: Jj}
        for a in (i, j):
            if a == 0:
                continue
            ra = slice(4 * (a - 1), 4 * a)
            g[ra] += J[a].T @ Om @ e
            for b in (i, j):
                if b == 0:
                    continue
                H[ra, 4 * (b - 1):4 * b] += J[a].T @ Om @ J[b]
    return F, g, H


def solve(subs, pts, x0, reg_pairs, factors, sigma_reg=0.05, max_iter=20, lambda0=1e-4, tol_step=1e-8):
    """Levenberg-Marquardt on Eq. (1).  Returns the poses (N, 4) and a stats
    dict: iterations (solves), accepted steps, initial and final F,
    converged flag."""
    x = np.array(x0, float).copy()
    F, g, H = linearize(subs, pts, x, reg_pairs, factors, sigma_reg)
    F0 = F
    mu, nu = lambda0, 2.0
    it = acc = 0
    converged = False
    while it < max_iter:
        it += 1
        A = H + mu * np.diag(np.diag(H))
        L = np.linalg.cholesky(A)
        delta = -np.linalg.solve(L.T, np.linalg.solve(L, g))
        if np.max(np.abs(delta)) < tol_step:
            converged = True
            break
        xn = x.copy()
        xn[1:] += delta.reshape(-1, 4)
        Fn, gn, Hn = linearize(subs, pts, xn, reg_pairs, factors, sigma_reg)
        pred = -(2.0 * float(delta @ g) + float(delta @ H @ delta))
        rho = (F - Fn) / pred if pred > 0 else -1.0
        if rho > 0:
            x, F, g, H = xn, Fn, gn, Hn
            acc += 1
            mu *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
        else:
            mu *= nu
            nu *= 2.0
    return x, {"iterations": it, "accepted": acc, "cost_init": F0, "cost_final": F, "converged": converged}
