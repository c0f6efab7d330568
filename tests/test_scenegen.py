"""Input generator checks: the renderer against analytic intersections, the
noise model's statistics and the counter-based generator's published
known-answer vectors."""
import math
import os

import numpy as np
import pytest

import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, rhs = line.split(":")
        rows.append(([int(x, 16) for x in lhs.split()], [int(x, 16) for x in rhs.split()]))
    return rows


def test_philox_known_answers():
    for lhs, rhs in _kat("philox4x32_10_kat.txt"):
        assert sg.philox4x32_10(lhs[:4], lhs[4:]) == rhs


def test_wall_depth_is_exact():
    # a fronto-parallel wall at z0: every pixel sees depth z0 (no noise)
    scene, cam = sg.wall_scene(1.37, H=24, W=32, f=20.0)
    d = sg.render(scene, cam, np.eye(4), seed=0, frame=0)
    assert np.all(d == np.float32(1.37))


def test_sphere_centre_pixel():
    scene = sg.Scene(spheres=np.array([[0.0, 0.0, 3.0, 0.5]]))
    cam = sg.Camera(H=11, W=11, fx=10.0, fy=10.0, cx=5.0, cy=5.0, max_range=10.0)
    d = sg.render(scene, cam, np.eye(4), seed=0, frame=0)
    assert d[5, 5] == np.float32(2.5)
    # off-centre pixel: ray (u, v, 1) hits the sphere at the analytic root
    u, v = (6 - 5.0) / 10.0, (5 - 5.0) / 10.0
    a = u * u + v * v + 1
    b = -2 * 3.0
    c = 9.0 - 0.25
    t = (-b - math.sqrt(b * b - 4 * a * c)) / (2 * a)
    assert abs(float(d[5, 6]) - t) < 1e-6


def test_box_and_range():
    scene = sg.Scene(boxes=np.array([[-1.0, -1.0, 2.0, 1.0, 1.0, 3.0]]))
    cam = sg.Camera(H=5, W=5, fx=2.0, fy=2.0, cx=2.0, cy=2.0, max_range=1.5)
    d = sg.render(scene, cam, np.eye(4), seed=0, frame=0)
    assert np.all(d == 0)  # beyond max range
    cam.max_range = 10.0
    d = sg.render(scene, cam, np.eye(4), seed=0, frame=0)
    assert d[2, 2] == np.float32(2.0)


def test_noise_statistics_and_invalid_fraction():
    scene, cam = sg.wall_scene(2.0, H=200, W=200, f=150.0)
    cam.noise_model, cam.noise_a, cam.invalid_frac = 2, 0.0012, 0.1
    d = sg.render(scene, cam, np.eye(4), seed=2, frame=3)
    valid = d > 0
    n = d.size
    frac_invalid = 1 - valid.mean()
    assert abs(frac_invalid - 0.1) < 3 * math.sqrt(0.1 * 0.9 / n)
    e = d[valid].astype(np.float64) - 2.0
    sigma = 0.0012 * 4.0
    assert abs(e.mean()) < 4 * sigma / math.sqrt(e.size)
    assert abs(e.std() / sigma - 1.0) < 0.02


def test_seed_reproducible_and_frame_dependent():
    w = sg.tiny()
    a = w.frame(3)
    b = w.frame(3)
    c = sg.render(w.scene, w.cam, w.poses[3], w.seed, 4)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_workload_shapes():
    w = sg.tiny()
    assert w.poses.shape == (20, 4, 4) and (w.cam.H, w.cam.W) == (120, 160)
    assert np.allclose(w.poses[:, :3, 3][:, 2], 1.2)
    assert np.allclose(np.linalg.norm(w.poses[:, :2, 3], axis=1), 1.0)
    r = sg.room()
    assert r.poses.shape == (300, 4, 4) and (r.cam.H, r.cam.W) == (480, 640)
    steps = np.linalg.norm(np.diff(r.poses[:, :3, 3], axis=0), axis=1)
    assert np.allclose(steps, 0.01, atol=2e-4)
    for T in r.poses:  # rotations are proper
        assert np.allclose(T[:3, :3] @ T[:3, :3].T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(T[:3, :3]) - 1) < 1e-12
