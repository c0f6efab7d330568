"""Pins of the oracle's projective TSDF integration and block allocation
(paper Sec. III-C projection mapping, Sec. III-D count / allocate / update).

Each check is against something other than the oracle's own formula: an
FP64 brute-force enumeration over a large voxel cube, closed forms for planes
of constant depth, and invariants (idempotence, averaging, frame order)."""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg


def _rot(yaw, pitch, roll):
    return sg.rot_z(yaw) @ sg.rot_y(pitch) @ sg.rot_x(roll)


def _pose(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def _brute_force_valid(T_cs, K, depth, vs, tau, max_range, lo, hi):
    """FP64 projective validity of every voxel of the cube [lo, hi]^3 and the
    distance to each.  Returns (voxel indices, sdf, margin) where margin is
    the distance of the decision from its nearest boundary."""
    H, W = depth.shape
    r = np.arange(lo, hi + 1)
    I = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    c = (I + 0.5) * vs
    p = c @ T_cs[:3, :3].T + T_cs[:3, 3]
    z = p[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = K[0] * p[:, 0] / z + K[2]
        v = K[1] * p[:, 1] / z + K[3]
    ok = z > 0
    uf = np.floor(u + 0.5)
    vf = np.floor(v + 0.5)
    ok &= (uf >= 0) & (uf < W) & (vf >= 0) & (vf < H)
    col = np.where(ok, uf, 0).astype(np.int64)
    row = np.where(ok, vf, 0).astype(np.int64)
    d = depth[row, col].astype(np.float64)
    ok &= (d > 0) & (d <= max_range)
    sdf = d - z
    ok &= sdf >= -tau
    # margin from the pixel-rounding and truncation decisions
    mu = np.minimum(np.abs((u + 0.5) - np.round(u + 0.5)), np.abs((v + 0.5) - np.round(v + 0.5)))
    margin = np.minimum(mu, np.abs(sdf + tau) * 100)
    return I[ok], sdf[ok], I, margin


def _voxel_table(exp):
    """dict voxel index -> (D, W) for observed voxels of an oracle export."""
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    D = exp["D"].reshape(-1)
    W = exp["W"].reshape(-1)
    m = W > 0
    return {tuple(c): (d, w) for c, d, w in zip(coords[m], D[m], W[m])}


@pytest.mark.parametrize("fp64", [False, True])
def test_constant_depth_plane_closed_form(fp64):
    """A depth image of constant z0 is a plane fronto-parallel to the camera:
    D(i) = min(z0 - z_cam(i), tau) for every valid voxel, W = 1, and the
    allocated blocks are exactly those holding a valid voxel of an FP64
    brute-force enumeration over a cube far larger than the frustum."""
    vs, tau, max_range = 0.05, 0.2, 5.0
    H, W = 12, 16
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    T_wc = _pose(_rot(0.7, -0.3, 0.2), [0.31, -0.17, 0.93])
    T_ws = _pose(_rot(-0.4, 0.1, 0.05), [0.11, 0.23, -0.07])
    z0 = 0.83
    depth = np.full((H, W), z0, np.float32)
    s = orc.Submap(orc.Params(vs=vs, trunc_vox=4, max_range=max_range, fp64=fp64), T_ws)
    st = s.integrate(depth, K, T_wc)
    T_cs = np.linalg.inv(T_wc) @ T_ws
    Iv, sdf, _, _ = _brute_force_valid(T_cs, K, depth, vs, tau, max_range, -70, 70)
    # the cube must contain the whole valid set with room to spare
    assert Iv.min() > -70 and Iv.max() < 70
    exp = s.export()
    tab = _voxel_table(exp)
    got = set(tab)
    want = {tuple(x) for x in Iv}
    assert got == want
    assert st["n_valid"] == len(want)
    blocks = {tuple(b) for b in np.floor_divide(Iv, 8)}
    assert {tuple(b) for b in orc.unpack_key(exp["keys"])} == blocks
    for x, sd in zip(map(tuple, Iv), sdf):
        D, Wt = tab[x]
        assert Wt == 1.0
        assert abs(D - min(sd, tau)) < (1e-12 if fp64 else 2e-6)


def test_tiny_workload_matches_fp64_brute_force_blocks():
    """Frame 0 of the tiny workload: the oracle's allocated block set equals
    the blocks of the FP64 brute-force valid set, except for voxels whose
    decision sits within rounding distance of a pixel edge or the
    truncation limit."""
    w = sg.tiny()
    d = w.frame(0)
    s = orc.Submap(orc.Params(vs=0.05, trunc_vox=4, max_range=5.0))
    s.integrate(d, w.cam.K, w.poses[0])
    exp = s.export()
    T_cs = np.linalg.inv(w.poses[0])
    Iv, sdf, Iall, margin = _brute_force_valid(T_cs, w.cam.K, d, 0.05, 0.2, 5.0, -48, 72)
    tab = _voxel_table(exp)
    want = {tuple(x) for x in Iv}
    got = set(tab)
    diff = want.symmetric_difference(got)
    close = {tuple(x) for x in Iall[margin < 1e-4]}
    assert diff <= close, "validity differs away from decision boundaries"
    assert len(diff) <= 3


def test_new_blocks_ascending_key_order_and_indices():
    w = sg.tiny()
    s = orc.Submap(orc.Params())
    prev = np.zeros(0, np.uint64)
    for f in range(6):
        st = s.integrate(w.frame(f), w.cam.K, w.poses[f])
        keys = s.export()["keys"]
        assert np.array_equal(keys[: len(prev)], prev)
        new = keys[len(prev):]
        assert len(new) == st["n_new"]
        assert np.all(np.diff(new.astype(np.uint64)) > 0)
        assert len(np.unique(keys)) == len(keys)
        prev = keys


def test_idempotent_double_integration():
    """(D * 1 + D) / 2 == D exactly, so integrating a frame twice leaves D
    bitwise unchanged and sets W = 2."""
    w = sg.tiny()
    d = w.frame(0)
    s = orc.Submap(orc.Params())
    s.integrate(d, w.cam.K, w.poses[0])
    e1 = s.export()
    s.integrate(d, w.cam.K, w.poses[0])
    e2 = s.export()
    assert np.array_equal(e1["keys"], e2["keys"])
    m = e1["W"] > 0
    assert np.array_equal(e1["D"][m], e2["D"][m])
    assert np.all(e2["W"][m] == 2.0)


def test_average_of_constant_depth_frames():
    """F frames of constant depth z_f from one pose: D is the mean of the
    truncated distances for voxels valid in every frame."""
    vs, tau = 0.05, 0.2
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    T_wc = _pose(_rot(0.2, 0.1, -0.3), [0.05, 0.02, -0.03])
    zs = [0.80, 0.83, 0.79, 0.86, 0.81]
    s = orc.Submap(orc.Params(vs=vs, trunc_vox=4))
    for z in zs:
        s.integrate(np.full((12, 16), z, np.float32), K, T_wc)
    exp = s.export()
    tab = _voxel_table(exp)
    T_cs = np.linalg.inv(T_wc)
    checked = 0
    for x, (D, Wt) in tab.items():
        if Wt != len(zs):
            continue
        zc = (T_cs[:3, :3] @ ((np.array(x) + 0.5) * vs) + T_cs[:3, 3])[2]
        want = np.mean([min(z - zc, tau) for z in zs])
        assert abs(D - want) < 2e-6
        checked += 1
    assert checked > 100


def test_frame_order_invariance_fp64():
    """The update is commutative (Sec. III-D): in binary64 the state after
    the same frames in another order agrees to 1e-12 (keyed by voxel)."""
    w = sg.tiny()
    frames = [w.frame(f) for f in range(5)]
    tabs = []
    for order in ([0, 1, 2, 3, 4], [3, 0, 4, 2, 1]):
        s = orc.Submap(orc.Params(fp64=True))
        for f in order:
            s.integrate(frames[f], w.cam.K, w.poses[f])
        tabs.append(_voxel_table(s.export()))
    assert set(tabs[0]) == set(tabs[1])
    for k, (D, Wt) in tabs[0].items():
        D2, W2 = tabs[1][k]
        assert W2 == Wt
        assert abs(D2 - D) < 1e-12


@pytest.mark.parametrize("bad", [0.0, np.nan, 5.01, np.inf, -1.0])
def test_depth_values_outside_range_are_ignored(bad):
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    s = orc.Submap(orc.Params(max_range=5.0))
    st = s.integrate(np.full((12, 16), bad, np.float32), K, np.eye(4))
    assert s.n_blocks == 0 and st["n_valid"] == 0


def test_truncation_clamp_and_behind_surface():
    """Voxels in front of the surface by more than tau hold +tau; voxels more
    than tau behind are never touched."""
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    s = orc.Submap(orc.Params(vs=0.05, trunc_vox=4))
    s.integrate(np.full((12, 16), 1.0, np.float32), K, np.eye(4))
    tab = _voxel_table(s.export())
    zs = np.array([(k[2] + 0.5) * 0.05 for k in tab])
    Ds = np.array([v[0] for v in tab.values()])
    assert zs.max() <= 1.2 + 1e-9
    assert np.all(Ds[zs < 0.79] == np.float32(0.2))
    assert np.all(Ds >= -0.2 - 1e-7)


def test_fp16_storage_rounds_each_store():
    """binary16 storage: every stored D and W is a binary16 value, and the
    first update of a voxel stores the binary16 rounding of its distance."""
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    d = np.full((12, 16), 0.9137, np.float32)
    s16 = orc.Submap(orc.Params(fp16=True))
    s32 = orc.Submap(orc.Params())
    s16.integrate(d, K, np.eye(4))
    s32.integrate(d, K, np.eye(4))
    e16, e32 = s16.export(), s32.export()
    m = e32["W"] > 0
    assert np.array_equal(e16["D"][m], e32["D"][m].astype(np.float16).astype(np.float64))


def test_binary16_conversion_matches_ieee():
    """The oracle's binary32 -> binary16 rounding equals numpy's IEEE
    round-to-nearest-even conversion, including subnormals, overflow and
    ties; binary16 -> binary32 is exact for every half value."""
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    xs = bits.view(np.float32)
    # add values near every half tie and the subnormal range
    halves = np.arange(0, 2 ** 16, dtype=np.uint32).astype(np.uint16).view(np.float16).astype(np.float32)
    extra = np.concatenate([halves, np.nextafter(halves, np.float32(np.inf)), np.nextafter(halves, np.float32(-np.inf)),
                            (halves[:-1] + halves[1:]) / 2])
    for x in np.concatenate([xs, extra]):
        if np.isnan(x):
            assert np.isnan(orc.h2f(orc.f2h(float(x))))
            continue
        with np.errstate(over="ignore"):
            want = np.float32(x).astype(np.float16).view(np.uint16)
        assert orc.f2h(float(x)) == int(want), x
    for h in range(2 ** 16):
        v = np.uint16(h).view(np.float16).astype(np.float32)
        got = orc.h2f(h)
        assert (np.isnan(v) and math.isnan(got)) or got == v


def test_pose_cam_sub_against_matrix_inverse():
    T_wc = _pose(_rot(0.7, -0.3, 0.2), [0.31, -0.17, 0.93])
    T_ws = _pose(_rot(-0.4, 0.1, 0.05), [0.11, 0.23, -0.07])
    assert np.allclose(orc.pose_cam_sub(T_wc, T_ws), np.linalg.inv(T_wc) @ T_ws, atol=1e-15)


def test_mix64_known_answers():
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_kat.txt")
    n = 0
    for line in open(p):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split(":")
        assert orc.mix64(int(a, 16)) == int(b, 16)
        n += 1
    assert n == 4


def test_packed_key_order_is_lexicographic():
    rng = np.random.default_rng(3)
    b = rng.integers(-1000, 1000, size=(500, 3))
    k = orc.pack_key(b[:, 0], b[:, 1], b[:, 2])
    assert np.array_equal(orc.unpack_key(k), b)
    order_k = np.argsort(k, kind="stable")
    order_lex = np.lexsort((b[:, 2], b[:, 1], b[:, 0]))
    assert np.array_equal(b[order_k], b[order_lex])
