"""Pins of the oracle's raycast integration (Sec. III-C: a ray from the
optical centre through each observed point updates every voxel it crosses up
to the truncation distance behind the point; Sec. III-D: allocate the new
blocks, then merge the frame's contributions per voxel).

The grid walk is checked against a brute-force slab test; the per-voxel
merge against closed forms on single rays along a voxel column; the
paper's "every point counts" against the voxel holding the optical centre,
which every ray of a frame crosses."""
import math

import numpy as np
import pytest

import oracle as orc

VS = 0.05
TAU = 0.2


def _slab(o, u, s0, s1, i, vs):
    """Parameter interval of the segment o + s u, s in [s0, s1], inside the
    closed cube of voxel i (binary64), or None."""
    lo, hi = s0, s1
    for a in range(3):
        b0, b1 = i[a] * vs, (i[a] + 1) * vs
        if u[a] == 0.0:
            if not (b0 <= o[a] <= b1):
                return None
            continue
        t0, t1 = (b0 - o[a]) / u[a], (b1 - o[a]) / u[a]
        if t0 > t1:
            t0, t1 = t1, t0
        lo, hi = max(lo, t0), min(hi, t1)
    return (lo, hi) if lo <= hi else None


def _random_rays(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        o = rng.uniform(-0.3, 0.3, 3).astype(np.float32)
        u = rng.normal(size=3)
        u = (u / np.linalg.norm(u)).astype(np.float32)
        s0 = np.float32(rng.uniform(0.0, 0.2))
        s1 = np.float32(s0 + rng.uniform(0.05, 0.9))
        yield o, u, s0, s1


def test_walk_is_the_set_of_crossed_voxels():
    """Every voxel the segment passes through for more than 1e-6 m is
    walked, every walked voxel is touched by the segment (to 1e-5 m), the
    walk is a face-connected chain, and it is ordered by entry parameter."""
    for o, u, s0, s1 in _random_rays(300, 11):
        walk = orc.ray_walk32(o, u, s0, s1, VS)
        o64, u64 = o.astype(np.float64), u.astype(np.float64)
        got = {tuple(v) for v in walk}
        assert len(got) == len(walk), "a voxel walked twice"
        p0, p1 = o64 + float(s0) * u64, o64 + float(s1) * u64
        lo = np.floor(np.minimum(p0, p1) / VS).astype(int) - 1
        hi = np.floor(np.maximum(p0, p1) / VS).astype(int) + 1
        want = set()
        for x in range(lo[0], hi[0] + 1):
            for y in range(lo[1], hi[1] + 1):
                for z in range(lo[2], hi[2] + 1):
                    iv = _slab(o64, u64, float(s0), float(s1), (x, y, z), VS)
                    if iv and iv[1] - iv[0] > 1e-6:
                        want.add((x, y, z))
        assert want <= got, sorted(want - got)
        entries = []
        for v in walk:
            iv = _slab(o64, u64, float(s0) - 1e-5, float(s1) + 1e-5, v, VS + 0.0)
            assert iv is not None, ("walked voxel not on the segment", v)
            entries.append(iv[0])
        assert np.all(np.diff(entries) >= -1e-6)
        steps = np.abs(np.diff(walk, axis=0)).sum(axis=1)
        assert np.all(steps == 1), "consecutive voxels must share a face"


def test_walk_along_an_axis():
    """A ray along +z from inside voxel (0, 0, 0) crosses exactly the column
    voxels k = 0 .. floor((o_z + s1) / vs)."""
    o = np.array([0.012, 0.013, 0.007], np.float32)
    u = np.array([0.0, 0.0, 1.0], np.float32)
    walk = orc.ray_walk32(o, u, 0.0, 1.2, VS)
    last = int(math.floor((0.007 + 1.2) / VS))
    assert np.array_equal(walk, np.array([[0, 0, k] for k in range(last + 1)]))
    walk = orc.ray_walk32(o, -u, 0.0, 0.3, VS)  # and along -z
    assert np.array_equal(walk, np.array([[0, 0, -k] for k in range(int(math.floor((0.3 - 0.007) / VS)) + 2)]))


def _one_ray_frame(Z, o, fp64=False, carve=True, mode=0):
    """A 1x1 depth image whose only ray runs along +z from o to depth Z."""
    s = orc.Submap(orc.Params(vs=VS, trunc_vox=4, max_range=5.0, d_max=2.0, fp64=fp64, integrator=1,
                              ray_carve=carve, weight_mode=mode))
    T = np.eye(4)
    T[:3, 3] = o
    st = s.integrate(np.full((1, 1), Z, np.float32), np.array([10.0, 10.0, 0.0, 0.0], np.float32), T)
    return s, st


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("carve", [True, False])
def test_single_ray_closed_form(fp64, carve):
    """Voxel k of the column gets sdf = Z - (c_k - o_z) once, clamped to tau,
    for every voxel from the start of the segment (the optical centre, or
    tau before the point) to the last one with sdf >= -tau."""
    o = (0.012, 0.013, 0.007)
    Z = float(np.float32(1.03))
    s, st = _one_ray_frame(Z, o, fp64=fp64, carve=carve)
    e = s.export()
    c = orc.voxel_coords(e["keys"]).reshape(-1, 3)
    W = e["W"].reshape(-1)
    D = e["D"].reshape(-1)
    hit = W > 0
    assert np.all(W[hit] == 1.0)
    assert np.all(c[hit][:, 0] == 0) and np.all(c[hit][:, 1] == 0)
    k = np.sort(c[hit][:, 2])
    zc = (k + 0.5) * VS
    sdf = Z - (zc - o[2])
    k0 = 0 if carve else int(math.floor((o[2] + Z - TAU) / VS))
    kend = int(math.floor((o[2] + Z + TAU) / VS))
    want_k = [q for q in range(k0, kend + 1) if Z - ((q + 0.5) * VS - o[2]) >= -TAU]
    assert list(k) == want_k
    order = np.argsort(c[hit][:, 2])
    tol = 1e-12 if fp64 else 1e-6
    assert np.allclose(D[hit][order], np.minimum(sdf, TAU), rtol=0, atol=tol)
    assert st["n_valid"] == len(want_k) and st["n_voxels"] == len(want_k)


@pytest.mark.parametrize("fp64", [False, True])
def test_two_frames_weighted_mean(fp64):
    """Two single-ray frames at depths Z1 and Z2 along the same line: every
    voxel both reach holds D = sum(t w) / sum(w) with w = 1 or 1 / Z^2."""
    o = (0.012, 0.013, 0.007)
    Z1, Z2 = float(np.float32(1.03)), float(np.float32(1.61))
    K = np.array([10.0, 10.0, 0.0, 0.0], np.float32)
    T = np.eye(4)
    T[:3, 3] = o
    for mode in (0, 1):
        s = orc.Submap(orc.Params(vs=VS, fp64=fp64, integrator=1, weight_mode=mode))
        s.integrate(np.full((1, 1), Z1, np.float32), K, T)
        s.integrate(np.full((1, 1), Z2, np.float32), K, T)
        e = s.export()
        c = orc.voxel_coords(e["keys"]).reshape(-1, 3)
        W, D = e["W"].reshape(-1), e["D"].reshape(-1)
        w1, w2 = (1.0, 1.0) if mode == 0 else (1 / Z1 ** 2, 1 / Z2 ** 2)
        zc = (c[:, 2] + 0.5) * VS - o[2]
        both = (Z1 - zc >= -TAU) & (W > 0)
        assert both.sum() > 15
        t1, t2 = np.minimum(Z1 - zc[both], TAU), np.minimum(Z2 - zc[both], TAU)
        tol = 1e-12 if fp64 else 2e-6
        assert np.allclose(W[both], w1 + w2, rtol=tol, atol=0)
        assert np.allclose(D[both], (t1 * w1 + t2 * w2) / (w1 + w2), rtol=0, atol=tol)


def test_every_point_counts_at_the_optical_centre():
    """All rays of a frame start in the voxel holding the optical centre, so
    with weight 1 it gains exactly one weight per valid pixel (here all but
    the invalid ones), at distance tau."""
    rng = np.random.default_rng(5)
    depth = rng.uniform(0.6, 3.0, (12, 16)).astype(np.float32)
    depth[3, 4] = 0.0
    depth[7, 9] = 9.0  # beyond max_range
    depth[5, 5] = np.nan
    K = np.array([12.0, 12.0, 7.5, 5.5], np.float32)
    T = np.eye(4)
    T[:3, :3] = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])  # camera looks along +x
    T[:3, 3] = (0.021, 0.033, 0.017)
    s = orc.Submap(orc.Params(vs=VS, integrator=1))
    s.integrate(depth, K, T)
    e = s.export()
    keys = e["keys"]
    bk = orc.pack_key(0, 0, 0)
    b = int(np.nonzero(keys == bk)[0][0])
    lin = 0 + 8 * 0 + 64 * 0
    assert e["W"][b, lin] == 16 * 12 - 3
    assert e["D"][b, lin] == np.float32(TAU)


def test_blocks_new_in_key_order_and_never_empty():
    """After one frame on an empty submap every allocated block holds an
    observed voxel, and buffer indices follow ascending packed keys; a second
    frame appends its new blocks in key order after the first frame's."""
    rng = np.random.default_rng(9)
    K = np.array([12.0, 12.0, 7.5, 5.5], np.float32)
    s = orc.Submap(orc.Params(vs=VS, integrator=1, ray_carve=False))
    st1 = s.integrate(rng.uniform(0.8, 2.5, (12, 16)).astype(np.float32), K, np.eye(4))
    e = s.export()
    assert np.all(np.diff(e["keys"].astype(np.uint64)) > 0)
    assert np.all((e["W"] > 0).any(axis=1))
    T = np.eye(4)
    T[:3, 3] = (0.4, 0.0, 0.0)
    st2 = s.integrate(rng.uniform(0.8, 2.5, (12, 16)).astype(np.float32), K, T)
    e2 = s.export()
    n1 = st1["n_new"]
    assert np.array_equal(e2["keys"][:n1], e["keys"])
    assert np.all(np.diff(e2["keys"][n1:].astype(np.uint64)) > 0) and st2["n_new"] == len(e2["keys"]) - n1


def test_binary32_and_binary64_agree():
    """The binary32 and binary64 oracles agree where their grid walks agree.
    Walk ties (a ray grazing a voxel edge, an optical centre on a voxel
    boundary) change which voxels some rays cross, so the total weight
    agrees to 1 %, and on voxels with equal weight the 99th percentile of
    |D32 - D64| stays below 1e-6 m."""
    import scenegen as sg
    w = sg.tiny(n_frames=3)
    a = orc.Submap(orc.Params(integrator=1))
    b = orc.Submap(orc.Params(integrator=1, fp64=True))
    for f in range(3):
        a.integrate(w.frame(f), w.cam.K, w.poses[f])
        b.integrate(w.frame(f), w.cam.K, w.poses[f])
    ea, eb = a.export(), b.export()
    ka = {int(k): i for i, k in enumerate(ea["keys"])}
    common = [(ka[int(k)], j) for j, k in enumerate(eb["keys"]) if int(k) in ka]
    assert len(common) > 0.99 * len(eb["keys"])
    ia, ib = np.array(common).T
    Wa, Wb = ea["W"][ia], eb["W"][ib]
    assert abs(Wa.sum() - Wb.sum()) < 0.01 * Wb.sum()
    same = (Wa == Wb) & (Wa > 0)
    assert same.sum() > 0.8 * (Wb > 0).sum()
    assert np.percentile(np.abs(ea["D"][ia][same] - eb["D"][ib][same]), 99) < 1e-6


def _walk_alt(o, u, s0, s1, vs, mode):
    """The traversal with other roundings of the crossing parameters:
    mode "recip" multiplies by the binary32 reciprocal of u_a, mode "f64"
    forms and compares the parameters in binary64 (from the same binary32
    inputs).  Both stay within 2^-22 relative of the exact quotient."""
    f = np.float32
    vs = f(vs)
    i = [int(math.floor(f(o[a] + f(f(s0) * u[a])) / vs)) for a in range(3)]
    step = [1 if u[a] > 0 else (-1 if u[a] < 0 else 0) for a in range(3)]
    iu = [f(f(1.0) / u[a]) if step[a] else f(0) for a in range(3)]
    out = []
    cap = 3 * int(math.ceil(f(f(s1) - f(s0)) / vs)) + 6
    while len(out) < cap:
        out.append(tuple(i))
        sn = []
        for a in range(3):
            if not step[a]:
                sn.append(math.inf)
                continue
            b = f(f(i[a] + (step[a] > 0)) * vs)
            if mode == "recip":
                sn.append(float(f(f(b - o[a]) * iu[a])))
            else:
                sn.append((float(b) - float(o[a])) / float(u[a]))
        a = 0
        if sn[1] < sn[a]:
            a = 1
        if sn[2] < sn[a]:
            a = 2
        if not (sn[a] < float(s1)):
            break
        i[a] += step[a]
    return out


def _near_tie_rays(n, seed):
    """Rays whose x and y crossings nearly coincide at every boundary: equal
    direction components and origin offsets up to a few ulps apart."""
    rng = np.random.default_rng(seed)
    for k in range(n):
        x = np.float32(rng.uniform(0.0, 0.05))
        o = np.array([x, x, rng.uniform(0.0, 0.05)], np.float32)
        o[1] = np.nextafter(o[1], np.float32(1.0) if k % 3 else np.float32(-1.0)) if k % 2 else o[1]
        c = rng.uniform(-0.5, 0.5)
        u = np.array([1.0, 1.0 + rng.choice([0.0, 1e-7, -1e-7, 3e-7]), c])
        u = (u / np.linalg.norm(u)).astype(np.float32)
        s1 = np.float32(rng.uniform(0.3, 1.5))
        yield o, u, np.float32(0.0), s1


def test_fragile_steps_cover_other_faithful_roundings():
    """Walks whose crossing parameters are rounded differently (but still
    faithfully) differ from the oracle's walk only in voxels the oracle
    recorded as fragile; rays away from ties record nothing."""
    differing = 0
    for o, u, s0, s1 in list(_near_tie_rays(400, 21)) + list(_random_rays(200, 22)):
        walk, frag = orc.ray_walk32(o, u, s0, s1, VS, fragile=True)
        got = {tuple(v) for v in walk}
        fr = {tuple(v) for v in frag}
        for mode in ("recip", "f64"):
            alt = set(_walk_alt(o, u, s0, s1, VS, mode))
            diff = alt ^ got
            assert diff <= fr, (mode, sorted(diff - fr)[:4])
            differing += bool(diff)
    assert differing > 20  # the near-tie rays do exercise the margin


def test_exact_tie_records_both_neighbours():
    """A ray with equal x and y components through a point with equal x and
    y offsets crosses every x and y boundary at the same parameter: the walk
    moves x first (the tie rule), and each tie records the two voxels a
    step could enter (x or y first), never the corner both reach."""
    o = np.array([0.013, 0.013, 0.021], np.float32)
    u = np.array([1.0, 1.0, 0.0], np.float32) / np.float32(np.sqrt(2.0))
    u = u.astype(np.float32)
    walk, frag = orc.ray_walk32(o, u, 0.0, 0.3, VS, fragile=True)
    steps = np.diff(walk, axis=0)
    assert np.all(steps[0::2] == [1, 0, 0]) and np.all(steps[1::2] == [0, 1, 0])
    fr = {tuple(v) for v in frag}
    for k in range(0, len(walk) - 1, 2):
        i = walk[k]
        if k + 2 < len(walk):
            assert (i[0] + 1, i[1], i[2]) in fr and (i[0], i[1] + 1, i[2]) in fr
            assert (i[0] + 1, i[1] + 1, i[2]) not in fr
    _, none = orc.ray_walk32(o, np.array([0.6, 0.8, 0.0], np.float32), 0.0, 0.3, VS, fragile=True)
    assert len(none) == 0
