"""Pins of the oracle's incremental (wavefront) ESDF (Sec. III-E: changed
voxels seed per-block work, blocks are swept along every axis, faces pass
better distances to neighbouring blocks until nothing changes).

The propagation keeps, per voxel, a parent site and its squared distance.
Pinned: a single site gives the exact squared distance everywhere within R;
every parent is a site at the stored distance (so k never undercuts the
exact EDT); the result is a fixed point of the face-neighbour offer; a
removed site (raise) hands its voxels to the remaining one exactly; and on
the tiny sequence the field equals the exact EDT on almost every voxel."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg

VS = 0.05
R = 8  # d_max = 0.4 m


def _cube(nb=3, sites=((12, 11, 10),)):
    """nb^3 blocks from the origin, every voxel observed at D = 0.2 m (outside
    the band, not a site) except the given site voxels (D = 0)."""
    keys = []
    for bx in range(nb):
        for by in range(nb):
            for bz in range(nb):
                keys.append(int(orc.pack_key(bx, by, bz)))
    keys = np.array(sorted(keys), np.uint64)
    D = np.full((len(keys), 512), 0.2)
    W = np.ones((len(keys), 512))
    pos = {int(k): j for j, k in enumerate(keys)}
    for (x, y, z) in sites:
        j = pos[int(orc.pack_key(x // 8, y // 8, z // 8))]
        D[j, (x & 7) + 8 * (y & 7) + 64 * (z & 7)] = 0.0
    return keys, D, W


def _field(keys, D, W, mode):
    s = orc.Submap(orc.Params(vs=VS, trunc_vox=2, d_max=R * VS, esdf_mode=mode))
    s.import_blocks(keys, D, W)
    s.update_esdf()
    return s


def _coords(keys):
    return orc.voxel_coords(keys).reshape(-1, 3)


def _k(s):
    """Squared distances of a cube field; the export marks band voxels -1,
    and in these fields the band voxels are exactly the sites (k = 0)."""
    k = s.export()["ksq"].reshape(-1).astype(np.int64)
    return np.where(k < 0, 0, k)


def test_single_site_is_exact_within_R():
    keys, D, W = _cube()
    c = _coords(keys)
    k_true = ((c - np.array([12, 11, 10])) ** 2).sum(axis=1)
    k = _k(_field(keys, D, W, 1))
    inside = k_true <= R * R
    assert np.array_equal(k[inside], k_true[inside])
    assert np.all(k[~inside] == R * R + 1)


def test_parents_are_sites_and_distances_never_undercut_the_exact_edt():
    rng = np.random.default_rng(3)
    sites = [tuple(rng.integers(0, 24, 3)) for _ in range(12)]
    keys, D, W = _cube(sites=sites)
    kw = _k(_field(keys, D, W, 1))
    ke = _k(_field(keys, D, W, 0))
    assert np.all(kw >= ke)
    c = _coords(keys)
    S = np.array(sites)
    d2 = ((c[:, None, :] - S[None, :, :]) ** 2).sum(axis=2)
    has = kw <= R * R
    # the stored distance is the squared distance to some site
    assert np.all((d2[has] == kw[has][:, None]).any(axis=1))
    assert (kw == ke).mean() > 0.99


def test_result_is_a_fixed_point_of_the_neighbour_offer():
    """No voxel could improve by taking the parent site of a face neighbour
    u: that site lies within sqrt(k(u)) + 1 of v, so wherever this bound is
    inside R, k(v) <= (sqrt(k(u)) + 1)^2 holds at the fixed point."""
    rng = np.random.default_rng(4)
    sites = [tuple(rng.integers(0, 24, 3)) for _ in range(6)]
    keys, D, W = _cube(sites=sites)
    k = _k(_field(keys, D, W, 1))
    c = _coords(keys)
    grid = np.full((24, 24, 24), -1, np.int64)
    grid[c[:, 0], c[:, 1], c[:, 2]] = k
    for a in range(3):
        u = np.take(grid, range(1, 24), axis=a).astype(float)
        v = np.take(grid, range(0, 23), axis=a).astype(float)
        for x, y in ((u, v), (v, u)):
            ok = (x >= 0) & ((np.sqrt(np.maximum(x, 0)) + 1) ** 2 <= R * R)
            bound = (np.sqrt(x[ok]) + 1) ** 2
            yv = np.where(y[ok] > R * R, np.inf, y[ok])
            assert np.all(yv <= bound + 1e-9)


def test_removed_site_hands_its_voxels_over():
    """Two sites, the first no longer observed: the propagation gives the
    single-site field of the second on every observed voxel within R.  (The
    incremental raise itself is covered by the tiny sequence below, where
    sites appear and vanish between updates.)"""
    a, b = (5, 5, 5), (18, 17, 16)
    keys, D, W = _cube(sites=(a, b))
    pos = {int(k): j for j, k in enumerate(keys)}
    j = pos[int(orc.pack_key(a[0] // 8, a[1] // 8, a[2] // 8))]
    W2 = W.copy()
    W2[j, (a[0] & 7) + 8 * (a[1] & 7) + 64 * (a[2] & 7)] = 0.0  # no longer observed
    sub = orc.Submap(orc.Params(vs=VS, trunc_vox=2, d_max=R * VS, esdf_mode=1))
    sub.import_blocks(keys, D, W2)  # the site at a is gone; import restarts the state
    sub.update_esdf()
    c = _coords(keys)
    k_b = ((c - np.array(b)) ** 2).sum(axis=1)
    k = _k(sub)
    inside = k_b <= R * R
    obs = W2.reshape(-1) > 0
    assert np.array_equal(k[inside & obs], k_b[inside & obs])


def test_incremental_raise_on_the_tiny_sequence():
    """Frames integrated between incremental updates: every parent stays a
    current site (distances never undercut the exact EDT), and the field
    equals the exact EDT on more than 99 % of observed voxels with errors
    below one voxel."""
    w = sg.tiny()
    a = orc.Submap(orc.Params())
    b = orc.Submap(orc.Params(esdf_mode=1))
    for f in range(20):
        a.integrate(w.frame(f), w.cam.K, w.poses[f])
        b.integrate(w.frame(f), w.cam.K, w.poses[f])
        if f % 4 == 3:
            a.update_esdf()
            st = b.esdf_wavefront()
            assert st["rounds"] >= 1
            ea, eb = a.export(), b.export()
            m = ea["ksq"] >= 0
            assert np.array_equal(np.isnan(ea["phi"]), np.isnan(eb["phi"]))
            assert np.all(eb["ksq"][m] >= ea["ksq"][m])
            obs = ~np.isnan(ea["phi"])
            d = np.abs(ea["phi"][obs] - eb["phi"][obs])
            assert (d == 0).mean() > 0.99 and d.max() < 0.05
