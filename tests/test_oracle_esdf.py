"""Pins of the oracle's ESDF (paper Sec. I: Euclidean distance to the nearest
obstacle built from the TSDF, reusing the distances inside the truncation
band; Sec. III-E: an exact EDT in the PBA lineage).

Checked against O(N * S) brute force on small grids, closed forms for a
single site and a plane of sites, the 1-Lipschitz property and the analytic
SDF of a noise-free scene."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg


def _grid_submap(params, shape_blocks, D, W, origin_block=(0, 0, 0), drop=()):
    """Import a dense box of blocks (minus `drop`) with voxel values given by
    arrays D, W of shape 8 * shape_blocks (x, y, z)."""
    keys, Ds, Ws, coords = [], [], [], []
    l = np.arange(512)
    off = np.stack([l & 7, (l >> 3) & 7, l >> 6], axis=1)
    for bx in range(shape_blocks[0]):
        for by in range(shape_blocks[1]):
            for bz in range(shape_blocks[2]):
                if (bx, by, bz) in drop:
                    continue
                b = np.array([bx, by, bz]) + origin_block
                keys.append(orc.pack_key(b[0], b[1], b[2]))
                loc = 8 * np.array([bx, by, bz]) + off
                Ds.append(D[loc[:, 0], loc[:, 1], loc[:, 2]])
                Ws.append(W[loc[:, 0], loc[:, 1], loc[:, 2]])
    s = orc.Submap(params)
    s.import_blocks(np.array(keys, np.uint64), np.stack(Ds), np.stack(Ws))
    return s


def _expected_from_definition(exp, params):
    """phi and k straight from the definition, brute force over all sites."""
    vs_f = np.float32(params.vs)
    tau_f = np.float32(params.trunc_vox * params.vs * (1.0 - 1.0 / 1024.0))
    dmax_f = np.float32(params.d_max)
    R = int(round(params.d_max / params.vs))
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    D = exp["D"].reshape(-1).astype(np.float32)
    W = exp["W"].reshape(-1).astype(np.float32)
    obs = W > 0
    site = obs & (np.abs(D) <= vs_f)
    band = obs & (np.abs(D) < tau_f)
    S = coords[site]
    k = np.full(len(D), -1, np.int64)
    phi = np.full(len(D), np.nan, np.float32)
    phi[band] = D[band]
    todo = np.nonzero(obs & ~band)[0]
    for j in todo:
        if len(S):
            kk = int(np.min(np.sum((S - coords[j]) ** 2, axis=1)))
        else:
            kk = R * R + 1
        sg_ = np.float32(1.0) if D[j] > 0 else np.float32(-1.0)
        if kk > R * R:
            k[j] = R * R + 1
            phi[j] = sg_ * dmax_f
        else:
            k[j] = kk
            phi[j] = sg_ * min(dmax_f, vs_f * np.sqrt(np.float32(kk)))
    return k, phi


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_esdf_matches_brute_force_on_small_grids(seed):
    rng = np.random.default_rng(seed)
    shape = (3, 3, 2)
    n = 8 * np.array(shape)
    D = rng.uniform(-0.2, 0.6, size=n)
    # sparse sites: most voxels far from the surface
    D[rng.uniform(size=n) < 0.9] = 0.45
    W = rng.choice([0.0, 1.0, 2.0], p=[0.2, 0.4, 0.4], size=n)
    params = orc.Params(vs=0.05, trunc_vox=4, d_max=0.4)  # R = 8 inside a 24-voxel box
    s = _grid_submap(params, shape, D, W, origin_block=(-1, 2, -3), drop={(1, 1, 0), (2, 0, 1)})
    s.update_esdf()
    exp = s.export()
    k_want, phi_want = _expected_from_definition(exp, params)
    k_got = exp["ksq"].reshape(-1)
    phi_got = exp["phi"].reshape(-1).astype(np.float32)
    assert np.array_equal(k_got, k_want)
    assert np.array_equal(np.isnan(phi_got), np.isnan(phi_want))
    m = ~np.isnan(phi_want)
    assert np.array_equal(phi_got[m], phi_want[m])


def test_single_site_closed_form():
    shape = (4, 4, 4)
    n = 8 * np.array(shape)
    D = np.full(n, 0.5)
    W = np.ones(n)
    s_ = (13, 17, 9)
    D[s_] = 0.0
    params = orc.Params(vs=0.05, trunc_vox=4, d_max=2.0)
    s = _grid_submap(params, shape, D, W)
    s.update_esdf()
    exp = s.export()
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    k = exp["ksq"].reshape(-1)
    phi = exp["phi"].reshape(-1)
    d2 = np.sum((coords - np.array(s_)) ** 2, axis=1)
    far = d2 > 0
    assert np.array_equal(k[far], d2[far])
    want = np.minimum(np.float32(2.0), np.float32(0.05) * np.sqrt(d2[far].astype(np.float32)))
    assert np.array_equal(phi[far].astype(np.float32), want)


def test_plane_of_sites_closed_form():
    shape = (3, 3, 4)
    n = 8 * np.array(shape)
    D = np.full(n, 0.5)
    W = np.ones(n)
    D[:, :, 11] = 0.01  # a plane of sites at z index 11
    s = _grid_submap(orc.Params(vs=0.05, d_max=2.0), shape, D, W)
    s.update_esdf()
    exp = s.export()
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    k = exp["ksq"].reshape(-1)
    m = coords[:, 2] != 11
    assert np.array_equal(k[m], (coords[m, 2] - 11) ** 2)


def test_band_membership_does_not_depend_on_precision():
    """Voxels clamped to tau in every observation are outside the band in the
    binary32, binary64 and binary16 modes alike, although their stored D
    rounds differently (binary16 0.2 is below 0.2)."""
    K = np.array([11.0, 12.5, 7.37, 5.61], np.float32)
    outs = []
    for kw in (dict(), dict(fp64=True), dict(fp16=True)):
        s = orc.Submap(orc.Params(**kw))
        for z in (1.1, 1.13, 1.08):
            s.integrate(np.full((12, 16), z, np.float32), K, np.eye(4))
        s.update_esdf()
        outs.append(s.export())
    k = [o["ksq"] for o in outs]
    assert np.array_equal(k[0], k[1]) and np.array_equal(k[0], k[2])
    assert np.count_nonzero(k[0] > 0) > 500


def test_no_sites_gives_dmax_and_unobserved_is_nan():
    shape = (2, 2, 2)
    n = 8 * np.array(shape)
    D = np.full(n, -0.3)
    W = np.ones(n)
    W[0, 0, 0] = 0
    s = _grid_submap(orc.Params(vs=0.05, d_max=2.0), shape, D, W)
    s.update_esdf()
    phi = s.export()["phi"].reshape(-1)
    assert np.isnan(phi[0])
    assert np.all(phi[1:] == np.float32(-2.0))


def test_lipschitz_and_band_copy_on_tiny_workload():
    w = sg.tiny()
    s = orc.Submap(orc.Params())
    for f in range(w.n_frames):
        s.integrate(w.frame(f), w.cam.K, w.poses[f])
    s.update_esdf()
    exp = s.export()
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    k = exp["ksq"].reshape(-1)
    D = exp["D"].reshape(-1)
    W = exp["W"].reshape(-1)
    phi = exp["phi"].reshape(-1)
    band = (W > 0) & (np.abs(D) < np.float32(0.2 * (1.0 - 1.0 / 1024.0)))
    assert np.array_equal(phi[band], D[band])
    # voxels at the truncation limit are outside the band
    clamped = (W > 0) & (D == np.float32(0.2))
    assert clamped.sum() > 1000 and np.all(k[clamped] >= 0)
    # 1-Lipschitz between axis neighbours that both carry an exact k
    lut = {tuple(c): kk for c, kk in zip(coords, k) if 0 <= kk <= 1600}
    checked = 0
    for c, kk in list(lut.items())[:200000]:
        for a in range(3):
            nb = list(c)
            nb[a] += 1
            k2 = lut.get(tuple(nb))
            if k2 is not None:
                assert abs(np.sqrt(kk) - np.sqrt(k2)) <= 1.0 + 1e-12
                checked += 1
    assert checked > 10000


def test_esdf_against_analytic_sdf_noise_free():
    """Noise-free tiny room: for observed voxels outside the band, phi is a
    distance to a site, and a site's |D| <= vs bounds its true distance to
    within the projective slack (z-differences shrink by the cosine of the
    ray angle, here <= 1.2 at the image corners, plus the pixel footprint), so
    phi >= SDF - 1.5 vs everywhere since SDF is 1-Lipschitz.  Where the
    nearest surface is observed the two agree to within vs + vs sqrt(3) / 2;
    surfaces never seen (sphere backs) make the rest."""
    w = sg.tiny(noise=False)
    s = orc.Submap(orc.Params())
    for f in range(w.n_frames):
        s.integrate(w.frame(f), w.cam.K, w.poses[f])
    s.update_esdf()
    exp = s.export()
    coords = orc.voxel_coords(exp["keys"]).reshape(-1, 3)
    D = exp["D"].reshape(-1)
    W = exp["W"].reshape(-1)
    phi = exp["phi"].reshape(-1)
    m = (W > 0) & (np.abs(D) >= np.float32(0.2 * (1.0 - 1.0 / 1024.0))) & (phi > 0) & (phi < 1.9)
    c = (coords[m] + 0.5) * 0.05
    sdf = w.scene.sdf(c)
    assert np.all(phi[m] >= sdf - 1.5 * 0.05)
    close = np.abs(phi[m] - sdf) <= 0.05 + 0.05 * np.sqrt(3) / 2
    assert close.mean() > 0.8
