"""Pins of the oracle's proposal-network code and coarse summaries: bf16
rounding at ties, the convolution against an independent numpy
implementation, backpropagation against central finite differences (binary64
toy network) and the summary of a linear field (exact under trilinear
interpolation)."""
import numpy as np
import pytest

import oracle as orc


def test_bf16_rounding_ties_to_even():
    one = 1.0
    ulp = 2.0 ** -7  # bf16 spacing at 1
    assert orc.bf16_round(one) == one
    assert orc.bf16_round(one + ulp / 2) == one            # tie -> even (1.0)
    assert orc.bf16_round(one + 3 * ulp / 2) == one + 2 * ulp  # tie -> even (1 + 2 ulp)
    assert orc.bf16_round(one + ulp / 2 + 2 ** -20) == one + ulp
    assert orc.bf16_round(-2.0 - 2.0 ** -7) == -2.0         # tie at 2 (spacing 2^-6) -> even
    assert orc.bf16_round(3.0e38) == pytest.approx(3.0e38, rel=2 ** -8)


def _numpy_conv(x, w, b, stride):
    """3x3x3 convolution with zero padding 1 (NDHWC), straight from the
    definition with numpy slicing."""
    n, D, _, _, cin = x.shape
    cout = w.shape[0]
    Do = (D + 2 - 3) // stride + 1
    xp = np.zeros((n, D + 2, D + 2, D + 2, cin))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    wk = w.reshape(cout, 3, 3, 3, cin)
    y = np.zeros((n, Do, Do, Do, cout)) + b
    for kd in range(3):
        for kh in range(3):
            for kw in range(3):
                sl = xp[:, kd:kd + stride * (Do - 1) + 1:stride, kh:kh + stride * (Do - 1) + 1:stride,
                        kw:kw + stride * (Do - 1) + 1:stride, :]
                y += np.einsum("ndhwc,oc->ndhwo", sl, wk[:, kd, kh, kw, :])
    return np.maximum(y, 0.0)


def _toy():
    layers = [(3, 4, 8, 8, 1), (4, 6, 8, 4, 2)]
    return layers, 6


def test_forward_matches_numpy_convolution():
    layers, feat = _toy()
    rng = np.random.default_rng(1)
    p = rng.normal(size=orc.net_num_params(layers, feat)).astype(np.float32) * 0.3
    x = rng.uniform(-1, 1, size=(2, 8, 8, 8, 3)).astype(np.float32)
    out = orc.net_forward(p, x, layers, feat, bf16=False)
    # numpy reference
    o = 0
    a = x.astype(np.float64)
    for (ci, co, di, do, st) in layers:
        nw = co * 27 * ci
        w = p[o:o + nw].astype(np.float64).reshape(co, 27 * ci)
        b = p[o + nw:o + nw + co].astype(np.float64)
        o += nw + co
        a = _numpy_conv(a, w, b, st)
    pooled = a.reshape(2, -1, feat).mean(axis=1)
    fw = p[o:o + 5 * feat].astype(np.float64).reshape(5, feat)
    fb = p[o + 5 * feat:o + 5 * feat + 5].astype(np.float64)
    want = pooled @ fw.T + fb
    assert np.allclose(out, want, rtol=1e-12, atol=1e-12)


def test_backprop_matches_finite_differences():
    layers, feat = _toy()
    rng = np.random.default_rng(2)
    p = (rng.normal(size=orc.net_num_params(layers, feat)) * 0.3).astype(np.float32)
    x = rng.uniform(-1, 1, size=(2, 8, 8, 8, 3)).astype(np.float32)
    y = rng.normal(size=(2, 5)).astype(np.float32)
    loss, g = orc.net_loss_grad(p, x, y, 3.0, layers, feat, bf16=False)
    assert loss > 0
    idx = np.concatenate([rng.choice(len(p), size=40, replace=False), [len(p) - 1, len(p) - 8, 0]])
    def fd(i, h):
        # the divisor is the perturbation actually stored in binary32
        pp, pm = p.copy(), p.copy()
        pp[i] += np.float32(h)
        pm[i] -= np.float32(h)
        lp, _ = orc.net_loss_grad(pp, x, y, 3.0, layers, feat, bf16=False)
        lm, _ = orc.net_loss_grad(pm, x, y, 3.0, layers, feat, bf16=False)
        return (lp - lm) / (float(pp[i]) - float(pm[i]))

    for i in idx:
        # A step can straddle a ReLU kink somewhere downstream; the loss is
        # piecewise smooth, so a smaller step must then agree.
        ok = False
        for h in (2.0 ** -12, 2.0 ** -16, 2.0 ** -20):
            d = fd(i, h)
            if abs(d - g[i]) <= 1e-5 * max(1.0, abs(g[i])) + 1e-7:
                ok = True
                break
        assert ok, (i, d, g[i])


def test_bf16_mode_close_to_binary64():
    layers, feat = _toy()
    rng = np.random.default_rng(3)
    p = (rng.normal(size=orc.net_num_params(layers, feat)) * 0.3).astype(np.float32)
    x = rng.uniform(-1, 1, size=(2, 8, 8, 8, 3)).astype(np.float32)
    a = orc.net_forward(p, x, layers, feat, bf16=False)
    b = orc.net_forward(p, x, layers, feat, bf16=True)
    assert np.allclose(a, b, rtol=0.05, atol=0.02)


def test_summary_of_a_linear_field():
    """phi = D inside the band; for D linear in the voxel centres the
    trilinear value at any point equals the linear function there."""
    params = orc.Params(vs=0.1, trunc_vox=4, d_max=3.0)
    keys, Ds, Ws = [], [], []
    l = np.arange(512)
    off = np.stack([l & 7, (l >> 3) & 7, l >> 6], axis=1)
    for bx in range(-3, 3):
        for by in range(-3, 3):
            for bz in range(-2, 2):
                keys.append(orc.pack_key(bx, by, bz))
                c = (8 * np.array([bx, by, bz]) + off + 0.5) * 0.1
                Ds.append(0.05 * c[:, 0] - 0.03 * c[:, 1] + 0.02 * c[:, 2] + 0.01)
                Ws.append(np.full(512, 2.0))
    s = orc.Submap(params)
    s.import_blocks(np.array(keys, np.uint64), np.stack(Ds), np.stack(Ws))
    s.update_esdf()
    T = np.eye(4)
    T[:3, 3] = [0.013, -0.021, 0.007]
    out = orc.summary(s, T, cell=0.1)
    cidx = np.arange(32768)
    g = np.stack([cidx & 31, (cidx >> 5) & 31, cidx >> 10], axis=1)
    q = ((g + 0.5) - 16.0) * 0.1 + T[:3, 3]
    inside = np.all(np.abs(q) < 1.55, axis=1) & (np.abs(q[:, 2]) < 1.55)
    want = (0.05 * q[:, 0] - 0.03 * q[:, 1] + 0.02 * q[:, 2] + 0.01) / 3.0
    m = out[:, 1] == 1
    assert m.sum() > 10000 and np.all(m[inside & (np.abs(q[:, 2]) < 1.5)])
    assert np.allclose(out[m, 0], want[m], atol=1e-6)  # phi stored in binary32
