"""GPU parity of the learned pose proposal: coarse ESDF summaries, the bf16
matrix-core network (forward and gradients) and the proposal-then-refine
driver, each through the C ABI against the oracle on the same seeded
inputs.

Bars: summary values within 2e-5 (binary32 vs binary64 trilinear weights;
values are phi / d_max in [-1, 1]) and masks equal except at cells whose
sample lies within 1e-4 voxel of a voxel-centre plane (the binary32 map
position can then select the neighbouring corner set); network outputs within
1e-3 of the output scale (the oracle rounds activations and weights to bf16
as the kernels do; a one-ulp difference in the accumulation order can still
flip a bf16 rounding, 2^-8 relative, so the bar sits well above the FP32
against binary64 summation difference); gradients within 1e-2 relative L2
per tensor against binary64 backpropagation through the oracle's bf16
forward pass (the kernels round the upstream gradient to bf16 for the matrix
cores).  The driver with a zero cost threshold must give exactly what plain
multi-start gives (every pair falls back); with turned priors it refines the
proposal of least cost at the proposal."""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_21149_amd as cv
    return cv


def _ctx(cv):
    return cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)


def _tiny_submaps(cv, ctx, with_oracle=True):
    import torch
    w = sg.tiny()
    fr = w.frames()
    dev = torch.from_numpy(fr).cuda()
    A, B = ctx.submap_create(), ctx.submap_create()
    rA = orc.Submap(orc.Params(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0)) if with_oracle else None
    rB = orc.Submap(orc.Params(vs=0.05, trunc_vox=4, max_range=5.0, d_max=2.0)) if with_oracle else None
    for f in range(20):
        for _ in range(2):
            ctx.integrate_depth(A if f < 12 else B, dev[f], w.cam.K, w.poses[f])
            if with_oracle:
                (rA if f < 12 else rB).integrate(fr[f], w.cam.K, w.poses[f])
    for f in range(8, 14):  # overlap
        ctx.integrate_depth(B if f < 12 else A, dev[f], w.cam.K, w.poses[f])
        if with_oracle:
            (rB if f < 12 else rA).integrate(fr[f], w.cam.K, w.poses[f])
    ctx.update_esdf(A)
    ctx.update_esdf(B)
    if with_oracle:
        rA.update_esdf()
        rB.update_esdf()
    return A, B, rA, rB


def _near_plane(T, cell, vs):
    """Cells whose sample point lies within 1e-4 voxel of a plane through
    voxel centres along some axis (x, y or z)."""
    c = np.arange(32768)
    g = np.stack([c & 31, (c >> 5) & 31, c >> 10], axis=1).astype(np.float64)
    q = (g + 0.5 - 16.0) * cell
    p = q @ T[:3, :3].T + T[:3, 3]
    u = p / vs - 0.5
    return np.any(np.abs(u - np.round(u)) < 1e-4, axis=1)


def test_summaries_parity(cv):
    import torch
    ctx = _ctx(cv)
    A, B, rA, rB = _tiny_submaps(cv, ctx)
    Ts = [np.eye(4), orc.se3_exp(np.array([0.13, -0.07, 0.02, 0.05, -0.03, 0.7]))]
    for T in Ts:
        for cell, sm, rs in ((0.05, A, rA), (0.11, B, rB)):
            out = torch.zeros((32768, 4), dtype=torch.float32, device="cuda")
            ctx.summaries([(sm, T, cell, out, 2)])
            g = out.cpu().numpy().astype(np.float64)
            r = orc.summary(rs, T, cell)
            assert np.all(g[:, :2] == 0), "other channels must be left untouched"
            bad = (g[:, 3] != r[:, 1]) & ~_near_plane(T, cell, 0.05)
            assert not bad.any(), np.flatnonzero(bad)[:10]
            both = (g[:, 3] == 1) & (r[:, 1] == 1)
            assert both.sum() > 1000
            assert np.abs(g[both, 2] - r[both, 0]).max() <= 2e-5
            assert np.all(g[g[:, 3] == 0, 2] == 0)
    ctx.close()


def _inputs(n, seed):
    """Summary-like network inputs: values in [-1, 1] with masks, the masked
    cells zero, in blobs (smooth fields) rather than white noise."""
    rng = np.random.default_rng(seed)
    c = np.arange(32)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    x = np.zeros((n, 32, 32, 32, 4), np.float32)
    for b in range(n):
        for side in range(2):
            a, bb, cc = rng.normal(size=3)
            field = np.sin(0.2 * a * X + 0.3 * bb * Y) * np.cos(0.25 * cc * Z) + 0.1 * rng.normal(size=X.shape)
            mask = (np.sin(0.15 * X + rng.uniform(0, 6)) + np.cos(0.2 * Y) + 0.5 * np.cos(0.1 * Z)) > -0.3
            v = np.clip(field, -1, 1) * mask
            # the (z, y, x) grid index order of NDHWC: x fastest
            x[b, :, :, :, 2 * side] = v.transpose(2, 1, 0)
            x[b, :, :, :, 2 * side + 1] = mask.transpose(2, 1, 0)
    return x


def test_network_forward_parity(cv):
    import torch
    ctx = _ctx(cv)
    net = cv.Net(ctx, seed=7)
    p = net.get_params()
    assert len(p) == orc.net_num_params()
    x = _inputs(2, 11)
    g = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    r = orc.net_forward(p, x, bf16=True)
    scale = np.abs(r).max()
    assert scale > 1e-3
    print("forward: max |gpu - oracle| / max |oracle| = %.3g" % (np.abs(g - r).max() / scale))
    # the oracle rounds activations and weights to bf16 as the kernels do; what
    # is left is FP32 against binary64 accumulation order (measured 5.5e-5)
    assert np.abs(g - r).max() <= 1e-3 * scale, (g, r)
    # a different batch size gives the same per-sample outputs
    g1 = net.forward(torch.from_numpy(x[1:]).cuda()).cpu().numpy()
    assert np.array_equal(g1[0], g[1].astype(np.float32))
    ctx.close()


def test_network_gradients_parity(cv):
    import torch
    ctx = _ctx(cv)
    net = cv.Net(ctx, seed=9)
    p = net.get_params()
    x = _inputs(2, 13)
    y = np.array([[0.5, -1.0, 0.2, 0.8, 0.6], [-2.0, 0.3, -0.1, -0.6, 0.8]], np.float32)
    loss_g, grad_g = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 3.0)
    loss_r, grad_r = orc.net_loss_grad(p, x, y, 3.0, bf16=True)
    assert abs(loss_g - loss_r) <= 0.02 * loss_r
    o = 0
    sizes = []
    for (ci, co, di, do, st) in orc.NET_LAYERS:
        sizes += [co * 27 * ci, co]
    sizes += [5 * orc.NET_FEAT, 5]
    errs = []
    for k, sz in enumerate(sizes):
        a, b = grad_g[o:o + sz].astype(np.float64), grad_r[o:o + sz]
        errs.append(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12))
        o += sz
    print("gradient rel-L2 per tensor:", " ".join(f"{e:.2e}" for e in errs))
    # the kernels also round the upstream gradient to bf16 for the matrix
    # cores (the oracle does not): measured at most 3.6e-3
    assert max(errs) <= 1e-2, errs
    assert o == len(p)
    ctx.close()


def test_training_reduces_the_loss(cv):
    import torch
    ctx = _ctx(cv)
    net = cv.Net(ctx, seed=3)
    x = torch.from_numpy(_inputs(4, 17)).cuda()
    y = torch.tensor([[1.0, -0.5, 0.1, 1.0, 0.0], [-1.0, 0.5, 0.0, 0.0, 1.0],
                      [0.3, 0.3, -0.2, -1.0, 0.0], [0.0, -1.2, 0.1, 0.0, -1.0]], device="cuda")
    p0 = net.get_params()
    losses = [net.train_step(x, y, 1e-3) for _ in range(40)]
    assert losses[-1] < 0.5 * losses[0], losses
    p1 = net.get_params()
    assert not np.array_equal(p0, p1)
    # set_params restores the exact forward
    net.set_params(p0)
    net2 = cv.Net(ctx, seed=3)
    assert np.array_equal(net.forward(x).cpu().numpy(), net2.forward(x).cpu().numpy())
    ctx.close()


def test_learned_driver_fallback_equals_multistart(cv):
    ctx = _ctx(cv)
    A, B, _, _ = _tiny_submaps(cv, ctx, with_oracle=False)
    net = cv.Net(ctx, seed=1)
    T0s = [orc.se3_exp(np.array([0.02, 0.01, -0.01, 0.0, 0.0, 0.5])),
           orc.se3_exp(np.array([-0.05, 0.03, 0.0, 0.0, 0.0, -0.2]))]
    pairs = [(A, B, T) for T in T0s]
    Tl, cl, sl = ctx.align_learned(net, pairs, 0.1, 0.0, n_starts=8)
    Tb, cb, sb = ctx.align_batch(pairs, n_starts=8)
    # an infinite threshold keeps the refined proposal: a converged pose
    Ti, ci, si = ctx.align_learned(net, pairs, 0.1, math.inf, n_starts=8)
    for k in range(2):
        assert si[k]["best_start"] == -1 and si[k]["status"] in (cv.OK, cv.NOT_CONVERGED)
        R = Ti[k][:3, :3]
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-9)
    # every pair falls back; the refined proposal competes with the starts
    # under the multi-start rule and keeps ties, so the result is whichever
    # of the two has the lower cost, never a higher cost than the refined pose
    for k in range(2):
        if cb[k] < ci[k]:
            assert np.array_equal(Tl[k], Tb[k]) and cl[k] == cb[k]
            assert sl[k]["best_start"] == sb[k]["best_start"]
        else:
            assert np.array_equal(Tl[k], Ti[k]) and cl[k] == ci[k] and sl[k]["best_start"] == -1
    ctx.close()


def test_context_close_before_net(cv):
    """Destroying a context frees the device memory of its networks; a net
    handle that outlives its context is rejected by every call and can still
    be destroyed (regression: the net's destroy used to read the freed
    context's stream)."""
    import ctypes
    import torch
    from paper_2410_21149_amd.covox import _lib
    ctx = _ctx(cv)
    net = cv.Net(ctx, seed=5)
    n_params = net.num_params
    x = torch.zeros((1, 32, 32, 32, 4), dtype=torch.float32, device="cuda")
    net.forward(x)
    h = net.handle
    # the C call order of a binding that does not close its nets: context first
    _lib.covox_destroy(ctx.handle)
    ctx.handle = None
    assert _lib.covox_net_num_params(h) == n_params
    out = torch.empty((1, 5), dtype=torch.float32, device="cuda")
    assert _lib.covox_net_forward(h, ctypes.c_void_p(x.data_ptr()), 1, ctypes.c_void_p(out.data_ptr())) == cv.EINVAL
    buf = np.zeros(n_params, np.float32)
    assert _lib.covox_net_get_params(h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n_params) == cv.EINVAL
    _lib.covox_net_destroy(h)
    net.handle = None
    # the binding closes a context's nets with it
    ctx2 = _ctx(cv)
    net2 = cv.Net(ctx2, seed=6)
    ctx2.close()
    assert net2.handle is None
    del net2
    torch.cuda.synchronize()


def test_propose_then_refine_equals_driver(cv):
    """With an infinite threshold the driver's pose is the single-start
    refinement of the network's proposal."""
    ctx = _ctx(cv)
    A, B, _, _ = _tiny_submaps(cv, ctx, with_oracle=False)
    net = cv.Net(ctx, seed=4)
    pairs = [(A, B, orc.se3_exp(np.array([0.03, -0.02, 0.0, 0.0, 0.0, 0.3]))),
             (B, A, orc.se3_exp(np.array([-0.02, 0.01, 0.01, 0.0, 0.0, -0.2])))]
    Tp = ctx.propose(net, pairs, 0.1)
    for k in range(2):
        R = Tp[k][:3, :3]
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-9) and np.allclose(Tp[k][3], [0, 0, 0, 1])
    Tl, cl, sl = ctx.align_learned(net, pairs, 0.1, math.inf)
    Tr, cr, sr = ctx.align_batch([(a, b, Tp[k]) for k, (a, b, _) in enumerate(pairs)], n_starts=1)
    assert np.array_equal(Tl, Tr) and np.array_equal(cl, cr)
    ctx.close()


def test_turned_priors_pick_then_refine(cv):
    """n_rot = 4: the prior turned by 0, 90, 180 and 270 degrees about the
    summary grid centre gives four proposals (the first that of the prior
    itself); with an infinite threshold the driver refines the proposal of
    least cost at the proposal (residual counts of at least n_min and half
    the largest), as calls of the parts in turn give it."""
    ctx = _ctx(cv)
    A, B, _, _ = _tiny_submaps(cv, ctx, with_oracle=False)
    net = cv.Net(ctx, seed=4)
    pairs = [(A, B, orc.se3_exp(np.array([0.03, -0.02, 0.0, 0.0, 0.0, 0.3]))),
             (B, A, orc.se3_exp(np.array([-0.02, 0.01, 0.01, 0.0, 0.0, -2.2])))]
    P4 = ctx.propose(net, pairs, 0.1, n_rot=4)
    assert P4.shape == (2, 4, 4, 4)
    assert np.array_equal(P4[:, 0], ctx.propose(net, pairs, 0.1))
    Tl, cl, sl = ctx.align_learned(net, pairs, 0.1, math.inf, n_rot=4)
    for i, (a, b, _) in enumerate(pairs):
        ctx.set_params(max_iter=0)  # the cost at each proposal, no update
        _, c0, s0 = ctx.align_batch([(a, b, P4[i, k]) for k in range(4)], n_starts=1)
        ctx.set_params(max_iter=30)
        ok = [s["n_used"] >= 100 for s in s0]
        nmax = max([s["n_used"] for s, o in zip(s0, ok) if o], default=0)
        cand = [k for k in range(4) if ok[k] and 2 * s0[k]["n_used"] >= nmax]
        best = min(cand, key=lambda k: (c0[k], k)) if cand else 0
        Tr, cr, sr = ctx.align_batch([(a, b, P4[i, best])], n_starts=1)
        assert np.array_equal(Tl[i], Tr[0]) and cl[i] == cr[0], (i, best)
    with pytest.raises(cv.CovoxError):
        ctx.align_learned(net, pairs, 0.1, math.inf, n_rot=0)
    # 70 items cross the 64-pair chunk of four turned priors: one call equals
    # two calls on parts of the list (every item stands alone)
    rng = np.random.default_rng(5)
    many = [(A, B, orc.se3_exp(np.concatenate([rng.uniform(-0.05, 0.05, 3), [0, 0], rng.uniform(-3, 3, 1)])))
            if k % 2 == 0 else (B, A, orc.se3_exp(np.concatenate([rng.uniform(-0.05, 0.05, 3), [0, 0],
                                                                   rng.uniform(-3, 3, 1)])))
            for k in range(70)]
    Pm = ctx.propose(net, many, 0.1, n_rot=4)
    assert np.array_equal(Pm, np.concatenate([ctx.propose(net, many[:30], 0.1, n_rot=4),
                                              ctx.propose(net, many[30:], 0.1, n_rot=4)]))
    Tm, cm, _ = ctx.align_learned(net, many, 0.1, 0.01, n_rot=4)
    T1, c1, _ = ctx.align_learned(net, many[:30], 0.1, 0.01, n_rot=4)
    T2, c2, _ = ctx.align_learned(net, many[30:], 0.1, 0.01, n_rot=4)
    assert np.array_equal(Tm, np.concatenate([T1, T2])) and np.array_equal(cm, np.concatenate([c1, c2]))
    ctx.close()


def test_training_items_use_the_ground_truth_prior(cv):
    """With zero re-framing ranges every prior is the ground truth and every
    target the identity correction, so a step with learning rate 0 reports
    the loss of the summaries at T_gt against (0, 0, 0, 1, 0)."""
    import torch
    ctx = _ctx(cv)
    A, B, _, _ = _tiny_submaps(cv, ctx, with_oracle=False)
    net = cv.Net(ctx, seed=2)
    p0 = net.get_params()
    T_gt = np.eye(4)
    L = ctx.train_proposal(net, [(A, B, T_gt)], steps=2, batch=3, lr=0.0, cell=0.1, trans_xy=0.0, trans_z=0.0,
                           yaw=0.0, tilt=0.0)
    assert np.array_equal(net.get_params(), p0)  # Adam with lr 0
    pbar = ctx.export_points(A).astype(np.float64).mean(axis=0)
    G = np.eye(4)
    G[:3, 3] = pbar
    x = torch.zeros((3, 32, 32, 32, 4), dtype=torch.float32, device="cuda")
    for b in range(3):
        ctx.summaries([(A, G, 0.1, x[b].view(32768, 4), 0), (B, np.linalg.inv(T_gt) @ G, 0.1, x[b].view(32768, 4), 2)])
    y = torch.tensor([[0.0, 0.0, 0.0, 1.0, 0.0]] * 3, device="cuda")
    loss, _ = net.gradients(x, y, 3.0)
    assert np.allclose(L, loss, rtol=1e-4), (L, loss)
    # non-zero ranges: the parameters move and the losses stay finite
    L2 = ctx.train_proposal(net, [(A, B, T_gt), (B, A, T_gt)], steps=3, batch=4, lr=1e-3, cell=0.1)
    assert np.all(np.isfinite(L2)) and not np.array_equal(net.get_params(), p0)
    ctx.close()
