"""Prepared alignment sets (covox_align_prepare / launch / collect): the same
poses, costs and statistics as covox_align_batch bit for bit, eager and
replayed from a captured graph (several replays with eager work between
them), and the version checks that keep a set or a graph from aligning
submaps that changed after the set was prepared."""
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


def _maps(cv):
    """A: tiny-room frames 0-9, B: 10-19 (each twice, every fifth frame of
    the other half once), C: frames 0-5 (for unrelated eager work)."""
    import torch
    w = sg.tiny()
    dev = torch.from_numpy(w.frames()).cuda()
    ctx = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=8192)
    A, B, C = ctx.submap_create(), ctx.submap_create(), ctx.submap_create()
    for f in range(20):
        for _ in range(2):
            ctx.integrate_depth(A if f < 10 else B, dev[f], w.cam.K, w.poses[f])
        if f % 5 == 0:
            ctx.integrate_depth(B if f < 10 else A, dev[f], w.cam.K, w.poses[f])
    for f in range(6):
        ctx.integrate_depth(C, dev[f], w.cam.K, w.poses[f])
    for s in (A, B, C):
        ctx.update_esdf(s)
    return ctx, w, dev, A, B, C


def _pairs(A, B, n=6):
    rng = np.random.default_rng(4)
    out = []
    for k in range(n):
        xi = np.concatenate([rng.uniform(-0.05, 0.05, 3), rng.uniform(-0.03, 0.03, 3)])
        out.append((A, B, orc.se3_exp(xi)) if k % 2 == 0 else (B, A, orc.se3_exp(xi)))
    return out


def _same(a, b):
    Ta, ca, sa = a
    Tb, cb, sb = b
    assert np.array_equal(Ta, Tb)
    assert np.array_equal(ca, cb)
    assert sa == sb


@pytest.mark.parametrize("solver", ["gn", "lm"])
def test_set_equals_align_batch(cv, solver):
    ctx, w, dev, A, B, C = _maps(cv)
    if solver == "lm":
        ctx.set_params(align_solver=cv.LEVENBERG_MARQUARDT)
    pairs = _pairs(A, B)
    for n_starts in (1, 8):
        ref = ctx.align_batch(pairs, n_starts)
        st = ctx.align_prepare(pairs, n_starts)
        st.launch()
        _same(st.collect(), ref)
        st.launch()  # a second launch over the same device problems
        _same(st.collect(), ref)
        # the set keeps the solver it was prepared with
        ctx.set_params(align_solver=cv.GAUSS_NEWTON if solver == "lm" else cv.LEVENBERG_MARQUARDT)
        st.launch()
        _same(st.collect(), ref)
        ctx.set_params(align_solver=cv.LEVENBERG_MARQUARDT if solver == "lm" else cv.GAUSS_NEWTON)
        st.close()
    ctx.close()


def test_graph_replays_equal_eager(cv):
    ctx, w, dev, A, B, C = _maps(cv)
    pairs = _pairs(A, B, 8)
    ref = ctx.align_batch(pairs, 8)
    other = [(A, B, orc.se3_exp(np.array([0.1, 0.0, 0.0, 0.0, 0.0, math.radians(20)])))]
    ref_other = ctx.align_batch(other, 1)
    st = ctx.align_prepare(pairs, 8)  # never launched eagerly: the results come from the replays
    T0s, c0s, s0s = st.collect()  # before any run: the starts, unmoved, not converged
    assert np.all(np.isinf(c0s)) and all(x["status"] == cv.NOT_CONVERGED and x["iterations"] == 0 for x in s0s)
    ctx.graph_begin()
    st.launch()
    g = ctx.graph_end()
    for rep in range(3):
        g.launch()
        _same(st.collect(), ref)
        # eager work between replays: another batch, and mapping into C
        _same(ctx.align_batch(other, 1), ref_other)
        ctx.integrate_depth(C, dev[6 + rep], w.cam.K, w.poses[6 + rep])
        ctx.update_esdf(C)
    g.close()
    st.close()
    ctx.close()


def test_changed_submaps_are_refused(cv):
    ctx, w, dev, A, B, C = _maps(cv)
    pairs = _pairs(A, B, 2)
    st = ctx.align_prepare(pairs, 1)
    ctx.graph_begin()
    st.launch()
    g = ctx.graph_end()
    g.launch()
    ref = st.collect()
    # a capture that aligns A and also changes it is refused
    ctx.graph_begin()
    st.launch()
    ctx.update_esdf(A)
    with pytest.raises(cv.CovoxError):
        ctx.graph_end()
    # B changes: the set and the graph refuse to run; results stay as they were
    ctx.integrate_depth(B, dev[3], w.cam.K, w.poses[3])
    ctx.update_esdf(B)
    with pytest.raises(cv.CovoxError):
        st.launch()
    with pytest.raises(cv.CovoxError):
        g.launch()
    _same(st.collect(), ref)
    # a set prepared now runs, eagerly and captured
    st2 = ctx.align_prepare(pairs, 1)
    st2.launch()
    r2 = st2.collect()
    _same(r2, ctx.align_batch(pairs, 1))
    g.close()
    st.close()
    st2.close()
    ctx.close()


def test_set_outlives_its_context_as_a_handle(cv):
    ctx, w, dev, A, B, C = _maps(cv)
    st = ctx.align_prepare(_pairs(A, B, 2), 1)
    ctx.close()
    st.close()  # frees nothing more, and does not touch the closed context
