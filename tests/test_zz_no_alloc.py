"""The network forward pass that allocates nothing
(covox_net_forward_noalloc), through the C ABI, against the allocating
covox_net_forward on the same inputs.

Both run the same kernels on the same weights, so the outputs must be equal
bit for bit; they are also held to the forward pass's oracle bar (2 % of the
output scale, bf16 activations).  Two calls in a row, the second with fewer
pairs, check that nothing of the first call's activations leaks into the
second.  A batch above the stated maximum is refused without a launch."""
import numpy as np
import pytest

import oracle as orc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_21149_amd as cv
    return cv


def _inputs(n, seed):
    """Summary-like inputs: smooth fields in [-1, 1] with masks, masked cells 0."""
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
            x[b, :, :, :, 2 * side] = v.transpose(2, 1, 0)
            x[b, :, :, :, 2 * side + 1] = mask.transpose(2, 1, 0)
    return x


def test_forward_noalloc_matches_allocating_forward(cv):
    import torch
    ctx = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=1024)
    net = cv.Net(ctx, seed=21)
    p = net.get_params()
    nmax = cv.NET_NOALLOC_MAX_PAIRS
    x = _inputs(nmax, 5)
    xd = torch.from_numpy(x).cuda()
    # first call: the full batch; second call: three pairs taken from the end
    for sl in (slice(0, nmax), slice(nmax - 3, nmax)):
        xs = xd[sl].contiguous()
        out = torch.full((xs.shape[0], 5), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(xs, out)
        ref = net.forward(xs)
        torch.cuda.synchronize()
        g, r = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), np.abs(g - r).max()
        o = orc.net_forward(p, x[sl], bf16=True)
        assert np.abs(g.astype(np.float64) - o).max() <= 0.02 * np.abs(o).max()
    # a batch beyond the maximum is refused
    big = torch.zeros((nmax + 1, 32, 32, 32, 4), dtype=torch.float32, device="cuda")
    out = torch.zeros((nmax + 1, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(cv.CovoxError) as e:
        net.forward_noalloc(big, out)
    assert e.value.code == cv.EINVAL
    assert torch.count_nonzero(out).item() == 0
    net.close()
    ctx.close()


def test_forward_noalloc_two_contexts_share_the_device_array(cv):
    """A second context on the same GPU uses the same array; sequential calls
    from the two give the outputs of their own nets."""
    import torch
    c1 = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=1024)
    c2 = cv.Context(voxel_size=0.05, trunc_vox=4, max_range=5.0, d_max=2.0, block_capacity=1024)
    n1, n2 = cv.Net(c1, seed=3), cv.Net(c2, seed=4)
    x = torch.from_numpy(_inputs(2, 9)).cuda()
    o1 = torch.empty((2, 5), dtype=torch.float32, device="cuda")
    o2 = torch.empty((1, 5), dtype=torch.float32, device="cuda")
    n1.forward_noalloc(x, o1)
    torch.cuda.synchronize()
    n2.forward_noalloc(x[:1].contiguous(), o2)
    torch.cuda.synchronize()
    assert np.array_equal(o1.cpu().numpy(), n1.forward(x).cpu().numpy())
    assert np.array_equal(o2.cpu().numpy(), n2.forward(x[:1].contiguous()).cpu().numpy())
    for h in (n1, n2):
        h.close()
    c1.close()
    c2.close()
