"""Pins of the FP64 oracle of the depthwise-separable convolution (CPU).

Pinned by: the dense 3x3x3 convolution with a diagonal weight tensor (itself
pinned to brute force), torch's grouped convolution (groups = channels) and
its autograd in float64, the adjoint identity, central finite differences of
the composed operator, and a planted mistake (flipped taps) that the dense
comparison catches."""
import numpy as np
import pytest

from oracle import dwsep, net

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _rand(rng, C=4, n=5, Co=3):
    x = rng.standard_normal((C, n, n, n))
    wd = rng.standard_normal((C, 3, 3, 3))
    bd = rng.standard_normal(C)
    wp = rng.standard_normal((Co, C))
    bp = rng.standard_normal(Co)
    return x, wd, bd, wp, bp


def test_depthwise_equals_dense_conv_with_diagonal_weights():
    rng = np.random.default_rng(0)
    x, wd, bd, _, _ = _rand(rng)
    C = x.shape[0]
    dense = np.zeros((C, C, 3, 3, 3))
    for c in range(C):
        dense[c, c] = wd[c]
    np.testing.assert_allclose(dwsep.dwconv3d(x, wd, bd), net.conv3d(x, dense, bd),
                               rtol=1e-12, atol=1e-12)


def test_depthwise_matches_torch_grouped_conv_and_autograd():
    rng = np.random.default_rng(1)
    x, wd, bd, _, _ = _rand(rng, C=6, n=6)
    C = x.shape[0]
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(wd[:, None], requires_grad=True)   # [C, 1, 3, 3, 3]
    bt = torch.tensor(bd, requires_grad=True)
    yt = F.conv3d(xt[None], wt, bt, padding=1, groups=C)[0]
    np.testing.assert_allclose(dwsep.dwconv3d(x, wd, bd), yt.detach().numpy(), rtol=1e-11,
                               atol=1e-11)
    g = rng.standard_normal(x.shape)
    (yt * torch.tensor(g)).sum().backward()
    gx, gw, gb = dwsep.dwconv3d_backward(x, wd, g)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gw, wt.grad.numpy()[:, 0], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_depthwise_adjoint_identity():
    rng = np.random.default_rng(2)
    x, wd, _, _, _ = _rand(rng, C=3, n=7)
    g = rng.standard_normal(x.shape)
    lhs = (dwsep.dwconv3d(x, wd, np.zeros(3)) * g).sum()
    gx, _, _ = dwsep.dwconv3d_backward(x, wd, g)
    assert lhs == pytest.approx((gx * x).sum(), rel=1e-12)


def test_pointwise_equals_dense_1x1_conv():
    rng = np.random.default_rng(3)
    x, _, _, wp, bp = _rand(rng)
    np.testing.assert_allclose(dwsep.pwconv3d(x, wp, bp),
                               net.conv3d(x, wp[:, :, None, None, None], bp), rtol=1e-12,
                               atol=1e-12)
    g = rng.standard_normal((wp.shape[0],) + x.shape[1:])
    gx, gw, gb = dwsep.pwconv3d_backward(x, wp, g)
    rx, rw, rb = net.conv3d_backward(x, wp[:, :, None, None, None], g)
    np.testing.assert_allclose(gx, rx, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gw, rw[:, :, 0, 0, 0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gb, rb, rtol=1e-12, atol=1e-12)


def test_composition_matches_torch_and_finite_differences():
    rng = np.random.default_rng(4)
    x, wd, bd, wp, bp = _rand(rng, C=4, n=5, Co=3)
    C = x.shape[0]
    y, d = dwsep.dwsep_conv3d(x, wd, bd, wp, bp)
    ref = F.conv3d(F.conv3d(torch.tensor(x)[None], torch.tensor(wd[:, None]), torch.tensor(bd),
                            padding=1, groups=C),
                   torch.tensor(wp[:, :, None, None, None]), torch.tensor(bp))[0].numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-11)
    R = rng.standard_normal(y.shape)
    gx, gwd, gbd, gwp, gbp = dwsep.dwsep_conv3d_backward(x, wd, wp, d, R)
    f = lambda xx, a, b_, c, e: (dwsep.dwsep_conv3d(xx, a, b_, c, e)[0] * R).sum()
    h = 1e-6
    for grad, k in ((gx, 0), (gwd, 1), (gbd, 2), (gwp, 3), (gbp, 4)):
        args = [x, wd, bd, wp, bp]
        v = rng.standard_normal(args[k].shape)
        plus = list(args)
        minus = list(args)
        plus[k] = args[k] + h * v
        minus[k] = args[k] - h * v
        fd = (f(*plus) - f(*minus)) / (2 * h)
        assert fd == pytest.approx((grad * v).sum(), rel=1e-6), k


def test_planted_tap_flip_is_caught():
    rng = np.random.default_rng(5)
    x, wd, bd, _, _ = _rand(rng)
    C = x.shape[0]
    dense = np.zeros((C, C, 3, 3, 3))
    for c in range(C):
        dense[c, c] = wd[c]
    flipped = dwsep.dwconv3d(x, wd[:, ::-1, ::-1, ::-1], bd)
    assert not np.allclose(flipped, net.conv3d(x, dense, bd))


def _sep_and_dense_thetas(rng, levels, C):
    """A depthwise-separable network whose depthwise convolutions are the
    identity (centre tap 1, bias 0) and the dense network it then equals:
    each dense 3x3x3 convolution is zero except its centre tap, which holds
    the pointwise weights."""
    ts_ = rng.standard_normal(net.n_params(levels, C, sep=True)) * 0.3
    Ps = net.unpack(ts_, levels, C, sep=True)
    td = np.zeros(net.n_params(levels, C))
    Pd = net.unpack(td, levels, C)
    for mod, d in Ps.items():
        for name, v in d.items():
            if name.endswith(".dw"):
                v[...] = 0.0
                v[:, 1, 1, 1] = 1.0
            elif name.endswith(".dwb"):
                v[...] = 0.0
    for mod, d in Pd.items():
        for name, v in d.items():
            if name in ("conv1.w", "conv2.w"):
                v[:, :, 1, 1, 1] = Ps[mod][name[:-2] + ".pw"]
            elif name in ("conv1.b", "conv2.b"):
                v[...] = Ps[mod][name[:-2] + ".pwb"]
            else:
                v[...] = Ps[mod][name]
    return ts_, td


def test_separable_network_with_identity_depthwise_equals_dense_network():
    rng = np.random.default_rng(6)
    n, L, C = 8, 2, 4
    ts_, td = _sep_and_dense_thetas(rng, L, C)
    Z = rng.standard_normal(n ** 3)
    ys, cs = net.forward(ts_, Z, n, L, C, sep=True)
    yd, cd = net.forward(td, Z, n, L, C)
    np.testing.assert_allclose(ys, yd, rtol=1e-10, atol=1e-10)
    g = rng.standard_normal((n, n, n))
    gs = net.unpack(net.backward(g, ts_, cs, n, L, C, sep=True), L, C, sep=True)
    gd = net.unpack(net.backward(g, td, cd, n, L, C), L, C)
    for mod, d in gd.items():
        for name, v in d.items():
            if name in ("conv1.w", "conv2.w"):
                ref, got = v[:, :, 1, 1, 1], gs[mod][name[:-2] + ".pw"]
            elif name in ("conv1.b", "conv2.b"):
                ref, got = v, gs[mod][name[:-2] + ".pwb"]
            else:
                ref, got = v, gs[mod][name]
            np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9, err_msg=mod + "." + name)


def test_separable_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    n, L, C = 4, 2, 4
    th = rng.standard_normal(net.n_params(L, C, sep=True)) * 0.3
    Z = rng.standard_normal(n ** 3)
    R = rng.standard_normal((n, n, n))
    y, cache = net.forward(th, Z, n, L, C, sep=True)
    g = net.backward(R, th, cache, n, L, C, sep=True)
    f = lambda t: (net.forward(t, Z, n, L, C, sep=True)[0] * R).sum()
    h = 1e-6
    P = net.unpack(np.arange(th.size, dtype=np.float64), L, C, sep=True)
    for mod, name in (("enc0", "conv1.dw"), ("dec0", "conv2.pw"), ("enc1", "conv1.dwb"),
                      (None, None)):
        v = np.zeros_like(th)
        if mod is None:
            v = rng.standard_normal(th.size)
        else:
            idx = P[mod][name].astype(int).ravel()
            v[idx] = rng.standard_normal(idx.size)
        fd = (f(th + h * v) - f(th - h * v)) / (2 * h)
        assert fd == pytest.approx(float(g @ v), rel=1e-6), (mod, name)


@pytest.mark.parametrize("dil", [2, 3])
def test_dilated_depthwise_matches_torch_and_autograd(dil):
    rng = np.random.default_rng(20 + dil)
    x, wd, bd, _, _ = _rand(rng, C=4, n=7)
    C = x.shape[0]
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(wd[:, None], requires_grad=True)
    bt = torch.tensor(bd, requires_grad=True)
    yt = F.conv3d(xt[None], wt, bt, padding=dil, dilation=dil, groups=C)[0]
    np.testing.assert_allclose(dwsep.dwconv3d(x, wd, bd, dil), yt.detach().numpy(),
                               rtol=1e-11, atol=1e-11)
    g = rng.standard_normal(x.shape)
    (yt * torch.tensor(g)).sum().backward()
    gx, gw, gb = dwsep.dwconv3d_backward(x, wd, g, dil)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gw, wt.grad.numpy()[:, 0], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_dilation_beyond_the_grid_leaves_only_the_centre_tap():
    """With dil >= n every off-centre tap falls outside the grid."""
    rng = np.random.default_rng(23)
    x, wd, bd, _, _ = _rand(rng, C=4, n=3)
    y = dwsep.dwconv3d(x, wd, bd, dil=3)
    np.testing.assert_allclose(y, bd[:, None, None, None] + wd[:, 1, 1, 1, None, None, None] * x,
                               rtol=1e-14, atol=1e-14)
