"""Pins of the oracle network's 3D-FastResUNet modules (CPU): the attention
units on the decoder skips and the sigmoid tail, alone and together with the
depthwise-separable convolutions and the SE units.

Pinned by: the attention unit against an independent torch float64
formulation (2x2x2 average pool, 1x1x1 convolutions, ReLU, sigmoid, nearest
interpolation, autograd), with non-symmetric weights and a skip and gating
signal of equal width so that a transposed weight or swapped inputs change
the result; saturated attention gates reducing the network to the plain one
(same image, same gradient, zero attention gradients); the sigmoid tail
equal to tanh of half the linear tail's output (2 sigmoid(t) - 1 = tanh(t/2));
and central finite differences of every module's parameters."""
import numpy as np
import pytest

from oracle import net


def _fd(th, f, g, idx_sets, rng, h=1e-6):
    for ii in idx_sets:
        v = np.zeros_like(th)
        if ii is None:
            v = rng.standard_normal(th.size)
        else:
            v[ii] = rng.standard_normal(ii.size)
        fd = (f(th + h * v) - f(th - h * v)) / (2 * h)
        # abs: the rounding floor of the difference quotient, ~eps |f| / h
        assert fd == pytest.approx(float(g @ v), rel=1e-6, abs=1e-9)


def _torch_attention(x, g, Q):
    """The attention unit written with torch float64 operations: gate on the
    gating signal's grid from the pooled skip, interpolated to the skip."""
    import torch
    import torch.nn.functional as F
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    X, G = t(x[None]), t(g[None])
    W = {k: t(v) for k, v in Q.items()}
    k1 = lambda w: w[:, :, None, None, None]
    a = (F.conv3d(F.avg_pool3d(X, 2), k1(W["att.wx"])) + F.conv3d(G, k1(W["att.wg"])) +
         W["att.b"].view(1, -1, 1, 1, 1))
    al = torch.sigmoid(F.conv3d(torch.relu(a), W["att.psi"].view(1, -1, 1, 1, 1)) +
                       W["att.bpsi"][0])
    return X, G, W, F.interpolate(al, scale_factor=2, mode="nearest") * X


def _att_inputs(c, cu, m, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((c, 2 * m, 2 * m, 2 * m))
    g = rng.standard_normal((cu, m, m, m))
    Q = {"att.wx": rng.standard_normal((c, c)), "att.wg": rng.standard_normal((c, cu)),
         "att.b": rng.standard_normal(c), "att.psi": rng.standard_normal(c),
         "att.bpsi": rng.standard_normal(1)}
    return x, g, Q, rng.standard_normal(x.shape)


@pytest.mark.parametrize("c,cu,m", [(4, 4, 3), (3, 6, 2)])
def test_attention_unit_matches_torch_float64(c, cu, m):
    x, g, Q, R = _att_inputs(c, cu, m, 20 + c + cu)
    y, cache = net.att_forward(x, g, Q)
    X, G, W, yt = _torch_attention(x, g, Q)
    np.testing.assert_allclose(y, yt.detach().numpy()[0], rtol=1e-12, atol=1e-13)
    gx, gg, grads = net.att_backward(R, Q, cache)
    import torch
    (yt * torch.tensor(R[None])).sum().backward()
    np.testing.assert_allclose(gx, X.grad.numpy()[0], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(gg, G.grad.numpy()[0], rtol=1e-11, atol=1e-12)
    for k in Q:
        np.testing.assert_allclose(grads[k], W[k].grad.numpy(), rtol=1e-11, atol=1e-12,
                                   err_msg=k)


def test_saturated_attention_gates_give_the_plain_network():
    rng = np.random.default_rng(10)
    n, L, C = 8, 3, 4
    th_a = rng.standard_normal(net.n_params(L, C, att=True)) * 0.3
    P = net.unpack(th_a, L, C, att=True)
    th = np.zeros(net.n_params(L, C))
    Pp = net.unpack(th, L, C)
    for mod, d in P.items():
        for name, v in d.items():
            if name in ("att.wx", "att.wg", "att.b"):
                v[...] = 0.0
            elif name == "att.bpsi":
                v[...] = 40.0
            elif not name.startswith("att."):
                Pp[mod][name][...] = v
    Z = rng.standard_normal(n ** 3)
    ya, ca = net.forward(th_a, Z, n, L, C, att=True)
    y, c = net.forward(th, Z, n, L, C)
    np.testing.assert_array_equal(ya, y)
    g = rng.standard_normal((n, n, n))
    Ga = net.unpack(net.backward(g, th_a, ca, n, L, C, att=True), L, C, att=True)
    G = net.unpack(net.backward(g, th, c, n, L, C), L, C)
    for mod, d in G.items():
        for name, v in d.items():
            np.testing.assert_allclose(Ga[mod][name], v, rtol=1e-12, atol=1e-14,
                                       err_msg=mod + "." + name)
    for mod, d in Ga.items():
        for name, v in d.items():
            if name.startswith("att."):
                assert not v.any(), mod + "." + name


def test_sigmoid_tail_is_tanh_of_half_the_linear_tail():
    rng = np.random.default_rng(11)
    n, L, C = 8, 2, 4
    th = rng.standard_normal(net.n_params(L, C)) * 0.3
    Z = rng.standard_normal(n ** 3)
    ys, _ = net.forward(th, Z, n, L, C, tail="sigmoid")
    yl, _ = net.forward(th, Z, n, L, C)
    np.testing.assert_allclose(ys, np.tanh(yl / 2), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("sep,r,att,tail", [(False, 0, True, "linear"),
                                            (False, 0, False, "sigmoid"),
                                            (True, 2, True, "sigmoid")])
def test_module_gradients_match_finite_differences(sep, r, att, tail):
    rng = np.random.default_rng(12 + 2 * att + r)
    n, L, C = 4, 2, 4
    th = rng.standard_normal(net.n_params(L, C, sep, r, att)) * 0.3
    Z = rng.standard_normal(n ** 3)
    R = rng.standard_normal((n, n, n))
    kw = dict(sep=sep, se_ratio=r, att=att, tail=tail)
    y, cache = net.forward(th, Z, n, L, C, **kw)
    g = net.backward(R, th, cache, n, L, C, **kw)
    f = lambda t: (net.forward(t, Z, n, L, C, **kw)[0] * R).sum()
    idx = net.unpack(np.arange(th.size, dtype=np.float64), L, C, sep, r, att)
    sets = [idx["tail"]["w"].astype(int).ravel(), None]
    if att:
        sets += [idx["dec0"][k].astype(int).ravel()
                 for k in ("att.wx", "att.wg", "att.b", "att.psi", "att.bpsi")]
    _fd(th, f, g, sets, rng)


def test_aspp_matches_torch_autograd():
    """The ASPP module against torch's float64 grouped, dilated and 1x1x1
    convolutions and autograd."""
    import torch
    F = torch.nn.functional
    rng = np.random.default_rng(30)
    c, n = 4, 6
    x = rng.standard_normal((c, n, n, n))
    Q = {k: rng.standard_normal(s) * 0.4 for k, s in net._aspp_shapes(c)}
    y, cache = net.aspp_forward(x, Q)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in Q.items()}
    xt = torch.tensor(x, requires_grad=True)
    pw = lambda t, w, b: F.conv3d(t[None], w[:, :, None, None, None], b)[0]
    br = [pw(xt, T["w0"], T["b0"])]
    for d in net.ASPP_RATES:
        dd = F.conv3d(xt[None], T["dw%d" % d][:, None], T["dwb%d" % d], padding=d, dilation=d,
                      groups=c)[0]
        br.append(pw(dd, T["pw%d" % d], T["pwb%d" % d]))
    yt = torch.relu(pw(torch.cat(br), T["wp"], T["bp"]))
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-11, atol=1e-11)
    g = rng.standard_normal(y.shape)
    (yt * torch.tensor(g)).sum().backward()
    gx, G = net.aspp_backward(g, Q, cache)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-10, atol=1e-11)
    for k in Q:
        np.testing.assert_allclose(G[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-11, err_msg=k)


def test_network_with_aspp_matches_finite_differences():
    rng = np.random.default_rng(31)
    n, L, C = 8, 2, 4
    kw = dict(aspp=True, sep=True)
    th = rng.standard_normal(net.n_params(L, C, sep=True, aspp=True)) * 0.3
    Z = rng.standard_normal(n ** 3)
    R = rng.standard_normal((n, n, n))
    y, cache = net.forward(th, Z, n, L, C, **kw)
    g = net.backward(R, th, cache, n, L, C, **kw)
    f = lambda t: (net.forward(t, Z, n, L, C, **kw)[0] * R).sum()
    idx = net.unpack(np.arange(th.size, dtype=np.float64), L, C, sep=True, aspp=True)
    sets = [idx["aspp"][k].astype(int).ravel() for k in ("w0", "dw2", "pw3", "wp", "dwb1")]
    _fd(th, f, g, sets + [None], rng)
