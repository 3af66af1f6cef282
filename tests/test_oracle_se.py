"""Pins of the FP64 oracle of the Squeeze-and-Excitation unit (CPU).

Pinned by: torch's own pooling, linear, ReLU and sigmoid in float64 and their
autograd; special cases with closed forms (zero excitation weights give a
gate of exactly 1/2; a constant input gives s = that constant); central
finite differences; and a planted mistake (the pooled mean's 1/V dropped
from the input gradient) that the finite differences catch."""
import numpy as np
import pytest

from oracle import se

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _rand(rng, C=8, H=2, n=5):
    x = rng.standard_normal((C, n, n, n))
    w1 = rng.standard_normal((H, C))
    b1 = rng.standard_normal(H)
    w2 = rng.standard_normal((C, H))
    b2 = rng.standard_normal(C)
    return x, w1, b1, w2, b2


def test_matches_torch_and_autograd():
    rng = np.random.default_rng(0)
    x, w1, b1, w2, b2 = _rand(rng)
    t = [torch.tensor(a, requires_grad=True) for a in (x, w1, b1, w2, b2)]
    s = F.adaptive_avg_pool3d(t[0][None], 1).flatten()
    e = torch.sigmoid(F.linear(torch.relu(F.linear(s, t[1], t[2])), t[3], t[4]))
    yt = t[0] * e[:, None, None, None]
    y, cache = se.se_forward(x, w1, b1, w2, b2)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    g = rng.standard_normal(x.shape)
    (yt * torch.tensor(g)).sum().backward()
    got = se.se_backward(x, w1, w2, cache, g)
    for a, b in zip(got, t):
        np.testing.assert_allclose(a, b.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_closed_forms():
    rng = np.random.default_rng(1)
    x, w1, b1, w2, b2 = _rand(rng)
    y, c = se.se_forward(x, w1, b1, np.zeros_like(w2), np.zeros_like(b2))
    np.testing.assert_array_equal(c["e"], np.full(x.shape[0], 0.5))
    np.testing.assert_allclose(y, 0.5 * x, rtol=0, atol=0)
    xc = np.broadcast_to(np.arange(8.0)[:, None, None, None], x.shape).copy()
    _, c = se.se_forward(xc, w1, b1, w2, b2)
    np.testing.assert_allclose(c["s"], np.arange(8.0), rtol=1e-15)


def _fd_check(backward):
    rng = np.random.default_rng(2)
    args = list(_rand(rng, C=6, H=3, n=4))
    R = rng.standard_normal(args[0].shape)
    f = lambda a: (se.se_forward(*a)[0] * R).sum()
    _, cache = se.se_forward(*args)
    grads = backward(args[0], args[1], args[3], cache, R)
    h = 1e-6
    ok = True
    for k, gk in zip((0, 1, 2, 3, 4), grads):
        v = rng.standard_normal(args[k].shape)
        p, m = list(args), list(args)
        p[k] = args[k] + h * v
        m[k] = args[k] - h * v
        fd = (f(p) - f(m)) / (2 * h)
        ok &= fd == pytest.approx(float((gk * v).sum()), rel=1e-6)
    return ok


def test_gradients_match_finite_differences():
    assert _fd_check(se.se_backward)


def test_planted_missing_mean_scale_is_caught():
    def bad(x, w1, w2, cache, gy):
        gx, a, b, c, d = se.se_backward(x, w1, w2, cache, gy)
        V = x[0].size
        e = cache["e"][:, None, None, None]
        gs_over_v = gx - gy * e
        return gy * e + gs_over_v * V, a, b, c, d   # 1/V dropped
    assert not _fd_check(bad)


def test_network_with_saturated_gates_equals_plain_network():
    """SE units whose gates are 1 (w2 = 0, b2 = 40: sigmoid(40) rounds to 1 in
    FP64) leave the network unchanged: same image, same gradient for every
    shared parameter, zero gradient for w1 and b1."""
    from oracle import net
    rng = np.random.default_rng(3)
    n, L, C, r = 8, 3, 4, 2
    th_se = rng.standard_normal(net.n_params(L, C, se_ratio=r)) * 0.3
    P = net.unpack(th_se, L, C, se_ratio=r)
    th = np.zeros(net.n_params(L, C))
    Pp = net.unpack(th, L, C)
    for mod, d in P.items():
        for name, v in d.items():
            if name == "se.w2":
                v[...] = 0.0
            elif name == "se.b2":
                v[...] = 40.0
            elif not name.startswith("se."):
                Pp[mod][name][...] = v
    Z = rng.standard_normal(n ** 3)
    y_se, c_se = net.forward(th_se, Z, n, L, C, se_ratio=r)
    y, c = net.forward(th, Z, n, L, C)
    np.testing.assert_array_equal(y_se, y)
    g = rng.standard_normal((n, n, n))
    G_se = net.unpack(net.backward(g, th_se, c_se, n, L, C, se_ratio=r), L, C, se_ratio=r)
    G = net.unpack(net.backward(g, th, c, n, L, C), L, C)
    for mod, d in G.items():
        for name, v in d.items():
            np.testing.assert_allclose(G_se[mod][name], v, rtol=1e-12, atol=1e-14,
                                       err_msg=mod + "." + name)
    for l in range(L):
        assert not G_se["enc%d" % l]["se.w1"].any() and not G_se["enc%d" % l]["se.b1"].any()


def test_network_with_se_units_matches_finite_differences():
    from oracle import net
    rng = np.random.default_rng(4)
    n, L, C, r = 4, 2, 4, 2
    th = rng.standard_normal(net.n_params(L, C, se_ratio=r)) * 0.3
    Z = rng.standard_normal(n ** 3)
    R = rng.standard_normal((n, n, n))
    y, cache = net.forward(th, Z, n, L, C, se_ratio=r)
    g = net.backward(R, th, cache, n, L, C, se_ratio=r)
    f = lambda t: (net.forward(t, Z, n, L, C, se_ratio=r)[0] * R).sum()
    idx = net.unpack(np.arange(th.size, dtype=np.float64), L, C, se_ratio=r)
    h = 1e-6
    for mod, name in (("enc0", "se.w1"), ("enc1", "se.w2"), ("enc1", "se.b1"),
                      ("enc0", "conv1.w"), (None, None)):
        v = np.zeros_like(th)
        if mod is None:
            v = rng.standard_normal(th.size)
        else:
            ii = idx[mod][name].astype(int).ravel()
            v[ii] = rng.standard_normal(ii.size)
        fd = (f(th + h * v) - f(th - h * v)) / (2 * h)
        assert fd == pytest.approx(float(g @ v), rel=1e-6), (mod, name)
