"""Pins of the oracle network's 3D-FastResUNet modules (CPU): the attention
units on the decoder skips and the sigmoid tail, alone and together with the
depthwise-separable convolutions and the SE units.

Pinned by: saturated attention gates reducing the network to the plain one
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
