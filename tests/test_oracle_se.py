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
