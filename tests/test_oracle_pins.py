"""Pins of the FP64 oracle against what the mathematics fixes.

Each test pins the oracle to something other than itself: brute-force loops,
torch's CPU float64 library operations and autograd, adjoint identities,
central finite differences, LayerNorm invariants, Adam's closed forms and the
least-squares limit of gradient descent on the data term.
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import tseit_synth as ts
from oracle import net, fit



@pytest.fixture(autouse=True)
def _float64_torch():
    # torch builds its reference tensors in float64 inside this module only;
    # the default is restored so GPU tests collected in the same process keep
    # float32 defaults
    prev = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(prev)


def _rng(s):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# convolution
# --------------------------------------------------------------------------

def _conv_brute(x, w, b):
    cin, n = x.shape[0], x.shape[1]
    cout, k = w.shape[0], w.shape[2]
    p = k // 2
    out = np.zeros((cout, n, n, n))
    for co, z, y, xx in itertools.product(range(cout), range(n), range(n), range(n)):
        s = b[co]
        for ci, dz, dy, dx in itertools.product(range(cin), range(k), range(k), range(k)):
            zz, yy, x3 = z + dz - p, y + dy - p, xx + dx - p
            if 0 <= zz < n and 0 <= yy < n and 0 <= x3 < n:
                s += w[co, ci, dz, dy, dx] * x[ci, zz, yy, x3]
        out[co, z, y, xx] = s
    return out


@pytest.mark.parametrize("k", [3, 1])
def test_conv_brute_force(k):
    r = _rng(1)
    x = r.standard_normal((2, 4, 4, 4))
    w = r.standard_normal((3, 2, k, k, k))
    b = r.standard_normal(3)
    np.testing.assert_allclose(net.conv3d(x, w, b), _conv_brute(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv_delta_kernel_is_identity():
    r = _rng(2)
    x = r.standard_normal((3, 5, 5, 5))
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(net.conv3d(x, w, np.zeros(3)), x)


def test_conv_matches_torch():
    r = _rng(3)
    x = r.standard_normal((5, 6, 6, 6))
    w = r.standard_normal((4, 5, 3, 3, 3))
    b = r.standard_normal(4)
    ref = F.conv3d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b), padding=1)[0].numpy()
    np.testing.assert_allclose(net.conv3d(x, w, b), ref, rtol=1e-11, atol=1e-11)


def test_conv_backward_adjoint_and_torch():
    r = _rng(4)
    x = r.standard_normal((3, 6, 6, 6))
    w = r.standard_normal((2, 3, 3, 3, 3))
    g = r.standard_normal((2, 6, 6, 6))
    gx, gw, gb = net.conv3d_backward(x, w, g)
    # <conv(x), g> = <x, conv^T(g)> (bias-free)
    lhs = (net.conv3d(x, w, np.zeros(2)) * g).sum()
    assert lhs == pytest.approx((x * gx).sum(), rel=1e-12)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.zeros(2, requires_grad=True)
    (F.conv3d(xt[None], wt, bt, padding=1)[0] * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gw, wt.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-11, atol=1e-11)


# --------------------------------------------------------------------------
# LayerNorm, pooling, up-sampling
# --------------------------------------------------------------------------

def test_layernorm_invariants_and_torch_group_norm():
    r = _rng(5)
    h = r.standard_normal((4, 5, 5, 5)) * 3.0 + 1.5
    g = r.standard_normal(4)
    beta = r.standard_normal(4)
    y, (xhat, rstd) = net.layer_norm(h, g, beta)
    assert abs(xhat.mean()) < 1e-14
    assert xhat.var() == pytest.approx(h.var() / (h.var() + 1e-5), rel=1e-12)
    ref = F.group_norm(torch.tensor(h)[None], 1, torch.tensor(g), torch.tensor(beta), eps=1e-5)[0]
    np.testing.assert_allclose(y, ref.numpy(), rtol=1e-11, atol=1e-12)


def test_layernorm_backward_torch():
    r = _rng(6)
    h = r.standard_normal((3, 4, 4, 4)) + 0.7
    g = r.standard_normal(3)
    beta = r.standard_normal(3)
    go = r.standard_normal((3, 4, 4, 4))
    _, cache = net.layer_norm(h, g, beta)
    gh, gg, gb = net.layer_norm_backward(go, g, cache)
    ht = torch.tensor(h, requires_grad=True)
    gt = torch.tensor(g, requires_grad=True)
    bt = torch.tensor(beta, requires_grad=True)
    (F.group_norm(ht[None], 1, gt, bt, eps=1e-5)[0] * torch.tensor(go)).sum().backward()
    np.testing.assert_allclose(gh, ht.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gg, gt.grad.numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-11, atol=1e-12)


def test_pool_and_up_against_torch_and_adjoints():
    r = _rng(7)
    x = r.standard_normal((3, 8, 8, 8))
    np.testing.assert_allclose(net.avgpool2(x), F.avg_pool3d(torch.tensor(x)[None], 2)[0].numpy(),
                               rtol=1e-13)
    s = r.standard_normal((3, 4, 4, 4))
    np.testing.assert_array_equal(
        net.up2(s), F.interpolate(torch.tensor(s)[None], scale_factor=2, mode="nearest")[0].numpy())
    # <up(s), x> = <s, up^T(x)> and <pool(x), s> = <x, pool^T(s)>
    assert (net.up2(s) * x).sum() == pytest.approx((s * net.up2_backward(x)).sum(), rel=1e-12)
    assert (net.avgpool2(x) * s).sum() == pytest.approx((x * net.avgpool2_backward(s)).sum(), rel=1e-12)


# --------------------------------------------------------------------------
# the whole network
# --------------------------------------------------------------------------

def _torch_net(theta, Z, n, levels, C):
    """The same architecture written with torch.nn.functional (float64 CPU)."""
    P = {}
    off = 0
    for name, shape, _ in ts.param_specs(levels, C):
        k = int(np.prod(shape))
        P[name] = theta[off:off + k].view(shape)
        off += k

    def ln(h, pre):
        return F.group_norm(h, 1, P[pre + ".g"], P[pre + ".beta"], eps=1e-5)

    def block(x, pre):
        h = F.relu(ln(F.conv3d(x, P[pre + ".conv1.w"], P[pre + ".conv1.b"], padding=1), pre + ".norm1"))
        h = ln(F.conv3d(h, P[pre + ".conv2.w"], P[pre + ".conv2.b"], padding=1), pre + ".norm2")
        s = F.conv3d(x, P[pre + ".proj.w"], P[pre + ".proj.b"]) if pre + ".proj.w" in P else x
        return F.relu(h + s)

    z = Z.view(1, 1, n, n, n)
    a = F.relu(ln(F.conv3d(z, P["stem.conv.w"], P["stem.conv.b"], padding=1), "stem.norm"))
    enc = []
    x = a
    for l in range(levels):
        if l:
            x = F.avg_pool3d(enc[-1], 2)
        enc.append(block(x, "enc%d" % l))
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        d = block(torch.cat([F.interpolate(d, scale_factor=2, mode="nearest"), enc[l]], 1), "dec%d" % l)
    return F.conv3d(d, P["tail.w"], P["tail.b"])[0, 0]


def test_layouts_agree():
    for L, C in [(2, 8), (3, 16), (4, 32), (3, 8)]:
        a = [(m + "." + p, s) for m, ps in net.module_list(L, C) for p, s in ps]
        b = [(nm, s) for nm, s, _ in ts.param_specs(L, C)]
        assert a == b
        assert net.n_params(L, C) == ts.param_count(L, C)


@pytest.mark.parametrize("n,L,C", [(8, 2, 2), (16, 3, 4)])
def test_network_forward_backward_vs_torch_autograd(n, L, C):
    r = _rng(8)
    theta = ts.kaiming_theta(L, C, 11, fp32=False)
    # perturb gains/shifts/biases so every parameter class is non-trivial
    theta = theta + 0.1 * r.standard_normal(theta.size)
    Z = r.standard_normal(n ** 3)
    go = r.standard_normal((n, n, n))
    out, cache = net.forward(theta, Z, n, L, C)
    g = net.backward(go, theta, cache, n, L, C)
    tt = torch.tensor(theta, requires_grad=True)
    ref = _torch_net(tt, torch.tensor(Z), n, L, C)
    np.testing.assert_allclose(out, ref.detach().numpy(), rtol=1e-10, atol=1e-10)
    (ref * torch.tensor(go)).sum().backward()
    np.testing.assert_allclose(g, tt.grad.numpy(), rtol=1e-9, atol=1e-10)


def test_full_loss_gradient_finite_differences():
    """Central FD of the data term of Eq. (4) w.r.t. sampled theta entries."""
    n, L, C = 8, 2, 2
    r = _rng(9)
    J, mask = ts.sensitivity_matrix(n, 1)
    J = J[:40]
    theta = ts.kaiming_theta(L, C, 3, fp32=False) + 0.05 * r.standard_normal(ts.param_count(L, C))
    Z = r.standard_normal(n ** 3)
    dv = r.standard_normal(40) * 0.1
    pr = fit.Problem(J, mask, Z, n, L, C)
    L0, g, _ = pr.loss_and_grad(theta, dv)
    # every parameter tensor gets sampled
    idx = []
    off = 0
    for _, shape, _ in ts.param_specs(L, C):
        k = int(np.prod(shape))
        idx += list(off + r.choice(k, size=min(k, 3), replace=False))
        off += k
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (pr.loss_and_grad(tp, dv)[0] - pr.loss_and_grad(tm, dv)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=2e-5, abs=1e-9), i


# --------------------------------------------------------------------------
# data term and Adam
# --------------------------------------------------------------------------

def test_data_loss_least_squares_limit():
    """Gradient descent on sigma alone (identity network) from 0 converges to
    the minimum-norm least-squares solution of J sigma = dv."""
    r = _rng(10)
    J = r.standard_normal((12, 30))
    dv = r.standard_normal(12)
    s = np.zeros(30)
    M = J.shape[0]
    step = 0.9 * M / (2.0 * np.linalg.norm(J, 2) ** 2)
    for _ in range(20000):
        _, gs = fit.data_loss(J, dv, s)
        s -= step * gs
    ref = np.linalg.lstsq(J, dv, rcond=None)[0]
    np.testing.assert_allclose(s, ref, rtol=1e-8, atol=1e-10)
    L, _ = fit.data_loss(J, dv, ref)
    assert L < 1e-20


def test_data_loss_value():
    J = np.array([[1.0, 2.0], [0.0, -1.0], [3.0, 1.0]])
    s = np.array([0.5, -1.0])
    dv = np.array([1.0, 0.0, 2.0])
    # r = [-1.5 - 1, 1 - 0, 0.5 - 2] = [-2.5, 1, -1.5]
    L, g = fit.data_loss(J, dv, s)
    assert L == pytest.approx((6.25 + 1 + 2.25) / 3)
    np.testing.assert_allclose(g, (2 / 3) * J.T @ np.array([-2.5, 1.0, -1.5]))


def test_adam_first_step_closed_form():
    r = _rng(11)
    th = r.standard_normal(50)
    g = r.standard_normal(50)
    lr = 1e-3
    th1, m, v, t = fit.adam_step(th, g, np.zeros(50), np.zeros(50), 0, lr)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert t == 1


def test_adam_constant_gradient_steps_are_equal():
    r = _rng(12)
    th = r.standard_normal(20)
    g = r.standard_normal(20)
    m = np.zeros(20)
    v = np.zeros(20)
    t = 0
    prev = th
    for _ in range(30):
        th, m, v, t = fit.adam_step(th, g, m, v, t, 1e-2)
        np.testing.assert_allclose(prev - th, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-14)
        prev = th


def test_tpp_schedule_composes():
    """fit_sequence(frames) equals manual run/reset/run on the same State."""
    p = ts.make_problem(8, 1, 2, 2, 5, frames=2, breathing=True)
    pr = fit.Problem(p["J"], p["mask"], p["Z"], 8, 2, 2)
    imgs, losses, st = fit.fit_sequence(pr, p["theta0"], p["dv"], [3, 2], 1e-3)
    s2 = fit.State(p["theta0"])
    l0 = fit.run(pr, s2, p["dv"][0], 3, 1e-3)
    s2.reset_optimizer()
    l1 = fit.run(pr, s2, p["dv"][1], 2, 1e-3)
    assert losses == [l0, l1]
    np.testing.assert_array_equal(st.theta, s2.theta)
    np.testing.assert_array_equal(imgs[1], pr.image(s2.theta))
    # masked voxels are exactly zero in every image
    assert np.all(imgs[:, p["mask"] == 0] == 0.0)
