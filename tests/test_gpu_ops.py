"""GPU tests of the standalone operators and their autograd wrappers.

Each operator's forward and backward (the library's HIP kernels) is compared
with the FP64 oracle's layer and with central finite differences of the GPU
forward; the network composed from the operators is compared with the oracle
gradient and with the fused fitting iteration, and with recomputed
activations at 64^3 it must give the same gradient as without.
"""
import numpy as np
import pytest

import tseit_synth as ts
from oracle import net as onet
from tests.gpu_util import make_ctx, oracle_problem, problem, record, rel

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-6, "bf16x3": 2e-5}


def cl(x):
    """(C, n, n, n) -> channels-last (n^3, C)."""
    return np.ascontiguousarray(x.reshape(x.shape[0], -1).T)


def cf(x, n):
    """channels-last (n^3, C) -> (C, n, n, n)."""
    return np.ascontiguousarray(np.asarray(x).T.reshape(-1, n, n, n))


def dev(a, grad=False):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda",
                        requires_grad=grad)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("cin,cout,k", [(8, 16, 3), (16, 8, 3), (24, 16, 1), (32, 32, 3)])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_conv3d_operator_matches_oracle_and_finite_differences(lib, cin, cout, k, prec):
    import torch
    from paper_2507_14046_amd import ops
    n = 8
    rng = np.random.default_rng(1000 * cin + 10 * cout + k)
    x = rng.standard_normal((cin, n, n, n)).astype(np.float32)
    w = (0.2 * rng.standard_normal((cout, cin, k, k, k))).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    R = rng.standard_normal((cout, n, n, n)).astype(np.float32)
    f64 = lambda a: a.astype(np.float64)
    yref = onet.conv3d(f64(x), f64(w), f64(b))
    gxr, gwr, gbr = onet.conv3d_backward(f64(x), f64(w), f64(R))
    X, W, B = dev(cl(x), True), dev(w, True), dev(b, True)
    Y = ops.Conv3dFn.apply(X, W, B, prec)
    Y.backward(dev(cl(R)))
    e = dict(y=rel(cf(host(Y), n), yref), gx=rel(cf(host(X.grad), n), gxr),
             gw=rel(host(W.grad), gwr), gb=rel(host(B.grad), gbr))
    # central differences of f = <R, conv(x, w)> along random directions (the
    # map is linear in x and in w, so they are exact up to rounding)
    vx = rng.standard_normal(x.shape).astype(np.float32)
    vw = (0.2 * rng.standard_normal(w.shape)).astype(np.float32)
    Rh = f64(cl(R))

    def f(xx, ww):
        with torch.no_grad():
            return float((host(ops.Conv3dFn.apply(dev(cl(xx)), dev(ww), dev(b), prec)) * Rh).sum())

    h = 0.5
    fd_x = (f(x + h * vx, w) - f(x - h * vx, w)) / (2 * h)
    fd_w = (f(x, w + h * vw) - f(x, w - h * vw)) / (2 * h)
    an_x = float((host(X.grad) * f64(cl(vx))).sum())
    an_w = float((host(W.grad) * f64(vw)).sum())
    e["fd_x"] = abs(fd_x - an_x) / abs(an_x)
    e["fd_w"] = abs(fd_w - an_w) / abs(an_w)
    record("op_conv3d", cin=cin, cout=cout, k=k, prec=prec, **e)
    for key in ("y", "gx", "gw", "gb"):
        assert e[key] < TOL[prec], (key, e)
    assert e["fd_x"] < 1e-4 and e["fd_w"] < 1e-4, e


@pytest.mark.parametrize("C", [8, 32])
@pytest.mark.parametrize("with_skip", [False, True])
def test_layernorm_relu_operator_matches_oracle_and_finite_differences(lib, C, with_skip):
    import torch
    from paper_2507_14046_amd import ops
    n = 8
    rng = np.random.default_rng(7 * C + with_skip)
    x = (0.5 + 2.0 * rng.standard_normal((C, n, n, n))).astype(np.float32)
    g = (1.0 + 0.3 * rng.standard_normal(C)).astype(np.float32)
    be = (0.2 * rng.standard_normal(C)).astype(np.float32)
    sk = rng.standard_normal((C, n, n, n)).astype(np.float32) if with_skip else None
    R = rng.standard_normal((C, n, n, n)).astype(np.float32)
    f64 = lambda a: a.astype(np.float64)
    z, cache = onet.layer_norm(f64(x), f64(g), f64(be))
    if with_skip:
        z = z + f64(sk)
    yref = onet.relu(z)
    gz = onet.relu_backward(f64(R), yref)
    gxr, ggr, gbr = onet.layer_norm_backward(gz, f64(g), cache)
    X, G, Be = dev(cl(x), True), dev(g, True), dev(be, True)
    S = dev(cl(sk), True) if with_skip else None
    Y = ops.LayerNormReLUFn.apply(X, G, Be, S)
    Y.backward(dev(cl(R)))
    e = dict(y=rel(cf(host(Y), n), yref), gx=rel(cf(host(X.grad), n), gxr),
             gg=rel(host(G.grad), ggr), gbeta=rel(host(Be.grad), gbr))
    if with_skip:
        e["gskip"] = rel(cf(host(S.grad), n), gz)
    # central differences of f = <R, y(x)> with the ReLU active everywhere
    # (skip = +6), summed in FP64 on the host
    big = np.full((C, n, n, n), 6.0, np.float32)
    Rh = f64(cl(R))
    Xs = dev(cl(x), True)
    Ys = ops.LayerNormReLUFn.apply(Xs, dev(g), dev(be), dev(cl(big)))
    Ys.backward(dev(cl(R)))
    v = rng.standard_normal(x.shape).astype(np.float32)

    def f(xx):
        with torch.no_grad():
            return float((host(ops.LayerNormReLUFn.apply(dev(cl(xx)), dev(g), dev(be),
                                                         dev(cl(big)))) * Rh).sum())

    h = 1e-2
    fd = (f(x + h * v) - f(x - h * v)) / (2 * h)
    an = float((host(Xs.grad) * f64(cl(v))).sum())
    e["fd_x"] = abs(fd - an) / abs(an)
    record("op_ln_relu", C=C, skip=with_skip, **e)
    for key in ("y", "gx", "gg", "gbeta", "gskip"):
        if key in e:
            assert e[key] < 2e-5, (key, e)
    assert e["fd_x"] < 1e-3, e


@pytest.mark.parametrize("M,n", [(208, 8), (928, 16)])
def test_measurement_operator_and_adjoint(lib, M, n):
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(M + n)
    Q = n ** 3
    J = rng.standard_normal((M, Q)).astype(np.float32) / np.sqrt(Q)
    s = rng.standard_normal(Q).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    S = dev(s, True)
    P = ops.MeasureFn.apply(S, dev(J))
    P.backward(dev(g))
    J64 = J.astype(np.float64)
    e = dict(p=rel(host(P), J64 @ s), jt=rel(host(S.grad), J64.T @ g))
    # adjoint identity and central differences (exact for a linear map)
    e["adjoint"] = abs(float(host(P) @ g) - float(s @ host(S.grad))) / abs(float(host(P) @ g))
    v = rng.standard_normal(Q).astype(np.float32)
    with torch.no_grad():
        fp = float(host(ops.MeasureFn.apply(dev(s + v), dev(J))) @ g)
        fm = float(host(ops.MeasureFn.apply(dev(s - v), dev(J))) @ g)
    e["fd"] = abs((fp - fm) / 2 - float(host(S.grad) @ v)) / abs(float(host(S.grad) @ v))
    record("op_measure", M=M, n=n, **e)
    assert e["p"] < 2e-6 and e["jt"] < 2e-6 and e["adjoint"] < 1e-5 and e["fd"] < 1e-4, e


def _ops_grad(p, recompute=False, precision="fp32"):
    import torch
    from paper_2507_14046_amd import ops
    net = ops.DIPNet(p["n"], p["levels"], p["base_ch"], precision=precision, recompute=recompute)
    th = dev(p["theta0"], True)
    loss = net.loss(th, dev(p["Z"]), dev(p["mask"].astype(np.float32)), dev(p["J"]),
                    dev(p["dv"][0]))
    loss.backward()
    torch.cuda.synchronize()
    return float(loss), host(th.grad)


@pytest.mark.parametrize("shape", [(8, 1, 2, 8), (16, 1, 2, 8), (16, 2, 3, 16)])
def test_operator_network_gradient_matches_oracle_and_fused(lib, shape):
    n, rings, L, C = shape
    p = problem(n, rings, L, C, 50 + n + L)
    loss, g = _ops_grad(p)
    pr = oracle_problem(p)
    L0, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    ctx = make_ctx(lib, [p])
    ctx.run(1)
    gf = ctx.get_grad(0).astype(np.float64)
    ctx.close()
    e = dict(loss=abs(loss - L0) / L0, grad_vs_oracle=rel(g, gref), grad_vs_fused=rel(g, gf))
    record("ops_network", n=n, levels=L, C=C, **e)
    assert e["loss"] < 1e-5 and e["grad_vs_oracle"] < 2e-4 and e["grad_vs_fused"] < 2e-4, e


def test_recomputed_activations_at_64cubed(lib):
    """64^3 / 4 levels / 32 channels: ResBlock activations recomputed in the
    backward give the same gradient (bitwise: the kernels are deterministic)
    with less peak memory, and the fused iteration's gradient agrees."""
    import torch
    c = ts.CONFIGS["c2"]
    p = problem(c["n"], c["rings"], c["levels"], c["base_ch"], c["seed"])
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    l_keep, g_keep = _ops_grad(p, recompute=False)
    peak_keep = torch.cuda.max_memory_allocated() - base
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    l_rec, g_rec = _ops_grad(p, recompute=True)
    peak_rec = torch.cuda.max_memory_allocated() - base
    ctx = make_ctx(lib, [p])
    ctx.run(1)
    gf = ctx.get_grad(0).astype(np.float64)
    ctx.close()
    e = dict(peak_mib_keep=peak_keep / 2 ** 20, peak_mib_recompute=peak_rec / 2 ** 20,
             grad_vs_fused=rel(g_rec, gf))
    record("recompute_64", **e)
    assert l_keep == l_rec
    np.testing.assert_array_equal(g_keep, g_rec)
    assert peak_rec < peak_keep, e
    assert e["grad_vs_fused"] < 1e-3, e


@pytest.mark.parametrize("M", [1, 208, 928, 5000])
def test_mse_loss_operator_matches_fp64(lib, M):
    """d2ip_op_mse_loss: the data term (1/M) sum (p - dv)^2 reduced in FP64 on
    the device, and its gradient (2/M)(p - dv), against FP64 on the host; the
    autograd wrapper passes the gradient on."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(M)
    p = rng.standard_normal(M).astype(np.float32)
    dv = (p + 1e-3 * rng.standard_normal(M)).astype(np.float32)  # small residuals
    P, DV = dev(p, True), dev(dv)
    loss = ops.MSELossFn.apply(P, DV)
    loss.backward()
    r = p.astype(np.float64) - dv.astype(np.float64)
    want = float(r @ r) / M
    got = float(loss)
    assert loss.dtype == torch.float64
    record("op_mse_loss", M=M, rel=abs(got - want) / want)
    assert abs(got - want) / want < 1e-6, (got, want)
    np.testing.assert_allclose(host(P.grad), 2.0 * r / M, rtol=1e-6, atol=1e-6 * np.abs(2 * r / M).max())


def _cl(x):
    return np.ascontiguousarray(x.reshape(x.shape[0], -1).T)


def _cf(x, n):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).T.reshape(-1, n, n, n))


@pytest.mark.parametrize("n,Cu,Cs", [(8, 16, 8), (6, 4, 12), (32, 32, 16), (2, 4, 4)])
def test_pool_and_up_concat_operators_match_oracle(lib, n, Cu, Cs):
    """d2ip_op_pool2_* and d2ip_op_up2_concat_* against the oracle's
    avgpool2 / up2 and their adjoints (FP64)."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(n * 100 + Cu + Cs)
    m = n // 2
    x = rng.standard_normal((Cs, n, n, n)).astype(np.float32)
    d = rng.standard_normal((Cu, m, m, m)).astype(np.float32)
    f64 = lambda a: a.astype(np.float64)
    X, D = dev(_cl(x), True), dev(_cl(d), True)
    Y = ops.Pool2Fn.apply(X)
    R = rng.standard_normal((Cs, m, m, m)).astype(np.float32)
    Y.backward(dev(_cl(R)))
    assert rel(_cf(host(Y), m), onet.avgpool2(f64(x))) < 1e-6
    assert rel(_cf(host(X.grad), n), onet.avgpool2_backward(f64(R))) < 1e-6
    E = dev(_cl(x), True)
    Cat = ops.Up2ConcatFn.apply(D, E)
    want = np.concatenate([onet.up2(f64(d)), f64(x)], axis=0)
    assert rel(_cf(host(Cat), n), want) == 0.0
    G = rng.standard_normal((Cu + Cs, n, n, n)).astype(np.float32)
    Cat.backward(dev(_cl(G)))
    assert rel(_cf(host(D.grad), m), onet.up2_backward(f64(G[:Cu]))) < 1e-6
    assert rel(_cf(host(E.grad), n), f64(G[Cu:])) == 0.0


@pytest.mark.parametrize("sig", [False, True])
@pytest.mark.parametrize("n,C", [(8, 8), (6, 16), (32, 16), (16, 256), (1, 256), (3, 4)])
def test_head_operator_matches_oracle(lib, n, C, sig):
    """d2ip_op_head_*: the 1x1x1 conv to one channel (linear or the sigmoid
    tail 2 sigmoid(t) - 1), masked, and its gradients, against the oracle's
    conv3d / conv3d_backward and the sigmoid's derivative (FP64)."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(7 * n + C + sig)
    x = rng.standard_normal((C, n, n, n)).astype(np.float32)
    w = (rng.standard_normal((1, C, 1, 1, 1)) / np.sqrt(C)).astype(np.float32)
    b = rng.standard_normal(1).astype(np.float32)
    mask = (rng.random(n ** 3) < 0.8).astype(np.float32)
    R = rng.standard_normal(n ** 3).astype(np.float32)
    f64 = lambda a: a.astype(np.float64)
    t = onet.conv3d(f64(x), f64(w), f64(b))[0].ravel()
    if sig:
        sg = 1.0 / (1.0 + np.exp(-t))
        want, gt = 2.0 * sg - 1.0, f64(R) * f64(mask) * 2.0 * sg * (1.0 - sg)
    else:
        want, gt = t, f64(R) * f64(mask)
    want = want * f64(mask)
    gxr, gwr, gbr = onet.conv3d_backward(f64(x), f64(w), gt.reshape(1, n, n, n))
    X, W, B = dev(_cl(x), True), dev(w, True), dev(b, True)
    out = ops.HeadFn.apply(X, W, B, dev(mask), sig)
    out.backward(dev(R))
    e = dict(y=rel(host(out), want), gx=rel(_cf(host(X.grad), n), gxr), gw=rel(host(W.grad), gwr),
             gb=rel(host(B.grad), gbr))
    record("op_head", n=n, C=C, sigmoid=sig, **e)
    for k, v in e.items():
        assert v < 2e-6, (k, e)


@pytest.mark.parametrize("n,c,cu", [(8, 8, 16), (6, 4, 8), (16, 16, 32), (32, 32, 64),
                                    (16, 64, 128), (2, 4, 4), (4, 12, 8), (10, 20, 44),
                                    (4, 64, 4), (6, 4, 128), (8, 128, 256), (6, 72, 136),
                                    (4, 256, 512), (8, 32, 160)])
def test_attention_operator_matches_oracle(lib, n, c, cu):
    """d2ip_op_attention_*: the attention unit (gate on the coarse grid from the
    pooled skip, interpolated) and its gradients against the oracle's
    att_forward / att_backward (FP64); ragged last block at 6^3 (27 coarse
    voxels), the widest channels at 16^3, a one-voxel coarse grid (2^3),
    channel counts off the 16-wide matrix-core tiles (12, 20, 44: partial row
    and column tiles, K = c + cu padded to a multiple of 16), the extreme
    c / cu mixes, and wide channels (above 64 / 128: the composed form on the
    pointwise GEMMs, up to 256 / 512)."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(n + 10 * c + cu)
    m = n // 2
    x = rng.standard_normal((c, n, n, n)).astype(np.float32)
    g = rng.standard_normal((cu, m, m, m)).astype(np.float32)
    Q = {"att.wx": (rng.standard_normal((c, c)) / np.sqrt(c)).astype(np.float32),
         "att.wg": (rng.standard_normal((c, cu)) / np.sqrt(cu)).astype(np.float32),
         "att.b": (0.1 * rng.standard_normal(c)).astype(np.float32),
         "att.psi": (rng.standard_normal(c) / np.sqrt(c)).astype(np.float32),
         "att.bpsi": (0.1 * rng.standard_normal(1)).astype(np.float32)}
    R = rng.standard_normal((c, n, n, n)).astype(np.float32)
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    Q64 = {k: f64(v) for k, v in Q.items()}
    yr, cache = onet.att_forward(f64(x), f64(g), Q64)
    gxr, ggr, gr = onet.att_backward(f64(R), Q64, cache)
    X, G = dev(_cl(x), True), dev(_cl(g), True)
    P = {k: dev(v, True) for k, v in Q.items()}
    Y = ops.AttentionFn.apply(X, G, P["att.wx"], P["att.wg"], P["att.b"], P["att.psi"],
                             P["att.bpsi"])
    Y.backward(dev(_cl(R)))
    e = dict(y=rel(_cf(host(Y), n), yr), gx=rel(_cf(host(X.grad), n), gxr),
             gg=rel(_cf(host(G.grad), m), ggr))
    for k in Q:
        e[k] = rel(host(P[k].grad), gr[k])
    record("op_attention", n=n, c=c, cu=cu, **e)
    for k, v in e.items():
        assert v < 1e-5, (k, e)


@pytest.mark.parametrize("V,cs", [(1000, (8, 16, 4, 12)), (4 ** 3, (64, 64, 64, 64)),
                                  (17, (4,))])
def test_channel_concat_and_relu_operators(lib, V, cs):
    """d2ip_op_channel_copy (concatenation along channels and the split of the
    gradient) bitwise against numpy; d2ip_op_relu_* bitwise against
    max(x, 0) and the gradient masked where the output is positive (exact
    zeros included, whose derivative is taken as 0)."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(V + sum(cs))
    xs = [rng.standard_normal((V, c)).astype(np.float32) for c in cs]
    X = [dev(x, True) for x in xs]
    cat = ops.ChannelConcatFn.apply(*X)
    want = np.concatenate(xs, axis=1)
    want[::3, 0] = 0.0                      # exact zeros at the kink
    G = rng.standard_normal(want.shape).astype(np.float32)
    np.testing.assert_array_equal(host(cat), np.concatenate(xs, axis=1))
    Z = dev(want, True)
    y = ops.ReLUFn.apply(Z)
    np.testing.assert_array_equal(host(y), np.maximum(want, 0.0))
    y.backward(dev(G))
    np.testing.assert_array_equal(host(Z.grad), np.where(want > 0, G, 0.0))
    cat.backward(dev(G))
    off = 0
    for x, c in zip(X, cs):
        np.testing.assert_array_equal(host(x.grad), G[:, off:off + c])
        off += c
