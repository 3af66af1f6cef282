"""GPU tests of the depthwise 3x3x3 convolution and the pointwise 1x1x1
convolution (forward, input and weight gradients) and of their composition,
the depthwise-separable convolution, against the FP64 oracle
(oracle/dwsep.py).

Depthwise cases span every channel-quad blocking the kernels pick (C/4 odd,
even, a multiple of 4 and of 8, several channel chunks), ragged tiles in x, y
and z and the degenerate one- and two-voxel grids; pointwise cases span
ragged row blocks, column tiles and k stages and several voxel chunks of the
weight gradient; both run the 64^3 x 64 workload that the benchmark times
(there sampled outputs and the full weight gradients)."""
import numpy as np
import pytest

from oracle import dwsep
from tests.gpu_util import record, rel

pytestmark = pytest.mark.gpu

# FP32 against FP64: the forward and input gradient sum 27 products per
# value; the weight and bias gradients sum n^3 products per value in a fixed
# tree, whose rounding grows with the depth of the tree (log2 of the sum's
# length), not with its length.
TOL_Y = 2e-6
TOL_W = 1e-5


def cl(x):
    return np.ascontiguousarray(x.reshape(x.shape[0], -1).T)


def cf(x, n):
    return np.ascontiguousarray(np.asarray(x).T.reshape(-1, n, n, n))


def dev(a, grad=False):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda",
                        requires_grad=grad)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _case(n, C, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((C, n, n, n)).astype(np.float32)
    w = (0.3 * rng.standard_normal((C, 3, 3, 3))).astype(np.float32)
    b = rng.standard_normal(C).astype(np.float32)
    g = rng.standard_normal((C, n, n, n)).astype(np.float32)
    return x, w, b, g


@pytest.mark.parametrize("n,C", [(1, 4), (2, 8), (5, 12), (8, 16), (13, 24), (9, 32), (11, 64),
                                 (16, 4), (17, 8), (20, 40)])
def test_depthwise_matches_oracle(lib, n, C):
    from paper_2507_14046_amd import ops
    x, w, b, g = _case(n, C, 7000 + 100 * n + C)
    f = lambda a: a.astype(np.float64)
    yref = dwsep.dwconv3d(f(x), f(w), f(b))
    gxr, gwr, gbr = dwsep.dwconv3d_backward(f(x), f(w), f(g))
    X, W, B = dev(cl(x), True), dev(w[:, None], True), dev(b, True)
    Y = ops.DWConv3dFn.apply(X, W, B)
    Y.backward(dev(cl(g)))
    e = dict(y=rel(cf(host(Y), n), yref), gx=rel(cf(host(X.grad), n), gxr),
             gw=rel(host(W.grad)[:, 0], gwr), gb=rel(host(B.grad), gbr))
    record("dwconv3d", n=n, C=C, **e)
    assert e["y"] < TOL_Y and e["gx"] < TOL_Y, e
    assert e["gw"] < TOL_W and e["gb"] < TOL_W, e


def test_depthwise_adjoint_and_determinism(lib):
    """<g, dw(x)> = <dw^T(g), x> with zero bias, and two backward passes give
    the same bits."""
    import torch
    from paper_2507_14046_amd import ops
    n, C = 12, 16
    x, w, _, g = _case(n, C, 4242)
    X, W, G = dev(cl(x)), dev(w), dev(cl(g))
    Y = ops.DWConv3dFn.apply(X, W, None)
    outs = []
    for _ in range(2):
        Xg, Wg = X.clone().requires_grad_(True), W.clone().requires_grad_(True)
        ops.DWConv3dFn.apply(Xg, Wg, None).backward(G)
        outs.append((Xg.grad.clone(), Wg.grad.clone()))
    lhs = float((Y.double() * G.double()).sum())
    rhs = float((outs[0][0].double() * X.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("n,C,Co", [(1, 4, 4), (5, 8, 12), (8, 64, 64), (17, 100, 132),
                                    (10, 36, 8), (20, 16, 72)])
def test_pointwise_matches_oracle(lib, n, C, Co):
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(500 + n + C + Co)
    x = rng.standard_normal((C, n, n, n)).astype(np.float32)
    w = (0.2 * rng.standard_normal((Co, C))).astype(np.float32)
    b = rng.standard_normal(Co).astype(np.float32)
    g = rng.standard_normal((Co, n, n, n)).astype(np.float32)
    f = lambda a: a.astype(np.float64)
    yref = dwsep.pwconv3d(f(x), f(w), f(b))
    gxr, gwr, gbr = dwsep.pwconv3d_backward(f(x), f(w), f(g))
    X, W, B = dev(cl(x), True), dev(w, True), dev(b, True)
    Y = ops.PWConv3dFn.apply(X, W, B)
    Y.backward(dev(cl(g)))
    e = dict(y=rel(cf(host(Y), n), yref), gx=rel(cf(host(X.grad), n), gxr),
             gw=rel(host(W.grad), gwr), gb=rel(host(B.grad), gbr))
    record("pwconv3d", n=n, C=C, Co=Co, **e)
    assert e["y"] < TOL_Y and e["gx"] < TOL_Y, e
    assert e["gw"] < TOL_W and e["gb"] < TOL_W, e


@pytest.mark.parametrize("C,Co", [(16, 24), (32, 8), (12, 20)])
def test_depthwise_separable_composition_matches_oracle(lib, C, Co):
    from paper_2507_14046_amd import ops
    n = 10
    rng = np.random.default_rng(90 + C + Co)
    x, wd, bd, _ = _case(n, C, 91 + C)
    wp = (0.2 * rng.standard_normal((Co, C))).astype(np.float32)
    bp = rng.standard_normal(Co).astype(np.float32)
    R = rng.standard_normal((Co, n, n, n)).astype(np.float32)
    f = lambda a: a.astype(np.float64)
    yref, d = dwsep.dwsep_conv3d(f(x), f(wd), f(bd), f(wp), f(bp))
    refs = dwsep.dwsep_conv3d_backward(f(x), f(wd), f(wp), d, f(R))
    X, WD, BD = dev(cl(x), True), dev(wd, True), dev(bd, True)
    WP, BP = dev(wp, True), dev(bp, True)
    Y = ops.dwsep_conv3d(X, WD, BD, WP, BP)
    Y.backward(dev(cl(R)))
    got = (cf(host(X.grad), n), host(WD.grad), host(BD.grad), host(WP.grad), host(BP.grad))
    e = dict(y=rel(cf(host(Y), n), yref))
    for k, gg, rr in zip(("gx", "gwd", "gbd", "gwp", "gbp"), got, refs):
        e[k] = rel(gg, rr)
    record("dwsep_conv3d", C=C, Co=Co, **e)
    assert e["y"] < TOL_Y and e["gx"] < TOL_Y, e
    assert max(e["gwd"], e["gbd"], e["gwp"], e["gbp"]) < TOL_W, e


def test_pointwise_full_size_workload(lib):
    """64^3 x 64 -> 64: sampled output rows and input-gradient rows against
    the definition at those voxels, the full weight and bias gradients
    against the oracle."""
    from paper_2507_14046_amd import ops
    n, C, Co = 64, 64, 64
    rng = np.random.default_rng(646464)
    x = rng.standard_normal((n ** 3, C)).astype(np.float32)
    w = (0.2 * rng.standard_normal((Co, C))).astype(np.float32)
    b = rng.standard_normal(Co).astype(np.float32)
    g = rng.standard_normal((n ** 3, Co)).astype(np.float32)
    X, W, B = dev(x, True), dev(w, True), dev(b, True)
    Y = ops.PWConv3dFn.apply(X, W, B)
    Y.backward(dev(g))
    y, gx = host(Y), host(X.grad)
    f = lambda a: a.astype(np.float64)
    rows = np.concatenate([[0, n ** 3 - 1, 4095, 4096, 127, 128], rng.integers(0, n ** 3, 200)])
    ey = rel(y[rows], f(x[rows]) @ f(w).T + f(b))
    eg = rel(gx[rows], f(g[rows]) @ f(w))
    e = dict(y_rows=ey, gx_rows=eg, gw=rel(host(W.grad), f(g).T @ f(x)),
             gb=rel(host(B.grad), f(g).sum(axis=0)))
    record("pwconv3d_64", **e)
    assert ey < TOL_Y and eg < TOL_Y, e
    assert e["gw"] < TOL_W and e["gb"] < TOL_W, e


def _dw_at(xp, w, b, c, z, y, x):
    """Depthwise output at one voxel from the zero-padded input (FP64)."""
    return b[c] + (w[c] * xp[c, z:z + 3, y:y + 3, x:x + 3]).sum()


def test_depthwise_full_size_workload(lib):
    """64^3 x 64: sampled forward and input-gradient outputs against the
    oracle's definition at those voxels, the full weight and bias gradients
    against the oracle."""
    from paper_2507_14046_amd import ops
    n, C = 64, 64
    x, w, b, g = _case(n, C, 64064)
    X, W, B = dev(cl(x), True), dev(w, True), dev(b, True)
    Y = ops.DWConv3dFn.apply(X, W, B)
    Y.backward(dev(cl(g)))
    y, gx = host(Y), host(X.grad)
    f = lambda a: a.astype(np.float64)
    xp = np.pad(f(x), ((0, 0), (1, 1), (1, 1), (1, 1)))
    gp = np.pad(f(g), ((0, 0), (1, 1), (1, 1), (1, 1)))
    wf = f(w[:, ::-1, ::-1, ::-1])  # input gradient = taps reversed
    rng = np.random.default_rng(5)
    pts = [(0, 0, 0), (63, 63, 63), (0, 63, 31), (31, 0, 63)]
    pts += [tuple(v) for v in rng.integers(0, n, (60, 3))]
    ey = eg = 0.0
    for (z, yy, xx) in pts:
        v = (z * n + yy) * n + xx
        for c in rng.integers(0, C, 4):
            ry = _dw_at(xp, f(w), f(b), c, z, yy, xx)
            rg = _dw_at(gp, wf, np.zeros(C), c, z, yy, xx)
            ey = max(ey, abs(y[v, c] - ry) / (1 + abs(ry)))
            eg = max(eg, abs(gx[v, c] - rg) / (1 + abs(rg)))
    _, gwr, gbr = dwsep.dwconv3d_backward(f(x), f(w), f(g))
    e = dict(y_sampled=ey, gx_sampled=eg, gw=rel(host(W.grad), gwr), gb=rel(host(B.grad), gbr))
    record("dwconv3d_64", **e)
    assert ey < 1e-5 and eg < 1e-5, e
    assert e["gw"] < TOL_W and e["gb"] < TOL_W, e


@pytest.mark.parametrize("shape", [(8, 1, 2, 8), (16, 2, 3, 16)])
def test_separable_network_gradient_matches_oracle(lib, shape):
    """The autograd network with depthwise-separable ResBlock convolutions
    (every conv on the library's kernels): loss and theta gradient against
    the FP64 oracle network of the same layout."""
    import torch
    from oracle import fit, net
    from paper_2507_14046_amd import ops
    from tests.gpu_util import problem
    n, rings, L, C = shape
    p = problem(n, rings, L, C, 70 + n + L)
    rng = np.random.default_rng(71 + n)
    th = (0.3 * rng.standard_normal(net.n_params(L, C, sep=True))).astype(np.float32)
    model = ops.DIPNet(n, L, C, conv="dwsep")
    T = dev(th, True)
    loss = model.loss(T, dev(p["Z"]), dev(p["mask"].astype(np.float32)), dev(p["J"]),
                      dev(p["dv"][0]))
    loss.backward()
    torch.cuda.synchronize()
    pr = fit.Problem(p["J"], p["mask"], p["Z"], n, L, C, sep=True)
    L0, gref, _ = pr.loss_and_grad(th.astype(np.float64), p["dv"][0].astype(np.float64))
    e = dict(loss=abs(float(loss.detach()) - L0) / L0, grad=rel(host(T.grad), gref))
    record("dwsep_network", n=n, levels=L, C=C, **e)
    assert e["loss"] < 1e-5 and e["grad"] < 2e-4, e


@pytest.mark.parametrize("n,C,dil", [(8, 16, 2), (5, 12, 3), (4, 8, 5), (16, 64, 2), (9, 4, 1)])
def test_dilated_depthwise_matches_oracle(lib, n, C, dil):
    """The atrous depthwise convolution (direct kernel) against the oracle,
    including a dilation past the grid (only the centre tap left) and
    dilation 1, which must agree with the streaming kernels as well."""
    import ctypes
    import torch
    from paper_2507_14046_amd import ops
    x, w, b, g = _case(n, C, 5000 + 10 * n + C + dil)
    f = lambda a: a.astype(np.float64)
    yref = dwsep.dwconv3d(f(x), f(w), f(b), dil)
    gxr, gwr, gbr = dwsep.dwconv3d_backward(f(x), f(w), f(g), dil)
    X, W, B = dev(cl(x), True), dev(w, True), dev(b, True)
    if dil == 1:  # force the direct kernel through the C-ABI
        from paper_2507_14046_amd import _lib as L
        y1 = torch.empty_like(X)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        L.check(L.load().d2ip_op_dwconv3d_dilated_forward(
            P(X), P(W), P(B), P(y1), n, C, 1,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        Y = y1
        ys = ops.DWConv3dFn.apply(X, W, B)
        assert rel(host(Y), host(ys)) < TOL_Y
    else:
        Y = ops.DWConv3dFn.apply(X, W, B, dil)
        Y.backward(dev(cl(g)))
    e = dict(y=rel(cf(host(Y), n), yref))
    if dil != 1:
        e.update(gx=rel(cf(host(X.grad), n), gxr), gw=rel(host(W.grad), gwr),
                 gb=rel(host(B.grad), gbr))
    record("dwconv3d_dilated", n=n, C=C, dil=dil, **e)
    assert e["y"] < TOL_Y and e.get("gx", 0) < TOL_Y, e
    assert e.get("gw", 0) < TOL_W and e.get("gb", 0) < TOL_W, e
