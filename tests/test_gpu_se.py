"""GPU tests of the Squeeze-and-Excitation unit (forward and backward through
the C-ABI) against the FP64 oracle (oracle/se.py): channel counts with one,
three, 16 and 256 quads (every column-sum lane layout), hidden widths down to
1, ragged and one-voxel grids, and the 64^3 x 64 workload the benchmark
times, compared in full."""
import numpy as np
import pytest

from oracle import se
from tests.gpu_util import record, rel

pytestmark = pytest.mark.gpu

# FP32 against FP64: the gate is one sigmoid of short dot products; the
# weight gradients hang on column sums over n^3 voxels (fixed-order tree).
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


@pytest.mark.parametrize("n,C,H", [(1, 4, 1), (5, 12, 3), (8, 16, 4), (13, 64, 16),
                                   (16, 1024, 64), (64, 64, 16)])
def test_se_matches_oracle(lib, n, C, H):
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(900 + n + C + H)
    x = (1.0 + rng.standard_normal((C, n, n, n))).astype(np.float32)  # nonzero means
    w1 = (rng.standard_normal((H, C)) / np.sqrt(C)).astype(np.float32)
    b1 = (0.1 * rng.standard_normal(H)).astype(np.float32)
    w2 = (rng.standard_normal((C, H)) / np.sqrt(H)).astype(np.float32)
    b2 = (0.1 * rng.standard_normal(C)).astype(np.float32)
    g = rng.standard_normal((C, n, n, n)).astype(np.float32)
    f = lambda a: a.astype(np.float64)
    yref, cache = se.se_forward(f(x), f(w1), f(b1), f(w2), f(b2))
    refs = se.se_backward(f(x), f(w1), f(w2), cache, f(g))
    T = [dev(cl(x), True)] + [dev(a, True) for a in (w1, b1, w2, b2)]
    Y = ops.SEFn.apply(*T)
    Y.backward(dev(cl(g)))
    got = [cf(host(T[0].grad), n)] + [host(t.grad) for t in T[1:]]
    e = dict(y=rel(cf(host(Y), n), yref))
    for k, a, b in zip(("gx", "gw1", "gb1", "gw2", "gb2"), got, refs):
        e[k] = rel(a, b)
    record("se", n=n, C=C, H=H, **e)
    assert e["y"] < TOL_Y and e["gx"] < TOL_Y, e
    assert max(e["gw1"], e["gb1"], e["gw2"], e["gb2"]) < TOL_W, e


@pytest.mark.parametrize("shape,sep", [((8, 1, 2, 8), False), ((16, 2, 3, 16), False),
                                       ((16, 2, 3, 16), True)])
def test_network_with_se_units_matches_oracle(lib, shape, sep):
    """The autograd network with an SE unit after every encoder block (and
    dense or depthwise-separable convs): loss and theta gradient against the
    FP64 oracle network of the same layout."""
    import torch
    from oracle import fit, net
    from paper_2507_14046_amd import ops
    from tests.gpu_util import problem
    n, rings, L, C = shape
    r = 4
    p = problem(n, rings, L, C, 80 + n + L)
    rng = np.random.default_rng(81 + n + sep)
    th = (0.3 * rng.standard_normal(net.n_params(L, C, sep, r))).astype(np.float32)
    model = ops.DIPNet(n, L, C, conv="dwsep" if sep else "dense", se_ratio=r)
    T = dev(th, True)
    loss = model.loss(T, dev(p["Z"]), dev(p["mask"].astype(np.float32)), dev(p["J"]),
                      dev(p["dv"][0]))
    loss.backward()
    torch.cuda.synchronize()
    pr = fit.Problem(p["J"], p["mask"], p["Z"], n, L, C, sep=sep, se_ratio=r)
    L0, gref, _ = pr.loss_and_grad(th.astype(np.float64), p["dv"][0].astype(np.float64))
    e = dict(loss=abs(float(loss.detach()) - L0) / L0, grad=rel(host(T.grad), gref))
    record("se_network", n=n, levels=L, C=C, sep=sep, **e)
    assert e["loss"] < 1e-5 and e["grad"] < 2e-4, e


@pytest.mark.parametrize("shape,sep,r,att,tail,aspp", [
    ((8, 1, 2, 8), False, 0, True, "linear", False),
    ((8, 1, 2, 8), False, 0, False, "sigmoid", False),
    ((16, 2, 3, 16), False, 0, False, "linear", True),
    ((16, 2, 3, 16), True, 4, True, "sigmoid", True)])
def test_network_modules_match_oracle(lib, shape, sep, r, att, tail, aspp):
    """Attention units on the decoder skips, the sigmoid tail, the ASPP module,
    and all of the 3D-FastResUNet modules together (depthwise-separable
    convs, SE units, ASPP, attention units, sigmoid tail): loss and theta
    gradient of the autograd network against the FP64 oracle network of the
    same layout."""
    import torch
    from oracle import fit, net
    from paper_2507_14046_amd import ops
    from tests.gpu_util import problem
    n, rings, L, C = shape
    p = problem(n, rings, L, C, 90 + n + L)
    rng = np.random.default_rng(91 + n + 2 * att + r)
    th = (0.3 * rng.standard_normal(net.n_params(L, C, sep, r, att, aspp))).astype(np.float32)
    model = ops.DIPNet(n, L, C, conv="dwsep" if sep else "dense", se_ratio=r, att=att,
                       tail=tail, aspp=aspp)
    T = dev(th, True)
    loss = model.loss(T, dev(p["Z"]), dev(p["mask"].astype(np.float32)), dev(p["J"]),
                      dev(p["dv"][0]))
    loss.backward()
    torch.cuda.synchronize()
    pr = fit.Problem(p["J"], p["mask"], p["Z"], n, L, C, sep=sep, se_ratio=r, att=att,
                     tail=tail, aspp=aspp)
    L0, gref, _ = pr.loss_and_grad(th.astype(np.float64), p["dv"][0].astype(np.float64))
    e = dict(loss=abs(float(loss.detach()) - L0) / L0, grad=rel(host(T.grad), gref))
    record("modules_network", n=n, levels=L, C=C, sep=sep, se_ratio=r, att=att, tail=tail,
           aspp=aspp, **e)
    assert e["loss"] < 1e-5 and e["grad"] < 2e-4, e


def test_se_and_pointwise_backward_are_bitwise_repeatable(lib):
    """The voxel sums of the SE unit and of the pointwise weight gradient are
    reduced in a fixed order: two backward passes give the same bits."""
    import torch
    from paper_2507_14046_amd import ops
    rng = np.random.default_rng(77)
    n, C, H = 24, 32, 8
    x = dev(rng.standard_normal((n ** 3, C)))
    g = dev(rng.standard_normal((n ** 3, C)))
    w1, b1 = dev(rng.standard_normal((H, C)) / 6), dev(rng.standard_normal(H))
    w2, b2 = dev(rng.standard_normal((C, H)) / 3), dev(rng.standard_normal(C))
    wp, bp = dev(rng.standard_normal((C, C)) / 6), dev(rng.standard_normal(C))
    outs = []
    for _ in range(2):
        T = [t.clone().requires_grad_(True) for t in (x, w1, b1, w2, b2, wp, bp)]
        y = ops.PWConv3dFn.apply(ops.SEFn.apply(*T[:5]), T[5], T[6])
        y.backward(g)
        outs.append([t.grad.clone() for t in T])
    for a, b in zip(*outs):
        assert torch.equal(a, b)
