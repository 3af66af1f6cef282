"""The BF16 forms against the FP64 oracle fed the operands the kernels round.

A BF16 convolution pass rounds its two operands to bfloat16 (round to nearest
even) and accumulates the exact products in FP32; the BF16x3 passes split each
operand x into hi = bf16(x) and lo = bf16(x - hi) and add hi*hi + hi*lo +
lo*hi.  Feeding the FP64 oracle's convolution the same rounded operands
leaves only the FP32 accumulation order between the two, so every output value
must agree to 1e-5 of the output's largest magnitude: a kernel fault (a wrong
tap, channel or tile) cannot hide behind the operand rounding.  The bias
gradient is summed from the unrounded gradient on the GPU, and so here.

At the network level the oracle runs with every convolution wrapped the same
way (the linear tail, FP32 on the GPU, unwrapped), so the BF16 form's image
and one-iteration gradient can be told apart from the FP64 oracle's by
operand rounding alone.  The rounding helpers are written here, from the definition
of the bfloat16 format (the upper 16 bits of an FP32 value, rounded to nearest
even).
"""
import ctypes

import numpy as np
import pytest

import tseit_synth as ts
from oracle import net as onet
from tests.gpu_util import oracle_problem, per_tensor_rel, problem, record, rel

pytestmark = pytest.mark.gpu

# the oracle's own convolutions (the network-level test wraps the module's)
_CONV3D, _CONV3D_BWD = onet.conv3d, onet.conv3d_backward


def bf16(a):
    """FP64/FP32 values -> the FP32 value of their bfloat16 rounding: first to
    FP32 (as the GPU holds them), then to nearest even on the upper 16 bits."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def split3(a):
    hi = bf16(a)
    lo = bf16(np.asarray(a, dtype=np.float32).astype(np.float64) - hi)
    return hi, lo


def conv_ref(x, w, b, prec):
    """Oracle forward on the rounded operands of one pass."""
    if prec == "bf16":
        return _CONV3D(bf16(x), bf16(w), b)
    (xh, xl), (wh, wl) = split3(x), split3(w)
    z = np.zeros_like(b)
    return _CONV3D(xh, wh, b) + _CONV3D(xh, wl, z) + _CONV3D(xl, wh, z)


def conv_bwd_ref(x, w, g, prec):
    """(gx, gw, gb) of the oracle on the rounded operands of each pass."""
    gb = g.reshape(g.shape[0], -1).sum(axis=1)
    if prec == "bf16":
        gx = _CONV3D_BWD(x, bf16(w), bf16(g))[0]
        gw = _CONV3D_BWD(bf16(x), w, bf16(g), need_gx=False)[1]
        return gx, gw, gb
    (xh, xl), (wh, wl), (gh, gl) = split3(x), split3(w), split3(g)
    gx = (_CONV3D_BWD(x, wh, gh)[0] + _CONV3D_BWD(x, wl, gh)[0] +
          _CONV3D_BWD(x, wh, gl)[0])
    f = lambda xx, gg: _CONV3D_BWD(xx, w, gg, need_gx=False)[1]
    gw = f(xh, gh) + f(xh, gl) + f(xl, gh)
    return gx, gw, gb


def cl(x):
    return np.ascontiguousarray(x.reshape(x.shape[0], -1).T)


def cf(x, n):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).T.reshape(-1, n, n, n))


# (n, cin, cout, taps): the convolutions of the 32^3 / 3-level / 16-channel
# network (stem with its input padded to 8 channels, encoder and decoder
# blocks, 1x1x1 projections) and the 64^3 decoder level-0 conv (96 -> 32)
SHAPES = [(32, 8, 16, 27), (32, 16, 16, 27), (16, 16, 32, 27), (8, 32, 64, 27),
          (16, 96, 32, 27), (32, 48, 16, 27), (16, 16, 32, 1), (32, 48, 16, 1),
          (64, 96, 32, 27)]
PREC = {"bf16": 1, "bf16x3": 2}


def _max_rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_%dto%d_k%d" % s)
def test_bf16_conv_passes_match_oracle_on_rounded_operands(lib, shape, prec):
    import torch
    from paper_2507_14046_amd import _lib as L
    lb = L.load()
    n, cin, cout, taps = shape
    k = 3 if taps == 27 else 1
    rng = np.random.default_rng(n * 7919 + cin * 31 + cout + taps)
    x = rng.standard_normal((cin, n, n, n)).astype(np.float32)
    w = (rng.standard_normal((cout, cin, k, k, k)) / np.sqrt(cin * taps)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    g = rng.standard_normal((cout, n, n, n)).astype(np.float32)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    X, W, B, G = dev(cl(x)), dev(w), dev(b), dev(cl(g))
    Y, GX, GW, GB = (torch.empty(n ** 3, cout, device="cuda"),
                     torch.empty_like(X), torch.empty_like(W), torch.empty_like(B))
    nb = ctypes.c_size_t()
    L.check(lb.d2ip_op_conv3d_bytes(n, cin, cout, taps, PREC[prec], ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print("bf16 rounding: %s %s" % (shape, prec), flush=True)
    L.check(lb.d2ip_op_conv3d_forward(P(X), P(W), P(B), P(Y), n, cin, cout, taps, PREC[prec],
                                      P(ws), nb.value, sp))
    L.check(lb.d2ip_op_conv3d_backward(P(X), P(W), P(G), P(GX), P(GW), P(GB), n, cin, cout, taps,
                                       PREC[prec], P(ws), nb.value, sp))
    torch.cuda.synchronize()
    f64 = lambda a: a.astype(np.float64)
    y_r = conv_ref(f64(x), f64(w), f64(b), prec)
    gx_r, gw_r, gb_r = conv_bwd_ref(f64(x), f64(w), f64(g), prec)
    h = lambda t: t.cpu().numpy().astype(np.float64)
    got = dict(y=cf(h(Y), n), gx=cf(h(GX), n), gw=h(GW), gb=h(GB))
    want = dict(y=y_r, gx=gx_r, gw=gw_r, gb=gb_r)
    e = {key: _max_rel(got[key], want[key]) for key in got}
    # for context: the same outputs against the unrounded FP64 oracle
    y_0 = _CONV3D(f64(x), f64(w), f64(b))
    e["y_vs_unrounded"] = _max_rel(got["y"], y_0)
    record("bf16_rounded_pass", shape=shape, prec=prec, **e)
    for key in ("y", "gx", "gw", "gb"):
        assert e[key] <= 1e-5, (key, e)


def _emulating_oracle(monkeypatch, prec):
    """Wrap the oracle's convolutions so that they see the rounded operands
    the BF16 form's kernels see (the 1-output-channel tail is FP32 on the GPU
    and stays unwrapped)."""
    f0, b0 = _CONV3D, _CONV3D_BWD

    def fwd(x, w, b):
        return f0(x, w, b) if w.shape[0] == 1 else conv_ref(x, w, b, prec)

    def bwd(x, w, g, need_gx=True):
        if w.shape[0] == 1:
            return b0(x, w, g, need_gx)
        gx, gw, gb = conv_bwd_ref(x, w, g, prec)
        return (gx if need_gx else None), gw, gb
    monkeypatch.setattr(onet, "conv3d", fwd)
    monkeypatch.setattr(onet, "conv3d_backward", bwd)


@pytest.mark.parametrize("cfg", ["c0", "c1"])
def test_bf16_network_is_the_rounded_operands_network(lib, monkeypatch, cfg):
    """The pure BF16 form's forward image and one-iteration gradient against
    the FP64 oracle and against the oracle on the same rounded operands.

    On the shallow 16^3 / 2-level network every rounding decision of the two
    coincides and they agree to FP32 accumulation.  On the 32^3 / 3-level
    network a few activations lie within FP32 rounding of a bfloat16 rounding
    boundary; the two round them differently, the changed values move later
    activations across further boundaries, and the match is lost at the
    bfloat16 level (measured: image 1.8e-3) -- yet the rounded-operand oracle
    still accounts for most of the distance to the FP64 oracle (gradient
    1.9e-2 -> 6.6e-3, worst tensor 0.63 -> 1.9e-2)."""
    from tests.gpu_util import make_ctx
    c = ts.CONFIGS[cfg]
    p = problem(c["n"], c["rings"], c["levels"], c["base_ch"], c["seed"])
    ctx = make_ctx(lib, [p], "bf16")
    img = ctx.read_image(0)
    loss = ctx.run(1)[0]
    g = ctx.get_grad(0)
    ctx.close()
    th0, dv = p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64)
    pr = oracle_problem(p)
    img64 = pr.image(th0)
    L64, g64, _ = pr.loss_and_grad(th0, dv)
    _emulating_oracle(monkeypatch, "bf16")
    imgr = pr.image(th0)
    Lr, gr, _ = pr.loss_and_grad(th0, dv)
    per64 = per_tensor_rel(g, g64, c["levels"], c["base_ch"])
    perr = per_tensor_rel(g, gr, c["levels"], c["base_ch"])
    w64 = max(per64.items(), key=lambda kv: kv[1])
    wr = max(perr.items(), key=lambda kv: kv[1])
    e = dict(image_vs_fp64=rel(img, img64), image_vs_rounded=rel(img, imgr),
             loss_vs_fp64=abs(loss - L64) / L64, loss_vs_rounded=abs(loss - Lr) / Lr,
             grad_vs_fp64=rel(g, g64), grad_vs_rounded=rel(g, gr),
             worst_vs_fp64=w64, worst_vs_rounded=wr)
    record("bf16_network_rounded_oracle", cfg=cfg, **e)
    if cfg == "c0":
        assert e["image_vs_rounded"] < 1e-5, e
        assert e["loss_vs_rounded"] < 1e-5, e
        assert e["grad_vs_rounded"] < 1e-3, e
    else:
        assert e["image_vs_rounded"] < e["image_vs_fp64"] / 2, e
        assert e["grad_vs_rounded"] < e["grad_vs_fp64"] / 2, e
        assert wr[1] < w64[1] / 10, e
