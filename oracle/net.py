"""FP64 oracle of the image prior phi(theta | Z): forward and exact backward.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy; it shares no
code with the GPU library and is imported only by the tests, the smoke check
and the CPU baseline leg of the benchmark.

The network is the paper's DIP image prior (Eq. (3); 3D convolutions,
residual connections and LayerNorm, Sec. III-D) in the plain residual U-Net
reading used throughout this project:

  stem   : a = relu(LN(conv3(Z)))
  enc_0  : ResBlock(C -> C) on a
  enc_l  : ResBlock(c_{l-1} -> c_l) on avgpool2(enc_{l-1}),  l = 1 .. L-1
  dec_l  : ResBlock(3 c_l -> c_l) on concat[up2(dec_{l+1}), enc_l],
           l = L-2 .. 0, with dec_{L-1} = enc_{L-1}
  tail   : y = conv1(dec_0) (C -> 1); the image is mask * y

  ResBlock(x): h1 = conv3(x); a1 = relu(LN1(h1)); h2 = conv3(a1);
               out = relu(LN2(h2) + skip(x)), skip = 1x1x1 conv if the channel
               count changes, identity otherwise.

With sep=True every ResBlock conv3 is the depthwise-separable convolution of
the lightweight backbone (Sec. III-D; oracle/dwsep.py): a per-channel 3x3x3
convolution with a bias, then a 1x1x1 convolution with a bias.  With
se_ratio = r > 0 a Squeeze-and-Excitation unit (Sec. III-D; oracle/se.py) of
hidden width c // r gates the output of every encoder block (enc_l above
stands for the gated output wherever it is used).  With att=True an additive
attention unit (att_forward) gates each decoder skip enc_l by the up-sampled
dec_{l+1} before the concatenation; with tail="sigmoid" the image is
2 sigmoid(conv1(dec_0)) - 1 (the paper's sigmoid tail, shifted and scaled so
that negative changes are representable); with aspp=True the ASPP module
(aspp_forward) transforms the bottleneck enc_{L-1} before the decoder.

Conventions: arrays are channel-first [C, n, n, n] in (z, y, x) order; conv3
is a 3x3x3 cross-correlation with zero padding 1; LN normalises over all of
(C, z, y, x) with the biased variance, eps = 1e-5 inside the square root, and
a per-channel affine (gamma, beta); avgpool2 averages 2x2x2 blocks; up2
repeats every voxel into a 2x2x2 block (nearest neighbour); relu'(0) = 0.
"""
import numpy as np

from . import dwsep, se

LN_EPS = 1e-5


# ----------------------------------------------------------------------------
# parameter unpacking (own copy of the flat layout: modules stem, enc_0..,
# dec_{L-2}..dec_0, tail; per conv W[Cout][Cin][k][k][k] then b; per norm
# gamma then beta; ResBlock order conv1, norm1, conv2, norm2, proj)
# ----------------------------------------------------------------------------

def _conv_shapes(name, cin, cout, sep):
    """A ResBlock's 3x3x3 convolution: dense (w, b), or with sep the
    depthwise-separable form (depthwise dw [cin, 3, 3, 3] and dwb [cin], then
    pointwise pw [cout, cin] and pwb [cout]; Sec. III-D)."""
    if sep:
        return [(name + ".dw", (cin, 3, 3, 3)), (name + ".dwb", (cin,)),
                (name + ".pw", (cout, cin)), (name + ".pwb", (cout,))]
    return [(name + ".w", (cout, cin, 3, 3, 3)), (name + ".b", (cout,))]


def _block_shapes(cin, cout, sep=False):
    shapes = (_conv_shapes("conv1", cin, cout, sep) +
              [("norm1.g", (cout,)), ("norm1.beta", (cout,))] +
              _conv_shapes("conv2", cout, cout, sep) +
              [("norm2.g", (cout,)), ("norm2.beta", (cout,))])
    if cin != cout:
        shapes += [("proj.w", (cout, cin, 1, 1, 1)), ("proj.b", (cout,))]
    return shapes


def se_hidden(c, se_ratio):
    """Hidden width of an SE unit on c channels with reduction ratio r."""
    return max(1, c // se_ratio)


def _se_shapes(c, se_ratio):
    if not se_ratio:
        return []
    h = se_hidden(c, se_ratio)
    return [("se.w1", (h, c)), ("se.b1", (h,)), ("se.w2", (c, h)), ("se.b2", (c,))]


def _att_shapes(c, c_up, att):
    if not att:
        return []
    return [("att.wx", (c, c)), ("att.wg", (c, c_up)), ("att.b", (c,)), ("att.psi", (c,)),
            ("att.bpsi", (1,))]


ASPP_RATES = (1, 2, 3)  # dilations of the atrous branches at the bottleneck


def _aspp_shapes(c):
    shapes = [("w0", (c, c)), ("b0", (c,))]
    for d in ASPP_RATES:
        shapes += [("dw%d" % d, (c, 3, 3, 3)), ("dwb%d" % d, (c,)), ("pw%d" % d, (c, c)),
                   ("pwb%d" % d, (c,))]
    return shapes + [("wp", (c, c * (1 + len(ASPP_RATES)))), ("bp", (c,))]


def aspp_forward(x, Q):
    """ASPP at the bottleneck (Sec. III-D): a 1x1x1 branch and one
    depthwise-separable atrous branch per rate in ASPP_RATES, concatenated,
    projected by a 1x1x1 conv and passed through a ReLU."""
    br = [dwsep.pwconv3d(x, Q["w0"], Q["b0"])]
    ds = []
    for d in ASPP_RATES:
        dd = dwsep.dwconv3d(x, Q["dw%d" % d], Q["dwb%d" % d], d)
        ds.append(dd)
        br.append(dwsep.pwconv3d(dd, Q["pw%d" % d], Q["pwb%d" % d]))
    cat = np.concatenate(br, axis=0)
    y = relu(dwsep.pwconv3d(cat, Q["wp"], Q["bp"]))
    return y, dict(x=x, ds=ds, cat=cat, y=y)


def aspp_backward(gy, Q, c):
    """(gx, {param grads}) of aspp_forward."""
    G = {}
    gz = relu_backward(gy, c["y"])
    gcat, G["wp"], G["bp"] = dwsep.pwconv3d_backward(c["cat"], Q["wp"], gz)
    k = c["x"].shape[0]
    gx, G["w0"], G["b0"] = dwsep.pwconv3d_backward(c["x"], Q["w0"], gcat[:k])
    for i, d in enumerate(ASPP_RATES):
        gb = gcat[(i + 1) * k:(i + 2) * k]
        gd, G["pw%d" % d], G["pwb%d" % d] = dwsep.pwconv3d_backward(c["ds"][i], Q["pw%d" % d], gb)
        gxi, G["dw%d" % d], G["dwb%d" % d] = dwsep.dwconv3d_backward(c["x"], Q["dw%d" % d], gd, d)
        gx = gx + gxi
    return gx, G


def module_list(levels, base_ch, sep=False, se_ratio=0, att=False, tail="linear", aspp=False):
    """[(module name, [(param name, shape)])] in flat order.  With sep every
    ResBlock convolution is depthwise-separable; the stem (one input channel)
    and the 1x1x1 projections and tail stay dense.  With se_ratio r > 0 every
    encoder ResBlock is followed by a Squeeze-and-Excitation unit of hidden
    width c // r (its parameters end the encoder module).  With att every
    decoder module ends with an attention unit on its skip input (wx [c][c],
    wg [c][c_up], b [c], psi [c], bpsi [1]).  With aspp an ASPP module on the
    bottleneck follows the encoder modules.  `tail` changes no parameter."""
    ch = [base_ch * 2 ** l for l in range(levels)]
    mods = [("stem", [("conv.w", (base_ch, 1, 3, 3, 3)), ("conv.b", (base_ch,)),
                      ("norm.g", (base_ch,)), ("norm.beta", (base_ch,))])]
    mods.append(("enc0", _block_shapes(ch[0], ch[0], sep) + _se_shapes(ch[0], se_ratio)))
    for l in range(1, levels):
        mods.append(("enc%d" % l, _block_shapes(ch[l - 1], ch[l], sep) +
                     _se_shapes(ch[l], se_ratio)))
    if aspp:
        mods.append(("aspp", _aspp_shapes(ch[-1])))
    for l in range(levels - 2, -1, -1):
        mods.append(("dec%d" % l, _block_shapes(ch[l + 1] + ch[l], ch[l], sep) +
                     _att_shapes(ch[l], ch[l + 1], att)))
    mods.append(("tail", [("w", (1, base_ch, 1, 1, 1)), ("b", (1,))]))
    return mods


def n_params(levels, base_ch, sep=False, se_ratio=0, att=False, aspp=False):
    return sum(int(np.prod(s)) for _, ps in
               module_list(levels, base_ch, sep, se_ratio, att, aspp=aspp) for _, s in ps)


def unpack(theta, levels, base_ch, sep=False, se_ratio=0, att=False, aspp=False):
    """Flat theta -> {module: {param: view}} (views into theta)."""
    out, off = {}, 0
    for mod, ps in module_list(levels, base_ch, sep, se_ratio, att, aspp=aspp):
        d = {}
        for name, shape in ps:
            k = int(np.prod(shape))
            d[name] = theta[off:off + k].reshape(shape)
            off += k
        out[mod] = d
    assert off == theta.size, (off, theta.size)
    return out


# ----------------------------------------------------------------------------
# layers (forward and backward)
# ----------------------------------------------------------------------------

def conv3d(x, w, b):
    """out[co] = b[co] + sum_{ci, dz, dy, dx} w[co, ci, dz, dy, dx] *
    x[ci, z+dz-1, y+dy-1, x+dx-1] (zeros outside); w is k x k x k, k in {1, 3}."""
    cin, n = x.shape[0], x.shape[1]
    k = w.shape[2]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p)))
    out = np.zeros((w.shape[0], n ** 3))
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                win = xp[:, dz:dz + n, dy:dy + n, dx:dx + n].reshape(cin, -1)
                # (a tap's weight slice is copied to a contiguous block so the
                # product is one BLAS call)
                out += np.ascontiguousarray(w[:, :, dz, dy, dx]) @ win
    out += b[:, None]
    return out.reshape(w.shape[0], n, n, n)


def conv3d_backward(x, w, gout, need_gx=True):
    """Gradients of conv3d w.r.t. x, w and b given gout = dL/dout."""
    cin, n = x.shape[0], x.shape[1]
    cout, k = w.shape[0], w.shape[2]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p)))
    g2 = gout.reshape(cout, -1)
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp) if need_gx else None
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                win = xp[:, dz:dz + n, dy:dy + n, dx:dx + n].reshape(cin, -1)
                gw[:, :, dz, dy, dx] = g2 @ win.T
                if need_gx:
                    gxp[:, dz:dz + n, dy:dy + n, dx:dx + n] += \
                        (np.ascontiguousarray(w[:, :, dz, dy, dx].T) @ g2).reshape(cin, n, n, n)
    gb = g2.sum(axis=1)
    gx = gxp[:, p:p + n, p:p + n, p:p + n] if need_gx else None
    return gx, gw, gb


def layer_norm(h, g, beta, eps=LN_EPS):
    mu = h.mean()
    var = ((h - mu) ** 2).mean()
    rstd = 1.0 / np.sqrt(var + eps)
    xhat = (h - mu) * rstd
    return g[:, None, None, None] * xhat + beta[:, None, None, None], (xhat, rstd)


def layer_norm_backward(gout, g, cache):
    xhat, rstd = cache
    gg = (gout * xhat).sum(axis=(1, 2, 3))
    gbeta = gout.sum(axis=(1, 2, 3))
    gxhat = gout * g[:, None, None, None]
    gh = rstd * (gxhat - gxhat.mean() - xhat * (gxhat * xhat).mean())
    return gh, gg, gbeta


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(gout, y):
    return gout * (y > 0.0)


def avgpool2(x):
    c, n = x.shape[0], x.shape[1]
    m = n // 2
    return x.reshape(c, m, 2, m, 2, m, 2).mean(axis=(2, 4, 6))


def avgpool2_backward(gout):
    return np.repeat(np.repeat(np.repeat(gout, 2, 1), 2, 2), 2, 3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 1), 2, 2), 2, 3)


def up2_backward(gout):
    c, n = gout.shape[0], gout.shape[1]
    m = n // 2
    return gout.reshape(c, m, 2, m, 2, m, 2).sum(axis=(2, 4, 6))


# ----------------------------------------------------------------------------
# blocks and the whole network
# ----------------------------------------------------------------------------

def _conv3(x, P, name):
    """A ResBlock convolution (dense or depthwise-separable, by its
    parameters); returns the output and the depthwise output (or None)."""
    if name + ".w" in P:
        return conv3d(x, P[name + ".w"], P[name + ".b"]), None
    y, d = dwsep.dwsep_conv3d(x, P[name + ".dw"], P[name + ".dwb"], P[name + ".pw"],
                              P[name + ".pwb"])
    return y, d


def _conv3_backward(x, P, name, g, d, G):
    """Input gradient of _conv3; its parameter gradients go into G."""
    if name + ".w" in P:
        gx, G[name + ".w"], G[name + ".b"] = conv3d_backward(x, P[name + ".w"], g)
        return gx
    gx, G[name + ".dw"], G[name + ".dwb"], G[name + ".pw"], G[name + ".pwb"] = \
        dwsep.dwsep_conv3d_backward(x, P[name + ".dw"], P[name + ".pw"], d, g)
    return gx


def resblock_forward(x, P):
    h1, d1 = _conv3(x, P, "conv1")
    n1, c1 = layer_norm(h1, P["norm1.g"], P["norm1.beta"])
    a1 = relu(n1)
    h2, d2 = _conv3(a1, P, "conv2")
    n2, c2 = layer_norm(h2, P["norm2.g"], P["norm2.beta"])
    s = conv3d(x, P["proj.w"], P["proj.b"]) if "proj.w" in P else x
    y = relu(n2 + s)
    return y, dict(x=x, a1=a1, c1=c1, c2=c2, y=y, d1=d1, d2=d2)


def resblock_backward(gy, P, cache):
    G = {}
    gz = relu_backward(gy, cache["y"])
    gh2, G["norm2.g"], G["norm2.beta"] = layer_norm_backward(gz, P["norm2.g"], cache["c2"])
    ga1 = _conv3_backward(cache["a1"], P, "conv2", gh2, cache["d2"], G)
    gn1 = relu_backward(ga1, cache["a1"])
    gh1, G["norm1.g"], G["norm1.beta"] = layer_norm_backward(gn1, P["norm1.g"], cache["c1"])
    gx = _conv3_backward(cache["x"], P, "conv1", gh1, cache["d1"], G)
    if "proj.w" in P:
        gxs, G["proj.w"], G["proj.b"] = conv3d_backward(cache["x"], P["proj.w"], gz)
        gx = gx + gxs
    else:
        gx = gx + gz
    return gx, G


def att_forward(x, g, Q):
    """Attention unit of one decoder up-sampling stage (Sec. III-D: the stage
    is an attention mechanism, followed by interpolation and a ResConv3D
    block).  x [c, n, n, n] is the encoder skip, g [c_up, n/2, n/2, n/2] the
    coarser decoder output (the gating signal), on its own grid.  The gate is
    formed on g's grid from the skip averaged over 2x2x2 cells:
    a = wx pool2(x) + wg g + b, q = relu(a), alpha = sigmoid(psi . q + bpsi)
    (one coefficient per coarse voxel); it is then interpolated (nearest
    neighbour, x2) to the skip's grid, and the output is alpha * x."""
    c = x.shape[0]
    xs = avgpool2(x)
    Xs, G = xs.reshape(c, -1), g.reshape(g.shape[0], -1)
    a = Q["att.wx"] @ Xs + Q["att.wg"] @ G + Q["att.b"][:, None]
    q = np.maximum(a, 0.0)
    al = 1.0 / (1.0 + np.exp(-(Q["att.psi"] @ q + Q["att.bpsi"][0])))
    alf = up2(al.reshape((1,) + g.shape[1:]))
    return alf * x, dict(x=x, Xs=Xs, G=G, a=a, q=q, al=al, alf=alf)


def att_backward(gout, Q, c):
    """(gx, gg, {param grads}) of att_forward given gout = dL/d(output); gg is
    on the gating signal's (coarse) grid."""
    x, Xs, G, a, q, al, alf = c["x"], c["Xs"], c["G"], c["a"], c["q"], c["al"], c["alf"]
    galf = (gout * x).sum(axis=0, keepdims=True)    # dL/d(interpolated alpha)
    gal = up2_backward(galf).reshape(-1)             # to the coarse coefficients
    gt = gal * al * (1.0 - al)                       # through the sigmoid
    gq = np.outer(Q["att.psi"], gt)
    ga = gq * (a > 0)                                # through the ReLU
    grads = {"att.wx": ga @ Xs.T, "att.wg": ga @ G.T, "att.b": ga.sum(axis=1),
             "att.psi": q @ gt, "att.bpsi": np.array([gt.sum()])}
    m = x.shape[1] // 2
    gxs = (Q["att.wx"].T @ ga).reshape((x.shape[0], m, m, m))
    gx = alf * gout + avgpool2_backward(gxs)
    gg = (Q["att.wg"].T @ ga).reshape((G.shape[0], m, m, m))
    return gx, gg, grads


def forward(theta, Z, n, levels, base_ch, sep=False, se_ratio=0, att=False, tail="linear",
            aspp=False):
    """phi(theta | Z) before masking, as an (n, n, n) array, plus the cache
    (sep: depthwise-separable ResBlock convolutions; se_ratio: SE units after
    the encoder blocks; see module_list)."""
    P = unpack(theta, levels, base_ch, sep, se_ratio, att, aspp)
    z = Z.reshape(1, n, n, n)
    hs = conv3d(z, P["stem"]["conv.w"], P["stem"]["conv.b"])
    ns, cs = layer_norm(hs, P["stem"]["norm.g"], P["stem"]["norm.beta"])
    a = relu(ns)
    cache = dict(z=z, stem=(a, cs))
    enc = []
    x = a
    for l in range(levels):
        if l > 0:
            x = avgpool2(enc[-1])
        y, cache["enc%d" % l] = resblock_forward(x, P["enc%d" % l])
        if se_ratio:
            Q = P["enc%d" % l]
            y_in = y
            y, cse = se.se_forward(y_in, Q["se.w1"], Q["se.b1"], Q["se.w2"], Q["se.b2"])
            cache["se%d" % l] = (y_in, cse)
        enc.append(y)
    d = enc[-1]
    if aspp:
        d, cache["aspp"] = aspp_forward(d, P["aspp"])
    for l in range(levels - 2, -1, -1):
        skip = enc[l]
        if att:  # the gate on the coarse grid, before the interpolation
            skip, cache["att%d" % l] = att_forward(skip, d, P["dec%d" % l])
        u = up2(d)
        x = np.concatenate([u, skip], axis=0)
        d, cache["dec%d" % l] = resblock_forward(x, P["dec%d" % l])
    out = conv3d(d, P["tail"]["w"], P["tail"]["b"])
    cache["d0"] = d
    if tail == "sigmoid":
        # the sigmoid tail, shifted and scaled to (-1, 1) so that the negative
        # conductivity changes stay representable: 2 sigmoid(t) - 1
        sg = 1.0 / (1.0 + np.exp(-out))
        cache["tail_sg"] = sg
        out = 2.0 * sg - 1.0
    return out[0], cache


def backward(gout, theta, cache, n, levels, base_ch, sep=False, se_ratio=0, att=False,
             tail="linear", aspp=False):
    """d(loss)/d(theta) as a flat array, given gout = d(loss)/d(phi) (n, n, n)."""
    P = unpack(theta, levels, base_ch, sep, se_ratio, att, aspp)
    grad = np.zeros(theta.size, dtype=np.float64)
    Gv = unpack(grad, levels, base_ch, sep, se_ratio, att, aspp)
    go = gout.reshape(1, n, n, n)
    if tail == "sigmoid":
        sg = cache["tail_sg"]
        go = go * 2.0 * sg * (1.0 - sg)
    gd, gtw, gtb = conv3d_backward(cache["d0"], P["tail"]["w"], go)
    Gv["tail"]["w"][...] = gtw
    Gv["tail"]["b"][...] = gtb
    # decoder, from dec_0 up to dec_{L-2}; gd is d(loss)/d(dec_l output)
    genc = [np.zeros(1)] * levels
    for l in range(0, levels - 1):
        gx, G = resblock_backward(gd, P["dec%d" % l], cache["dec%d" % l])
        for k, v in G.items():
            Gv["dec%d" % l][k][...] = v
        c_up = base_ch * 2 ** (l + 1)
        gu = gx[:c_up]
        gskip = gx[c_up:]
        gd = up2_backward(gu)                  # to dec_{l+1} (or enc_{L-1})
        if att:  # the skip passed through the attention unit, gated from dec_{l+1}
            gskip, gg, Ga = att_backward(gskip, P["dec%d" % l], cache["att%d" % l])
            for k, v in Ga.items():
                Gv["dec%d" % l][k][...] = v
            gd = gd + gg
        genc[l] = gskip                        # skip contribution to enc_l
    if aspp:  # gd is d(loss)/d(ASPP output): back through the module
        gd, Ga = aspp_backward(gd, P["aspp"], cache["aspp"])
        for k, v in Ga.items():
            Gv["aspp"][k][...] = v
    # encoder, from the bottleneck down; gd is d(loss)/d(enc_{L-1} output)
    genc[levels - 1] = gd
    gy = genc[levels - 1]
    for l in range(levels - 1, -1, -1):
        if se_ratio:  # through the SE unit that follows the block
            Q, y_in, cse = P["enc%d" % l], cache["se%d" % l][0], cache["se%d" % l][1]
            gy, gw1, gb1, gw2, gb2 = se.se_backward(y_in, Q["se.w1"], Q["se.w2"], cse, gy)
            Ge = Gv["enc%d" % l]
            Ge["se.w1"][...], Ge["se.b1"][...] = gw1, gb1
            Ge["se.w2"][...], Ge["se.b2"][...] = gw2, gb2
        gx, G = resblock_backward(gy, P["enc%d" % l], cache["enc%d" % l])
        for k, v in G.items():
            Gv["enc%d" % l][k][...] = v
        if l > 0:
            gy = genc[l - 1] + avgpool2_backward(gx)
        else:
            ga = gx
    a, cs = cache["stem"]
    gn = relu_backward(ga, a)
    gh, Gv["stem"]["norm.g"][...], Gv["stem"]["norm.beta"][...] = \
        layer_norm_backward(gn, P["stem"]["norm.g"], cs)
    _, gw, gb = conv3d_backward(cache["z"], P["stem"]["conv.w"], gh, need_gx=False)
    Gv["stem"]["conv.w"][...] = gw
    Gv["stem"]["conv.b"][...] = gb
    return grad
