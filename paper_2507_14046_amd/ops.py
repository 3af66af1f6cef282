"""PyTorch autograd operators over the library's standalone kernels.

``Conv3dFn``, ``DWConv3dFn``, ``PWConv3dFn``, ``SEFn``, ``LayerNormReLUFn``
and ``MeasureFn`` wrap the op-level C-ABI (include/d2ip.h): their forward and
backward passes are the library's HIP kernels (implicit-GEMM convolutions
with the input and weight gradients, the depthwise 3x3x3 and pointwise 1x1x1
convolutions of the depthwise-separable convolution and their gradients, the
Squeeze-and-Excitation unit, the whole-volume LayerNorm + ReLU and its
backward, J sigma and J^T g).  ``DIPNet``
composes the prior of Eq. (3) from them (with ``conv="dwsep"`` every ResBlock
convolution is the depthwise-separable one of Sec. III-D, with ``se_ratio`` an
SE unit gates every encoder block, with ``att`` an attention unit gates every
decoder skip, with ``aspp`` an ASPP module transforms the bottleneck, and
``tail="sigmoid"`` gives the image 2 sigmoid(t) - 1); pooling, up-sampling, channel
concatenation and the 1x1x1 output head are plain tensor operations of the
model around the operators.  With ``recompute=True`` every ResBlock's
activations are dropped after the forward and recomputed during the backward
(``torch.utils.checkpoint``), trading one more forward for activation memory.

Activations are channels-last 2-D tensors [n^3, C] (voxel v = (z*n + y)*n + x).
"""
import ctypes

import numpy as np

from . import _lib as L

_PREC = {"fp32": L.PLAIN_FP32, "bf16": L.BF16_CONV, "bf16x3": L.BF16X3_CONV}


def _torch():
    import torch
    return torch


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(t):
    return ctypes.c_void_p(_torch().cuda.current_stream(t.device).cuda_stream)


def _a16(t):
    """t contiguous and 16-byte aligned (the float4 kernels' requirement):
    views into a flat parameter vector can start anywhere, so copy those."""
    if t is None:
        return None
    t = t.contiguous()
    return t if t.data_ptr() % 16 == 0 else t.clone()


def _workspace(fn, *args, device):
    torch = _torch()
    nb = ctypes.c_size_t()
    L.check(fn(*args, ctypes.byref(nb)))
    return torch.empty(nb.value, dtype=torch.uint8, device=device), nb.value


def _grid_n(V):
    n = round(V ** (1.0 / 3.0))
    if n ** 3 != V:
        raise ValueError("activations must hold n^3 voxels")
    return n


class Conv3dFn:
    """y = conv3d(x, w, b): x [n^3, cin], w [cout, cin, k, k, k] (k 3 or 1), b [cout]."""

    @staticmethod
    def apply(x, w, b, precision="fp32"):
        return _conv_fn().apply(x, w, b, precision)


class LayerNormReLUFn:
    """y = relu(LayerNorm(x) * gamma + beta + skip) over all n^3 x C values."""

    @staticmethod
    def apply(x, gamma, beta, skip=None):
        return _ln_fn().apply(x, gamma, beta, skip)


class DWConv3dFn:
    """y = depthwise conv3d(x, w, b): x [n^3, C] (C % 4 == 0), w [C, 1, 3, 3, 3] or
    [C, 3, 3, 3], b [C] or None (Sec. III-D's depthwise-separable convolution,
    first half); dil > 1 spaces the taps dil voxels apart (atrous)."""

    @staticmethod
    def apply(x, w, b=None, dil=1):
        return _dw_fn().apply(x, w, b, dil)


class PWConv3dFn:
    """y = pointwise conv3d(x, w, b) as an FP32 matrix-core GEMM: x [n^3, C],
    w [Cout, C] or [Cout, C, 1, 1, 1], b [Cout] or None (C, Cout % 4 == 0)."""

    @staticmethod
    def apply(x, w, b=None):
        return _pw_fn().apply(x, w, b)


def dwsep_conv3d(x, wd, bd, wp, bp):
    """Depthwise-separable convolution: the depthwise 3x3x3 convolution, then
    the pointwise 1x1x1 one, both on the library's kernels."""
    return PWConv3dFn.apply(DWConv3dFn.apply(x, wd, bd), wp, bp)


class SEFn:
    """y = SE(x): the Squeeze-and-Excitation unit of Sec. III-D on x [n^3, C]
    (C % 4 == 0): gate e = sigmoid(w2 relu(w1 mean(x) + b1) + b2), w1 [H, C],
    w2 [C, H]; y = x * e."""

    @staticmethod
    def apply(x, w1, b1, w2, b2):
        return _se_fn().apply(x, w1, b1, w2, b2)


class MeasureFn:
    """p = J sigma (J dense [M, Q]); its backward is g_sigma = J^T g_p."""

    @staticmethod
    def apply(sigma, J):
        return _measure_fn().apply(sigma, J)


_FNS = {}


def _conv_fn():
    if "conv" in _FNS:
        return _FNS["conv"]
    torch = _torch()

    class _Conv(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, w, b, precision):
            lib = L.load()
            x, w = x.contiguous(), w.contiguous()
            b = b.contiguous() if b is not None else None
            V, cin = x.shape
            cout, taps = w.shape[0], w[0, 0].numel()
            n = _grid_n(V)
            prec = _PREC[precision]
            ws, nb = _workspace(lib.d2ip_op_conv3d_bytes, n, cin, cout, taps, prec,
                                device=x.device)
            y = torch.empty(V, cout, dtype=torch.float32, device=x.device)
            L.check(lib.d2ip_op_conv3d_forward(_p(x), _p(w), _p(b), _p(y), n, cin, cout, taps,
                                               prec, _p(ws), nb, _stream(x)))
            ctx.save_for_backward(x, w)
            ctx.meta = (n, cin, cout, taps, prec, b is not None)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, w = ctx.saved_tensors
            n, cin, cout, taps, prec, has_b = ctx.meta
            gy = _a16(gy)
            need_x, need_w, need_b = ctx.needs_input_grad[:3]
            gx = torch.empty_like(x) if need_x else None
            gw = torch.empty_like(w) if need_w else None
            gb = torch.empty(cout, dtype=torch.float32, device=x.device) if (need_b and has_b) \
                else None
            ws, nb = _workspace(lib.d2ip_op_conv3d_bytes, n, cin, cout, taps, prec,
                                device=x.device)
            L.check(lib.d2ip_op_conv3d_backward(_p(x), _p(w), _p(gy), _p(gx), _p(gw), _p(gb), n,
                                                cin, cout, taps, prec, _p(ws), nb, _stream(x)))
            return gx, gw, gb, None

    _FNS["conv"] = _Conv
    return _Conv


def _dw_fn():
    if "dw" in _FNS:
        return _FNS["dw"]
    torch = _torch()

    class _DW(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, w, b, dil):
            lib = L.load()
            x, w, b = _a16(x), w.contiguous(), _a16(b)
            V, C = x.shape
            if w.numel() != 27 * C:
                raise ValueError("w must hold C x 27 taps")
            n = _grid_n(V)
            y = torch.empty_like(x)
            if dil == 1:
                L.check(lib.d2ip_op_dwconv3d_forward(_p(x), _p(w), _p(b), _p(y), n, C,
                                                     _stream(x)))
            else:
                L.check(lib.d2ip_op_dwconv3d_dilated_forward(_p(x), _p(w), _p(b), _p(y), n, C,
                                                             dil, _stream(x)))
            ctx.save_for_backward(x, w)
            ctx.meta = (n, C, b is not None, dil)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, w = ctx.saved_tensors
            n, C, has_b, dil = ctx.meta
            gy = _a16(gy)
            need_x, need_w, need_b = ctx.needs_input_grad[:3]
            gx = torch.empty_like(x) if need_x else None
            gw = torch.empty_like(w) if need_w else None
            gb = torch.empty(C, dtype=torch.float32, device=x.device) if (need_b and has_b) \
                else None
            ws, nb = (None, 0)
            if dil == 1:
                if gw is not None or gb is not None:
                    ws, nb = _workspace(lib.d2ip_op_dwconv3d_bytes, n, C, device=x.device)
                L.check(lib.d2ip_op_dwconv3d_backward(_p(x), _p(w), _p(gy), _p(gx), _p(gw),
                                                      _p(gb), n, C, _p(ws), nb, _stream(x)))
            else:
                if gw is not None or gb is not None:
                    ws, nb = _workspace(lib.d2ip_op_dwconv3d_dilated_bytes, n, C, dil,
                                        device=x.device)
                L.check(lib.d2ip_op_dwconv3d_dilated_backward(_p(x), _p(w), _p(gy), _p(gx),
                                                              _p(gw), _p(gb), n, C, dil, _p(ws),
                                                              nb, _stream(x)))
            return gx, gw, gb, None

    _FNS["dw"] = _DW
    return _DW


def _pw_fn():
    if "pw" in _FNS:
        return _FNS["pw"]
    torch = _torch()

    class _PW(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, w, b):
            lib = L.load()
            x, w = _a16(x), _a16(w)
            b = b.contiguous() if b is not None else None
            V, cin = x.shape
            cout = w.shape[0]
            if w.numel() != cout * cin:
                raise ValueError("w must be [Cout, C] (or [Cout, C, 1, 1, 1])")
            n = _grid_n(V)
            y = torch.empty(V, cout, dtype=torch.float32, device=x.device)
            L.check(lib.d2ip_op_pwconv3d_forward(_p(x), _p(w), _p(b), _p(y), n, cin, cout,
                                                 _stream(x)))
            ctx.save_for_backward(x, w)
            ctx.meta = (n, cin, cout, b is not None)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, w = ctx.saved_tensors
            n, cin, cout, has_b = ctx.meta
            gy = _a16(gy)
            need_x, need_w, need_b = ctx.needs_input_grad[:3]
            gx = torch.empty_like(x) if need_x else None
            gw = torch.empty_like(w) if need_w else None
            gb = torch.empty(cout, dtype=torch.float32, device=x.device) if (need_b and has_b) \
                else None
            ws, nb = (None, 0)
            if gw is not None or gb is not None:
                ws, nb = _workspace(lib.d2ip_op_pwconv3d_bytes, n, cin, cout, device=x.device)
            L.check(lib.d2ip_op_pwconv3d_backward(_p(x), _p(w), _p(gy), _p(gx), _p(gw), _p(gb),
                                                  n, cin, cout, _p(ws), nb, _stream(x)))
            return gx, gw, gb

    _FNS["pw"] = _PW
    return _PW


def _se_fn():
    if "se" in _FNS:
        return _FNS["se"]
    torch = _torch()

    class _SE(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, w1, b1, w2, b2):
            lib = L.load()
            x = _a16(x)
            w1, b1, w2, b2 = (t.contiguous() for t in (w1, b1, w2, b2))
            V, C = x.shape
            H = w1.shape[0]
            n = _grid_n(V)
            ws, nb = _workspace(lib.d2ip_op_se_bytes, n, C, H, device=x.device)
            y = torch.empty_like(x)
            L.check(lib.d2ip_op_se_forward(_p(x), _p(w1), _p(b1), _p(w2), _p(b2), _p(y), n, C,
                                           H, _p(ws), nb, _stream(x)))
            ctx.save_for_backward(x, w1, b1, w2, b2)
            ctx.meta = (n, C, H)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, w1, b1, w2, b2 = ctx.saved_tensors
            n, C, H = ctx.meta
            gy = _a16(gy)
            need = ctx.needs_input_grad[:5]
            outs = [torch.empty_like(t) if nd else None
                    for t, nd in zip((x, w1, b1, w2, b2), need)]
            ws, nb = _workspace(lib.d2ip_op_se_bytes, n, C, H, device=x.device)
            L.check(lib.d2ip_op_se_backward(_p(x), _p(w1), _p(b1), _p(w2), _p(b2), _p(gy),
                                            *[_p(o) for o in outs], n, C, H, _p(ws), nb,
                                            _stream(x)))
            return tuple(outs)

    _FNS["se"] = _SE
    return _SE


def _ln_fn():
    if "ln" in _FNS:
        return _FNS["ln"]
    torch = _torch()

    class _LN(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, gamma, beta, skip):
            lib = L.load()
            x = _a16(x)
            skip = _a16(skip) if skip is not None else None
            V, C = x.shape
            n = _grid_n(V)
            ws, nb = _workspace(lib.d2ip_op_ln_relu_bytes, n, C, device=x.device)
            y = torch.empty_like(x)
            L.check(lib.d2ip_op_ln_relu_forward(_p(x), _p(gamma.contiguous()),
                                                _p(beta.contiguous()), _p(skip), _p(y), n, C,
                                                _p(ws), nb, _stream(x)))
            ctx.save_for_backward(x, y, gamma)
            ctx.meta = (n, C, skip is not None)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, y, gamma = ctx.saved_tensors
            n, C, has_skip = ctx.meta
            gy = _a16(gy)
            gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
            gskip = torch.empty_like(x) if (has_skip and ctx.needs_input_grad[3]) else None
            need_gb = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
            ggb = torch.empty(2 * C, dtype=torch.float32, device=x.device) if need_gb else None
            ws, nb = _workspace(lib.d2ip_op_ln_relu_bytes, n, C, device=x.device)
            L.check(lib.d2ip_op_ln_relu_backward(_p(x), _p(y), _p(gamma.contiguous()), _p(gy),
                                                 _p(gx), _p(gskip), _p(ggb), n, C, _p(ws), nb,
                                                 _stream(x)))
            gg = ggb[:C] if need_gb else None
            gbeta = ggb[C:] if need_gb else None
            return gx, gg, gbeta, gskip

    _FNS["ln"] = _LN
    return _LN


def _measure_fn():
    if "j" in _FNS:
        return _FNS["j"]
    torch = _torch()

    class _J(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sigma, J):
            lib = L.load()
            sigma, J = sigma.contiguous(), J.contiguous()
            M, Q = J.shape
            p = torch.empty(M, dtype=torch.float32, device=J.device)
            L.check(lib.d2ip_op_j_forward(_p(J), _p(sigma), _p(p), M, Q, _stream(J)))
            ctx.save_for_backward(J)
            return p

        @staticmethod
        def backward(ctx, gp):
            lib = L.load()
            (J,) = ctx.saved_tensors
            M, Q = J.shape
            out = torch.empty(Q, dtype=torch.float32, device=J.device)
            ws, nb = _workspace(lib.d2ip_op_jt_bytes, M, Q, device=J.device)
            L.check(lib.d2ip_op_jt(_p(J), _p(gp.contiguous()), _p(out), M, Q, _p(ws), nb,
                                   _stream(J)))
            return out, None

    _FNS["j"] = _J
    return _J


class Pool2Fn:
    """y = 2x2x2 average pool of x [n^3, C] -> [(n/2)^3, C] (library kernel)."""

    @staticmethod
    def apply(x):
        return _pool_fn().apply(x)


class Up2ConcatFn:
    """cat = [nearest-up x2 of d [(n/2)^3, Cu], e [n^3, Cs]] (library kernel)."""

    @staticmethod
    def apply(d, e):
        return _upcat_fn().apply(d, e)


class HeadFn:
    """out [n^3] = mask * (w . x[v] + b), or mask * (2 sigmoid(.) - 1) with
    sigmoid=True: the output head (library kernels)."""

    @staticmethod
    def apply(x, w, b, mask=None, sigmoid=False):
        return _head_fn().apply(x, w, b, mask, sigmoid)


class AttentionFn:
    """Attention unit of a decoder stage (library kernels): the skip x [n^3, c]
    gated by coefficients formed on the grid of the coarser decoder output
    g [(n/2)^3, cu] from the pooled skip, then interpolated to x's grid."""

    @staticmethod
    def apply(x, g, wx, wg, b, psi, bpsi):
        return _att_fn().apply(x, g, wx, wg, b, psi, bpsi)


class ChannelConcatFn:
    """[x0 | x1 | ...] along channels of channels-last tensors [V, c_i]
    (library channel-range copies, forward and backward)."""

    @staticmethod
    def apply(*xs):
        return _chcat_fn().apply(*xs)


class ReLUFn:
    """max(x, 0) on the library's kernels."""

    @staticmethod
    def apply(x):
        return _relu_fn().apply(x)


def _chcat_fn():
    if "chcat" in _FNS:
        return _FNS["chcat"]
    torch = _torch()

    class _ChCat(torch.autograd.Function):
        @staticmethod
        def forward(ctx, *xs):
            lib = L.load()
            xs = [_a16(x) for x in xs]
            V = xs[0].shape[0]
            cs = [int(x.shape[1]) for x in xs]
            if any(x.shape[0] != V or x.dim() != 2 for x in xs):
                raise ValueError("tensors must be [V, c] with the same V")
            out = torch.empty(V, sum(cs), dtype=xs[0].dtype, device=xs[0].device)
            off = 0
            for x, c in zip(xs, cs):
                L.check(lib.d2ip_op_channel_copy(_p(x), c, 0, _p(out), out.shape[1], off, c, V,
                                                 _stream(x)))
                off += c
            ctx.cs = cs
            return out

        @staticmethod
        def backward(ctx, g):
            lib = L.load()
            g = _a16(g)
            V, out, off = g.shape[0], [], 0
            for c in ctx.cs:
                gi = torch.empty(V, c, dtype=g.dtype, device=g.device)
                L.check(lib.d2ip_op_channel_copy(_p(g), g.shape[1], off, _p(gi), c, 0, c, V,
                                                 _stream(g)))
                out.append(gi)
                off += c
            return tuple(out)

    _FNS["chcat"] = _ChCat
    return _ChCat


def _relu_fn():
    if "relu" in _FNS:
        return _FNS["relu"]
    torch = _torch()

    class _ReLU(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            lib = L.load()
            x = _a16(x)
            y = torch.empty_like(x)
            L.check(lib.d2ip_op_relu_forward(_p(x), _p(y), x.numel(), _stream(x)))
            ctx.save_for_backward(y)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            (y,) = ctx.saved_tensors
            gy = _a16(gy)
            gx = torch.empty_like(gy)
            L.check(lib.d2ip_op_relu_backward(_p(y), _p(gy), _p(gx), y.numel(), _stream(gy)))
            return gx

    _FNS["relu"] = _ReLU
    return _ReLU


def _pool_fn():
    if "pool" in _FNS:
        return _FNS["pool"]
    torch = _torch()

    class _Pool(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            lib = L.load()
            x = _a16(x)
            n, C = _grid_n(x.shape[0]), x.shape[1]
            y = torch.empty((n // 2) ** 3, C, dtype=x.dtype, device=x.device)
            L.check(lib.d2ip_op_pool2_forward(_p(x), _p(y), n, C, _stream(x)))
            ctx.n = n
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            gy = _a16(gy)
            C = gy.shape[1]
            gx = torch.empty(ctx.n ** 3, C, dtype=gy.dtype, device=gy.device)
            L.check(lib.d2ip_op_pool2_backward(_p(gy), _p(gx), ctx.n, C, _stream(gy)))
            return gx

    _FNS["pool"] = _Pool
    return _Pool


def _upcat_fn():
    if "upcat" in _FNS:
        return _FNS["upcat"]
    torch = _torch()

    class _UpCat(torch.autograd.Function):
        @staticmethod
        def forward(ctx, d, e):
            lib = L.load()
            d, e = _a16(d), _a16(e)
            n, Cu, Cs = _grid_n(e.shape[0]), d.shape[1], e.shape[1]
            cat = torch.empty(n ** 3, Cu + Cs, dtype=e.dtype, device=e.device)
            L.check(lib.d2ip_op_up2_concat_forward(_p(d), Cu, _p(e), Cs, n, _p(cat), _stream(e)))
            ctx.dims = (n, Cu, Cs)
            return cat

        @staticmethod
        def backward(ctx, gcat):
            lib = L.load()
            n, Cu, Cs = ctx.dims
            gcat = _a16(gcat)
            gd = torch.empty((n // 2) ** 3, Cu, dtype=gcat.dtype, device=gcat.device)
            ge = torch.empty(n ** 3, Cs, dtype=gcat.dtype, device=gcat.device)
            L.check(lib.d2ip_op_up2_concat_backward(_p(gcat), Cu, Cs, n, _p(gd), _p(ge),
                                                    _stream(gcat)))
            return gd, ge

    _FNS["upcat"] = _UpCat
    return _UpCat


def _head_fn():
    if "head" in _FNS:
        return _FNS["head"]
    torch = _torch()

    class _Head(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, w, b, mask, sigmoid):
            lib = L.load()
            wshape = w.shape
            x, w, b = _a16(x), _a16(w.reshape(-1)), b.contiguous()
            n, C = _grid_n(x.shape[0]), x.shape[1]
            m = mask.contiguous() if mask is not None else None
            out = torch.empty(n ** 3, dtype=x.dtype, device=x.device)
            L.check(lib.d2ip_op_head_forward(_p(x), _p(w), _p(b), _p(m), _p(out), n, C,
                                             int(bool(sigmoid)), _stream(x)))
            ctx.save_for_backward(x, w, b, m if m is not None else torch.empty(0))
            ctx.sigmoid, ctx.has_mask, ctx.wshape = bool(sigmoid), m is not None, wshape
            return out

        @staticmethod
        def backward(ctx, gout):
            lib = L.load()
            x, w, b, m = ctx.saved_tensors
            n, C = _grid_n(x.shape[0]), x.shape[1]
            gx, gw, gb = torch.empty_like(x), torch.empty_like(w), torch.empty_like(b)
            ws, nb = _workspace(lib.d2ip_op_head_bytes, n, C, device=x.device)
            L.check(lib.d2ip_op_head_backward(
                _p(x), _p(w), _p(b), _p(m) if ctx.has_mask else None, _p(gout.contiguous()),
                _p(gx), _p(gw), _p(gb), n, C, int(ctx.sigmoid), _p(ws), nb, _stream(x)))
            return gx, gw.view(ctx.wshape), gb, None, None

    _FNS["head"] = _Head
    return _Head


def _att_fn():
    if "att" in _FNS:
        return _FNS["att"]
    torch = _torch()

    class _Att(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, g, wx, wg, b, psi, bpsi):
            lib = L.load()
            x, g, wx, wg = _a16(x), _a16(g), _a16(wx), _a16(wg)
            b, psi, bpsi = (t.contiguous() for t in (b, psi, bpsi))
            n, c, cu = _grid_n(x.shape[0]), x.shape[1], g.shape[1]
            y = torch.empty_like(x)
            ws, nb = _workspace(lib.d2ip_op_attention_bytes, n, c, cu, device=x.device)
            L.check(lib.d2ip_op_attention_forward(_p(x), _p(g), _p(wx), _p(wg), _p(b), _p(psi),
                                                  _p(bpsi), _p(y), None, n, c, cu, _p(ws), nb,
                                                  _stream(x)))
            ctx.save_for_backward(x, g, wx, wg, b, psi, bpsi)
            return y

        @staticmethod
        def backward(ctx, gy):
            lib = L.load()
            x, g, wx, wg, b, psi, bpsi = ctx.saved_tensors
            n, c, cu = _grid_n(x.shape[0]), x.shape[1], g.shape[1]
            gy = _a16(gy)
            gx, gg = torch.empty_like(x), torch.empty_like(g)
            grads = [torch.empty_like(t) for t in (wx, wg, b, psi, bpsi)]
            ws, nb = _workspace(lib.d2ip_op_attention_bytes, n, c, cu, device=x.device)
            L.check(lib.d2ip_op_attention_backward(
                _p(x), _p(g), _p(wx), _p(wg), _p(b), _p(psi), _p(bpsi), _p(gy), _p(gx), _p(gg),
                *[_p(t) for t in grads], n, c, cu, _p(ws), nb, _stream(x)))
            return (gx, gg, *grads)

    _FNS["att"] = _Att
    return _Att


class MSELossFn:
    """(1/M) sum (p - dv)^2 as a float64 scalar tensor: reduced in FP64 on the
    device by the library (the data term of Eq. (4)); gradient (2/M)(p - dv)."""

    @staticmethod
    def apply(p, dv):
        return _mse_fn().apply(p, dv)


def _mse_fn():
    if "mse" in _FNS:
        return _FNS["mse"]
    torch = _torch()

    class _MSE(torch.autograd.Function):
        @staticmethod
        def forward(ctx, p, dv):
            lib = L.load()
            p, dv = p.contiguous(), dv.contiguous()
            if p.dtype != torch.float32 or dv.dtype != torch.float32 or p.numel() != dv.numel():
                raise TypeError("p and dv must be float32 tensors of equal size")
            loss = torch.empty((), dtype=torch.float64, device=p.device)
            gp = torch.empty_like(p)
            L.check(lib.d2ip_op_mse_loss(_p(p), _p(dv), _p(gp), _p(loss), p.numel(),
                                         _stream(p)))
            ctx.save_for_backward(gp)
            return loss

        @staticmethod
        def backward(ctx, gl):
            (gp,) = ctx.saved_tensors
            return gp * gl.to(torch.float32), None

    _FNS["mse"] = _MSE
    return _MSE


# ----------------------------------------------------------------------------
# the prior of Eq. (3) composed from the operators
# ----------------------------------------------------------------------------

ASPP_RATES = (1, 2, 3)  # dilations of the ASPP module's atrous branches


def param_shapes(levels, base_ch, sep=False, se_ratio=0, att=False, aspp=False):
    """(name, shape) of every parameter tensor in the canonical flat order:
    stem, encoder ResBlocks 0..L-1, decoder ResBlocks L-2..0, head; in a
    module each conv's W [Cout][Cin][k][k][k] then b, each norm gamma then
    beta, in the order conv1, norm1, conv2, norm2, projection.  With sep each
    ResBlock 3x3x3 conv is depthwise-separable (Sec. III-D): depthwise
    [Cin][3][3][3] and its bias, then pointwise [Cout][Cin] and its bias.
    With se_ratio r > 0 each encoder module ends with an SE unit's w1 [H][c],
    b1, w2 [c][H], b2 (H = max(1, c // r)); with att each decoder module ends
    with an attention unit's wx [c][c], wg [c][c_up], b [c], psi [c], bpsi [1]."""
    C = base_ch
    ch = [C << l for l in range(levels)]
    out = [("stem.w", (C, 1, 3, 3, 3)), ("stem.b", (C,)), ("stem.g", (C,)), ("stem.beta", (C,))]

    def conv(name, k, a, b):
        if sep:
            return [(name + ".dw" + k, (a, 3, 3, 3)), (name + ".dwb" + k, (a,)),
                    (name + ".pw" + k, (b, a)), (name + ".pwb" + k, (b,))]
        return [(name + ".w" + k, (b, a, 3, 3, 3)), (name + ".b" + k, (b,))]

    def block(name, a, b):
        s = (conv(name, "1", a, b) + [(name + ".g1", (b,)), (name + ".beta1", (b,))] +
             conv(name, "2", b, b) + [(name + ".g2", (b,)), (name + ".beta2", (b,))])
        if a != b:
            s += [(name + ".wp", (b, a, 1, 1, 1)), (name + ".bp", (b,))]
        return s

    def se_unit(name, c):
        if not se_ratio:
            return []
        h = max(1, c // se_ratio)
        return [(name + ".sw1", (h, c)), (name + ".sb1", (h,)), (name + ".sw2", (c, h)),
                (name + ".sb2", (c,))]

    out += block("enc0", C, C) + se_unit("enc0", C)
    for l in range(1, levels):
        out += block("enc%d" % l, ch[l - 1], ch[l]) + se_unit("enc%d" % l, ch[l])
    def att_unit(name, c, c_up):
        if not att:
            return []
        return [(name + ".awx", (c, c)), (name + ".awg", (c, c_up)), (name + ".ab", (c,)),
                (name + ".apsi", (c,)), (name + ".abpsi", (1,))]

    if aspp:  # on the bottleneck, between the encoder and decoder modules
        c = ch[-1]
        out += [("aspp.w0", (c, c)), ("aspp.b0", (c,))]
        for d in ASPP_RATES:
            out += [("aspp.dw%d" % d, (c, 3, 3, 3)), ("aspp.dwb%d" % d, (c,)),
                    ("aspp.pw%d" % d, (c, c)), ("aspp.pwb%d" % d, (c,))]
        out += [("aspp.wp", (c, c * (1 + len(ASPP_RATES)))), ("aspp.bp", (c,))]
    for l in range(levels - 2, -1, -1):
        out += block("dec%d" % l, ch[l + 1] + ch[l], ch[l]) + att_unit("dec%d" % l, ch[l],
                                                                       ch[l + 1])
    out += [("head.w", (1, C, 1, 1, 1)), ("head.b", (1,))]
    return out


class DIPNet:
    """sigma = mask * phi(theta | Z) built from the operators; theta is one
    flat tensor in the canonical order (gradients flow to it through views)."""

    def __init__(self, n, levels, base_ch, precision="fp32", recompute=False, conv="dense",
                 se_ratio=0, att=False, tail="linear", aspp=False):
        if conv not in ("dense", "dwsep"):
            raise ValueError("conv must be 'dense' or 'dwsep'")
        if tail not in ("linear", "sigmoid"):
            raise ValueError("tail must be 'linear' or 'sigmoid'")
        self.att, self.tail = att, tail  # attention units on the skips; output head
        self.n, self.L, self.C = n, levels, base_ch
        self.precision = precision
        self.recompute = recompute
        self.sep = conv == "dwsep"  # depthwise-separable ResBlock convs (FP32)
        self.se_ratio = se_ratio    # SE units gating the encoder blocks (0: none)
        self.aspp = aspp  # ASPP module at the bottleneck
        self.shapes = param_shapes(levels, base_ch, self.sep, se_ratio, att, aspp)
        self.size = int(sum(np.prod(s) for _, s in self.shapes))

    def views(self, theta):
        out, off = {}, 0
        for name, shape in self.shapes:
            k = int(np.prod(shape))
            out[name] = theta[off:off + k].view(*shape)
            off += k
        return out

    def _conv3(self, P, name, k, x):
        if self.sep:
            return dwsep_conv3d(x, P[name + ".dw" + k], P[name + ".dwb" + k], P[name + ".pw" + k],
                                P[name + ".pwb" + k])
        return Conv3dFn.apply(x, P[name + ".w" + k], P[name + ".b" + k], self.precision)

    def _block(self, P, name, x, n):
        prec = self.precision
        h1 = self._conv3(P, name, "1", x)
        a1 = LayerNormReLUFn.apply(h1, P[name + ".g1"], P[name + ".beta1"])
        h2 = self._conv3(P, name, "2", a1)
        s = Conv3dFn.apply(x, P[name + ".wp"], P[name + ".bp"], prec) if name + ".wp" in P else x
        return LayerNormReLUFn.apply(h2, P[name + ".g2"], P[name + ".beta2"], s)

    def _run_block(self, P, name, x, n):
        if not self.recompute:
            return self._block(P, name, x, n)
        from torch.utils.checkpoint import checkpoint
        return checkpoint(lambda t: self._block(P, name, t, n), x, use_reentrant=False)

    def forward(self, theta, Z, mask):
        """theta [P], Z [n^3] noise input, mask [n^3] (0/1) -> sigma [n^3]."""
        torch = _torch()
        P = self.views(theta)
        n, L = self.n, self.L
        # the 1-channel stem input is padded to 8 channels (zero weights)
        z8 = torch.zeros(n ** 3, 8, dtype=torch.float32, device=Z.device)
        z8[:, 0] = Z
        w8 = torch.cat([P["stem.w"], torch.zeros(self.C, 7, 3, 3, 3, dtype=theta.dtype,
                                                 device=theta.device)], dim=1)
        h = Conv3dFn.apply(z8, w8, P["stem.b"], self.precision)
        x = LayerNormReLUFn.apply(h, P["stem.g"], P["stem.beta"])
        skips = []
        for l in range(L):
            nl = n >> l
            if l > 0:
                x = Pool2Fn.apply(x)
            x = self._run_block(P, "enc%d" % l, x, nl)
            if self.se_ratio:
                e = "enc%d" % l
                x = SEFn.apply(x, P[e + ".sw1"], P[e + ".sb1"], P[e + ".sw2"], P[e + ".sb2"])
            skips.append(x)
        if self.aspp:
            x = self._aspp(P, x)
        for l in range(L - 2, -1, -1):
            nl = n >> l
            s = skips[l]
            if self.att:  # the gate on the coarse grid, then the interpolation
                s = self._attend(P, "dec%d" % l, s, x, nl)
            x = Up2ConcatFn.apply(x, s)
            x = self._run_block(P, "dec%d" % l, x, nl)
        return HeadFn.apply(x, P["head.w"], P["head.b"], mask, self.tail == "sigmoid")

    def _aspp(self, P, x):
        """ASPP on the bottleneck: a 1x1x1 branch and one depthwise-separable
        atrous branch per rate, concatenated, projected (1x1x1), ReLU."""
        br = [PWConv3dFn.apply(x, P["aspp.w0"], P["aspp.b0"])]
        for d in ASPP_RATES:
            t = DWConv3dFn.apply(x, P["aspp.dw%d" % d], P["aspp.dwb%d" % d], d)
            br.append(PWConv3dFn.apply(t, P["aspp.pw%d" % d], P["aspp.pwb%d" % d]))
        return ReLUFn.apply(PWConv3dFn.apply(ChannelConcatFn.apply(*br), P["aspp.wp"],
                                             P["aspp.bp"]))

    def _attend(self, P, d, s, g, n):
        """Attention unit of a decoder stage (Sec. III-D: attention, then
        interpolation) on the library's kernels: the skip s (n^3 grid) gated
        by sigmoid(psi . relu(wx pool2(s) + wg g + b) + bpsi), formed on the
        grid of the coarser decoder output g and interpolated (nearest, x2)."""
        return AttentionFn.apply(s, g, P[d + ".awx"], P[d + ".awg"], P[d + ".ab"],
                                 P[d + ".apsi"], P[d + ".abpsi"])

    def loss(self, theta, Z, mask, J, dv):
        """(1/M) sum (J sigma - dv)^2 (float64 scalar), with J sigma, J^T and
        the FP64 loss reduction on the library's kernels."""
        sigma = self.forward(theta, Z, mask)
        return MSELossFn.apply(MeasureFn.apply(sigma, J), dv)
