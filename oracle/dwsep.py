"""FP64 oracle of the depthwise-separable 3D convolution of the paper's
lightweight backbone (Sec. III-D; Sec. I: 3D-FastResUNet uses depthwise
separable convolutions to cut the cost of each convolution).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A depthwise-separable convolution is a per-channel 3x3x3 convolution followed
by a 1x1x1 convolution that mixes channels:

  depthwise:  d[c]  = bd[c]  + sum_{dz,dy,dx} wd[c, dz, dy, dx] x[c, z+dz-1, y+dy-1, x+dx-1]
  pointwise:  y[co] = bp[co] + sum_c wp[co, c] d[c]

with zeros outside the grid (the cross-correlation and padding convention of
``net.conv3d``).  Arrays are channel-first [C, n, n, n].
"""
import numpy as np


def dwconv3d(x, w, b, dil=1):
    """Depthwise 3x3x3 convolution: x [C, n, n, n], w [C, 3, 3, 3], b [C]; with
    dil > 1 the taps sit dil voxels apart (atrous convolution, as in the ASPP
    branches): out[c, v] = b[c] + sum_t w[c, t] x[c, v + dil (t - 1)]."""
    n, d = x.shape[1], dil
    xp = np.pad(x, ((0, 0), (d, d), (d, d), (d, d)))
    out = np.broadcast_to(b[:, None, None, None], x.shape).astype(np.float64).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                oz, oy, ox = dz * d, dy * d, dx * d
                out += w[:, dz, dy, dx, None, None, None] * xp[:, oz:oz + n, oy:oy + n, ox:ox + n]
    return out


def dwconv3d_backward(x, w, gout, dil=1):
    """(gx, gw, gb) of dwconv3d given gout = dL/dout."""
    n, d = x.shape[1], dil
    xp = np.pad(x, ((0, 0), (d, d), (d, d), (d, d)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                oz, oy, ox = dz * d, dy * d, dx * d
                win = xp[:, oz:oz + n, oy:oy + n, ox:ox + n]
                gw[:, dz, dy, dx] = (gout * win).sum(axis=(1, 2, 3))
                gxp[:, oz:oz + n, oy:oy + n, ox:ox + n] += w[:, dz, dy, dx, None, None, None] * gout
    gb = gout.sum(axis=(1, 2, 3))
    return gxp[:, d:n + d, d:n + d, d:n + d], gw, gb


def pwconv3d(x, w, b):
    """Pointwise (1x1x1) convolution: x [C, n, n, n], w [Cout, C], b [Cout]."""
    c, n = x.shape[0], x.shape[1]
    return (w @ x.reshape(c, -1) + b[:, None]).reshape(w.shape[0], n, n, n)


def pwconv3d_backward(x, w, gout):
    c, n = x.shape[0], x.shape[1]
    g2 = gout.reshape(w.shape[0], -1)
    gx = (w.T @ g2).reshape(c, n, n, n)
    return gx, g2 @ x.reshape(c, -1).T, g2.sum(axis=1)


def dwsep_conv3d(x, wd, bd, wp, bp):
    """Depthwise 3x3x3 then pointwise 1x1x1; returns (y, d)."""
    d = dwconv3d(x, wd, bd)
    return pwconv3d(d, wp, bp), d


def dwsep_conv3d_backward(x, wd, wp, d, gout):
    """(gx, gwd, gbd, gwp, gbp) given the depthwise output d and gout."""
    gd, gwp, gbp = pwconv3d_backward(d, wp, gout)
    gx, gwd, gbd = dwconv3d_backward(x, wd, gd)
    return gx, gwd, gbd, gwp, gbp
