"""FP64 oracle of the Squeeze-and-Excitation unit of the paper's
3D-FastResUNet (Sec. III-D: three SE units gate the channels of the
encoder; the unit follows its cited definition, ref. [43]).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

  squeeze:     s[c] = (1 / V) sum_v x[c, v]                (global average pool)
  excitation:  z = relu(W1 s + b1)       W1 [H, C], b1 [H]
               e = sigmoid(W2 z + b2)    W2 [C, H], b2 [C]
  scale:       y[c, v] = e[c] x[c, v]

Arrays are channel-first [C, n, n, n]; V = n^3.  The hidden width H (C / r
for a reduction ratio r) is a parameter.
"""
import numpy as np


def sigmoid(t):
    return 1.0 / (1.0 + np.exp(-t))


def se_forward(x, w1, b1, w2, b2):
    """Returns y and the cache (s, z, e) the backward needs."""
    C = x.shape[0]
    s = x.reshape(C, -1).mean(axis=1)
    z = np.maximum(w1 @ s + b1, 0.0)
    e = sigmoid(w2 @ z + b2)
    y = x * e[:, None, None, None]
    return y, dict(s=s, z=z, e=e)


def se_backward(x, w1, w2, cache, gy):
    """(gx, gw1, gb1, gw2, gb2) given gy = dL/dy."""
    C = x.shape[0]
    V = x[0].size
    s, z, e = cache["s"], cache["z"], cache["e"]
    ge = (gy * x).reshape(C, -1).sum(axis=1)     # dL/de
    ga2 = ge * e * (1.0 - e)                     # through the sigmoid
    gw2, gb2 = np.outer(ga2, z), ga2
    gz = w2.T @ ga2
    ga1 = gz * (z > 0)                           # through the ReLU (relu'(0) = 0)
    gw1, gb1 = np.outer(ga1, s), ga1
    gs = w1.T @ ga1                              # dL/ds
    gx = gy * e[:, None, None, None] + (gs / V)[:, None, None, None]
    return gx, gw1, gb1, gw2, gb2
