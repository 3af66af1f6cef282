"""Canonical flat layout of the network parameters theta, used to draw theta_0.

Network (reading of Sec. III-D for a plain 3D residual U-Net with L levels and
C base channels; level l has c_l = C * 2**l channels on an (n >> l)^3 grid):

  stem            conv3(1 -> C), norm
  enc_0           ResBlock(C -> C)
  enc_l, l >= 1   ResBlock(c_{l-1} -> c_l)        (input: 2x2x2 average pool)
  dec_l, l = L-2 .. 0
                  ResBlock(c_{l+1} + c_l -> c_l)  (input: [nearest-up x2, skip])
  tail            conv1(C -> 1)

ResBlock(a -> b): conv3(a -> b), norm, conv3(b -> b), norm, and a 1x1x1
projection conv(a -> b) on the skip path when a != b.

Flat order: modules as listed above; inside a module each conv contributes
W[Cout][Cin][kz][ky][kx] then b[Cout], each norm gamma[C] then beta[C], in the
order conv1, norm1, conv2, norm2, proj.  Kind is one of "w", "b", "g", "beta".
"""


def _resblock(prefix, cin, cout):
    s = [(prefix + ".conv1.w", (cout, cin, 3, 3, 3), "w"),
         (prefix + ".conv1.b", (cout,), "b"),
         (prefix + ".norm1.g", (cout,), "g"),
         (prefix + ".norm1.beta", (cout,), "beta"),
         (prefix + ".conv2.w", (cout, cout, 3, 3, 3), "w"),
         (prefix + ".conv2.b", (cout,), "b"),
         (prefix + ".norm2.g", (cout,), "g"),
         (prefix + ".norm2.beta", (cout,), "beta")]
    if cin != cout:
        s += [(prefix + ".proj.w", (cout, cin, 1, 1, 1), "w"),
              (prefix + ".proj.b", (cout,), "b")]
    return s


def param_specs(levels, base_ch):
    """List of (name, shape, kind) in flat order."""
    C = base_ch
    ch = [C << l for l in range(levels)]
    s = [("stem.conv.w", (C, 1, 3, 3, 3), "w"), ("stem.conv.b", (C,), "b"),
         ("stem.norm.g", (C,), "g"), ("stem.norm.beta", (C,), "beta")]
    s += _resblock("enc0", C, C)
    for l in range(1, levels):
        s += _resblock("enc%d" % l, ch[l - 1], ch[l])
    for l in range(levels - 2, -1, -1):
        s += _resblock("dec%d" % l, ch[l + 1] + ch[l], ch[l])
    s += [("tail.w", (1, C, 1, 1, 1), "w"), ("tail.b", (1,), "b")]
    return s


def param_count(levels, base_ch):
    total = 0
    for _, shape, _ in param_specs(levels, base_ch):
        k = 1
        for d in shape:
            k *= d
        total += k
    return total
