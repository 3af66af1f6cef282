"""The pins catch plausible mistakes: each test plants one mistake in the
oracle (CPU only, via monkeypatch) and checks that a pin then fails."""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import net, fit


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_ln_backward_missing_term(monkeypatch):
    def bad(gout, g, cache):
        xhat, rstd = cache
        gxhat = gout * g[:, None, None, None]
        gh = rstd * (gxhat - gxhat.mean())
        return gh, (gout * xhat).sum(axis=(1, 2, 3)), gout.sum(axis=(1, 2, 3))
    monkeypatch.setattr(net, "layer_norm_backward", bad)
    _fails(pins.test_layernorm_backward_torch)
    _fails(pins.test_network_forward_backward_vs_torch_autograd, 8, 2, 2)


def test_conv_backward_unflipped_taps(monkeypatch):
    orig = net.conv3d_backward

    def bad(x, w, gout, need_gx=True):
        return orig(x, w[:, :, ::-1, ::-1, ::-1].copy(), gout, need_gx)[0], \
            orig(x, w, gout, need_gx)[1], orig(x, w, gout, need_gx)[2]
    monkeypatch.setattr(net, "conv3d_backward", bad)
    _fails(pins.test_conv_backward_adjoint_and_torch)


def test_conv_forward_transposed_tap(monkeypatch):
    orig = net.conv3d

    def bad(x, w, b):
        return orig(x, np.ascontiguousarray(w.transpose(0, 1, 2, 4, 3)), b)
    monkeypatch.setattr(net, "conv3d", bad)
    _fails(pins.test_conv_matches_torch)


def test_adam_without_bias_correction(monkeypatch):
    def bad(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        t += 1
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        return theta - lr * m / (np.sqrt(v) + eps), m, v, t
    monkeypatch.setattr(fit, "adam_step", bad)
    _fails(pins.test_adam_first_step_closed_form)


def test_data_loss_sign(monkeypatch):
    def bad(J, dv, sigma):
        r = J @ sigma - dv
        return float(r @ r) / J.shape[0], -(2.0 / J.shape[0]) * (J.T @ r)
    monkeypatch.setattr(fit, "data_loss", bad)
    _fails(pins.test_data_loss_value)


def test_up_backward_mean_instead_of_sum(monkeypatch):
    def bad(gout):
        c, n = gout.shape[0], gout.shape[1]
        m = n // 2
        return gout.reshape(c, m, 2, m, 2, m, 2).mean(axis=(2, 4, 6))
    monkeypatch.setattr(net, "up2_backward", bad)
    _fails(pins.test_pool_and_up_against_torch_and_adjoints)
    _fails(pins.test_network_forward_backward_vs_torch_autograd, 8, 2, 2)


def test_skip_gradient_dropped(monkeypatch):
    orig = net.resblock_backward

    def bad(gy, P, cache):
        gx, G = orig(gy, P, cache)
        if "proj.w" not in P:
            gz = net.relu_backward(gy, cache["y"])
            gx = gx - gz
        return gx, G
    monkeypatch.setattr(net, "resblock_backward", bad)
    _fails(pins.test_network_forward_backward_vs_torch_autograd, 8, 2, 2)


def _attention_pin():
    import tests.test_oracle_modules as mods
    mods.test_attention_unit_matches_torch_float64(4, 4, 3)


def test_attention_transposed_skip_weight(monkeypatch):
    orig = net.att_forward

    def bad(x, g, Q):
        return orig(x, g, dict(Q, **{"att.wx": np.ascontiguousarray(Q["att.wx"].T)}))
    monkeypatch.setattr(net, "att_forward", bad)
    _fails(_attention_pin)


def test_attention_swapped_skip_and_gate(monkeypatch):
    def bad(x, g, Q):
        c = x.shape[0]
        xs = net.avgpool2(x)
        Xs, G = xs.reshape(c, -1), g.reshape(g.shape[0], -1)
        a = Q["att.wx"] @ G + Q["att.wg"] @ Xs + Q["att.b"][:, None]   # inputs swapped
        q = np.maximum(a, 0.0)
        al = 1.0 / (1.0 + np.exp(-(Q["att.psi"] @ q + Q["att.bpsi"][0])))
        alf = net.up2(al.reshape((1,) + g.shape[1:]))
        return alf * x, dict(x=x, Xs=Xs, G=G, a=a, q=q, al=al, alf=alf)
    monkeypatch.setattr(net, "att_forward", bad)
    _fails(_attention_pin)
