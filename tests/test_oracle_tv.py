"""Pins of the FP64 4D-TV oracle (Sec. III-E, Eqs. (11)-(14)) against closed
forms, brute force and finite differences, and planted mistakes each pin catches."""
import math

import numpy as np
import pytest

import tseit_synth as ts
from oracle import fit, tv


def test_constant_image_spatial_tv_is_sqrt_eps():
    s = np.full((5, 5, 5), 0.7)
    R, g = tv.spatial(s, 1e-8)
    assert R == pytest.approx(1e-4, rel=1e-12)
    assert np.abs(g).max() == 0.0


def test_ramp_closed_form():
    """s = a * x: interior voxels differ by a along x only; the last column
    has no forward neighbour."""
    n, a, eps = 6, 0.3, 1e-8
    x = np.arange(n, dtype=np.float64)
    s = np.broadcast_to(a * x, (n, n, n)).copy()
    R, g = tv.spatial(s, eps)
    q = math.sqrt(a * a + eps)
    expect = ((n - 1) * n * n * q + n * n * math.sqrt(eps)) / n ** 3
    assert R == pytest.approx(expect, rel=1e-13)
    # gradient: -a/q at x = 0, +a/q at x = n-1, 0 inside (divided by V)
    gx = g[0, 0, :] * n ** 3
    assert gx[0] == pytest.approx(-a / q, rel=1e-12)
    assert gx[-1] == pytest.approx(a / q, rel=1e-12)
    assert np.abs(gx[1:-1]).max() < 1e-12


def test_spatial_matches_brute_force_loops():
    rng = np.random.default_rng(3)
    n, eps = 4, 1e-3
    s = rng.standard_normal((n, n, n))
    tot = 0.0
    for z in range(n):
        for y in range(n):
            for x in range(n):
                dz = s[z + 1, y, x] - s[z, y, x] if z + 1 < n else 0.0
                dy = s[z, y + 1, x] - s[z, y, x] if y + 1 < n else 0.0
                dx = s[z, y, x + 1] - s[z, y, x] if x + 1 < n else 0.0
                tot += math.sqrt(dz * dz + dy * dy + dx * dx + eps)
    assert tv.spatial(s, eps)[0] == pytest.approx(tot / n ** 3, rel=1e-13)


def test_temporal_closed_forms():
    n, c, eps = 4, 0.25, 1e-8
    rng = np.random.default_rng(4)
    s = rng.standard_normal((n, n, n))
    R, g = tv.temporal(s, [s - c], [1.0], eps)
    assert R == pytest.approx(n ** 3 * math.sqrt(c * c + eps), rel=1e-12)
    assert np.allclose(g, c / math.sqrt(c * c + eps), rtol=1e-12)
    w = tv.temporal_weights(3, [1, 2])
    assert w.sum() == pytest.approx(1.0)
    assert w[1] / w[0] == pytest.approx(math.e, rel=1e-12)   # the newer frame weighs e times more
    assert tv.temporal(s, [], [], eps) == (0.0, pytest.approx(np.zeros_like(s)))


def test_tv4d_gradient_by_central_differences():
    rng = np.random.default_rng(5)
    n, eps = 5, 1e-4
    s = rng.standard_normal((n, n, n))
    hist = [s + 0.3 * rng.standard_normal(s.shape) for _ in range(3)]
    w = tv.temporal_weights(4, [1, 2, 3])
    _, g = tv.tv4d(s, hist, w, 0.7, 1.0, 0.1, eps)
    v = rng.standard_normal(s.shape)
    h = 1e-6
    fp = tv.tv4d(s + h * v, hist, w, 0.7, 1.0, 0.1, eps)[0]
    fm = tv.tv4d(s - h * v, hist, w, 0.7, 1.0, 0.1, eps)[0]
    assert (fp - fm) / (2 * h) == pytest.approx(float((g * v).sum()), rel=1e-7)


def test_full_loss_with_tv_by_central_differences():
    p = ts.make_problem(8, 1, 2, 8, 7, frames=2, breathing=True, fp32=False)
    pr = fit.Problem(p["J"], p["mask"], p["Z"], 8, 2, 8)
    th = p["theta0"]
    rng = np.random.default_rng(6)
    hist = [pr.image(th + 0.01 * rng.standard_normal(th.shape))]
    cfg = dict(history=hist, weights=tv.temporal_weights(2, [1]), lam=0.05, lam_s=1.0,
               lam_t=0.1, eps=1e-6)
    L, g, _ = pr.loss_and_grad(th, p["dv"][1], cfg)
    v = rng.standard_normal(th.shape)
    h = 1e-7  # the square roots near zero differences curve sharply
    Lp = pr.loss_and_grad(th + h * v, p["dv"][1], cfg)[0]
    Lm = pr.loss_and_grad(th - h * v, p["dv"][1], cfg)[0]
    assert (Lp - Lm) / (2 * h) == pytest.approx(float(g @ v), rel=2e-5)


def test_sequence_with_tv_uses_earlier_frames():
    """Frame 1 has no temporal term; from frame 2 on the earlier frames' final
    images enter the loss (the loss differs from the data-only run)."""
    p = ts.make_problem(8, 1, 2, 8, 8, frames=3, breathing=True, fp32=False)
    pr = fit.Problem(p["J"], p["mask"], p["Z"], 8, 2, 8)
    cfg = dict(lam=0.002, lam_s=1.0, lam_t=0.1, eps=1e-8)
    im_tv, l_tv, _ = fit.fit_sequence(pr, p["theta0"], p["dv"], [3, 2, 2], 1e-3, tv=cfg)
    im_0, l_0, _ = fit.fit_sequence(pr, p["theta0"], p["dv"], [3, 2, 2], 1e-3)
    s1 = im_tv[0].reshape(8, 8, 8)
    # first iteration of frame 1: data + spatial term only
    L_data = fit.data_loss(pr.J, p["dv"][0], pr.image(p["theta0"]))[0]
    Rs = tv.spatial(pr.image(p["theta0"]).reshape(8, 8, 8), 1e-8)[0]
    assert l_tv[0][0] == pytest.approx(L_data + 0.002 * Rs, rel=1e-12)
    assert l_tv[1][0] != l_0[1][0]
    assert s1.shape == (8, 8, 8)


# ---- planted mistakes ------------------------------------------------------

def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_mutation_backward_differences(monkeypatch):
    def bad(s):
        dz = np.zeros_like(s); dy = np.zeros_like(s); dx = np.zeros_like(s)
        dz[1:] = s[1:] - s[:-1]; dy[:, 1:] = s[:, 1:] - s[:, :-1]; dx[:, :, 1:] = s[:, :, 1:] - s[:, :, :-1]
        return dz, dy, dx
    monkeypatch.setattr(tv, "forward_diffs", bad)
    _fails(test_ramp_closed_form)


def test_mutation_reversed_temporal_weights(monkeypatch):
    orig = tv.temporal_weights
    monkeypatch.setattr(tv, "temporal_weights", lambda i, prev: orig(i, prev)[::-1])
    _fails(test_temporal_closed_forms)


def test_mutation_gradient_missing_neighbour_terms(monkeypatch):
    def bad(s, eps=tv.TV_EPS):
        dz, dy, dx = tv.forward_diffs(s)
        q = np.sqrt(dz * dz + dy * dy + dx * dx + eps)
        return float(q.sum()) / s.size, -(dz + dy + dx) / q / s.size
    monkeypatch.setattr(tv, "spatial", bad)
    _fails(test_tv4d_gradient_by_central_differences)
