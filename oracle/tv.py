"""FP64 oracle of the 4D total-variation regulariser (Sec. III-E).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For the current frame's image s (n^3 voxels, (z, y, x) order) and the
reconstructed images h_j of the previous frames j = 1 .. i-1:

  R_spatial(s)  = (1/V) sum_v sqrt(dz(v)^2 + dy(v)^2 + dx(v)^2 + eps)     (Eq. (12))
      forward differences dz(v) = s[z+1, y, x] - s[z, y, x] etc.; a
      difference whose neighbour lies outside the grid is 0 (the paper does
      not say; the image is zero-padded in no other place, so the boundary
      simply has fewer differences); V = n^3.
  R_temporal    = (1 / sum_j a_j) sum_j a_j sum_v sqrt((s[v] - h_j[v])^2 + eps)  (Eq. (13))
      a_j = exp(-(i - j)); with no previous frame the term is 0.
  R_4D-TV       = lambda_s R_spatial + lambda_t R_temporal                (Eq. (11))
  loss_i        = data term + lambda_TV R_4D-TV                           (Eq. (14))

Defaults follow Sec. IV-C: lambda_TV = 0.002, lambda_s = 1, lambda_t = 0.1;
eps (unstated) = 1e-8.
"""
import numpy as np

TV_LAMBDA = 0.002
TV_LAMBDA_S = 1.0
TV_LAMBDA_T = 0.1
TV_EPS = 1e-8


def forward_diffs(s):
    """(dz, dy, dx) of a 3-D array, 0 where the forward neighbour is outside."""
    dz = np.zeros_like(s)
    dy = np.zeros_like(s)
    dx = np.zeros_like(s)
    dz[:-1] = s[1:] - s[:-1]
    dy[:, :-1] = s[:, 1:] - s[:, :-1]
    dx[:, :, :-1] = s[:, :, 1:] - s[:, :, :-1]
    return dz, dy, dx


def spatial(s, eps=TV_EPS):
    """(R_spatial, dR/ds) for a 3-D image s."""
    V = s.size
    dz, dy, dx = forward_diffs(s)
    q = np.sqrt(dz * dz + dy * dy + dx * dx + eps)
    # each difference d(v) = s[v + e] - s[v] contributes d/q to v + e and -d/q to v
    g = -(dz + dy + dx) / q
    g[1:] += (dz / q)[:-1]
    g[:, 1:] += (dy / q)[:, :-1]
    g[:, :, 1:] += (dx / q)[:, :, :-1]
    return float(q.sum()) / V, g / V


def temporal_weights(i, prev_frames):
    """a_j = exp(-(i - j)) for the previous frames j (1-based), normalised."""
    a = np.array([np.exp(-(i - j)) for j in prev_frames])
    return a / a.sum()


def temporal(s, history, weights, eps=TV_EPS):
    """(R_temporal, dR/ds): history[k] is a previous image, weights[k] its
    normalised weight."""
    if len(history) == 0:
        return 0.0, np.zeros_like(s)
    R = 0.0
    g = np.zeros_like(s)
    for h, w in zip(history, weights):
        d = s - h
        q = np.sqrt(d * d + eps)
        R += w * float(q.sum())
        g += w * d / q
    return R, g


def tv4d(s, history, weights, lam=TV_LAMBDA, lam_s=TV_LAMBDA_S, lam_t=TV_LAMBDA_T, eps=TV_EPS):
    """(lambda_TV * R_4D-TV, its gradient) for a 3-D image s."""
    Rs, gs = spatial(s, eps)
    Rt, gt = temporal(s, history, weights, eps)
    return lam * (lam_s * Rs + lam_t * Rt), lam * (lam_s * gs + lam_t * gt)
