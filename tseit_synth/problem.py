"""Seeded synthetic problems: lungs, voltages, noise input Z and theta_0.

Recipes (synthetic stand-ins for the paper's data, Sec. IV-A):

* Lungs: two ellipsoids centred at (+-0.42, 0, 0) with semi-axes
  (0.28, 0.45, 0.60); the conductivity change is the amplitude inside them and
  0 elsewhere.  Single frames use amplitude -0.3; the time sequence uses
  a_t = -0.3 * (0.5 + 0.5 * sin(2*pi*t/25)), t = 0 .. T-1.
* Voltages: dv_t = J sigma_t + eta_t, with eta_t i.i.d. N(0, (0.01*RMS(J sigma_t))^2)
  drawn fresh per frame (1% noise).
* Noise input Z: N(0, 1), one channel, n^3 voxels, fixed for a sequence.  The
  paper draws Z from U(0, 1) (Eq. (3)); ``z_dist="uniform"`` gives that variant.
* theta_0: Kaiming (fan-in, ReLU gain) as the paper initialises its network
  (Sec. III-B): conv weights N(0, 2/(Cin*k^3)), biases 0, norm gains 1 and
  shifts 0.
* Seeds: numpy SeedSequence([seed, stream]) with PCG64; stream 0 draws
  theta_0, stream 1 draws Z, stream (2, t) draws the noise of frame t.

All arrays handed to the GPU are FP32-representable (``fp32=True``), so the
FP64 oracle sees exactly the same numbers after promotion.
"""
import functools
import math

import numpy as np

from .geometry import sensitivity_matrix, voxel_centres, cylinder_mask
from .layout import param_specs

LUNG_CENTRES = ((-0.42, 0.0, 0.0), (0.42, 0.0, 0.0))
LUNG_SEMI_AXES = (0.28, 0.45, 0.60)
LUNG_VALUE = -0.3
NOISE_FRACTION = 0.01
BREATH_PERIOD = 25.0


def _cfg(name, n, rings, levels, base_ch, iters, lr=1e-3, seed=0, frames=1,
         later_iters=0, sequences=1, seeds=None, breathing=False, desc=""):
    return dict(name=name, n=n, rings=rings, levels=levels, base_ch=base_ch,
                iters=iters, later_iters=later_iters, lr=lr, seed=seed,
                frames=frames, sequences=sequences,
                seeds=list(seeds) if seeds is not None else [seed],
                breathing=breathing, desc=desc)


def instance_mix(i):
    """Instance i of the uneven batch: grid, rings and base channels."""
    return (24, 32, 48)[i % 3], (1, 2)[(i // 3) % 2], (8, 16)[(i // 6) % 2]


CONFIGS = {
    "c0": _cfg("c0", 16, 1, 2, 8, 50, seed=0,
               desc="16^3 grid, 16 electrodes (208 meas), 2 levels, C=8, 50 Adam iters"),
    "c1": _cfg("c1", 32, 2, 3, 16, 500, seed=1,
               desc="32^3 grid, 32 electrodes (928 meas), 3 levels, C=16, 500 Adam iters"),
    "c2": _cfg("c2", 64, 2, 4, 32, 1000, seed=2,
               desc="64^3 grid, 32 electrodes (928 meas), 4 levels, C=32, 1000 Adam iters"),
    "c3": _cfg("c3", 32, 2, 3, 16, 500, later_iters=50, frames=100, sequences=8,
               seeds=range(300, 308), breathing=True,
               desc="8 sequences x 100 frames at 32^3, 500 then 50 iters/frame (TPP)"),
    "c4": dict(name="c4", iters=200, lr=1e-3, levels=3,
               instances=[dict(zip(("n", "rings", "base_ch"), instance_mix(i)),
                               seed=400 + i) for i in range(16)],
               desc="16 uneven single-frame instances (24/32/48^3, 208/928 meas, C 8/16), 200 iters"),
}


@functools.lru_cache(maxsize=4)
def _geometry64(n, rings):
    J, mask = sensitivity_matrix(n, rings, np.float64)
    J.setflags(write=False)
    mask.setflags(write=False)
    return J, mask


def make_geometry(n, rings, fp32=True):
    """(J, mask): J FP32 (or FP64 when fp32=False), mask uint8."""
    J64, mask = _geometry64(n, rings)
    if fp32:
        return J64.astype(np.float32), mask.copy()
    return J64.copy(), mask.copy()


def lung_mask(n):
    p = voxel_centres(n)
    inside = np.zeros(p.shape[0], dtype=bool)
    for c in LUNG_CENTRES:
        r2 = sum(((p[:, k] - c[k]) / LUNG_SEMI_AXES[k]) ** 2 for k in range(3))
        inside |= r2 <= 1.0
    return inside & cylinder_mask(n).astype(bool)


def breathing_amplitude(t):
    return LUNG_VALUE * (0.5 + 0.5 * math.sin(2.0 * math.pi * t / BREATH_PERIOD))


def true_sigma(n, amplitude=LUNG_VALUE):
    return np.where(lung_mask(n), amplitude, 0.0)


def _rng(seed, *stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *stream])))


def noise_input(n, seed, fp32=True, z_dist="normal"):
    g = _rng(seed, 1)
    if z_dist == "normal":
        z = g.standard_normal(n ** 3)
    elif z_dist == "uniform":
        z = g.random(n ** 3)
    else:
        raise ValueError(z_dist)
    return z.astype(np.float32) if fp32 else z


def kaiming_theta(levels, base_ch, seed, fp32=True):
    g = _rng(seed, 0)
    parts = []
    for _, shape, kind in param_specs(levels, base_ch):
        size = int(np.prod(shape))
        if kind == "w":
            fan_in = int(np.prod(shape[1:]))
            parts.append(g.standard_normal(size) * math.sqrt(2.0 / fan_in))
        elif kind == "g":
            parts.append(np.ones(size))
        else:
            parts.append(np.zeros(size))
    th = np.concatenate(parts)
    return th.astype(np.float32) if fp32 else th


def frame_voltages(J64, sigma, seed, frame):
    """dv = J sigma + 1% Gaussian noise (FP64)."""
    clean = J64 @ sigma
    rms = math.sqrt(float(np.mean(clean ** 2)))
    eta = _rng(seed, 2, frame).standard_normal(clean.shape[0]) * (NOISE_FRACTION * rms)
    return clean + eta


def make_problem(n, rings, levels, base_ch, seed, frames=1, breathing=False,
                 fp32=True, z_dist="normal"):
    """One instance: dict with J, mask, Z, theta0, dv (frames x M), sigma_true."""
    J64, mask = _geometry64(n, rings)
    sig = []
    dv = []
    for t in range(frames):
        amp = breathing_amplitude(t) if breathing else LUNG_VALUE
        s = true_sigma(n, amp)
        sig.append(s)
        dv.append(frame_voltages(J64, s, seed, t))
    ft = np.float32 if fp32 else np.float64
    return dict(
        n=n, rings=rings, levels=levels, base_ch=base_ch, seed=seed,
        J=J64.astype(ft), mask=mask.copy(),
        Z=noise_input(n, seed, fp32, z_dist),
        theta0=kaiming_theta(levels, base_ch, seed, fp32),
        dv=np.stack(dv).astype(ft), sigma_true=np.stack(sig),
    )
