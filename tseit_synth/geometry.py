"""Cylinder geometry, electrode layout and the synthetic sensitivity matrix J.

Reading of the paper (its J is FEM-derived, normalised and projected; Eq. (1),
Sec. II) for synthetic problems:

* Domain: the cube [-1, 1]^3 split into n^3 voxels; voxel centres at
  -1 + (2i + 1)/n along each axis.  Voxel flattening (the reshape operator V of
  Eq. (3)) is z-major, x fastest: q = (z*n + y)*n + x.
* The imaging region is the unit cylinder with axis z: a voxel is inside iff
  its centre has x^2 + y^2 <= 1.  Columns of J outside it are zero.
* Electrodes: 16 per ring at radius 1, angle 2*pi*k/16.  One ring at z = 0, or
  two aligned rings at z = -0.5 and z = +0.5 (the paper's 32 electrodes in two
  layers, Sec. IV-A).
* Adjacent protocol: drive pairs (k, k+1 mod 16) inside each ring; the measure
  pairs are the same set of adjacent pairs (over all rings) minus every pair
  sharing an electrode with the drive pair.  This gives 16*13 = 208 rows for
  one ring and 32*29 = 928 rows for two rings; rows are ordered drive-major,
  then by measure pair.
* Row of J for drive (a, b) and measure (m, n): G_a - G_b + G_m - G_n with
  G_e(x) = exp(-|x - e|^2 / (2 * 0.2^2)), masked, then scaled to unit L2 norm.
"""
import numpy as np

ELECTRODES_PER_RING = 16
GAUSS_WIDTH = 0.2


def electrode_positions(rings):
    """(rings*16, 3) electrode centres; electrode index = ring*16 + k."""
    if rings == 1:
        zs = [0.0]
    elif rings == 2:
        zs = [-0.5, 0.5]
    else:
        raise ValueError("rings must be 1 or 2")
    k = np.arange(ELECTRODES_PER_RING)
    ang = 2.0 * np.pi * k / ELECTRODES_PER_RING
    pos = []
    for z in zs:
        pos.append(np.stack([np.cos(ang), np.sin(ang), np.full_like(ang, z)], axis=1))
    return np.concatenate(pos, axis=0)


def drive_measure_pairs(rings):
    """List of ((a, b), (m, n)) electrode-index pairs, drive-major."""
    E = ELECTRODES_PER_RING
    adjacent = [(r * E + k, r * E + (k + 1) % E) for r in range(rings) for k in range(E)]
    rows = []
    for d in adjacent:
        for m in adjacent:
            if set(d) & set(m):
                continue
            rows.append((d, m))
    return rows


def voxel_centres(n):
    """(n^3, 3) array of (x, y, z) voxel centres in flattening order."""
    c = -1.0 + (2.0 * np.arange(n) + 1.0) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def cylinder_mask(n):
    """uint8 (n^3,) indicator of voxels whose centre lies in the unit cylinder."""
    p = voxel_centres(n)
    return (p[:, 0] ** 2 + p[:, 1] ** 2 <= 1.0).astype(np.uint8)


def sensitivity_matrix(n, rings, dtype=np.float64):
    """Synthetic J (M x n^3, row-major) and the voxel mask, generated in FP64."""
    pts = voxel_centres(n)
    mask = cylinder_mask(n)
    el = electrode_positions(rings)
    d2 = ((pts[None, :, :] - el[:, None, :]) ** 2).sum(axis=2)      # (E, Q)
    G = np.exp(-d2 / (2.0 * GAUSS_WIDTH ** 2))
    G *= mask[None, :]
    pairs = drive_measure_pairs(rings)
    J = np.empty((len(pairs), n ** 3), dtype=np.float64)
    for i, ((a, b), (m, nn)) in enumerate(pairs):
        row = G[a] - G[b] + G[m] - G[nn]
        J[i] = row / np.linalg.norm(row)
    return J.astype(dtype, copy=False), mask
