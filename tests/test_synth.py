"""Pins of the synthetic problem generator (geometry, J, lungs, noise, theta_0)."""
import math

import numpy as np
import pytest

import tseit_synth as ts
from tseit_synth.geometry import drive_measure_pairs


@pytest.mark.parametrize("rings,M", [(1, 208), (2, 928)])
def test_measurement_counts(rings, M):
    assert len(drive_measure_pairs(rings)) == M
    J, mask = ts.sensitivity_matrix(8, rings)
    assert J.shape == (M, 512)


@pytest.mark.parametrize("n,active", [(16, 3328), (32, 25984), (64, 206592)])
def test_mask_counts(n, active):
    assert int(ts.cylinder_mask(n).sum()) == active


def test_rows_unit_norm_and_masked_columns_zero():
    J, mask = ts.sensitivity_matrix(16, 2)
    assert np.abs(np.linalg.norm(J, axis=1) - 1.0).max() < 1e-12
    assert np.all(J[:, mask == 0] == 0.0)


def test_reciprocity():
    # the row of drive d / measure m equals the row of drive m / measure d
    pairs = drive_measure_pairs(2)
    J, _ = ts.sensitivity_matrix(8, 2)
    idx = {p: i for i, p in enumerate(pairs)}
    checked = 0
    for (d, m), i in idx.items():
        j = idx.get((m, d))
        if j is not None:
            np.testing.assert_allclose(J[i], J[j], rtol=0, atol=1e-15)
            checked += 1
    assert checked == len(pairs)


def test_row_against_direct_formula():
    # one row recomputed from the Gaussian recipe at one voxel
    n = 8
    J, mask = ts.sensitivity_matrix(n, 1)
    (a, b), (m, k) = drive_measure_pairs(1)[5]
    el = ts.electrode_positions(1)
    pts = ts.voxel_centres(n)
    G = lambda e: np.exp(-((pts - el[e]) ** 2).sum(1) / (2 * 0.2 ** 2))
    row = (G(a) - G(b) + G(m) - G(k)) * mask
    np.testing.assert_allclose(J[5], row / np.linalg.norm(row), rtol=1e-13, atol=1e-16)


def test_flatten_order():
    p = ts.voxel_centres(4)
    # x fastest, then y, then z
    assert p[1, 0] > p[0, 0] and p[1, 1] == p[0, 1] and p[1, 2] == p[0, 2]
    assert p[4, 1] > p[0, 1] and p[16, 2] > p[0, 2]


def test_noise_level_and_determinism():
    J, _ = ts.make_geometry(16, 1, fp32=False)
    s = ts.true_sigma(16)
    clean = J @ s
    dvs = np.stack([ts.frame_voltages(J, s, 7, t) for t in range(200)])
    rel = np.sqrt(((dvs - clean) ** 2).mean()) / np.sqrt((clean ** 2).mean())
    assert abs(rel - 0.01) < 0.0005
    np.testing.assert_array_equal(ts.frame_voltages(J, s, 7, 3), dvs[3])
    assert not np.array_equal(dvs[3], dvs[4])


def test_kaiming_variance_and_determinism():
    th = ts.kaiming_theta(3, 16, 1, fp32=False)
    off = 0
    for name, shape, kind in ts.param_specs(3, 16):
        k = int(np.prod(shape))
        seg = th[off:off + k]
        off += k
        if kind == "w" and k > 4000:
            fan_in = int(np.prod(shape[1:]))
            assert abs(seg.var() / (2.0 / fan_in) - 1.0) < 0.1, name
        elif kind == "g":
            assert np.all(seg == 1.0)
        elif kind in ("b", "beta"):
            assert np.all(seg == 0.0)
    assert off == th.size == 367425
    np.testing.assert_array_equal(th, ts.kaiming_theta(3, 16, 1, fp32=False))


def test_noise_input_moments():
    z = ts.noise_input(32, 5, fp32=False)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02
    u = ts.noise_input(32, 5, fp32=False, z_dist="uniform")
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def test_breathing_amplitude():
    assert ts.problem.breathing_amplitude(0) == pytest.approx(-0.15)
    assert ts.problem.breathing_amplitude(6.25) == pytest.approx(-0.3)
    assert abs(ts.problem.breathing_amplitude(18.75)) < 1e-15


def test_fp32_inputs_are_representable():
    p = ts.make_problem(16, 1, 2, 8, 0)
    for k in ("J", "Z", "theta0", "dv"):
        assert p[k].dtype == np.float32


def test_instance_mix_covers_all_combinations():
    combos = {ts.instance_mix(i) for i in range(12)}
    assert len(combos) == 12
    assert [ts.instance_mix(i) for i in range(12, 16)] == [ts.instance_mix(i) for i in range(4)]


def test_param_counts():
    assert ts.param_count(2, 8) == 21521
    assert ts.param_count(3, 16) == 367425
    assert ts.param_count(4, 32) == 5974785
    assert ts.param_count(3, 8) == 92257
