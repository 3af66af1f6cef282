"""Seeded synthetic tsEIT problems (inputs only).

This package draws every input that the fitting iteration consumes: the
sensitivity matrix J and voxel mask of a cylinder geometry, a ground-truth
conductivity change, the measured voltage differences, the fixed noise input Z
and the Kaiming-initialised network parameters theta_0.  It holds none of the
method's arithmetic (no network, no loss, no optimiser): both the FP64 oracle
and the GPU library receive the same arrays from here.

The paper's data (COMSOL thorax simulation, clinical recordings; Sec. IV-A/B)
is not available, so the recipes below stand in for it: a 16- or 32-electrode
cylinder with adjacent drive/measure pairs (the paper's 32 electrodes in two
layers, Sec. IV-A), two ellipsoidal lung inclusions whose amplitude varies
sinusoidally over the frames (the paper's sinusoidal lung volume, Sec. IV-A)
and 1% Gaussian measurement noise.
"""
from .geometry import (electrode_positions, drive_measure_pairs, voxel_centres,
                       cylinder_mask, sensitivity_matrix)
from .layout import param_specs, param_count
from .problem import (CONFIGS, make_geometry, lung_mask, true_sigma,
                      noise_input, kaiming_theta, frame_voltages, make_problem,
                      instance_mix)

__all__ = [
    "electrode_positions", "drive_measure_pairs", "voxel_centres",
    "cylinder_mask", "sensitivity_matrix", "param_specs", "param_count",
    "CONFIGS", "make_geometry", "lung_mask", "true_sigma", "noise_input",
    "kaiming_theta", "frame_voltages", "make_problem", "instance_mix",
]
