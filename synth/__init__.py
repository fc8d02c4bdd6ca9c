"""Seeded synthetic workloads and initial parameters.

This module is shared by the tests, the benchmark and the smoke check. It
builds inputs only: reference meshes with normals, per-frame target point
clouds, hyper-parameter sets and initial parameter values. It contains none
of the method's arithmetic (no grid lookup, decoder, loss, gradient,
preconditioner or optimizer code), so the CPU oracle and the HIP path stay
independent of each other and of this file.

The workloads stand in for the paper's datasets (DFAUST, AMA, DT4D), which
are not available: sizes follow the paper's scales (17-1000 frames, 2k-20k
points per frame, sensor noise well inside the stable range of the noise
ablation, Table 8).
"""
from .configs import config_c1, config_c2, config_c3, config_c5, config_small, config_by_name  # noqa: F401
from .meshes import icosphere, capsule_figure  # noqa: F401
from .workloads import make_workload, init_params, random_state  # noqa: F401
