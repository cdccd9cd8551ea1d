"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package renders images, ground-truth depth and surface normals of
piecewise-planar textured scenes along camera trajectories. It holds none of
the tracking method's arithmetic: no warp, residual, Jacobian or message rule
lives here, only ray casting and texture evaluation, so that both the CPU
oracle and the GPU path receive identical inputs from code neither of them
shares.
"""

from .scenes import (  # noqa: F401
    Camera,
    Plane,
    Scene,
    value_noise_texture,
    render,
    so3_exp,
    pose_from_motion,
    tiny_pair,
    make_sequence_scene,
    sequence_poses,
    render_sequence_frame,
    SequenceConfig,
    SEQUENCE_CONFIGS,
    batch_resolution,
)
from .noise import PPA_MILD, PPA_STRONG, SensorNoise, degrade, render_noisy_frame  # noqa: F401
