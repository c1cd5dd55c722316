"""Seeded synthetic scenes and cameras for the Gaussian-splatting hot path.

This package creates inputs only: Gaussian parameters, pinhole cameras and
camera trajectories drawn from fixed seeds.  It holds none of the method's
arithmetic (no projection, no compositing, no gradients), so both the FP64
CPU oracle and the GPU path can take their inputs from it without sharing any
computation.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    random_scene,
    surface_scene,
    jitter_means,
    look_camera,
    camera_from_pose,
    trajectory_cameras,
    lidar_stream,
    with_sh,
    perturb_camera,
    so3_exp,
    config1,
    config2,
    config3,
    config4,
    config5,
    CONFIG_NAMES,
)
