"""Seeded synthetic scenes and camera rigs shared by the GPU path, its tests and the oracle.

This package draws random numbers and lays them out; it contains none of the
training method's arithmetic (no projection, compositing, loss or solve).
"""
from .scenes import (  # noqa: F401
    Gaussians, Camera, CONFIGS, make_config, perturb, fibonacci_cameras,
    look_at_camera, pinhole_intrinsics, sh_coeffs_per_channel, Y00,
)
