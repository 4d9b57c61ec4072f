"""Seeded synthetic inputs shared by the oracle's tests, the GPU tests and the bench.

This package only draws random numbers and lays out scenes (plane parameters,
pinhole cameras, trajectories).  It holds none of the splatting arithmetic:
no ray-plane intersection, no splat weight, no compositing, no loss.
"""

from .scenes import (  # noqa: F401
    Camera,
    PlaneSet,
    random_planes,
    perturb_planes,
    tiny_camera,
    scaled_camera,
    degenerate_planes,
    stacked_planes,
    room_planes,
    room_trajectory,
    room_init_planes,
    room_batch_specs,
    quat_from_matrix,
    quat_mul,
)
