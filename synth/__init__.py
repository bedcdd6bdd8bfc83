"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package draws inputs only: surfel arrays, cameras and poses.  It holds none
of the rasterizer's arithmetic (no projection, blending, loss or Lie-group map),
so that the FP64 oracle and the HIP path can both consume its arrays without
sharing any code with each other.
"""

from .scenes import (  # noqa: F401
    Camera,
    SurfelSet,
    random_surfels,
    single_surfel,
    stacked_surfels,
    planar_carpet,
    Room,
    make_room,
    room_camera,
    perturb_pose,
    pose_error,
    look_at_pose,
    tiny_scene,
    PARAM_ROWS,
)
