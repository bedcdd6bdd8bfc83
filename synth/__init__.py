"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package draws inputs only: surfel arrays, cameras, poses, and the warm-start
network's initial weights, inputs and twists.  It holds none
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
from .nets import (  # noqa: F401
    LAYER_SHAPES,
    exact_inputs,
    exact_params,
    exact_targets,
    init_params,
    random_inputs,
    random_twists,
)
