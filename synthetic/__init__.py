"""Seeded synthetic inputs for the ray-traced Gaussian renderer.

This package only draws inputs: Gaussian scenes, pinhole-camera rays and a
triangle mesh. It holds none of the rendering arithmetic, so both the FP64
oracle and the HIP path can be fed from it without sharing any method code.
"""

from .scenes import (  # noqa: F401
    Scene,
    scene_config1,
    scene_config2,
    scene_config3,
    scene_config4,
    scene_config5,
    random_scene,
)
from .cameras import Camera, pinhole_rays, look_at_camera, fibonacci_cameras, circle_cameras  # noqa: F401
from .mesh import Mesh, mirror_mesh  # noqa: F401
from .workloads import WORKLOADS, workload  # noqa: F401
