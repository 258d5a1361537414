"""MI355X-native ray-traced Gaussian renderer (RaySplats, arXiv 2501.19196).

The hot path (BVH build, ray / confidence-ellipsoid traversal, depth-ordered
compositing and its adjoint) runs as hand-written HIP kernels for gfx950 in
librs.so behind the C ABI of include/raysplats.h; this package marshals torch
tensors into that ABI.
"""

from ._lib import RaySplatsError, LIB_PATH  # noqa: F401


def __getattr__(name):
    # the torch-facing wrappers load lazily so that `build` can run without a GPU
    if name in ("render", "Params", "Gaussians", "Rays", "build_bvh", "render_fwd", "render_bwd", "read_status",
                "download", "RaySplatsRender", "BVH", "workspace_bytes"):
        from . import renderer as _r
        return getattr(_r, name)
    raise AttributeError(name)
