"""ctypes view of the C ABI declared in include/raysplats.h.

Argument marshalling only: every step of the rendering runs in librs.so.
Loading fails loudly when the library has not been built.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RS_LIBRARY", os.path.join(_HERE, "librs.so"))

RS_OK = 0
RS_ERR_INVALID_ARG = -1
RS_ERR_WORKSPACE = -2
RS_ERR_HIP = -3
RS_ERR_BVH_MISMATCH = -4
RS_ERR_STACK_OVERFLOW = -5
RS_ERR_NONFINITE = -6
RS_ERR_UNSUPPORTED = -7
RS_ERR_LIST_POOL = -8

RS_BRUTE_FORCE = 1 << 0
RS_PERSISTENT = 1 << 1
RS_ZERO_COLOUR = 1 << 2
RS_COUNTERS = 1 << 3
RS_PAPER_GRADIENT = 1 << 4
RS_BUILD_LBVH = 1 << 5
RS_MAX_BOUNCES = 3
RS_MAX_VIEWS = 64

# Every symbol include/raysplats.h declares.
EXPORTS = ("rs_default_params", "rs_bvh_workspace_bytes", "rs_ray_state_bytes", "rs_build_bvh", "rs_render_fwd",
           "rs_render_bwd", "rs_read_status", "rs_read_counters", "rs_status_string", "rs_bvh_download",
           "rs_default_shading", "rs_build_mesh_bvh", "rs_trace_mesh", "rs_mesh_frame_bytes", "rs_render_mesh_fwd",
           "rs_render_mesh_bwd", "rs_autotune", "rs_default_loss_params", "rs_loss_workspace_bytes", "rs_loss",
           "rs_hit_lists_download", "rs_mesh_hit_lists_download", "rs_loss_noalloc", "rs_loss_noalloc_max_bytes")
RS_TUNE_MAX = 32


class rs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p)]


class rs_view(C.Structure):
    _fields_ = [("ray_offset", C.c_int64), ("width", C.c_int32), ("height", C.c_int32)]


class rs_rays(C.Structure):
    _fields_ = [("n", C.c_int64), ("origin", C.c_void_p), ("dir", C.c_void_p), ("t_max", C.c_void_p),
                ("bg", C.c_void_p), ("n_views", C.c_int32), ("views", C.POINTER(rs_view))]


class rs_params(C.Structure):
    _fields_ = [("Q", C.c_float), ("eps1", C.c_float), ("t_min", C.c_float), ("max_hits", C.c_int32),
                ("bg", C.c_float * 3), ("flags", C.c_uint32), ("kbuf", C.c_int32), ("stack_depth", C.c_int32),
                ("tile_width", C.c_int32), ("hit_list", C.c_int32), ("eps2", C.c_float)]


class rs_grads(C.Structure):
    _fields_ = [("d_mean", C.c_void_p), ("d_scale", C.c_void_p), ("d_quat", C.c_void_p),
                ("d_opacity", C.c_void_p), ("d_rgb", C.c_void_p)]


class rs_bvh(C.Structure):
    _fields_ = [("opaque", C.c_uint64 * 16)]


class rs_mesh(C.Structure):
    _fields_ = [("n_verts", C.c_int64), ("n_tris", C.c_int64), ("verts", C.c_void_p), ("tris", C.c_void_p),
                ("material", C.c_void_p)]


class rs_shading(C.Structure):
    _fields_ = [("light", C.c_float * 3), ("intensity", C.c_float), ("albedo", C.c_float),
                ("mirror_reflectance", C.c_float), ("mirror_diffuse", C.c_float), ("offset", C.c_float),
                ("max_bounces", C.c_int32), ("ior", C.c_float)]


class rs_tune(C.Structure):
    _fields_ = [("fwd", rs_params), ("bwd", rs_params), ("n", C.c_int32), ("kbuf", C.c_int32 * RS_TUNE_MAX),
                ("persistent", C.c_int32 * RS_TUNE_MAX), ("tile_width", C.c_int32 * RS_TUNE_MAX),
                ("ms_fwd", C.c_float * RS_TUNE_MAX), ("ms_bwd", C.c_float * RS_TUNE_MAX)]


class rs_loss_params(C.Structure):
    _fields_ = [("lambda_", C.c_float), ("radius", C.c_int32), ("sigma", C.c_float)]


class RaySplatsError(RuntimeError):
    pass


_lib = None


def lib():
    """Load librs.so (built by paper_2501_19196_amd.build). Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RaySplatsError(f"{LIB_PATH} is missing: build the HIP library first "
                             "(python -m paper_2501_19196_amd.build)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.rs_default_params.argtypes = [C.POINTER(rs_params)]
    L.rs_default_params.restype = None
    L.rs_bvh_workspace_bytes.argtypes = [C.c_int64]
    L.rs_bvh_workspace_bytes.restype = C.c_size_t
    L.rs_ray_state_bytes.argtypes = [C.c_int64, C.POINTER(rs_params)]
    L.rs_ray_state_bytes.restype = C.c_size_t
    L.rs_build_bvh.argtypes = [C.POINTER(rs_gaussians), C.POINTER(rs_params), P, C.c_size_t, C.POINTER(rs_bvh), P]
    L.rs_build_bvh.restype = C.c_int
    L.rs_render_fwd.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_gaussians), C.POINTER(rs_rays), C.POINTER(rs_params),
                                P, P, P]
    L.rs_render_fwd.restype = C.c_int
    L.rs_render_bwd.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_gaussians), C.POINTER(rs_rays), C.POINTER(rs_params),
                                P, P, C.POINTER(rs_grads), P]
    L.rs_render_bwd.restype = C.c_int
    L.rs_read_status.argtypes = [C.POINTER(rs_bvh), P]
    L.rs_read_status.restype = C.c_int
    L.rs_read_counters.argtypes = [C.POINTER(rs_bvh), P, P]
    L.rs_read_counters.restype = C.c_int
    L.rs_status_string.argtypes = [C.c_int]
    L.rs_status_string.restype = C.c_char_p
    L.rs_bvh_download.argtypes = [C.POINTER(rs_bvh), P, P, P, P, P, P, P]
    L.rs_bvh_download.restype = C.c_int
    L.rs_hit_lists_download.argtypes = [C.POINTER(rs_rays), C.POINTER(rs_params), P, P, C.c_int64, P, P, P, P,
                                        C.c_int32, P]
    L.rs_hit_lists_download.restype = C.c_int
    L.rs_mesh_hit_lists_download.argtypes = [C.POINTER(rs_rays), C.POINTER(rs_params), C.POINTER(rs_shading), P,
                                             C.c_int32, P, C.c_int64, P, P, P, C.c_int32, P]
    L.rs_mesh_hit_lists_download.restype = C.c_int
    L.rs_default_shading.argtypes = [C.POINTER(rs_shading)]
    L.rs_default_shading.restype = None
    L.rs_build_mesh_bvh.argtypes = [C.POINTER(rs_mesh), P, C.c_size_t, C.POINTER(rs_bvh), P]
    L.rs_build_mesh_bvh.restype = C.c_int
    L.rs_trace_mesh.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_rays), P, C.c_int, P, P, P]
    L.rs_trace_mesh.restype = C.c_int
    L.rs_mesh_frame_bytes.argtypes = [C.c_int64, C.POINTER(rs_params), C.POINTER(rs_shading)]
    L.rs_mesh_frame_bytes.restype = C.c_size_t
    L.rs_render_mesh_fwd.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_bvh), C.POINTER(rs_gaussians), C.POINTER(rs_mesh),
                                     C.POINTER(rs_shading), C.POINTER(rs_rays), C.POINTER(rs_params), P, P, P]
    L.rs_render_mesh_fwd.restype = C.c_int
    L.rs_render_mesh_bwd.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_bvh), C.POINTER(rs_gaussians), C.POINTER(rs_mesh),
                                     C.POINTER(rs_shading), C.POINTER(rs_rays), C.POINTER(rs_params), P, P,
                                     C.POINTER(rs_grads), P]
    L.rs_render_mesh_bwd.restype = C.c_int
    L.rs_autotune.argtypes = [C.POINTER(rs_bvh), C.POINTER(rs_gaussians), C.POINTER(rs_rays), C.POINTER(rs_params), P,
                              P, P, C.POINTER(rs_grads), C.c_int, C.POINTER(rs_tune), P]
    L.rs_autotune.restype = C.c_int
    L.rs_default_loss_params.argtypes = [C.POINTER(rs_loss_params)]
    L.rs_default_loss_params.restype = None
    L.rs_loss_workspace_bytes.argtypes = [C.c_int32, C.c_int32]
    L.rs_loss_workspace_bytes.restype = C.c_size_t
    L.rs_loss.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(rs_loss_params), P, P, P, P]
    L.rs_loss.restype = C.c_int
    L.rs_loss_noalloc.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(rs_loss_params), P, P, P]
    L.rs_loss_noalloc.restype = C.c_int
    L.rs_loss_noalloc_max_bytes.argtypes = []
    L.rs_loss_noalloc_max_bytes.restype = C.c_size_t
    _lib = L
    return L


def check(code, what):
    if code != RS_OK:
        msg = lib().rs_status_string(code).decode()
        raise RaySplatsError(f"{what} failed: {msg} ({code})")
    return code
