"""Torch-facing wrappers of the C ABI: device memory and streams come from
torch, every computation runs in librs.so. Also the autograd Function.

Names follow the paper: Q (ellipsoid quantile, Sec. 3), eps1 (transmittance
threshold) and max_hits (K_max, the per-ray hit cap, Sec. 3 "Color
Aggregation").
"""

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


@dataclass
class Params:
    Q: float = 11.3449
    eps1: float = 1e-4
    t_min: float = 0.0
    max_hits: int = 512
    bg: tuple = (0.0, 0.0, 0.0)
    flags: int = 0
    kbuf: int = 0
    stack_depth: int = 0
    tile_width: int = 0
    hit_list: int = 0
    eps2: float = 1e-4
    # wrapper-side only: the autograd Functions read the sticky device status
    # after each call (a stream synchronisation) and raise on a device error
    raise_on_status: bool = False

    def c(self):
        p = L.rs_params()
        p.Q, p.eps1, p.t_min, p.max_hits = float(self.Q), float(self.eps1), float(self.t_min), int(self.max_hits)
        for k in range(3):
            p.bg[k] = float(self.bg[k])
        p.flags = int(self.flags)
        p.kbuf = int(self.kbuf)
        p.stack_depth = int(self.stack_depth)
        p.tile_width = int(self.tile_width)
        p.hit_list = int(self.hit_list)
        p.eps2 = float(self.eps2)
        return p


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class Gaussians:
    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    rgb: torch.Tensor

    def c(self):
        n = self.mean.shape[0]
        for name in ("mean", "scale", "quat", "opacity", "rgb"):
            _dev(getattr(self, name), name)
        if self.mean.shape != (n, 3) or self.scale.shape != (n, 3) or self.quat.shape != (n, 4) or \
                self.opacity.shape != (n,) or self.rgb.shape != (n, 3):
            raise ValueError("gaussian arrays must be mean[n,3], scale[n,3], quat[n,4], opacity[n], rgb[n,3]")
        return L.rs_gaussians(n, _ptr(self.mean), _ptr(self.scale), _ptr(self.quat), _ptr(self.opacity),
                              _ptr(self.rgb))

    @property
    def n(self):
        return int(self.mean.shape[0])


@dataclass
class Rays:
    origin: torch.Tensor
    direction: torch.Tensor
    t_max: torch.Tensor = None
    bg: torch.Tensor = None
    views: list = field(default_factory=list)  # [(ray_offset, width, height)]

    def c(self):
        n = self.origin.shape[0]
        _dev(self.origin, "origin")
        _dev(self.direction, "direction")
        if self.origin.shape != (n, 3) or self.direction.shape != (n, 3):
            raise ValueError("rays must be origin[n,3], direction[n,3]")
        if self.t_max is not None:
            _dev(self.t_max, "t_max")
        if self.bg is not None:
            _dev(self.bg, "bg")
        nv = len(self.views)
        self._views = (L.rs_view * max(nv, 1))()
        for i, (off, w, h) in enumerate(self.views):
            self._views[i].ray_offset, self._views[i].width, self._views[i].height = int(off), int(w), int(h)
        return L.rs_rays(n, _ptr(self.origin), _ptr(self.direction), _ptr(self.t_max), _ptr(self.bg), nv,
                         C.cast(self._views, C.POINTER(L.rs_view)))

    @property
    def n(self):
        return int(self.origin.shape[0])


class BVH:
    """A built BVH: the caller-owned workspace tensor plus its descriptor."""

    def __init__(self, n, Q, workspace, desc):
        self.n, self.Q, self.workspace, self.desc = n, Q, workspace, desc


def state_bytes(n, params=None):
    pc = params.c() if params is not None else None
    return int(L.lib().rs_ray_state_bytes(int(n), C.byref(pc) if pc is not None else None))


def new_state(n, params, device="cuda"):
    """Ray state for render_fwd / render_bwd: a flat float32 buffer of
    rs_ray_state_bytes(n, params) bytes whose first 4 n floats are the final
    colour and transmittance of each ray (see state_colour)."""
    return torch.empty(max((state_bytes(n, params) + 3) // 4, 64), dtype=torch.float32, device=device)


def state_colour(state, n):
    """The [n, 4] (final colour, final transmittance) part of a ray state."""
    return state.reshape(-1)[:4 * n].view(n, 4)


def _check_state(state, n, params):
    """The C ABI takes the ray state without a size: check it here."""
    if state is None:
        return None
    state = _dev(state, "state") if state.dtype == torch.float32 else _dev(state, "state", state.dtype)
    need = state_bytes(n, params)
    have = state.numel() * state.element_size()
    if have < need:
        raise ValueError(f"ray state holds {have} bytes, rs_ray_state_bytes({n}, params) needs {need}")
    return state


def workspace_bytes(n):
    return int(L.lib().rs_bvh_workspace_bytes(int(n)))


def build_bvh(g: Gaussians, params: Params, workspace=None):
    lib = L.lib()
    nbytes = workspace_bytes(g.n)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=g.mean.device)
    desc = L.rs_bvh()
    gc, pc = g.c(), params.c()
    L.check(lib.rs_build_bvh(C.byref(gc), C.byref(pc), _ptr(workspace), C.c_size_t(workspace.numel()),
                             C.byref(desc), _stream()), "rs_build_bvh")
    return BVH(g.n, params.Q, workspace, desc)


def render_fwd(bvh: BVH, g: Gaussians, rays: Rays, params: Params, out=None, state=None, want_state=True):
    lib = L.lib()
    n = rays.n
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=rays.origin.device)
    if want_state and state is None:
        state = new_state(n, params, rays.origin.device)
    state = _check_state(state, n, params)
    gc, rc, pc = g.c(), rays.c(), params.c()
    L.check(lib.rs_render_fwd(C.byref(bvh.desc), C.byref(gc), C.byref(rc), C.byref(pc), _ptr(out), _ptr(state),
                              _stream()), "rs_render_fwd")
    return out, state


def render_bwd(bvh: BVH, g: Gaussians, rays: Rays, params: Params, grad_rgb, state, grads=None):
    lib = L.lib()
    grad_rgb = _dev(grad_rgb.contiguous(), "grad_rgb")
    if grad_rgb.numel() != 3 * rays.n:
        raise ValueError("grad_rgb must hold [n_rays, 3] values")
    if state is None:
        raise ValueError("render_bwd needs the ray state of the forward call")
    state = _check_state(state, rays.n, params)
    if grads is None:
        grads = (torch.empty_like(g.mean), torch.empty_like(g.scale), torch.empty_like(g.quat),
                 torch.empty_like(g.opacity), torch.empty_like(g.rgb))
    gr = L.rs_grads(*[_ptr(t) for t in grads])
    gc, rc, pc = g.c(), rays.c(), params.c()
    L.check(lib.rs_render_bwd(C.byref(bvh.desc), C.byref(gc), C.byref(rc), C.byref(pc), _ptr(grad_rgb),
                              _ptr(state), C.byref(gr), _stream()), "rs_render_bwd")
    return grads


def _params_from_c(cp, like):
    return Params(Q=like.Q, eps1=like.eps1, t_min=like.t_min, max_hits=like.max_hits, bg=tuple(like.bg),
                  flags=int(cp.flags), kbuf=int(cp.kbuf), stack_depth=int(cp.stack_depth),
                  tile_width=int(cp.tile_width), hit_list=int(cp.hit_list), eps2=like.eps2,
                  raise_on_status=like.raise_on_status)


def autotune(bvh: BVH, g: Gaussians, rays: Rays, params: Params, grad_rgb=None, reps=2):
    """Time the launch shapes (rs_autotune) on these inputs. Returns
    (fastest forward Params, fastest adjoint Params, rows of timings)."""
    n = rays.n
    dev = rays.origin.device
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    state = new_state(n, params, dev)
    gr = None
    keep = None
    if grad_rgb is not None:
        grad_rgb = _dev(grad_rgb.contiguous(), "grad_rgb")
        keep = (torch.empty_like(g.mean), torch.empty_like(g.scale), torch.empty_like(g.quat),
                torch.empty_like(g.opacity), torch.empty_like(g.rgb))
        gr = L.rs_grads(*[_ptr(t) for t in keep])
    res = L.rs_tune()
    gc, rc, pc = g.c(), rays.c(), params.c()
    L.check(L.lib().rs_autotune(C.byref(bvh.desc), C.byref(gc), C.byref(rc), C.byref(pc), _ptr(grad_rgb), _ptr(out),
                                _ptr(state), C.byref(gr) if gr is not None else None, int(reps), C.byref(res),
                                _stream()), "rs_autotune")
    rows = [dict(kbuf=res.kbuf[k], persistent=bool(res.persistent[k]), tile_width=res.tile_width[k],
                 ms_fwd=float(res.ms_fwd[k]), ms_bwd=float(res.ms_bwd[k])) for k in range(res.n)]
    return _params_from_c(res.fwd, params), _params_from_c(res.bwd, params), rows


def read_status(bvh: BVH):
    return int(L.lib().rs_read_status(C.byref(bvh.desc), _stream()))


def raise_on_status(bvh: BVH, what):
    """Synchronise and raise if a device-side check failed since the build."""
    code = read_status(bvh)
    if code != L.RS_OK:
        raise L.RaySplatsError(f"{what}: device status {L.lib().rs_status_string(code).decode()} ({code})")


COUNTER_NAMES = ("packets", "node_visits", "leaf_visits", "rounds", "lane_leaf_tests", "lane_hits_buffered",
                 "lane_composited", "lane_child_overlaps", "grad_groups", "list_packets", "list_composited",
                 "list_grad_groups", "list_rows", "adjoint_packets", "list_slots", "c15")


def read_counters(bvh: BVH):
    out = np.zeros(16, np.uint64)
    L.check(L.lib().rs_read_counters(C.byref(bvh.desc), out.ctypes.data_as(C.c_void_p), _stream()),
            "rs_read_counters")
    return dict(zip(COUNTER_NAMES, (int(x) for x in out)))


def _lists_out(m, cap):
    return (np.zeros(max(m, 1), np.int32), np.zeros(max(m, 1), np.int32), np.zeros(max(m, 1), np.int32),
            np.zeros((max(m, 1), cap), np.int32))


def hit_lists(rays: Rays, params: Params, state, cap=None, select=None):
    """Host copies of the stored hit lists of a ray state (rs_hit_lists_download),
    for every ray or for the ray indices in `select`: dict(count, stored, extra,
    ids[m, cap] with -1 padding)."""
    cap = int(cap or max(params.max_hits, 1))
    sel = None if select is None else np.ascontiguousarray(select, np.int64)
    m = rays.n if sel is None else len(sel)
    count, stored, extra, ids = _lists_out(m, cap)
    rc, pc = rays.c(), params.c()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    L.check(L.lib().rs_hit_lists_download(C.byref(rc), C.byref(pc), _ptr(state), None if sel is None else p(sel),
                                          m, p(count), p(stored), p(extra), p(ids), cap, _stream()),
            "rs_hit_lists_download")
    return dict(count=count[:m], stored=stored[:m], extra=extra[:m], ids=ids[:m])


def mesh_hit_lists(rays: Rays, params: Params, shading, frame, ray_set, cap=None, select=None):
    """Stored hit lists of ray set `ray_set` of a mesh frame (rs_mesh_hit_lists_download):
    0..B path levels, B+1..2B shadow levels."""
    cap = int(cap or max(params.max_hits, 1))
    sel = None if select is None else np.ascontiguousarray(select, np.int64)
    m = rays.n if sel is None else len(sel)
    count, stored, _, ids = _lists_out(m, cap)
    rc, pc, sc = rays.c(), params.c(), shading.c()
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    L.check(L.lib().rs_mesh_hit_lists_download(C.byref(rc), C.byref(pc), C.byref(sc), _ptr(frame), int(ray_set),
                                               None if sel is None else p(sel), m, p(count), p(stored), p(ids), cap,
                                               _stream()), "rs_mesh_hit_lists_download")
    return dict(count=count[:m], stored=stored[:m], ids=ids[:m])


def download(bvh: BVH):
    """Host copies of the built BVH (for tests)."""
    n = bvh.n
    ni = max(n - 1, 0)
    codes = np.zeros(max(n, 1), np.uint32)
    perm = np.zeros(max(n, 1), np.int32)
    child = np.zeros((max(ni, 1), 2), np.int32)
    boxes = np.zeros((max(ni, 1), 2, 6), np.float32)
    leaf_boxes = np.zeros((max(n, 1), 6), np.float32)
    bounds = np.zeros(6, np.float32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    L.check(L.lib().rs_bvh_download(C.byref(bvh.desc), p(codes), p(perm), p(child), p(boxes), p(leaf_boxes),
                                    p(bounds), _stream()), "rs_bvh_download")
    return dict(codes=codes[:n], perm=perm[:n], child=child[:ni], boxes=boxes[:ni], leaf_boxes=leaf_boxes[:n],
                bounds=bounds)


# ------------------------------------------------------------ mesh + Gaussians

@dataclass
class Mesh:
    verts: torch.Tensor            # [V, 3] float32
    tris: torch.Tensor             # [T, 3] int32
    material: torch.Tensor = None  # [T] int32: 0 diffuse, 1 mirror, 2 glass

    def c(self):
        _dev(self.verts, "verts")
        _dev(self.tris, "tris", torch.int32)
        if self.material is not None:
            _dev(self.material, "material", torch.int32)
        return L.rs_mesh(int(self.verts.shape[0]), int(self.tris.shape[0]), _ptr(self.verts), _ptr(self.tris),
                         _ptr(self.material))

    @property
    def n(self):
        return int(self.tris.shape[0])


@dataclass
class Shading:
    light: tuple = (2.0, -2.0, 5.0)
    intensity: float = 1.0
    albedo: float = 0.8
    mirror_reflectance: float = 0.8
    mirror_diffuse: float = 0.2
    offset: float = 1e-4
    max_bounces: int = 1
    ior: float = 1.5

    def c(self):
        s = L.rs_shading()
        for k in range(3):
            s.light[k] = float(self.light[k])
        s.intensity, s.albedo = float(self.intensity), float(self.albedo)
        s.mirror_reflectance, s.mirror_diffuse = float(self.mirror_reflectance), float(self.mirror_diffuse)
        s.offset = float(self.offset)
        s.max_bounces, s.ior = int(self.max_bounces), float(self.ior)
        return s


def build_mesh_bvh(mesh: Mesh, workspace=None):
    lib = L.lib()
    nbytes = workspace_bytes(mesh.n)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=mesh.verts.device)
    desc = L.rs_bvh()
    mc = mesh.c()
    L.check(lib.rs_build_mesh_bvh(C.byref(mc), _ptr(workspace), C.c_size_t(workspace.numel()), C.byref(desc),
                                  _stream()), "rs_build_mesh_bvh")
    return BVH(mesh.n, 0.0, workspace, desc)


def trace_mesh(mbvh: BVH, rays: Rays, t_limit=None, any_hit=False):
    n = rays.n
    t = torch.empty(n, dtype=torch.float32, device=rays.origin.device)
    tri = torch.empty(n, dtype=torch.int32, device=rays.origin.device)
    rc = rays.c()
    L.check(L.lib().rs_trace_mesh(C.byref(mbvh.desc), C.byref(rc), _ptr(t_limit), int(any_hit), _ptr(t), _ptr(tri),
                                  _stream()), "rs_trace_mesh")
    return t, tri


def mesh_frame(n, params=None, device="cuda", shading=None):
    pc = params.c() if params is not None else None
    sc = shading.c() if shading is not None else None
    nbytes = int(L.lib().rs_mesh_frame_bytes(int(n), C.byref(pc) if pc is not None else None,
                                             C.byref(sc) if sc is not None else None))
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def render_mesh_fwd(gbvh: BVH, mbvh: BVH, g: Gaussians, mesh: Mesh, shading: Shading, rays: Rays, params: Params,
                    out=None, frame=None):
    n = rays.n
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=rays.origin.device)
    if frame is None:
        frame = mesh_frame(n, params, rays.origin.device, shading)
    gc, mc, sc, rc, pc = g.c(), mesh.c(), shading.c(), rays.c(), params.c()
    L.check(L.lib().rs_render_mesh_fwd(C.byref(gbvh.desc), C.byref(mbvh.desc), C.byref(gc), C.byref(mc), C.byref(sc),
                                       C.byref(rc), C.byref(pc), _ptr(out), _ptr(frame), _stream()),
            "rs_render_mesh_fwd")
    return out, frame


def render_mesh_bwd(gbvh: BVH, mbvh: BVH, g: Gaussians, mesh: Mesh, shading: Shading, rays: Rays, params: Params,
                    grad_rgb, frame, grads=None):
    grad_rgb = _dev(grad_rgb.contiguous(), "grad_rgb")
    if grads is None:
        grads = (torch.empty_like(g.mean), torch.empty_like(g.scale), torch.empty_like(g.quat),
                 torch.empty_like(g.opacity), torch.empty_like(g.rgb))
    gr = L.rs_grads(*[_ptr(t) for t in grads])
    gc, mc, sc, rc, pc = g.c(), mesh.c(), shading.c(), rays.c(), params.c()
    L.check(L.lib().rs_render_mesh_bwd(C.byref(gbvh.desc), C.byref(mbvh.desc), C.byref(gc), C.byref(mc), C.byref(sc),
                                       C.byref(rc), C.byref(pc), _ptr(grad_rgb), _ptr(frame), C.byref(gr),
                                       _stream()), "rs_render_mesh_bwd")
    return grads


# ------------------------------------------------------------ training loss

def loss_workspace(width, height, device="cuda"):
    return torch.empty(max(int(L.lib().rs_loss_workspace_bytes(int(width), int(height))), 256), dtype=torch.uint8,
                       device=device)


def image_loss(img, target, width, height, lam=0.2, radius=5, sigma=1.5, grad=True, ws=None, out=None,
               grad_out=None):
    """(1 - lam) L2 + lam D-SSIM of one image ([height*width, 3] or [height, width, 3])
    against its target (rs_loss). Returns (loss[1], grad or None)."""
    img = _dev(img.contiguous(), "img")
    target = _dev(target.contiguous(), "target")
    lp = L.rs_loss_params(float(lam), int(radius), float(sigma))
    ws = ws if ws is not None else loss_workspace(width, height, img.device)
    loss = out if out is not None else torch.empty(1, dtype=torch.float32, device=img.device)
    g = (_dev(grad_out, "grad_out") if grad_out is not None else torch.empty_like(img)) if grad else None
    L.check(L.lib().rs_loss(_ptr(img), _ptr(target), int(width), int(height), C.byref(lp), _ptr(loss), _ptr(g),
                            _ptr(ws), _stream()), "rs_loss")
    return loss, g


class ImageLoss(torch.autograd.Function):
    """Scalar (1 - lam) L2 + lam D-SSIM of one image against its target
    (rs_loss); the gradient comes from the same launch."""

    @staticmethod
    def forward(ctx, img, target, width, height, lam=0.2, radius=5, sigma=1.5):
        loss, g = image_loss(img.detach(), target.detach(), width, height, lam, radius, sigma,
                             grad=img.requires_grad)
        ctx.save_for_backward(g if g is not None else img.new_zeros(0))
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (g * grad_out if g.numel() else None), None, None, None, None, None, None


class MeshRender(torch.autograd.Function):
    """Gaussians + triangle mesh with mirror reflections and shadows; the
    Gaussian BVH is rebuilt every forward, the mesh BVH is given."""

    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, rgb, origin, direction, mesh, mbvh, shading, params, views):
        g = Gaussians(mean.contiguous(), scale.contiguous(), quat.contiguous(), opacity.contiguous(),
                      rgb.contiguous())
        rays = Rays(origin.contiguous(), direction.contiguous(), views=list(views or []))
        gbvh = build_bvh(g, params)
        out, frame = render_mesh_fwd(gbvh, mbvh, g, mesh, shading, rays, params)
        if params.raise_on_status:
            raise_on_status(gbvh, "rs_render_mesh_fwd")
        ctx.saved = (gbvh, mbvh, g, mesh, shading, rays, params, frame)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        gbvh, mbvh, g, mesh, shading, rays, params, frame = ctx.saved
        dm, ds, dq, do, dc = render_mesh_bwd(gbvh, mbvh, g, mesh, shading, rays, params, grad_out.contiguous(), frame)
        if params.raise_on_status:
            raise_on_status(gbvh, "rs_render_mesh_bwd")
        return dm, ds, dq, do, dc, None, None, None, None, None, None, None


class RaySplatsRender(torch.autograd.Function):
    """rgb = render(mean, scale, quat, opacity, rgb; rays). The BVH is rebuilt
    in every forward (the parameters change every optimisation step); the
    backward replays the stored hit lists (params.hit_list > 0) or
    re-traverses the rays."""

    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, rgb, origin, direction, params, views):
        g = Gaussians(mean.contiguous(), scale.contiguous(), quat.contiguous(), opacity.contiguous(),
                      rgb.contiguous())
        rays = Rays(origin.contiguous(), direction.contiguous(), views=list(views or []))
        bvh = build_bvh(g, params)
        out, state = render_fwd(bvh, g, rays, params)
        if params.raise_on_status:
            raise_on_status(bvh, "rs_render_fwd")
        ctx.saved = (bvh, g, rays, params, state)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        bvh, g, rays, params, state = ctx.saved
        dm, ds, dq, do, dc = render_bwd(bvh, g, rays, params, grad_out.contiguous(), state)
        if params.raise_on_status:
            raise_on_status(bvh, "rs_render_bwd")
        return dm, ds, dq, do, dc, None, None, None, None


def render(mean, scale, quat, opacity, rgb, origin, direction, params=None, views=None):
    return RaySplatsRender.apply(mean, scale, quat, opacity, rgb, origin, direction, params or Params(), views)
