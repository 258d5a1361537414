"""Helpers shared by the GPU tests: move seeded inputs to the device and call
the HIP library through its C ABI (via the package's ctypes binding)."""

import numpy as np
import torch

from synthetic.cameras import pinhole_rays, concat_rays

import paper_2501_19196_amd as rs
from paper_2501_19196_amd import renderer as R


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gaussians(scene):
    return R.Gaussians(*(dev(a) for a in scene.arrays()))


def rays_of(origin, direction, views=None, t_max=None, bg=None):
    return R.Rays(dev(origin), dev(direction), None if t_max is None else dev(np.float32(t_max)),
                  None if bg is None else dev(np.float32(bg)), list(views or []))


def camera_rays(cams):
    o, d, views = concat_rays(cams)
    return o, d, [tuple(int(x) for x in v) for v in views]


def render(scene, origin, direction, params=None, views=None, t_max=None, bg=None, bvh=None, g=None):
    params = params or R.Params()
    g = g or gaussians(scene)
    bvh = bvh or R.build_bvh(g, params)
    rays = rays_of(origin, direction, views, t_max, bg)
    out, state = R.render_fwd(bvh, g, rays, params)
    torch.cuda.synchronize()
    status = R.read_status(bvh)
    return out.cpu().numpy(), state.cpu().numpy(), status, (bvh, g, rays)


def oracle_params(O, p):
    # the library takes float32 knobs: give the oracle the same values exactly
    f = lambda x: float(np.float32(x))
    return O.Params(Q=f(p.Q), eps1=f(p.eps1), t_min=f(p.t_min), max_hits=p.max_hits, bg=tuple(f(b) for b in p.bg),
                    zero_colour=bool(p.flags & 4))
