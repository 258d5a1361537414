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
    """Forward through the C ABI. Returns (rgb numpy, ray state (device tensor),
    status, (bvh, gaussians, rays))."""
    params = params or R.Params()
    g = g or gaussians(scene)
    bvh = bvh or R.build_bvh(g, params)
    rays = rays_of(origin, direction, views, t_max, bg)
    out, state = R.render_fwd(bvh, g, rays, params)
    torch.cuda.synchronize()
    status = R.read_status(bvh)
    return out.cpu().numpy(), state, status, (bvh, g, rays)


def colour_state(state, n):
    """(final colour, final T) [n, 4] of a ray state, on the host."""
    return R.state_colour(state, n).cpu().numpy()


def sequences(scene, origin, direction, params, cap=512, t_max=None, bg=None):
    """The GPU forward's composited Gaussian ids per ray, in order (stored hit
    lists of a forward over these rays alone; a ray's hits do not depend on the
    other rays of its packet). Returns (ids[n, cap] with -1 padding, counts)."""
    import dataclasses
    p = dataclasses.replace(params, hit_list=min(cap + 128, 4096), flags=params.flags & ~16)
    out, state, status, (bvh, g, rays) = render(scene, origin, direction, p, t_max=t_max, bg=bg)
    assert status == 0
    L = R.hit_lists(rays, p, state, cap=cap)
    assert np.array_equal(L["stored"], L["count"]), "the test pool is sized never to run out"
    return L["ids"], L["count"]


def oracle_params(O, p):
    # the library takes float32 knobs: give the oracle the same values exactly
    f = lambda x: float(np.float32(x))
    return O.Params(Q=f(p.Q), eps1=f(p.eps1), t_min=f(p.t_min), max_hits=p.max_hits, bg=tuple(f(b) for b in p.bg),
                    zero_colour=bool(p.flags & 4))


GROUPS = ("mean", "scale", "quat", "opacity", "rgb")


def assert_elementwise(got, ref, label, rel=1e-3):
    """Every entry of every parameter group: |g_gpu - g_oracle| <= rel |g_oracle|
    + rel max |g_oracle| (the floor keeps entries that are sums of nearly
    cancelling contributions from failing on float32 rounding alone)."""
    worst = {}
    for k in GROUPS:
        a, b = got[k], ref[k]
        scale = np.abs(b).max() if b.size else 0.0
        err = np.abs(a - b)
        bound = rel * np.abs(b) + rel * scale
        bad = err > bound
        worst[k] = float((err / np.maximum(np.abs(b) + scale, 1e-300)).max()) if b.size else 0.0
        if bad.any():
            i = np.unravel_index(np.argmax(err - bound), err.shape)
            raise AssertionError(f"{label} {k}: {int(bad.sum())} of {bad.size} entries outside the bound; "
                                 f"worst at {i}: gpu {a[i]:.6e} oracle {b[i]:.6e} (max |oracle| {scale:.3e})")
    norms = {k: float(np.linalg.norm(got[k] - ref[k]) / max(np.linalg.norm(ref[k]), 1e-300)) for k in GROUPS}
    print(label, "worst |err| / (|ref| + max|ref|):", {k: f"{v:.1e}" for k, v in worst.items()},
          "norm ratios:", {k: f"{v:.1e}" for k, v in norms.items()}, flush=True)
