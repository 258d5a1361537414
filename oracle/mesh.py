"""FP64 oracle of the mixed mesh + Gaussian workload (TEST INFRASTRUCTURE ONLY).

The paper shows meshes combined with Gaussians, with mirror reflections,
shadows and glass (Sec. 1, Figs. 1 and 3-6), but specifies no shading model.
This file is the definition both sides implement.

A pixel follows a chain of up to B + 1 path rays (B = max_bounces, 1..3);
path ray 0 is the camera ray. For path ray k with origin o, unit direction d:

  closest triangle hit t_k (Moller-Trumbore, no culling, t > 0); Gaussians
  with t1 < t_k composite (Eq. 3, K_max / eps1 rules) over a black background
  when it hits a triangle and over bg when it hits none: colour C_k,
  transmittance T_k.
  at a hit with k < B: P = o + t_k d, n_g = unit geometric normal (e1 x e2 of
  the triangle's vertex order), n = n_g turned to face the ray (n.d < 0),
  l = unit vector from P to the point light, and by material:
    diffuse (0): rho_d = 1, no continuation;
    mirror (1):  rho_d = mirror_diffuse; continuation along d - 2 (d.n) n
                 from P + offset n, weight w = mirror_reflectance;
    glass (2):   rho_d = 0; entering (d.n_g < 0) eta = 1 / ior, leaving
                 eta = ior; cos_i = -d.n, k = 1 - eta^2 (1 - cos_i^2);
                 k < 0 (total internal reflection): continuation along
                 d + 2 cos_i n from P + offset n, weight 1; else refraction
                 along eta d + (eta cos_i - sqrt(k)) n from P - offset n with
                 weight 1 - F, F = R0 + (1 - R0) (1 - c)^5 (Schlick),
                 R0 = ((1 - ior) / (1 + ior))^2, c = cos_i when entering and
                 sqrt(k) when leaving (the cosine on the optically thinner
                 side); the reflected part of glass is not traced.
  shadow ray (rho_d > 0 and n.l > 0): from P + offset n towards the light,
  length L; T_s = 0 if a triangle lies at 0 < t < L, else the transmittance
  of the Gaussians with t1 < L (colours 0, background 1, same rules);
  diffuse term D_k = rho_d albedo (n.l) I_light T_s.
  radiance R_k = C_k + T_k (D_k + w R_{k+1}) at a hit with k < B (R_{k+1} = 0
  without continuation), R_k = C_k otherwise (a hit of the last path ray is
  black); pixel = R_0.

With B = 1 this is the single-bounce model: primary, mirror reflection (seeing
Gaussians up to its own closest triangle, then black, or bg past the mesh) and
shadow rays. Spawned rays are rounded to float32 on both sides.

Gradients flow through the Gaussian hits of every ray: path ray k's upstream
gradient is W_k g (W_0 = 1, W_{k+1} = W_k T_k w) and its background in the
adjoint is D_k + w R_{k+1}; shadow ray k's transmittance gradient is
W_k T_k rho_d albedo (n.l) I_light sum(g).
"""

import numpy as np

from . import oracle as O

DIFFUSE, MIRROR, GLASS = 0, 1, 2


class Shading:
    def __init__(self, light=(2.0, -2.0, 5.0), intensity=1.0, albedo=0.8, mirror_reflectance=0.8,
                 mirror_diffuse=0.2, offset=1e-4, max_bounces=1, ior=1.5):
        self.light = np.asarray(light, np.float64)
        self.intensity = float(intensity)
        self.albedo = float(albedo)
        self.mirror_reflectance = float(mirror_reflectance)
        self.mirror_diffuse = float(mirror_diffuse)
        self.offset = float(offset)
        self.max_bounces = int(max_bounces)
        self.ior = float(ior)


def _normals(verts, tris, idx):
    v = verts.astype(np.float64)
    t = tris[idx]
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def glass_continuation(d, n_g, ior):
    """Continuation of unit rays d at a glass surface with unit geometric
    normals n_g: (direction, origin side +1 / -1 along the facing normal,
    weight, facing normal). FP64."""
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n_g = np.asarray(n_g, np.float64).reshape(-1, 3)
    c = np.einsum("ij,ij->i", d, n_g)
    entering = c < 0
    n = np.where(entering[:, None], n_g, -n_g)
    eta = np.where(entering, 1.0 / ior, ior)
    cos_i = -np.einsum("ij,ij->i", d, n)
    k = 1.0 - eta * eta * (1.0 - cos_i * cos_i)
    tir = k < 0
    ks = np.sqrt(np.maximum(k, 0.0))
    refr = eta[:, None] * d + (eta * cos_i - ks)[:, None] * n
    refl = d + 2.0 * cos_i[:, None] * n
    r0 = ((1.0 - ior) / (1.0 + ior)) ** 2
    cs = np.where(entering, cos_i, ks)
    F = r0 + (1.0 - r0) * (1.0 - cs) ** 5
    direction = np.where(tir[:, None], refl, refr)
    side = np.where(tir, 1.0, -1.0)
    weight = np.where(tir, 1.0, 1.0 - F)
    return direction, side, weight, n


def mesh_forward(scene, mesh, shading, origin, direction, params=None, threads=0):
    """Returns a dict with the pixel colours and every intermediate the
    adjoint and the parity tests need (per path level: its rays, C, T, the
    triangle hits, the continuation weight, the diffuse term and radiance)."""
    params = params or O.Params()
    B = shading.max_bounces
    o = np.asarray(origin, np.float32).astype(np.float64).reshape(-1, 3)
    d = np.asarray(direction, np.float32).astype(np.float64).reshape(-1, 3)
    n_r = o.shape[0]
    bg = np.asarray(params.bg, np.float64)
    material = np.asarray(mesh.mirror)
    sp = O.Params(Q=params.Q, eps1=params.eps1, t_min=params.t_min, max_hits=params.max_hits,
                  bg=(1.0, 1.0, 1.0), zero_colour=True)
    levels = []
    idx = np.arange(n_r)          # pixels whose chain reaches this level
    ro, rd = o, d                  # their rays (float32 values in float64)
    for k in range(B + 1):
        lv = dict(idx=idx, origin=ro, dir=rd)
        t_m, tri = O.mesh_closest(mesh.verts, mesh.tris, ro, rd, t_eps=0.0)
        hit = tri >= 0
        bg_k = np.where(hit[:, None], 0.0, bg[None, :])
        C, T, _ = O.render_fwd(scene, ro, rd, params, t_max=t_m, bg=bg_k, threads=threads)
        lv.update(t_max=t_m, tri=tri, hit=hit, bg=bg_k, C=C, T=T, w=np.zeros(len(idx)), D=np.zeros(len(idx)),
                  shad=dict(sel=np.zeros(0, np.int64), idx=np.zeros(0, np.int64)), nxt=np.zeros(0, np.int64))
        levels.append(lv)
        if k == B or not hit.any():
            break
        hi = np.nonzero(hit)[0]
        n_g = _normals(mesh.verts, mesh.tris, tri[hi])
        dd = rd[hi]
        face = np.where((np.einsum("ij,ij->i", n_g, dd) > 0)[:, None], -n_g, n_g)
        P = ro[hi] + t_m[hi, None] * dd
        mat = material[tri[hi]]
        rho_d = np.where(mat == MIRROR, shading.mirror_diffuse, np.where(mat == GLASS, 0.0, 1.0))
        # shadow rays
        Lv = shading.light[None, :] - P
        nl = np.maximum(0.0, np.einsum("ij,ij->i", face, Lv / np.linalg.norm(Lv, axis=1, keepdims=True)))
        ssel = (rho_d > 0) & (nl > 0)
        if ssel.any():
            so = P[ssel] + shading.offset * face[ssel]
            Ls = shading.light[None, :] - so
            dist = np.linalg.norm(Ls, axis=1)
            so32, sd32 = np.float32(so), np.float32(Ls / dist[:, None])
            t_b, tri_b = O.mesh_closest(mesh.verts, mesh.tris, so32.astype(np.float64), sd32.astype(np.float64),
                                        t_eps=0.0)
            dist32 = dist.astype(np.float32).astype(np.float64)
            blocked = (tri_b >= 0) & (t_b < dist32)
            _, T_s, _ = O.render_fwd(scene, so32, sd32, sp, t_max=dist32, threads=threads)
            T_s = np.where(blocked, 0.0, T_s)
            wd = rho_d[ssel] * shading.albedo * nl[ssel] * shading.intensity
            lv["D"][hi[ssel]] = wd * T_s
            lv["shad"] = dict(sel=hi[ssel], idx=idx[hi[ssel]], origin=so32, dir=sd32, t_max=dist32,
                              blocked=blocked, T=T_s, w=wd, params=sp)
        # continuation rays
        cdir = np.zeros_like(dd)
        cside = np.ones(len(hi))
        cw = np.zeros(len(hi))
        mir = mat == MIRROR
        if mir.any():
            cdir[mir] = dd[mir] - 2.0 * np.einsum("ij,ij->i", dd[mir], face[mir])[:, None] * face[mir]
            cw[mir] = shading.mirror_reflectance
        gl = mat == GLASS
        if gl.any():
            gd, gs, gw, _ = glass_continuation(dd[gl], n_g[gl], shading.ior)
            cdir[gl], cside[gl], cw[gl] = gd, gs, gw
        csel = cw > 0
        if not csel.any():
            break
        lv["w"][hi[csel]] = cw[csel]
        lv["nxt"] = hi[csel]
        co = P[csel] + (cside[csel] * shading.offset)[:, None] * face[csel]
        ro = np.float32(co).astype(np.float64)
        rd = np.float32(cdir[csel]).astype(np.float64)
        idx = idx[hi[csel]]
    # radiance bottom-up
    R_next = None
    for k in range(len(levels) - 1, -1, -1):
        lv = levels[k]
        R = lv["C"].copy()
        S = np.zeros_like(R)  # background of this path ray's adjoint: D + w R_{k+1}
        h = np.nonzero(lv["hit"])[0]
        S[h] += lv["D"][h, None]
        if R_next is not None and len(lv["nxt"]):
            S[lv["nxt"]] += lv["w"][lv["nxt"], None] * R_next
        R[h] += lv["T"][h, None] * S[h]
        lv["S"] = np.where(lv["hit"][:, None], S, lv["bg"])
        lv["R"] = R
        R_next = R
    l0 = levels[0]
    out = dict(rgb=l0["R"], levels=levels, t_mesh=l0["t_max"], tri=l0["tri"], C_p=l0["C"], T_p=l0["T"],
               bg_p=l0["bg"], shade=np.where(l0["hit"][:, None], l0["S"], 0.0), rho_m=l0["w"], shad=l0["shad"])
    # the first continuation (the mirror reflection of the single-bounce model)
    if len(levels) > 1:
        l1 = levels[1]
        out["refl"] = dict(idx=l1["idx"], origin=l1["origin"], dir=l1["dir"], t_max=l1["t_max"], bg=l1["bg"],
                           C=l1["C"], T=l1["T"])
    else:
        out["refl"] = dict(idx=np.zeros(0, np.int64))
    return out


def mesh_backward(scene, mesh, shading, origin, direction, grad_rgb, params=None, fwd=None, threads=0):
    """Gradients of sum <grad_rgb, pixel> with respect to the Gaussian parameters."""
    params = params or O.Params()
    fwd = fwd or mesh_forward(scene, mesh, shading, origin, direction, params, threads)
    g = np.asarray(grad_rgb, np.float64).reshape(-1, 3)
    grads = None
    W = np.ones(g.shape[0])   # path weight of each pixel at the current level (indexed by pixel)
    for k, lv in enumerate(fwd["levels"]):
        idx = lv["idx"]
        gk = g[idx] * W[idx, None]
        gg = O.render_bwd(scene, lv["origin"], lv["dir"], gk, params, t_max=lv["t_max"], bg=lv["S"],
                          threads=threads)
        grads = gg if grads is None else {key: grads[key] + gg[key] for key in grads}
        s = lv["shad"]
        if len(s["sel"]):
            sel = s["sel"]
            up = np.where(s["blocked"], 0.0, gk[sel].sum(axis=1) * lv["T"][sel] * s["w"])
            gs = np.zeros((len(sel), 3))
            gs[:, 0] = up
            gg = O.render_bwd(scene, s["origin"], s["dir"], gs, s["params"], t_max=s["t_max"], bg=None,
                              threads=threads)
            for key in grads:
                grads[key] += gg[key]
        if len(lv["nxt"]):
            nxt = lv["nxt"]
            W[idx[nxt]] = W[idx[nxt]] * lv["T"][nxt] * lv["w"][nxt]
    return grads
