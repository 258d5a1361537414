"""FP64 oracle of the mixed mesh + Gaussian workload (TEST INFRASTRUCTURE ONLY).

The paper shows meshes combined with Gaussians, with mirror reflections and
shadows (Sec. 1, Figs. 1 and 3-6), but specifies no shading model. This file
is the definition both sides implement:

  primary ray r: closest triangle hit t_m (Moller-Trumbore, no culling, t > 0);
      Gaussians composite over hits with t1 < t_m (Eq. 3, K_max / eps1 rules)
      giving colour C_p and transmittance T_p; with no triangle hit the pixel
      is C_p + T_p bg (the plain render).
  at a triangle hit: P = o + t_m d, n = the unit geometric normal facing the
      ray (n.d < 0), l = unit vector from P to the point light;
      mirror material: rho_m = mirror_reflectance, rho_d = mirror_diffuse;
      diffuse material: rho_m = 0, rho_d = 1.
  reflection ray (if rho_m > 0): origin P + offset n, direction d - 2 (d.n) n;
      its own closest triangle hit t_r bounds its Gaussians (t1 < t_r); it sees
      bg when it hits no triangle and black when it does (one bounce):
      C_r = C + T * (t_r finite ? 0 : bg).
  shadow ray (if rho_d > 0 and n.l > 0): origin P + offset n, direction to
      the light, length L; blocked (T_s = 0) by any triangle with 0 < t < L;
      otherwise T_s = transmittance of the Gaussians with t1 < L (colours 0,
      background 1, same K_max / eps1 rules).
  pixel = C_p + T_p * (rho_m C_r + rho_d * albedo * (n.l) * I_light * T_s).

Gradients flow through the Gaussian hits of all three rays: the primary's
background is the shade term, the reflection ray's upstream gradient is
T_p rho_m g, the shadow ray's is T_p rho_d albedo (n.l) I_light sum(g).
"""

import numpy as np

from . import oracle as O


class Shading:
    def __init__(self, light=(2.0, -2.0, 5.0), intensity=1.0, albedo=0.8, mirror_reflectance=0.8,
                 mirror_diffuse=0.2, offset=1e-4):
        self.light = np.asarray(light, np.float64)
        self.intensity = float(intensity)
        self.albedo = float(albedo)
        self.mirror_reflectance = float(mirror_reflectance)
        self.mirror_diffuse = float(mirror_diffuse)
        self.offset = float(offset)


def _normals(verts, tris, idx):
    v = verts.astype(np.float64)
    t = tris[idx]
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def mesh_forward(scene, mesh, shading, origin, direction, params=None, threads=0):
    """Returns a dict with the pixel colours and every intermediate the
    adjoint and the parity tests need."""
    params = params or O.Params()
    o = np.asarray(origin, np.float32).astype(np.float64).reshape(-1, 3)
    d = np.asarray(direction, np.float32).astype(np.float64).reshape(-1, 3)
    n_r = o.shape[0]
    bg = np.asarray(params.bg, np.float64)
    t_m, tri = O.mesh_closest(mesh.verts, mesh.tris, o, d, t_eps=0.0)
    hit = tri >= 0
    bg_p = np.where(hit[:, None], 0.0, bg[None, :])
    C_p, T_p, _ = O.render_fwd(scene, o, d, params, t_max=t_m, bg=bg_p, threads=threads)
    out = C_p.copy()
    shade = np.zeros((n_r, 3))
    rho_m = np.zeros(n_r)
    rho_d = np.zeros(n_r)
    nl = np.zeros(n_r)
    refl = dict(idx=np.zeros(0, np.int64))
    shad = dict(idx=np.zeros(0, np.int64))
    if hit.any():
        hi = np.nonzero(hit)[0]
        nrm = _normals(mesh.verts, mesh.tris, tri[hi])
        flip = np.einsum("ij,ij->i", nrm, d[hi]) > 0
        nrm[flip] *= -1.0
        P = o[hi] + t_m[hi, None] * d[hi]
        mirror = mesh.mirror[tri[hi]] == 1
        rho_m[hi] = np.where(mirror, shading.mirror_reflectance, 0.0)
        rho_d[hi] = np.where(mirror, shading.mirror_diffuse, 1.0)
        Lv = shading.light[None, :] - P
        lhat = Lv / np.linalg.norm(Lv, axis=1, keepdims=True)
        nl[hi] = np.maximum(0.0, np.einsum("ij,ij->i", nrm, lhat))
        # reflection rays
        rsel = rho_m[hi] > 0
        if rsel.any():
            ri = hi[rsel]
            ro = P[rsel] + shading.offset * nrm[rsel]
            dd = d[ri]
            rd = dd - 2.0 * np.einsum("ij,ij->i", dd, nrm[rsel])[:, None] * nrm[rsel]
            ro32, rd32 = np.float32(ro), np.float32(rd)
            t_r, tri_r = O.mesh_closest(mesh.verts, mesh.tris, ro32.astype(np.float64), rd32.astype(np.float64),
                                        t_eps=0.0)
            bg_r = np.where((tri_r >= 0)[:, None], 0.0, bg[None, :])
            C_r, T_r, _ = O.render_fwd(scene, ro32, rd32, params, t_max=t_r, bg=bg_r, threads=threads)
            shade[ri] += rho_m[ri, None] * C_r
            refl = dict(idx=ri, origin=ro32, dir=rd32, t_max=t_r, bg=bg_r, C=C_r, T=T_r)
        # shadow rays
        ssel = (rho_d[hi] > 0) & (nl[hi] > 0)
        if ssel.any():
            si = hi[ssel]
            so = P[ssel] + shading.offset * nrm[ssel]
            Ls = shading.light[None, :] - so
            dist = np.linalg.norm(Ls, axis=1)
            sd = Ls / dist[:, None]
            so32, sd32 = np.float32(so), np.float32(sd)
            t_b, tri_b = O.mesh_closest(mesh.verts, mesh.tris, so32.astype(np.float64), sd32.astype(np.float64),
                                        t_eps=0.0)
            dist32 = dist.astype(np.float32).astype(np.float64)
            blocked = (tri_b >= 0) & (t_b < dist32)
            sp = O.Params(Q=params.Q, eps1=params.eps1, t_min=params.t_min, max_hits=params.max_hits,
                          bg=(1.0, 1.0, 1.0), zero_colour=True)
            _, T_s, _ = O.render_fwd(scene, so32, sd32, sp, t_max=dist32, threads=threads)
            T_s = np.where(blocked, 0.0, T_s)
            w = rho_d[si] * shading.albedo * nl[si] * shading.intensity
            shade[si] += (w * T_s)[:, None]
            shad = dict(idx=si, origin=so32, dir=sd32, t_max=dist32, blocked=blocked, T=T_s, w=w, params=sp)
        out[hi] = C_p[hi] + T_p[hi, None] * shade[hi]
    return dict(rgb=out, C_p=C_p, T_p=T_p, t_mesh=t_m, tri=tri, bg_p=bg_p, shade=shade, rho_m=rho_m, refl=refl,
                shad=shad)


def mesh_backward(scene, mesh, shading, origin, direction, grad_rgb, params=None, fwd=None, threads=0):
    """Gradients of sum <grad_rgb, pixel> with respect to the Gaussian parameters."""
    params = params or O.Params()
    fwd = fwd or mesh_forward(scene, mesh, shading, origin, direction, params, threads)
    g = np.asarray(grad_rgb, np.float64).reshape(-1, 3)
    hit = fwd["tri"] >= 0
    # primary: the background of a mesh-hitting ray is its shade term
    bg_bwd = np.where(hit[:, None], fwd["shade"], np.asarray(params.bg, np.float64)[None, :])
    grads = O.render_bwd(scene, origin, direction, g, params, t_max=fwd["t_mesh"], bg=bg_bwd, threads=threads)
    r = fwd["refl"]
    if len(r["idx"]):
        gr = g[r["idx"]] * (fwd["T_p"][r["idx"]] * fwd["rho_m"][r["idx"]])[:, None]
        gg = O.render_bwd(scene, r["origin"], r["dir"], gr, params, t_max=r["t_max"], bg=r["bg"], threads=threads)
        for k in grads:
            grads[k] += gg[k]
    s = fwd["shad"]
    if len(s["idx"]):
        up = np.where(s["blocked"], 0.0, g[s["idx"]].sum(axis=1) * fwd["T_p"][s["idx"]] * s["w"])
        gs = np.zeros((len(s["idx"]), 3))
        gs[:, 0] = up
        gg = O.render_bwd(scene, s["origin"], s["dir"], gs, s["params"], t_max=s["t_max"], bg=None,
                          threads=threads)
        for k in grads:
            grads[k] += gg[k]
    return grads
