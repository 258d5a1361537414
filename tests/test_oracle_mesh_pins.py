"""Pins of the mesh + Gaussian oracle (oracle/mesh.py) against facts it does
not compute itself: an independent plane / barycentric triangle test, the
Lambert and mirror closed forms on a bare mesh, the identity between a
perfect mirror and the scene unioned with its mirror image, a shadow ray
through one Gaussian (transmittance 1 - opacity), a blocked shadow, and
central differences of the mesh adjoint. CPU only."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from synthetic import mesh as M
from synthetic import scenes
from synthetic.scenes import Scene


def _mesh(verts, tris, mirror):
    return M.Mesh(np.ascontiguousarray(np.asarray(verts, np.float32)), np.ascontiguousarray(np.asarray(tris, np.int32)),
                  np.ascontiguousarray(np.asarray(mirror, np.int32)))


def _plane(cells, half, mirror):
    v, t = M.subdivided_plane(cells, half)
    return _mesh(v, t, np.full(len(t), int(mirror)))


def _far_scene(n=1):
    """Gaussians nowhere near any ray of these tests (the bare-mesh cases)."""
    f = lambda a: np.asarray(a, np.float32)
    return Scene(f([[50.0, 50.0, 50.0]] * n), f([[0.01, 0.01, 0.01]] * n), f([[1, 0, 0, 0]] * n),
                 f([0.5] * n), f([[1, 1, 1]] * n))


def _brute_closest(verts, tris, o, d):
    """Plane intersection plus a barycentric solve per triangle (no Moller-Trumbore)."""
    v = verts.astype(np.float64)
    best_t = np.full(len(o), np.inf)
    best_f = np.full(len(o), -1)
    for f, (a, b, c) in enumerate(tris):
        A, B, Cc = v[a], v[b], v[c]
        n = np.cross(B - A, Cc - A)
        den = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            t = ((A - o) @ n) / den
        P = o + t[:, None] * d
        # barycentric coordinates from the 3x2 least-squares system P - A = u (B-A) + w (C-A)
        E = np.stack([B - A, Cc - A], axis=1)
        uw, *_ = np.linalg.lstsq(E, (P - A).T, rcond=None)
        u, w = uw
        inside = (u >= -1e-12) & (w >= -1e-12) & (u + w <= 1 + 1e-12) & (den != 0) & (t > 0)
        better = inside & (t < best_t)
        best_t[better] = t[better]
        best_f[better] = f
    return best_t, best_f


def test_mesh_closest_matches_barycentric_brute_force(orc):
    mesh = M.mirror_mesh(plane_cells=4, plane_half=2.0, sphere_subdiv=1, sphere_radius=0.6)
    rng = np.random.default_rng(0)
    o = rng.uniform(-1.5, 1.5, size=(400, 3)) + np.array([0.0, 0.0, 2.5])
    d = rng.normal(size=(400, 3))
    d[:, :2] *= 0.4
    d[:, 2] = -np.abs(d[:, 2]) - 0.3
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t, tri, amb = orc.mesh_closest(mesh.verts, mesh.tris, o, d, edge=1e-9, want_amb=True)
    tb, fb = _brute_closest(mesh.verts, mesh.tris, o, d)
    ok = ~amb
    assert ok.sum() > 350
    assert np.array_equal(tri[ok], fb[ok])
    hit = ok & (tri >= 0)
    assert hit.sum() > 200
    np.testing.assert_allclose(t[hit], tb[hit], rtol=1e-10)
    assert np.all(np.isinf(t[ok & (tri < 0)]))


def test_lambert_closed_form_on_bare_diffuse_plane(orc):
    """No Gaussian on any path: pixel = albedo (n.l) I on the plane, bg off it."""
    from oracle import mesh as OM
    mesh = _plane(3, 1.0, mirror=False)
    sh = OM.Shading(light=(0.3, -0.4, 2.0), intensity=1.7, albedo=0.6)
    rng = np.random.default_rng(1)
    xy = rng.uniform(-1.4, 1.4, size=(256, 2))
    o = np.column_stack([xy, np.full(256, 3.0)])
    d = np.tile([0.0, 0.0, -1.0], (256, 1))
    p = orc.Params(bg=(0.1, 0.2, 0.3))
    out = OM.mesh_forward(_far_scene(), mesh, sh, o, d, p)["rgb"]
    on = (np.abs(xy) < 1.0).all(axis=1)
    P = np.column_stack([xy, np.zeros(256)])
    L = np.asarray(sh.light) - P
    nl = L[:, 2] / np.linalg.norm(L, axis=1)
    want = np.where(on[:, None], (0.6 * 1.7 * nl)[:, None] * np.ones(3), [0.1, 0.2, 0.3])
    np.testing.assert_allclose(out, want, atol=1e-6)


def test_bare_mirror_sees_background_plus_diffuse(orc):
    """Mirror plane, no Gaussians: pixel = rho_m bg + rho_d albedo (n.l) I."""
    from oracle import mesh as OM
    mesh = _plane(2, 1.0, mirror=True)
    sh = OM.Shading(light=(-0.5, 0.5, 3.0), intensity=1.0, albedo=0.9, mirror_reflectance=0.7, mirror_diffuse=0.25)
    rng = np.random.default_rng(2)
    xy = rng.uniform(-0.9, 0.9, size=(64, 2))
    o = np.column_stack([xy - 0.5, np.full(64, 2.0)])
    d = np.column_stack([np.full(64, 0.25), np.zeros(64), np.full(64, -1.0)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    bg = np.array([0.2, 0.4, 0.6])
    out = OM.mesh_forward(_far_scene(), mesh, sh, o, d, orc.Params(bg=bg))["rgb"]
    t = o[:, 2] / -d[:, 2]
    P = o + t[:, None] * d
    on = (np.abs(P[:, :2]) < 1.0).all(axis=1)
    assert on.sum() > 40
    L = np.asarray(sh.light) - P
    nl = L[:, 2] / np.linalg.norm(L, axis=1)
    want = 0.7 * bg[None, :] + (0.25 * 0.9 * nl)[:, None]
    np.testing.assert_allclose(out[on], want[on], atol=1e-6)


def _mirror_image(sc):
    """Gaussians reflected in the plane z = 0: mean z -> -z and rotation M R F
    (M = F = diag(1, 1, -1)), a proper rotation with the same ellipsoid."""
    Mz = np.diag([1.0, 1.0, -1.0])
    q = sc.quat.astype(np.float64)
    R = Rotation.from_quat(np.column_stack([q[:, 1:], q[:, :1]])).as_matrix()
    R2 = Mz @ R @ Mz
    q2 = Rotation.from_matrix(R2).as_quat()
    out = sc.copy()
    out.mean = np.ascontiguousarray((sc.mean.astype(np.float64) @ Mz).astype(np.float32))
    out.quat = np.ascontiguousarray(np.column_stack([q2[:, 3:], q2[:, :3]]).astype(np.float32))
    return out


def test_perfect_mirror_equals_scene_union_mirror_image(orc):
    """A perfect mirror (rho_m = 1, rho_d = 0) at z = 0 shows, along the
    reflected ray, exactly what the straight ray would see in the mirrored
    scene. With no early stop (eps1 = 0, unbounded hits) the mixed render
    equals a plain render of scene + mirror image."""
    from oracle import mesh as OM
    sc = scenes.random_scene(3, 150, box=0.8, scale_lo=0.02, scale_hi=0.05)
    sc.mean[:, 2] = np.abs(sc.mean[:, 2]) + 0.3
    mesh = _plane(2, 4.0, mirror=True)
    sh = OM.Shading(mirror_reflectance=1.0, mirror_diffuse=0.0, offset=1e-6)
    rng = np.random.default_rng(4)
    tgt = np.column_stack([rng.uniform(-1.2, 1.2, size=(300, 2)), np.zeros(300)])
    o = np.tile([0.4, -0.3, 2.6], (300, 1))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o, d = np.float32(o).astype(np.float64), np.float32(d).astype(np.float64)
    p = orc.Params(eps1=0.0, max_hits=0, bg=(0.1, 0.2, 0.3))
    out = OM.mesh_forward(sc, mesh, sh, o, d, p)["rgb"]
    mi = _mirror_image(sc)
    union = Scene(*[np.ascontiguousarray(np.concatenate([a, b])) for a, b in zip(sc.arrays(), mi.arrays())])
    want, _, _ = orc.render_fwd(union, o, d, p)
    assert np.abs(want - np.float64(p.bg)).max() > 0.05  # the Gaussians are visible
    np.testing.assert_allclose(out, want, atol=2e-4)


def test_shadow_through_one_gaussian(orc):
    """Diffuse plane lit through one Gaussian centred on the shadow ray:
    T_s = 1 - opacity and the pixel is albedo (n.l) I (1 - opacity)."""
    from oracle import mesh as OM
    mesh = _plane(1, 2.0, mirror=False)
    sh = OM.Shading(light=(1.5, 0.0, 1.5), intensity=1.0, albedo=0.8, offset=1e-4)
    P = np.array([-0.5, 0.2, 0.0])
    so = P + np.array([0.0, 0.0, 1e-4])
    so = np.float32(so).astype(np.float64)
    c = so + 0.5 * (np.asarray(sh.light) - so)
    f = lambda a: np.asarray(a, np.float32)
    sc = Scene(f([c]), f([[0.05, 0.05, 0.05]]), f([[1, 0, 0, 0]]), f([0.6]), f([[0.3, 0.3, 0.3]]))
    c = sc.mean[0].astype(np.float64)
    o = np.array([[P[0], P[1], 4.0]])
    d = np.array([[0.0, 0.0, -1.0]])
    res = OM.mesh_forward(sc, mesh, sh, o, d, orc.Params())
    L = np.asarray(sh.light) - so
    nl = (np.asarray(sh.light) - P)
    nl = nl[2] / np.linalg.norm(nl)
    sdir = np.float32(L / np.linalg.norm(L)).astype(np.float64)
    # the shadow ray passes the centre at the distance float32 rounding leaves
    w = c - so
    dist2 = np.dot(w, w) - np.dot(w, sdir) ** 2 / np.dot(sdir, sdir)
    alpha = float(sc.opacity[0]) * np.exp(-0.5 * dist2 / float(sc.scale[0, 0]) ** 2)
    assert alpha == pytest.approx(0.6, rel=1e-4)
    np.testing.assert_allclose(res["shad"]["T"], [1 - alpha], rtol=1e-9)
    np.testing.assert_allclose(res["rgb"][0], 0.8 * nl * (1 - alpha), rtol=1e-6)


def test_shadow_blocked_by_mesh(orc):
    """A triangle between the point and the light turns its direct light off."""
    from oracle import mesh as OM
    pv, pt = M.subdivided_plane(1, 2.0)
    blocker_v = np.array([[-1.0, -1.0, 1.0], [1.0, -1.0, 1.0], [0.0, 1.0, 1.0]])
    mesh = _mesh(np.concatenate([pv, blocker_v]), np.concatenate([pt, [[4, 5, 6]]]), [0, 0, 0])
    sh = OM.Shading(light=(0.0, 0.0, 2.0))
    o = np.array([[0.0, -1.5, 0.5], [1.8, 1.8, 0.5]])
    d = np.array([[0.0, 0.2, -1.0], [0.0, 0.0, -1.0]])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    res = OM.mesh_forward(_far_scene(), mesh, sh, o, d, orc.Params())
    assert res["tri"][0] in (0, 1) and res["tri"][1] in (0, 1)
    assert np.all(res["rgb"][0] == 0.0)  # under the blocker
    P = o[1] + res["t_mesh"][1] * d[1]
    L = np.asarray(sh.light) - P
    assert res["rgb"][1][0] == pytest.approx(0.8 * L[2] / np.linalg.norm(L), rel=1e-6)  # beside it


def _mixed_case(seed):
    sc = scenes.random_scene(seed, 60, box=0.7, flat_frac=0.3, scale_lo=0.06, scale_hi=0.2)
    sc.mean[:, 2] = np.abs(sc.mean[:, 2]) + 0.35
    mesh = M.mirror_mesh(plane_cells=3, plane_half=2.0, sphere_subdiv=1, sphere_radius=0.3,
                         sphere_centre=(0.9, 0.9, 0.3))
    rng = np.random.default_rng(seed + 1)
    tgt = np.column_stack([rng.uniform(-1.0, 1.0, size=(150, 2)), np.zeros(150)])
    o = np.tile([0.2, -2.0, 2.2], (150, 1))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return sc, mesh, np.float32(o).astype(np.float64), np.float32(d).astype(np.float64), rng.normal(size=(150, 3))


@pytest.mark.parametrize("seed", [50])
def test_mesh_adjoint_matches_central_differences(orc, seed):
    """d(sum g . pixel)/dparam of the mixed render: primary, reflection and
    shadow hits all contribute (checked where two step sizes agree)."""
    from oracle import mesh as OM
    sc, mesh, o, d, g = _mixed_case(seed)
    sh = OM.Shading(light=(1.0, -1.0, 3.0))
    p = orc.Params(eps1=1e-4, max_hits=64, bg=(0.3, 0.5, 0.7))
    grads = OM.mesh_backward(sc, mesh, sh, o, d, g, p)
    loss = lambda s2: float(np.sum(OM.mesh_forward(s2, mesh, sh, o, d, p)["rgb"] * g))
    rng = np.random.default_rng(seed + 9)
    checked = 0
    for name in ("mean", "scale", "quat", "opacity", "rgb"):
        base = getattr(sc, name)
        for _ in range(8):
            i = rng.integers(0, sc.n)
            comp = None if name == "opacity" else rng.integers(0, 4 if name == "quat" else 3)
            if name == "scale" and base[i].min() < 1e-3:
                continue
            an = grads[name][i] if comp is None else grads[name][i, comp]
            v0 = float(base[i] if comp is None else base[i, comp])
            ests = []
            for h in (2.0 ** -15, 2.0 ** -16):
                step = h * max(abs(v0), 0.25)
                vals = []
                for sgn in (+1, -1):
                    s2 = sc.copy()
                    a2 = getattr(s2, name)
                    if comp is None:
                        a2[i] = np.float32(v0 + sgn * step)
                        actual = float(a2[i]) - v0
                    else:
                        a2[i, comp] = np.float32(v0 + sgn * step)
                        actual = float(a2[i, comp]) - v0
                    vals.append((loss(s2), actual))
                ests.append((vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1]))
            if abs(ests[0] - ests[1]) > 1e-5 * max(abs(ests[1]), 1e-2):
                continue
            fd = (4 * ests[1] - ests[0]) / 3
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-7), (name, i, comp)
            checked += 1
    assert checked >= 15


def test_mesh_adjoint_has_secondary_contributions(orc):
    """The reflection and shadow paths carry gradient: dropping them changes
    the result (guards against an adjoint that only replays the primary)."""
    from oracle import mesh as OM
    sc, mesh, o, d, g = _mixed_case(51)
    sh = OM.Shading(light=(1.0, -1.0, 3.0))
    p = orc.Params(bg=(0.3, 0.5, 0.7))
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, p)
    assert len(fwd["refl"]["idx"]) > 50 and len(fwd["shad"]["idx"]) > 50
    full = OM.mesh_backward(sc, mesh, sh, o, d, g, p, fwd=fwd)
    bg_bwd = np.where((fwd["tri"] >= 0)[:, None], fwd["shade"], np.float64(p.bg)[None, :])
    prim = orc.render_bwd(sc, o, d, g, p, t_max=fwd["t_mesh"], bg=bg_bwd)
    diff = np.abs(full["mean"] - prim["mean"]).max()
    assert diff > 1e-3 * np.abs(full["mean"]).max()
