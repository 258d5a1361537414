"""Pins of the multi-bounce / glass part of the mesh oracle (oracle/mesh.py)
against facts it does not compute itself: Snell's law, reversibility and the
Fresnel limits of the glass continuation; index-matched glass leaves a render
unchanged; a ray through a tilted glass slab leaves parallel to itself,
shifted by the textbook lateral displacement; a two-mirror periscope gives
rho^2 times a plain render along the final ray; central differences of the
chain adjoint. CPU only."""

import numpy as np
import pytest

from oracle import mesh as OM
from synthetic import mesh as M
from synthetic import scenes
from synthetic.scenes import Scene


def _mesh(verts, tris, mat):
    return M.Mesh(np.ascontiguousarray(np.asarray(verts, np.float32)), np.ascontiguousarray(np.asarray(tris, np.int32)),
                  np.ascontiguousarray(np.asarray(mat, np.int32)))


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def test_glass_continuation_snell_reversibility_fresnel():
    rng = np.random.default_rng(0)
    ior = 1.5
    n_g = np.tile([0.0, 0.0, 1.0], (500, 1))
    # entering from above (d.n_g < 0)
    th = rng.uniform(0.0, 1.45, size=500)
    ph = rng.uniform(0, 2 * np.pi, size=500)
    d = np.column_stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), -np.cos(th)])
    t, side, w, n = OM.glass_continuation(d, n_g, ior)
    np.testing.assert_allclose(np.linalg.norm(t, axis=1), 1.0, atol=1e-12)
    sin_i = np.linalg.norm(np.cross(d, n_g), axis=1)
    sin_t = np.linalg.norm(np.cross(t, n_g), axis=1)
    np.testing.assert_allclose(sin_i, ior * sin_t, atol=1e-12)
    assert np.all(side == -1) and np.all(t[:, 2] < 0)  # continues below the surface
    # reversibility: leaving along -t through the same surface gives -d
    t2, side2, w2, _ = OM.glass_continuation(-t, n_g, ior)
    np.testing.assert_allclose(t2, -d, atol=1e-12)
    np.testing.assert_allclose(w2, w, atol=1e-12)  # Schlick on the thinner side: same weight both ways
    # normal incidence: straight through, weight 1 - ((1 - ior) / (1 + ior))^2 = 0.96
    t3, _, w3, _ = OM.glass_continuation([[0.0, 0.0, -1.0]], [[0.0, 0.0, 1.0]], ior)
    np.testing.assert_allclose(t3, [[0.0, 0.0, -1.0]], atol=1e-15)
    assert w3[0] == pytest.approx(0.96, abs=1e-15)
    # grazing incidence: the transmitted weight goes to 0
    tg, _, wg, _ = OM.glass_continuation([_unit([1.0, 0.0, -1e-6])], [[0.0, 0.0, 1.0]], ior)
    assert wg[0] < 1e-5
    # total internal reflection leaving beyond the critical angle (sin > 1 / ior)
    thc = np.arcsin(1 / ior) + 0.05
    dl = np.array([[np.sin(thc), 0.0, np.cos(thc)]])  # inside, towards the surface (d.n_g > 0)
    tt, st, wt, nt = OM.glass_continuation(dl, [[0.0, 0.0, 1.0]], ior)
    np.testing.assert_allclose(tt, [[np.sin(thc), 0.0, -np.cos(thc)]], atol=1e-15)
    assert st[0] == 1 and wt[0] == 1.0


def _box_mesh(lo, hi, mat):
    v, t = M.box(lo, hi)
    return _mesh(v, t, np.full(len(t), mat))


def _scene_around(seed, n, box=(1.5, 1.5, 3.0)):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1, 1, size=(n, 3)) * np.asarray(box)
    sc = scenes.random_scene(seed, n, box=1.0)
    return Scene(np.float32(mean), sc.scale, sc.quat, sc.opacity, sc.rgb)


def test_index_matched_glass_is_invisible(orc):
    """A closed glass box of ior 1 hit at normal incidence passes every ray
    straight on with weight 1 (Schlick's R0 = 0): with no per-segment
    threshold (eps1 = 0, K_max unbounded) the chain renders what a plain
    render without the mesh renders."""
    mesh = _box_mesh((-1.2, -1.2, -1.0), (1.2, 1.2, 1.0), OM.GLASS)
    sc = _scene_around(1, 400)
    xs = np.linspace(-1.0, 1.0, 12)
    X, Y = np.meshgrid(xs, xs)
    o = np.column_stack([X.ravel() + 0.013, Y.ravel() - 0.007, np.full(X.size, 4.0)])
    d = np.tile([0.0, 0.0, -1.0], (len(o), 1))
    p = orc.Params(eps1=0.0, max_hits=0, bg=(0.2, 0.4, 0.6))
    sh = OM.Shading(max_bounces=2, ior=1.0, offset=1e-6)
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, p)
    assert len(fwd["levels"]) == 3 and len(fwd["levels"][2]["idx"]) == len(o)
    ref, _, _ = orc.render_fwd(sc, np.float32(o), np.float32(d), p)
    np.testing.assert_allclose(fwd["rgb"], ref, atol=1e-5)
    assert np.abs(ref - np.asarray(p.bg)).max() > 0.1  # the Gaussians are visible


def test_tilted_slab_lateral_displacement(orc):
    """Through a glass slab of thickness h at incidence theta the ray leaves
    parallel to itself, displaced by h sin(theta - theta_t) / cos(theta_t)."""
    h = 0.5
    mesh = _box_mesh((-50.0, -50.0, -h), (50.0, 50.0, 0.0), OM.GLASS)
    ior = 1.5
    th = np.deg2rad([10.0, 30.0, 50.0])
    d = np.column_stack([np.sin(th), np.zeros(3), -np.cos(th)])
    o = np.column_stack([np.zeros(3), np.zeros(3), np.full(3, 2.0)])
    sh = OM.Shading(max_bounces=2, ior=ior, offset=1e-7)
    fwd = OM.mesh_forward(Scene(*(np.float32(a) for a in ([[90, 90, 90]], [[0.01] * 3], [[1, 0, 0, 0]], [0.5],
                                                            [[1, 1, 1]]))), mesh, sh, o, d, orc.Params())
    l2 = fwd["levels"][2]
    assert len(l2["idx"]) == 3
    np.testing.assert_allclose(_unit(l2["dir"]), d, atol=1e-6)
    tht = np.arcsin(np.sin(th) / ior)
    want = h * np.sin(th - tht) / np.cos(tht)
    # distance of the exit point from the incoming line
    got = np.linalg.norm(np.cross(l2["origin"] - o, d), axis=1)
    np.testing.assert_allclose(got, want, atol=2e-5)
    # two interfaces, each transmitting 1 - F
    w = fwd["levels"][0]["w"] * fwd["levels"][1]["w"]
    assert np.all((w > 0.8) & (w < 1.0))


def _square(centre, u, v, half):
    c, u, v = (np.asarray(x, np.float64) for x in (centre, u, v))
    p = [c - half * u - half * v, c + half * u - half * v, c + half * u + half * v, c - half * u + half * v]
    return np.asarray(p), np.asarray([(0, 1, 2), (0, 2, 3)])


def test_periscope_two_mirrors(orc):
    """Rays along +x hit a 45-degree mirror at x = 0 (to +y), then one at
    y = 3 (back to +x): with no diffuse part and no Gaussians on the first two
    legs, the pixel is rho^2 times a plain render along the final leg."""
    s2 = np.sqrt(0.5)
    v1, t1 = _square((0.0, 0.0, 0.0), (s2, s2, 0.0), (0.0, 0.0, 1.0), 1.0)
    v2, t2 = _square((0.0, 3.0, 0.0), (s2, s2, 0.0), (0.0, 0.0, 1.0), 1.0)
    mesh = _mesh(np.concatenate([v1, v2]), np.concatenate([t1, t2 + 4]), np.ones(4, np.int32))
    rng = np.random.default_rng(3)
    n = 300
    mean = np.column_stack([rng.uniform(1.5, 6.0, n), 3.0 + rng.uniform(-0.4, 0.4, n), rng.uniform(-0.4, 0.4, n)])
    base = scenes.random_scene(3, n, box=1.0, scale_lo=0.05, scale_hi=0.2)
    sc = Scene(np.float32(mean), base.scale, base.quat, base.opacity, base.rgb)
    zs = np.linspace(-0.3, 0.3, 7)
    o = np.column_stack([np.full(7, -5.0), np.zeros(7), zs])
    d = np.tile([1.0, 0.0, 0.0], (7, 1))
    rho = 0.75
    sh = OM.Shading(max_bounces=2, mirror_reflectance=rho, mirror_diffuse=0.0, offset=1e-6)
    p = orc.Params(bg=(0.1, 0.2, 0.3))
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, p)
    # the final leg starts on the second mirror and runs along +x
    of = np.column_stack([np.zeros(7), np.full(7, 3.0), zs])
    ref, _, _ = orc.render_fwd(sc, np.float32(of), np.float32(d), p)
    np.testing.assert_allclose(fwd["rgb"], rho * rho * ref, atol=2e-5)
    assert np.abs(ref - np.asarray(p.bg)).max() > 0.05


def _chain_case(seed):
    sc = scenes.random_scene(seed, 250, box=1.0, scale_lo=0.03, scale_hi=0.12)
    sc.mean[:, 2] = np.abs(sc.mean[:, 2]) + 0.35
    mesh = M.glass_mesh(plane_cells=3, plane_half=2.0, sphere_subdiv=1, sphere_radius=0.35,
                        sphere_centre=(0.1, 0.2, 0.7), box_lo=(0.6, -1.0, 0.1), box_hi=(1.2, -0.4, 0.8))
    rng = np.random.default_rng(seed + 1)
    tgt = np.column_stack([rng.uniform(-1.0, 1.2, size=(150, 2)), rng.uniform(0.0, 0.6, size=150)])
    o = np.tile([0.2, -2.5, 2.0], (150, 1))
    d = _unit(tgt - o)
    return sc, mesh, np.float32(o).astype(np.float64), np.float32(d).astype(np.float64), rng.normal(size=(150, 3))


@pytest.mark.parametrize("bounces", [2, 3])
def test_chain_adjoint_matches_central_differences(orc, bounces):
    """d(sum g . pixel)/dparam through glass refractions, mirror bounces and
    shadow rays (checked where two step sizes agree)."""
    sc, mesh, o, d, g = _chain_case(60 + bounces)
    sh = OM.Shading(light=(1.0, -1.0, 3.0), max_bounces=bounces)
    p = orc.Params(eps1=1e-4, max_hits=64, bg=(0.3, 0.5, 0.7))
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, p)
    assert len(fwd["levels"]) == bounces + 1
    deep = fwd["levels"][-1]
    assert len(deep["idx"]) > 5  # some pixels reach the last level
    grads = OM.mesh_backward(sc, mesh, sh, o, d, g, p, fwd=fwd)
    loss = lambda s2: float(np.sum(OM.mesh_forward(s2, mesh, sh, o, d, p)["rgb"] * g))
    rng = np.random.default_rng(bounces)
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
            for hstep in (2.0 ** -15, 2.0 ** -16):
                step = hstep * max(abs(v0), 0.25)
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


def test_single_bounce_chain_is_the_mirror_model(orc):
    """max_bounces = 1 keeps the primary / reflection / shadow model: the
    reflection level sees Gaussians up to its own triangle, then black."""
    sc, mesh, o, d, _ = _chain_case(70)
    mesh = M.Mesh(mesh.verts, mesh.tris, np.where(mesh.mirror == 2, 0, mesh.mirror).astype(np.int32))
    sh = OM.Shading(light=(1.0, -1.0, 3.0), max_bounces=1)
    p = orc.Params(bg=(0.3, 0.5, 0.7))
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, p)
    r = fwd["refl"]
    assert len(r["idx"]) > 20
    hit = fwd["tri"] >= 0
    # pixel = C_p + T_p (rho_m C_r + D) on mesh hits
    want = fwd["C_p"].copy()
    shade = np.zeros_like(want)
    shade[r["idx"]] += fwd["rho_m"][r["idx"], None] * r["C"]
    s = fwd["shad"]
    shade[s["idx"]] += (s["w"] * s["T"])[:, None]
    want[hit] += fwd["T_p"][hit, None] * shade[hit]
    np.testing.assert_allclose(fwd["rgb"], want, rtol=1e-12, atol=1e-14)
