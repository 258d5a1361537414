"""Mesh + Gaussian path on the GPU against the FP64 oracle (oracle/mesh.py):
triangle tracing (closest and any hit), the mixed forward render with
reflection and shadow rays, and its adjoint.

Parity protocol: a pixel passes when it is within TOL of the oracle, or of
one of the oracle's rounding-level alternatives of one of its three rays
(primary, reflection, shadow). Rays that pass within 1e-5 (barycentric) of a
triangle edge may take another triangle in float32; they are counted and
capped, not compared."""

import numpy as np
import pytest
import torch

from synthetic import scenes
from synthetic import mesh as M
from synthetic.cameras import circle_cameras, concat_rays
from oracle import oracle as O
from oracle import mesh as OM

pytestmark = pytest.mark.gpu

TOL = 1e-4
REL = 1e-3
EDGE = 1e-5
GROUPS = ("mean", "scale", "quat", "opacity", "rgb")
# binary-exact shading constants, so both sides start from the same values
SHADE = dict(light=(2.0, -2.0, 5.0), intensity=1.0, albedo=0.75, mirror_reflectance=0.75, mirror_diffuse=0.25,
             offset=2.0 ** -13)


def _g():
    import tests._gpu as G
    from paper_2501_19196_amd import renderer as R
    return G, R


def _dev_mesh(R, G, mesh, with_material=True):
    return R.Mesh(G.dev(mesh.verts), G.dev(mesh.tris), G.dev(mesh.mirror) if with_material else None)


def _case(seed=5, n=3000, res=(40, 30), n_cams=2, mesh=None):
    sc = scenes.scene_config5(seed=seed, n=n)
    cams = circle_cameras(n_cams, 6.0, 3.0, res)
    o, d, views = concat_rays(cams)
    mesh = mesh or M.mirror_mesh(plane_cells=10, plane_half=3.0, sphere_subdiv=2)
    return sc, mesh, o, d, [tuple(int(x) for x in v) for v in views]


# ------------------------------------------------------------- tracing only

def test_trace_mesh_closest_matches_oracle():
    print("case trace closest", flush=True)
    G, R = _g()
    mesh = M.mirror_mesh()  # 5000 plane + 5120 sphere triangles
    _, _, o, d, views = _case(res=(64, 48), mesh=mesh)
    rng = np.random.default_rng(7)
    # plus rays from random points in every direction (both faces, inside the sphere)
    o2 = np.float32(rng.uniform(-2, 2, size=(4096, 3)) + [0, 0, 1.0])
    d2 = rng.normal(size=(4096, 3))
    d2 = np.float32(d2 / np.linalg.norm(d2, axis=1, keepdims=True))
    o, d = np.concatenate([o, o2]), np.concatenate([d, d2])
    mbvh = R.build_mesh_bvh(_dev_mesh(R, G, mesh))
    t, tri = R.trace_mesh(mbvh, G.rays_of(o, d))
    torch.cuda.synchronize()
    assert R.read_status(mbvh) == 0
    t, tri = t.cpu().numpy().astype(np.float64), tri.cpu().numpy().astype(np.int64)
    tr, trir, amb = O.mesh_closest(mesh.verts, mesh.tris, o, d, t_eps=0.0, edge=EDGE, want_amb=True)
    ok = ~amb
    print("edge-ambiguous", int(amb.sum()), "of", len(amb), flush=True)
    assert amb.mean() < 0.01
    assert np.array_equal(tri[ok], trir[ok])
    h = ok & (trir >= 0)
    assert h.sum() > 0.3 * len(h)
    np.testing.assert_allclose(t[h], tr[h], rtol=2e-5, atol=2e-6)
    assert np.all(np.isinf(t[ok & (trir < 0)]))


def test_trace_mesh_any_hit_and_limits():
    print("case trace any", flush=True)
    G, R = _g()
    mesh = M.mirror_mesh(plane_cells=12, sphere_subdiv=3)
    rng = np.random.default_rng(8)
    n = 5000
    o = np.float32(rng.uniform(-2, 2, size=(n, 3)) + [0, 0, 1.0])
    d = rng.normal(size=(n, 3))
    d = np.float32(d / np.linalg.norm(d, axis=1, keepdims=True))
    tr, trir, amb = O.mesh_closest(mesh.verts, mesh.tris, o, d, t_eps=0.0, edge=EDGE, want_amb=True)
    limit = np.where(np.isfinite(tr), tr * rng.uniform(0.5, 1.5, size=n), rng.uniform(0.1, 5, size=n))
    limit[:50] = 0.0     # skipped rays
    limit[50:100] = -1.0
    limit = np.float32(limit)
    mbvh = R.build_mesh_bvh(_dev_mesh(R, G, mesh))
    rays = G.rays_of(o, d)
    for any_hit in (0, 1):
        t, tri = R.trace_mesh(mbvh, rays, t_limit=G.dev(limit), any_hit=bool(any_hit))
        torch.cuda.synchronize()
        t, tri = t.cpu().numpy().astype(np.float64), tri.cpu().numpy()
        assert np.all(tri[:100] == -1) and np.all(np.isinf(t[:100]))
        want = trir >= 0
        want &= tr < limit
        near = amb | (np.abs(tr - limit) <= 1e-4 * (1 + np.abs(limit)))
        near[:100] = False
        got = tri >= 0
        assert np.array_equal(got[~near], want[~near]), any_hit
        # every reported hit is a real hit of that triangle inside (0, limit)
        assert np.all((t[got] > 0) & (t[got] < limit[got]))
        if not any_hit:
            ok = ~near & got
            assert np.array_equal(tri[ok], trir[ok])


def test_trace_mesh_empty_rays():
    G, R = _g()
    mesh = M.mirror_mesh(plane_cells=2, sphere_subdiv=0)
    mbvh = R.build_mesh_bvh(_dev_mesh(R, G, mesh))
    t, tri = R.trace_mesh(mbvh, G.rays_of(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32)))
    torch.cuda.synchronize()
    assert t.numel() == 0 and tri.numel() == 0


# --------------------------------------------------------- mixed rendering

def _oracle_mixed(sc, mesh, o, d, op):
    sh = OM.Shading(**SHADE)
    fwd = OM.mesh_forward(sc, mesh, sh, o, d, op)
    return sh, fwd


def _ambiguity(sc, mesh, o, d, op, fwd):
    """Per pixel: edge-ambiguous on any of its rays, and the Gaussian
    alternatives count of each ray set (1 = unambiguous)."""
    n = o.shape[0]
    _, _, amb = O.mesh_closest(mesh.verts, mesh.tris, o, d, t_eps=0.0, edge=EDGE, want_amb=True)
    edge = amb.copy()
    gauss = np.ones(n, bool)
    cnt, _ = O.alternatives_batch(sc, o, d, op, cap=2, t_max=fwd["t_mesh"], bg=fwd["bg_p"])
    gauss &= cnt == 1
    r = fwd["refl"]
    if len(r["idx"]):
        _, _, ar = O.mesh_closest(mesh.verts, mesh.tris, r["origin"], r["dir"], t_eps=0.0, edge=EDGE, want_amb=True)
        edge[r["idx"]] |= ar
        cnt, _ = O.alternatives_batch(sc, r["origin"], r["dir"], op, cap=2, t_max=r["t_max"], bg=r["bg"])
        gauss[r["idx"]] &= cnt == 1
    s = fwd["shad"]
    if len(s["idx"]):
        _, _, as_ = O.mesh_closest(mesh.verts, mesh.tris, s["origin"], s["dir"], t_eps=0.0, edge=EDGE, want_amb=True)
        edge[s["idx"]] |= as_
        cnt, _ = O.alternatives_batch(sc, s["origin"], s["dir"], s["params"], cap=2, t_max=s["t_max"])
        gauss[s["idx"]] &= (cnt == 1) | s["blocked"]
    return edge, gauss


def _explain(gpu, sc, o, d, op, fwd, bad):
    """Indices of `bad` pixels no single-ray alternative explains."""
    rgb = fwd["rgb"]
    cand = {int(k): [] for k in bad}
    # primary: the pixel is a plain render with background = shade term
    bgp = np.where((fwd["tri"] >= 0)[:, None], fwd["shade"], fwd["bg_p"])
    cnt, alts = O.alternatives_batch(sc, o[bad], d[bad], op, t_max=fwd["t_mesh"][bad], bg=bgp[bad])
    for j, k in enumerate(bad):
        cand[int(k)] += list(alts[j, :max(cnt[j], 0)])
    Tp = fwd["T_p"]
    r = fwd["refl"]
    pos = {int(k): j for j, k in enumerate(r["idx"])}
    sel = [pos[int(k)] for k in bad if int(k) in pos]
    if sel:
        sel = np.asarray(sel)
        cnt, alts = O.alternatives_batch(sc, r["origin"][sel], r["dir"][sel], op, t_max=r["t_max"][sel],
                                         bg=r["bg"][sel])
        for j, q in enumerate(sel):
            k = int(r["idx"][q])
            for a in alts[j, :max(cnt[j], 0)]:
                cand[k].append(rgb[k] + Tp[k] * fwd["rho_m"][k] * (a - r["C"][q]))
    s = fwd["shad"]
    pos = {int(k): j for j, k in enumerate(s["idx"])}
    sel = [pos[int(k)] for k in bad if int(k) in pos]
    if sel:
        sel = np.asarray(sel)
        cnt, alts = O.alternatives_batch(sc, s["origin"][sel], s["dir"][sel], s["params"], t_max=s["t_max"][sel])
        for j, q in enumerate(sel):
            k = int(s["idx"][q])
            if s["blocked"][q]:
                continue
            for a in alts[j, :max(cnt[j], 0)]:
                cand[k].append(rgb[k] + Tp[k] * s["w"][q] * (a[0] - s["T"][q]))
    left = []
    for k in bad:
        c = cand[int(k)]
        if not c or np.abs(np.asarray(c) - gpu[k]).max(axis=1).min() > TOL:
            left.append(int(k))
    return left


def _mixed_forward(sc, mesh, o, d, views, p, material=True):
    G, R = _g()
    g = G.gaussians(sc)
    gbvh = R.build_bvh(g, p)
    dm = _dev_mesh(R, G, mesh, material)
    mbvh = R.build_mesh_bvh(dm)
    rays = G.rays_of(o, d, views)
    out, frame = R.render_mesh_fwd(gbvh, mbvh, g, dm, R.Shading(**SHADE), rays, p)
    torch.cuda.synchronize()
    assert R.read_status(gbvh) == 0 and R.read_status(mbvh) == 0
    return out.cpu().numpy().astype(np.float64), (gbvh, mbvh, g, dm, rays, frame)


def _forward_parity(sc, mesh, o, d, views, p, label, material=True):
    G, R = _g()
    op = G.oracle_params(O, p)
    if not material:
        mesh = M.Mesh(mesh.verts, mesh.tris, np.zeros_like(mesh.mirror))
    gpu, ctx = _mixed_forward(sc, mesh, o, d, views, p, material)
    sh, fwd = _oracle_mixed(sc, mesh, o, d, op)
    err = np.abs(gpu - fwd["rgb"]).max(axis=1)
    _, _, amb = O.mesh_closest(mesh.verts, mesh.tris, o, d, t_eps=0.0, edge=EDGE, want_amb=True)
    bad = np.nonzero(err > TOL)[0]
    left = _explain(gpu, sc, o, d, op, fwd, bad) if len(bad) else []
    edge_left = [k for k in left if amb[k]]
    left = [k for k in left if not amb[k]]
    if left:
        # secondary-ray edge decisions
        edge, _ = _ambiguity(sc, mesh, o[left], d[left], op,
                             OM.mesh_forward(sc, mesh, sh, o[left], d[left], op))
        edge_left += [k for k, e in zip(left, edge) if e]
        left = [k for k, e in zip(left, edge) if not e]
    n_hit = int((fwd["tri"] >= 0).sum())
    print(label, "pixels", len(err), "mesh hits", n_hit, "refl", len(fwd["refl"]["idx"]), "shadow",
          len(fwd["shad"]["idx"]), "within", int((err <= TOL).sum()), "edge", len(edge_left), "unresolved", left,
          "max_err_ok", float(err[err <= TOL].max()), flush=True)
    assert n_hit > 0.2 * len(err)
    assert len(edge_left) <= max(2, 0.01 * len(err))
    assert not left
    return gpu, fwd, ctx


def test_mixed_forward_parity():
    print("case mixed fwd", flush=True)
    G, R = _g()
    sc, mesh, o, d, views = _case()
    _forward_parity(sc, mesh, o, d, views, R.Params(bg=(0.25, 0.5, 0.75)), "mixed")


def test_mixed_forward_all_diffuse_and_caps():
    print("case mixed fwd diffuse caps", flush=True)
    G, R = _g()
    sc, mesh, o, d, views = _case(seed=6, n=2000, res=(32, 24))
    _forward_parity(sc, mesh, o, d, views, R.Params(bg=(0.25, 0.5, 0.75)), "diffuse", material=False)
    _forward_parity(sc, mesh, o, d, views, R.Params(max_hits=4, eps1=0.01), "caps")


def test_mixed_forward_bare_mesh_lambert():
    """No Gaussian near any ray: the GPU pixel equals the closed-form shade."""
    print("case mixed bare", flush=True)
    G, R = _g()
    far = scenes.Scene(*(np.float32(a) for a in ([[40, 40, 40]], [[0.01] * 3], [[1, 0, 0, 0]], [0.5], [[1, 1, 1]])))
    _, mesh, o, d, views = _case(res=(32, 24))
    _forward_parity(far, mesh, o, d, views, R.Params(bg=(0.25, 0.5, 0.75)), "bare")


@pytest.mark.parametrize("hit_list", [0, 8, 256])
def test_mixed_gradients(hit_list):
    """Adjoint parity of the mixed render, recomputing or from stored lists
    (a capacity of 8 overflows on many rays, which then re-traverse)."""
    print("case mixed grads", hit_list, flush=True)
    G, R = _g()
    sc, mesh, o, d, views = _case(seed=7, n=2000, res=(32, 24))
    p = R.Params(bg=(0.25, 0.5, 0.75), hit_list=hit_list)
    op = G.oracle_params(O, p)
    sh, fwd = _oracle_mixed(sc, mesh, o, d, op)
    edge, gauss = _ambiguity(sc, mesh, o, d, op, fwd)
    mask = ~edge & gauss
    print("masked", int((~mask).sum()), "of", len(mask), flush=True)
    rng = np.random.default_rng(9)
    grad = np.float32(rng.normal(size=(o.shape[0], 3)) * mask[:, None])
    gpu, (gbvh, mbvh, g, dm, rays, frame) = _mixed_forward(sc, mesh, o, d, views, p)
    gg = R.render_mesh_bwd(gbvh, mbvh, g, dm, R.Shading(**SHADE), rays, p, G.dev(grad), frame)
    torch.cuda.synchronize()
    got = dict(zip(GROUPS, (t.cpu().numpy().astype(np.float64) for t in gg)))
    ref = OM.mesh_backward(sc, mesh, sh, o, d, grad.astype(np.float64), op, fwd=fwd)
    G.assert_elementwise(got, ref, f"mixed lists {hit_list}", REL)
    assert (~mask).mean() <= 0.02, int((~mask).sum())
    # the secondary rays carry part of the gradient
    bg_bwd = np.where((fwd["tri"] >= 0)[:, None], fwd["shade"], np.float64(op.bg)[None, :])
    prim = O.render_bwd(sc, o, d, grad.astype(np.float64), op, t_max=fwd["t_mesh"], bg=bg_bwd)
    assert np.linalg.norm(ref["mean"] - prim["mean"]) > 10 * REL * np.linalg.norm(ref["mean"])


def test_mesh_render_autograd_matches_direct_adjoint():
    print("case mixed autograd", flush=True)
    G, R = _g()
    sc, mesh, o, d, views = _case(seed=8, n=1500, res=(24, 16), n_cams=1)
    p = R.Params()
    dm = _dev_mesh(R, G, mesh)
    mbvh = R.build_mesh_bvh(dm)
    leaves = [G.dev(a).requires_grad_(True) for a in sc.arrays()]
    out = R.MeshRender.apply(*leaves, G.dev(o), G.dev(d), dm, mbvh, R.Shading(**SHADE), p, views)
    rng = np.random.default_rng(10)
    gout = G.dev(np.float32(rng.normal(size=(o.shape[0], 3))))
    (out * gout).sum().backward()
    gpu, (gbvh, mbvh2, g, dm2, rays, frame) = _mixed_forward(sc, mesh, o, d, views, p)
    np.testing.assert_array_equal(out.detach().cpu().numpy(), np.float32(gpu))
    direct = R.render_mesh_bwd(gbvh, mbvh2, g, dm2, R.Shading(**SHADE), rays, p, gout, frame)
    torch.cuda.synchronize()
    for leaf, dref in zip(leaves, direct):
        a, b = leaf.grad.cpu().numpy(), dref.cpu().numpy()
        # the same kernels in the same order; float atomics may reorder sums
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6 * np.abs(b).max())


@pytest.mark.timeout(900)
def test_mesh_workload_full_size_sampled():
    """500k Gaussians plus the 10k-triangle mirror mesh (subdivided plane and
    icosphere), 4 views of 1024x768 rendered in the benchmark's launch (the
    primary, reflection and shadow ray sets in one persistent launch, stored
    hit lists of 64 slots per ray), against the oracle on 4,096 seeded pixels:
    the forward under the mesh protocol, then the adjoint with the upstream
    gradient on those pixels, element by element. Pixels are left out of the
    gradient when a triangle decision is within rounding (edge) or when the
    composited sequence of any of the pixel's rays differs from the oracle's
    (each such pixel must have a Gaussian decision within rounding)."""
    from synthetic import workload
    print("case mesh workload sampled", flush=True)
    G, R = _g()
    w = workload(5)
    sc, mesh = w["scene"], w["mesh"]
    o, d, views = concat_rays(w["cams"])
    views = [tuple(int(x) for x in v) for v in views]
    p = R.Params(bg=(0.25, 0.5, 0.75), hit_list=64)
    op = G.oracle_params(O, p)
    gpu_all, (gbvh, mbvh, g, dm, rays, frame) = _mixed_forward(sc, mesh, o, d, views, p)
    rng = np.random.default_rng(51)
    sel = np.sort(rng.choice(o.shape[0], 4096, replace=False))
    os_, ds = o[sel], d[sel]
    sh, fwd = _oracle_mixed(sc, mesh, os_, ds, op)
    gpu = gpu_all[sel]
    # forward parity (mesh protocol)
    err = np.abs(gpu - fwd["rgb"]).max(axis=1)
    bad = np.nonzero(err > TOL)[0]
    left = _explain(gpu, sc, os_, ds, op, fwd, bad) if len(bad) else []
    edge, _ = _ambiguity(sc, mesh, os_, ds, op, fwd)
    unexplained = [k for k in left if not edge[k]]
    print("mesh workload: pixels", len(sel), "mesh hits", int((fwd["tri"] >= 0).sum()), "within", int((~(err > TOL)).sum()),
          "resolved", len(bad) - len(left), "edge", int(edge.sum()), "unexplained", unexplained, flush=True)
    assert not unexplained
    assert edge.mean() <= 0.01
    # the composited sequence of every ray set against the oracle's
    shade = R.Shading(**SHADE)
    n = len(sel)
    diff = np.zeros(n, bool)
    seqs = [(0, np.arange(n), O.render_lists(sc, os_, ds, op, cap=64, t_max=fwd["t_mesh"]))]
    r = fwd["refl"]
    if len(r["idx"]):
        seqs.append((1, r["idx"], O.render_lists(sc, r["origin"], r["dir"], op, cap=64, t_max=r["t_max"])))
    s = fwd["shad"]
    if len(s["idx"]):
        keep = ~s["blocked"]
        ids_s, L_s = O.render_lists(sc, s["origin"], s["dir"], s["params"], cap=64, t_max=s["t_max"])
        seqs.append((2, s["idx"][keep], (ids_s[keep], L_s[keep])))
    for ray_set, idx, (ids_o, L_o) in seqs:
        got = R.mesh_hit_lists(rays, p, shade, frame, ray_set, cap=64, select=sel)
        assert np.array_equal(got["stored"], got["count"])
        want_ids = np.full((n, 64), -1, np.int64)
        want_L = np.zeros(n, np.int64)
        want_ids[idx], want_L[idx] = ids_o, L_o
        d_set = (got["count"] != want_L) | np.any(got["ids"] != want_ids, axis=1)
        print("ray set", ray_set, "rays", len(idx), "differing", int(d_set.sum()), flush=True)
        if ray_set == 0 and (d_set & ~edge).any():
            # a camera ray whose sequence differs has a Gaussian decision within rounding
            k = np.nonzero(d_set & ~edge)[0]
            amb, _ = O.alternatives_batch(sc, os_[k], ds[k], op, cap=2, t_max=fwd["t_mesh"][k])
            assert np.all(amb != 1), k[amb == 1]
        diff |= d_set
    masked = diff | edge
    print("left out of the gradient:", int(masked.sum()), "of", n, flush=True)
    assert diff.mean() <= 0.02, int(diff.sum())
    rng2 = np.random.default_rng(52)
    gsel = np.float32(rng2.normal(size=(n, 3))) * (~masked)[:, None]
    grad = np.zeros((o.shape[0], 3), np.float32)
    grad[sel] = gsel
    gg = R.render_mesh_bwd(gbvh, mbvh, g, dm, shade, rays, p, G.dev(grad), frame)
    torch.cuda.synchronize()
    assert R.read_status(gbvh) == 0
    got = dict(zip(GROUPS, (t.cpu().numpy().astype(np.float64) for t in gg)))
    ref = OM.mesh_backward(sc, mesh, sh, os_, ds, gsel.astype(np.float64), op, fwd=fwd)
    G.assert_elementwise(got, ref, "mesh workload 4096 px", REL)
