"""Launch forms: many views in one launch, persistent queues, packet tile
shapes, the autotuner and HIP-graph capture of a whole training step. None of
them may change a rendered value; gradients may differ only by the order of
float atomics."""

import numpy as np
import pytest
import torch

from synthetic import scenes
from synthetic.cameras import fibonacci_cameras, concat_rays, circle_cameras
from synthetic import mesh as M

pytestmark = pytest.mark.gpu

GROUPS = ("mean", "scale", "quat", "opacity", "rgb")


def _g():
    import tests._gpu as G
    from paper_2501_19196_amd import renderer as R
    return G, R


def _multiview(n=20000):
    sc = scenes.scene_config3(seed=3, n=n)
    res = [(72, 56)] * 4 + [(37, 29)] * 4  # uneven sizes, ragged tiles
    cams = fibonacci_cameras(8, 4.0, res)
    o, d, views = concat_rays(cams)
    return sc, o, d, [tuple(int(x) for x in v) for v in views]


def _grads_close(a, b, rel=1e-5):
    for x, y in zip(a, b):
        x, y = x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
        den = np.linalg.norm(y)
        assert np.linalg.norm(x - y) <= rel * max(den, 1e-30), (np.linalg.norm(x - y), den)


def test_batched_views_equal_per_view_launches():
    print("case batched vs per-view", flush=True)
    G, R = _g()
    sc, o, d, views = _multiview()
    g = G.gaussians(sc)
    p = R.Params()
    bvh = R.build_bvh(g, p)
    rng = np.random.default_rng(0)
    grad = G.dev(np.float32(rng.normal(size=(o.shape[0], 3))))
    per_out, per_grads = [], None
    for off, w, h in views:
        sl = slice(off, off + w * h)
        rays = G.rays_of(o[sl], d[sl], [(0, w, h)])
        out, state = R.render_fwd(bvh, g, rays, p)
        gg = R.render_bwd(bvh, g, rays, p, grad[sl], state)
        per_out.append(out)
        per_grads = [t.clone() for t in gg] if per_grads is None else [a + b for a, b in zip(per_grads, gg)]
    per_out = torch.cat(per_out).cpu().numpy()
    rays = G.rays_of(o, d, views)
    for flags in (0, 2):
        for tw in (4, 8, 16, 32):
            q = R.Params(flags=flags, tile_width=tw)
            out, state = R.render_fwd(bvh, g, rays, q)
            np.testing.assert_array_equal(out.cpu().numpy(), per_out, err_msg=f"flags {flags} tile {tw}")
            gg = R.render_bwd(bvh, g, rays, q, grad, state)
            _grads_close(gg, per_grads)
    torch.cuda.synchronize()
    assert R.read_status(bvh) == 0


@pytest.mark.parametrize("hit_list", [0, 64])
def test_autotune_picks_a_listed_candidate_with_identical_output(hit_list):
    print("case autotune", hit_list, flush=True)
    G, R = _g()
    sc, o, d, views = _multiview(8000)
    g = G.gaussians(sc)
    p = R.Params(hit_list=hit_list)
    bvh = R.build_bvh(g, p)
    rays = G.rays_of(o, d, views)
    ref, state = R.render_fwd(bvh, g, rays, p)
    rng = np.random.default_rng(1)
    grad = G.dev(np.float32(rng.normal(size=(o.shape[0], 3))))
    ref_g = [t.clone() for t in R.render_bwd(bvh, g, rays, p, grad, state)]
    pf, pb, rows = R.autotune(bvh, g, rays, p, grad_rgb=grad, reps=1)
    print("autotune", pf, pb, flush=True)
    assert len(rows) == 20
    assert all(r["ms_fwd"] > 0 and r["ms_bwd"] > 0 for r in rows)
    best_f = min(rows, key=lambda r: r["ms_fwd"])
    assert (pf.kbuf, bool(pf.flags & 2), pf.tile_width) == (best_f["kbuf"], best_f["persistent"],
                                                            best_f["tile_width"])
    best_b = min(rows, key=lambda r: r["ms_bwd"])
    assert (pb.kbuf, bool(pb.flags & 2), pb.tile_width) == (best_b["kbuf"], best_b["persistent"],
                                                            best_b["tile_width"])
    assert pf.Q == p.Q and pf.eps1 == p.eps1 and pf.max_hits == p.max_hits and pf.hit_list == p.hit_list
    out, state2 = R.render_fwd(bvh, g, rays, pf)
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    _grads_close(R.render_bwd(bvh, g, rays, pb, grad, state2), ref_g)
    # forward-only tuning leaves bwd = fwd; rays without views try one tile shape
    pf2, pb2, rows2 = R.autotune(bvh, g, G.rays_of(o, d), p, reps=1)
    assert len(rows2) == 10 and pb2 == pf2 and all(r["ms_bwd"] == 0 for r in rows2)


@pytest.mark.parametrize("hit_list", [0, 128])
def test_graph_captured_training_step_replays_match_eager(hit_list):
    """Capture BVH rebuild + forward + L1 gradient + adjoint in one HIP graph;
    replays (with eager work and parameter updates in between) equal the eager
    step: forward bitwise, gradients to atomic-order rounding."""
    print("case graph step", hit_list, flush=True)
    G, R = _g()
    sc, o, d, views = _multiview(20000)
    g = G.gaussians(sc)
    p = R.Params(hit_list=hit_list)
    rays = G.rays_of(o, d, views)
    n, nr = sc.n, o.shape[0]
    ws = torch.empty(R.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    out = torch.empty((nr, 3), device="cuda")
    state = R.new_state(nr, p)
    grads = tuple(torch.empty_like(t) for t in (g.mean, g.scale, g.quat, g.opacity, g.rgb))
    target = torch.rand((nr, 3), device="cuda")

    held = {}

    def step():
        bvh = R.build_bvh(g, p, workspace=ws)
        R.render_fwd(bvh, g, rays, p, out=out, state=state)
        gr = torch.sign(out - target) * (1.0 / (3.0 * nr))
        R.render_bwd(bvh, g, rays, p, gr, state, grads=grads)
        held["bvh"] = bvh

    def eager():
        e_ws = torch.empty_like(ws)
        bvh = R.build_bvh(g, p, workspace=e_ws)
        o_, s_ = R.render_fwd(bvh, g, rays, p)
        gr = torch.sign(o_ - target) * (1.0 / (3.0 * nr))
        return o_, [t.clone() for t in R.render_bwd(bvh, g, rays, p, gr, s_)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for rep in range(4):
        if rep >= 2:  # an optimiser-like in-place update the graph must see
            with torch.no_grad():
                g.mean.add_(G.dev(np.float32(rng.normal(scale=1e-3, size=(n, 3)))))
                g.opacity.mul_(0.99)
        ref_out, ref_g = eager()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref_out.cpu().numpy(), err_msg=f"replay {rep}")
        _grads_close(grads, ref_g)
        # the status word of the replayed step's own workspace (the build clears it, the
        # render and adjoint of the same step set it): read without rebuilding
        assert R.read_status(held["bvh"]) == 0, f"replay {rep}"


def test_graph_captured_mesh_step_replays_match_eager():
    print("case graph mesh step", flush=True)
    G, R = _g()
    sc = scenes.scene_config5(seed=5, n=3000)
    cams = circle_cameras(2, 6.0, 3.0, (40, 30))
    o, d, views = concat_rays(cams)
    views = [tuple(int(x) for x in v) for v in views]
    mesh = M.mirror_mesh(plane_cells=10, sphere_subdiv=2)
    g = G.gaussians(sc)
    p = R.Params()
    dm = R.Mesh(G.dev(mesh.verts), G.dev(mesh.tris), G.dev(mesh.mirror))
    mbvh = R.build_mesh_bvh(dm)
    sh = R.Shading()
    rays = G.rays_of(o, d, views)
    nr = o.shape[0]
    ws = torch.empty(R.workspace_bytes(sc.n), dtype=torch.uint8, device="cuda")
    out = torch.empty((nr, 3), device="cuda")
    frame = R.mesh_frame(nr)
    grads = tuple(torch.empty_like(t) for t in (g.mean, g.scale, g.quat, g.opacity, g.rgb))
    gout = G.dev(np.float32(np.random.default_rng(3).normal(size=(nr, 3))))

    def step():
        bvh = R.build_bvh(g, p, workspace=ws)
        R.render_mesh_fwd(bvh, mbvh, g, dm, sh, rays, p, out=out, frame=frame)
        R.render_mesh_bwd(bvh, mbvh, g, dm, sh, rays, p, gout, frame, grads=grads)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        bvh = R.build_bvh(g, p)
        ref_out, fr = R.render_mesh_fwd(bvh, mbvh, g, dm, sh, rays, p)
        ref_g = [t.clone() for t in R.render_mesh_bwd(bvh, mbvh, g, dm, sh, rays, p, gout, fr)]
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref_out.cpu().numpy(), err_msg=f"replay {rep}")
        _grads_close(grads, ref_g)
