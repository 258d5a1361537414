"""Adjoint parity: GPU gradients (back-to-front replay from stored lists or by
re-traversal, wave-aggregated atomics) against the FP64 oracle adjoint, which
is itself pinned by central differences.

Every comparison is element by element: for each parameter group and every
entry, |g_gpu - g_oracle| <= 1e-3 |g_oracle| + 1e-3 max |g_oracle|.

A float32 renderer may legitimately composite a different hit sequence than
the FP64 oracle where a decision sits within rounding (a near-tangent ray, two
hits at nearly the same depth, T next to eps1). Such a pixel's gradient is that
of another valid sequence, so it is left out on both sides. Which pixels are
left out is decided by comparing the GPU's composited sequence (its stored hit
list) with the oracle's: every pixel that differs must be one the oracle flags
as within rounding of a decision, and at most 1 % may differ."""

import dataclasses

import numpy as np
import pytest
import torch

from synthetic import scenes, workload
from synthetic.cameras import look_at_camera, pinhole_rays
from oracle import oracle as O

pytestmark = pytest.mark.gpu

REL = 1e-3
GROUPS = ("mean", "scale", "quat", "opacity", "rgb")
MAX_DIFFERING = 0.01  # fraction of pixels whose GPU hit sequence may differ from the oracle's


def _g():
    import tests._gpu as G
    from paper_2501_19196_amd import renderer as R
    return G, R


def _differing_pixels(sc, o, d, p, label, cap=512, t_max=None, bg=None):
    """Pixels whose GPU composited sequence differs from the oracle's; checks
    that each of them is within rounding of a decision and that they are few."""
    G, R = _g()
    op = G.oracle_params(O, p)
    ids_g, cnt_g = G.sequences(sc, o, d, p, cap=cap, t_max=t_max, bg=bg)
    ids_o, L_o = O.render_lists(sc, o, d, op, cap=cap, t_max=t_max, bg=bg)
    diff = (cnt_g != L_o) | np.any(ids_g != ids_o, axis=1)
    n = len(diff)
    if diff.any():
        amb, _ = O.alternatives_batch(sc, o[diff], d[diff], op, max_events=3, cap=2)
        assert np.all(amb != 1), f"{label}: {int((amb == 1).sum())} pixels differ with no decision within rounding"
    print(label, "pixels whose hit sequence differs:", int(diff.sum()), "of", n, flush=True)
    assert diff.sum() <= max(MAX_DIFFERING * n, 1), (int(diff.sum()), n)
    return diff


def _assert_elementwise(got, ref, label, rel=REL):
    G, _ = _g()
    G.assert_elementwise(got, ref, label, rel)


def _grads_gpu(R, bvh, g, rays, p, grad, state):
    gg = R.render_bwd(bvh, g, rays, p, grad if torch.is_tensor(grad) else torch.from_numpy(np.float32(grad)).cuda(),
                      state)
    torch.cuda.synchronize()
    assert R.read_status(bvh) == 0
    return dict(zip(GROUPS, (t.cpu().numpy().astype(np.float64) for t in gg)))


def _grad_parity(sc, o, d, grad, p, views=None, label=""):
    """Element-wise parity of the adjoint for the upstream gradient `grad` over
    the rays (o, d) rendered with params p (and views)."""
    G, R = _g()
    op = G.oracle_params(O, p)
    diff = _differing_pixels(sc, o, d, p, label)
    grad = np.float32(grad * (~diff)[:, None])
    out, state, status, (bvh, g, rays) = G.render(sc, o, d, p, views=views)
    assert status == 0
    got = _grads_gpu(R, bvh, g, rays, p, grad, state)
    ref = O.render_bwd(sc, o, d, grad.astype(np.float64), op)
    _assert_elementwise(got, ref, label)
    return got, ref


def test_tiny_scene_gradients():
    print("case tiny grads", flush=True)
    G, R = _g()
    sc = scenes.random_scene(40, 48, box=0.6, scale_lo=0.05, scale_hi=0.25)
    cam = look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 24, 20, fov_y_deg=30)
    o, d = pinhole_rays(cam)
    rng = np.random.default_rng(1)
    for hit_list in (0, 64):
        _grad_parity(sc, o, d, rng.normal(size=(o.shape[0], 3)),
                     R.Params(bg=(0.1, 0.2, 0.3), max_hits=64, hit_list=hit_list), views=[(0, 24, 20)],
                     label=f"tiny lists {hit_list}")


@pytest.mark.parametrize("n,hit_list", [(1, 0), (1, 64), (3, 64), (3, 0)])
def test_one_gaussian_per_packet_gradients(n, hit_list):
    """Large Gaussians covering the whole view: every lane of a packet holds the
    same Gaussian at a step, the largest groups of the wave aggregation (and,
    for n = 1, a BVH whose root is a leaf)."""
    print("case big groups", n, hit_list, flush=True)
    G, R = _g()
    sc = scenes.random_scene(60 + n, n, box=0.1, scale_lo=0.8, scale_hi=1.2)
    cam = look_at_camera((0, 0, -4), (0, 0, 0), (0, 1, 0), 16, 16, fov_y_deg=20)
    o, d = pinhole_rays(cam)
    rng = np.random.default_rng(2)
    _, ref = _grad_parity(sc, o, d, rng.normal(size=(o.shape[0], 3)), R.Params(bg=(0.1, 0.2, 0.3), hit_list=hit_list),
                          views=[(0, 16, 16)], label="big groups")
    assert np.linalg.norm(ref["mean"]) > 0


@pytest.mark.parametrize("hit_list", [0, 512])
def test_config1_gradients(hit_list):
    print("case config1 grads", hit_list, flush=True)
    G, R = _g()
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    rng = np.random.default_rng(2)
    _grad_parity(w["scene"], o, d, rng.normal(size=(o.shape[0], 3)), R.Params(hit_list=hit_list), views=views,
                 label=f"config1 lists {hit_list}")


@pytest.mark.parametrize("hit_list", [0, 96])
def test_near_opaque_scene_gradients(hit_list):
    """Every opacity in [0.95, 0.999]: T falls by 20 to 1000 per hit, the regime
    where a front-to-back form that divides by 1 - alpha loses its digits."""
    print("case near-opaque grads", hit_list, flush=True)
    G, R = _g()
    sc = scenes.random_scene(80, 2000, box=0.9, flat_frac=0.3, scale_lo=0.03, scale_hi=0.15)
    rng = np.random.default_rng(81)
    sc.opacity[:] = np.float32(rng.uniform(0.95, 0.999, size=sc.n))
    cam = look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 48, 40, fov_y_deg=40)
    o, d = pinhole_rays(cam)
    for eps1 in (1e-4, 0.0):
        p = R.Params(hit_list=hit_list, eps1=eps1, max_hits=0 if eps1 == 0.0 else 512)
        _grad_parity(sc, o, d, rng.normal(size=(o.shape[0], 3)), p, views=[(0, 48, 40)],
                     label=f"near-opaque lists {hit_list} eps1 {eps1}")


@pytest.mark.parametrize("hit_list", [0, 64])
@pytest.mark.parametrize("eps1", [0.0, 1e-4])
def test_fully_opaque_hit_regression(hit_list, eps1):
    """Opacity exactly 1 on a ray through the mean: alpha = 1, T becomes 0.
    With eps1 = 0 and no K_max the ray keeps compositing hits whose T is 0; the
    gradient of the opaque hit still sees the colour behind it, and the hits in
    front of it get the T they had (the forward saves T where it reaches 0).
    Every value stays finite and equals the oracle's."""
    print("case opacity 1", hit_list, eps1, flush=True)
    G, R = _g()
    z = np.float32([-1.0, 0.0, 1.0, 2.0])
    # anisotropic and rotated, so every parameter group has a gradient (an isotropic
    # Gaussian's quaternion gradient is exactly zero)
    q = np.float32([[0.9, 0.2, -0.3, 0.1], [0.7, -0.4, 0.5, 0.2], [0.8, 0.1, 0.1, -0.5], [0.6, 0.3, 0.6, 0.4]])
    sc = scenes.Scene(np.float32([[0.0, 0.0, zz] for zz in z]),
                      np.float32([[0.3, 0.22, 0.35], [0.25, 0.4, 0.3], [0.2, 0.3, 0.28], [0.33, 0.26, 0.4]]), q,
                      np.float32([0.5, 1.0, 0.6, 0.7]),
                      np.float32([[0.9, 0.1, 0.2], [0.2, 0.8, 0.3], [0.1, 0.2, 0.9], [0.5, 0.5, 0.1]]))
    # rays through the means (alpha exactly 1 at the opaque one) and slightly off them
    offs = np.float32([[0.0, 0.0], [1e-5, 0.0], [0.02, -0.01], [0.05, 0.05], [0.1, 0.0], [-0.12, 0.07]])
    o = np.float32([[x, y, -3.0] for x, y in offs])
    d = np.float32([[0.0, 0.0, 1.0]] * len(offs))
    p = R.Params(hit_list=hit_list, eps1=eps1, max_hits=0, bg=(0.25, 0.5, 0.75))
    op = G.oracle_params(O, p)
    out, state, status, (bvh, g, rays) = G.render(sc, o, d, p)
    assert status == 0
    ref, T, L = O.render_fwd(sc, o, d, op)
    assert T[0] == 0.0 and L[0] == (4 if eps1 == 0.0 else 2)
    assert np.abs(out - ref).max() <= 1e-5
    rng = np.random.default_rng(90)
    grad = np.float32(rng.normal(size=(len(offs), 3)))
    got = _grads_gpu(R, bvh, g, rays, p, grad, state)
    refg = O.render_bwd(sc, o, d, grad.astype(np.float64), op)
    for k in GROUPS:
        assert np.all(np.isfinite(got[k])), k
    _assert_elementwise(got, refg, f"opacity 1 lists {hit_list} eps1 {eps1}")
    # the opaque Gaussian's opacity gradient sees the colour behind it (not 0/0)
    assert abs(refg["opacity"][1]) > 1e-3


@pytest.mark.parametrize("max_hits,eps1", [(3, 1e-4), (0, 0.0), (512, 0.3)])
def test_gradients_under_caps(max_hits, eps1):
    print("case grads caps", max_hits, eps1, flush=True)
    G, R = _g()
    sc = scenes.scene_config1()
    cam = look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 32, 32)
    o, d = pinhole_rays(cam)
    rng = np.random.default_rng(3)
    for hit_list in (0, 48):
        _grad_parity(sc, o, d, rng.normal(size=(o.shape[0], 3)),
                     R.Params(max_hits=max_hits, eps1=eps1, hit_list=hit_list), views=[(0, 32, 32)],
                     label=f"caps {max_hits} {eps1} lists {hit_list}")


def test_autograd_function_matches_adjoint():
    print("case autograd", flush=True)
    G, R = _g()
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    sc = w["scene"]
    params = [G.dev(a).requires_grad_(True) for a in sc.arrays()]
    p = R.Params(raise_on_status=True)
    out = R.render(*params, G.dev(o), G.dev(d), p, views)
    loss = out.abs().mean()
    loss.backward()
    torch.cuda.synchronize()
    grad = np.float32(np.sign(out.detach().cpu().numpy()) / out.numel())
    # the same adjoint called directly through the C ABI
    _, state, _, (bvh, g, rays) = G.render(sc, o, d, p, views=views)
    direct = _grads_gpu(R, bvh, g, rays, p, grad, state)
    for k, prm in zip(GROUPS, params):
        a = prm.grad.cpu().numpy().astype(np.float64)
        b = direct[k]
        # same kernels, so equal up to float32 atomic ordering
        assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(b), 1e-30), k
    # and the oracle agrees on the pixels with the oracle's hit sequence
    _grad_parity(sc, o, d, grad.astype(np.float64), p, views=views, label="autograd-ref")


def test_autograd_raises_on_device_status():
    """With raise_on_status the autograd Function reports a device-side error
    (here a traversal stack of depth 1) instead of returning a silent image."""
    print("case autograd status", flush=True)
    G, R = _g()
    from paper_2501_19196_amd import _lib as L
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    params = [G.dev(a) for a in w["scene"].arrays()]
    with pytest.raises(L.RaySplatsError, match="stack"):
        R.render(*params, G.dev(o), G.dev(d), R.Params(stack_depth=1, raise_on_status=True), views)


def test_persistent_backward_matches_plain():
    print("case persistent bwd", flush=True)
    G, R = _g()
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    rng = np.random.default_rng(4)
    grad = G.dev(np.float32(rng.normal(size=(o.shape[0], 3))))
    for hit_list in (0, 64):
        res = []
        for flags in (0, 2):
            p = R.Params(flags=flags, hit_list=hit_list)
            out, state, status, (bvh, g, rays) = G.render(w["scene"], o, d, p, views=views)
            res.append(_grads_gpu(R, bvh, g, rays, p, grad, state))
        for k in GROUPS:
            a, b = res[0][k], res[1][k]
            assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(a), 1e-12), (hit_list, k)


def test_config2_l1_loss_gradients_sampled():
    """Config-2 shape: L1 loss against a target rendered from a jittered copy,
    gradient restricted to a seeded sample of pixels."""
    print("case config2 L1 grads", flush=True)
    G, R = _g()
    w = workload(2)
    o, d, views = G.camera_rays(w["cams"])
    tgt, _, _, _ = G.render(w["target"], o, d, R.Params(), views=views)
    out, _, _, _ = G.render(w["scene"], o, d, R.Params(), views=views)
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(o.shape[0], 1200, replace=False))
    grad = np.sign(out[sel] - tgt[sel]) / (3.0 * o.shape[0])
    _grad_parity(w["scene"], o[sel], d[sel], grad, R.Params(), views=None, label="config2 sampled")


def _full_size_sampled(k, n_samples, seed, hit_list, label):
    """The full-size workload rendered and differentiated in the launch
    configuration the benchmark times (all its views in one launch, stored
    lists of capacity hit_list or re-traversal), with the upstream gradient of
    a mean L1 loss kept on a seeded sample of pixels only; the oracle computes
    the same sample's gradient pixel by pixel."""
    G, R = _g()
    w = workload(k)
    o, d, views = G.camera_rays(w["cams"])
    sc = w["scene"]
    p = R.Params(hit_list=hit_list, flags=2 if len(views) > 1 else 0)
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(o.shape[0], n_samples, replace=False))
    diff = _differing_pixels(sc, o[sel], d[sel], p, label)
    out, state, status, (bvh, g, rays) = G.render(sc, o, d, p, views=views)
    assert status == 0
    tgt = np.float32(np.clip(out + np.float32(rng.normal(scale=0.05, size=out.shape)), 0, 1))
    gsel = np.float32(np.sign(out[sel] - tgt[sel]) / (3.0 * o.shape[0]))
    gsel *= (~diff)[:, None]
    grad = np.zeros_like(out)
    grad[sel] = gsel
    got = _grads_gpu(R, bvh, g, rays, p, grad, state)
    ref = O.render_bwd(sc, o[sel], d[sel], gsel.astype(np.float64), G.oracle_params(O, p))
    _assert_elementwise(got, ref, label)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("hit_list", [64, 512, 0])
def test_scene_scale_sampled_gradients(hit_list):
    """1M Gaussians, 1920x1080, 8,000 sampled pixels (64 slots per ray: the benchmark's pool)."""
    print("case scene-scale sampled grads", hit_list, flush=True)
    _full_size_sampled(4, 8000, 41, hit_list, f"scene-scale 8000 px lists {hit_list}")


@pytest.mark.timeout(600)
def test_batch_8views_sampled_gradients():
    """300k Gaussians (40 % flat), 8 views of uneven size in one persistent launch."""
    print("case 8-view batch sampled grads", flush=True)
    _full_size_sampled(3, 8000, 43, 512, "8-view batch 8000 px")


# ------------------------------------------------- stored hit lists (store vs recompute)

@pytest.mark.parametrize("cap,max_hits", [(512, 512), (64, 512), (4, 0), (16, 64)])
def test_stored_hit_lists_match_recompute(cap, max_hits):
    """The list-replay adjoint (with re-traversal for the rays of packets that
    found the pool exhausted) gives the re-traversing adjoint's gradients; the
    forward is unchanged and its lists hold exactly the composited ids."""
    print("case hit lists", cap, max_hits, flush=True)
    G, R = _g()
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    sc = w["scene"]
    n = o.shape[0]
    rng = np.random.default_rng(11)
    grad = np.float32(rng.normal(size=(n, 3)))
    p0 = R.Params(max_hits=max_hits)
    out0, st0, _, (bvh0, g0_, rays0) = G.render(sc, o, d, p0, views=views)
    g0 = _grads_gpu(R, bvh0, g0_, rays0, p0, grad, st0)
    p = R.Params(max_hits=max_hits, hit_list=cap)
    out1, st1, status, (bvh, g1_, rays) = G.render(sc, o, d, p, views=views)
    assert status == 0
    g1 = _grads_gpu(R, bvh, g1_, rays, p, grad, st1)
    np.testing.assert_array_equal(out1, out0)
    np.testing.assert_array_equal(G.colour_state(st1, n), G.colour_state(st0, n))
    for k in GROUPS:
        assert np.linalg.norm(g1[k] - g0[k]) <= 1e-5 * max(np.linalg.norm(g0[k]), 1e-30), k
    lists = R.hit_lists(rays, p, st1, cap=512)
    op = G.oracle_params(O, p)
    ids_o, L_o = O.render_lists(sc, o, d, op, cap=512)
    full = lists["stored"] == lists["count"]
    if cap == 4:
        assert (~full).sum() > 0  # the pool ran out: those rays took the re-traversal
    if cap == 512:
        assert full.all()
    unamb, _ = O.alternatives_batch(sc, o, d, op, max_events=3, cap=2)
    checked = 0
    for r in np.nonzero((unamb == 1) & full)[0][::7]:
        assert lists["count"][r] == L_o[r], r
        np.testing.assert_array_equal(lists["ids"][r], ids_o[r])
        checked += 1
    assert checked > 50


def test_stored_hit_lists_oracle_parity_and_counters():
    print("case hit lists parity", flush=True)
    G, R = _g()
    w = workload(1)
    o, d, views = G.camera_rays(w["cams"])
    rng = np.random.default_rng(12)
    p = R.Params(hit_list=128)
    _grad_parity(w["scene"], o, d, rng.normal(size=(o.shape[0], 3)), p, views=views, label="lists")
    # work counters: the list adjoint replays exactly the forward's composited hits
    pc = R.Params(hit_list=512, flags=8)
    out, state, _, (bvh, g, rays) = G.render(w["scene"], o, d, pc, views=views)
    cf = R.read_counters(bvh)
    R.render_bwd(bvh, g, rays, pc, G.dev(np.float32(rng.normal(size=(o.shape[0], 3)))), state)
    cb = R.read_counters(bvh)
    assert cb["list_composited"] == cf["lane_composited"] > 0
    assert cb["lane_composited"] == cf["lane_composited"]  # no traversal adjoint ran
    assert cb["adjoint_packets"] == 0
    assert cf["list_rows"] >= cf["lane_composited"] / 64
    # dense rows: one id per composited hit plus a two-word lane mask per row
    assert cf["list_slots"] == cf["lane_composited"] + 2 * cf["list_rows"]


# ------------------------------------------- the paper's gradient variant (second threshold)

def _opaque(seed=70, n=3000):
    sc = scenes.random_scene(seed, n, box=0.8, flat_frac=0.3, scale_lo=0.03, scale_hi=0.15)
    rng = np.random.default_rng(seed + 1)
    sc.opacity[:] = np.float32(rng.uniform(0.3, 0.95, size=n))
    return sc


@pytest.mark.parametrize("eps2", [1e-3, 1.0])
def test_paper_gradient_matches_oracle(eps2):
    """RS_PAPER_GRADIENT: the forward image is unchanged, the second-phase
    counts equal the oracle's, and the gradients match the oracle's paper
    variant element by element on the pixels whose composited sequence, count
    and second phase are the oracle's (eps2 = 1 collects one hit at most)."""
    print("case paper gradient", eps2, flush=True)
    G, R = _g()
    sc = _opaque()
    cam = look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 40, 32, fov_y_deg=40)
    o, d = pinhole_rays(cam)
    views = [(0, 40, 32)]
    n = o.shape[0]
    rng = np.random.default_rng(71)
    grad = rng.normal(size=(n, 3))
    base = dict(eps1=2e-2, max_hits=128, hit_list=256, bg=(0.1, 0.2, 0.3))
    out0, _, _, _ = G.render(sc, o, d, R.Params(**base), views=views)
    p = R.Params(**base, flags=16, eps2=eps2)
    out1, st, status, (bvh, g, rays) = G.render(sc, o, d, p, views=views)
    assert status == 0
    np.testing.assert_array_equal(out1, out0)
    lists = R.hit_lists(rays, p, st, cap=256)
    L_gpu, x_gpu = lists["count"], lists["extra"]
    op = G.oracle_params(O, p)
    e2 = float(np.float32(eps2))
    ref_g, x_ref, near = O.render_bwd_paper(sc, o, d, np.zeros((n, 3)), op, eps2=e2)
    diff = _differing_pixels(sc, o, d, R.Params(**base), "paper variant")
    same = ~diff & ~near & (x_gpu == x_ref)
    print("rays with a second phase", int((x_ref > 0).sum()), "left out", int((~same).sum()), "of", n, flush=True)
    assert (x_ref > 0).sum() > 0.2 * n
    assert same.sum() > 0.9 * n
    gm = np.float32(grad * same[:, None])
    got = _grads_gpu(R, bvh, g, rays, p, gm, st)
    ref, _, _ = O.render_bwd_paper(sc, o, d, gm.astype(np.float64), op, eps2=e2)
    exact = O.render_bwd(sc, o, d, gm.astype(np.float64), op)
    _assert_elementwise(got, ref, f"paper eps2 {eps2}")
    if eps2 == 1.0:
        assert x_ref.max() == 1
    # the variant is visible in the opacity gradients (the last composited hits)
    assert np.linalg.norm(exact["opacity"] - ref["opacity"]) > 10 * REL * np.linalg.norm(ref["opacity"])


@pytest.mark.parametrize("group,eps,tol", [("rgb", 1e-2, 1e-4), ("opacity", 1e-2, 2e-3)])
def test_scene_scale_adjoint_directional_derivative(group, eps, tol):
    """At the full scene-scale size (1M Gaussians, 1920x1080, stored lists of
    capacity 512), the adjoint of F = sum_rays <g, C> along a random direction
    v matches the central difference of the forward, a property that holds at
    any size. F is linear in the colours, so the rgb case is exact up to float
    rounding. Opacities move T, so the opacity case turns off the eps1 and K_max
    stops (a stop that moves is a jump the difference would see): every ray
    composites all its hits, so long lists exhaust the pool and those packets
    take the re-traversal. Directions that the [0, 0.999] range of the
    opacities would clip are left out."""
    print("case directional", group, flush=True)
    G, R = _g()
    w = workload(4)
    o, d, views = G.camera_rays(w["cams"])
    sc = w["scene"]
    p = R.Params(hit_list=512) if group == "rgb" else R.Params(hit_list=512, eps1=0.0, max_hits=0)
    rng = np.random.default_rng(7)
    g = np.float32(rng.normal(size=(o.shape[0], 3)))
    v = np.float32(rng.normal(size=getattr(sc, group).shape))
    if group == "opacity":
        v[(sc.opacity - eps * np.abs(v) < 0) | (sc.opacity + eps * np.abs(v) > 0.999)] = 0.0
    rays = G.rays_of(o, d, views)

    def F(scene):
        gs = G.gaussians(scene)
        bvh = R.build_bvh(gs, p)
        out, state = R.render_fwd(bvh, gs, rays, p)
        torch.cuda.synchronize()
        assert R.read_status(bvh) == 0
        return float(np.sum(out.cpu().numpy().astype(np.float64) * g)), (bvh, gs, state)

    f0, (bvh, gs, state) = F(sc)
    got = _grads_gpu(R, bvh, gs, rays, p, g, state)
    analytic = float(np.sum(got[group] * v))

    def shifted(sign):
        arrs = {k: getattr(sc, k).copy() for k in GROUPS}
        arrs[group] = np.float32(arrs[group] + sign * eps * v)
        return type(sc)(*(arrs[k] for k in GROUPS))

    fp, _ = F(shifted(+1))
    fm, _ = F(shifted(-1))
    numeric = (fp - fm) / (2 * eps)
    print(group, "adjoint", analytic, "central difference", numeric, flush=True)
    assert abs(analytic - numeric) <= tol * max(abs(numeric), 1.0)
