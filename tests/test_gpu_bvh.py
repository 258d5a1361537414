"""BVH build on the GPU against the CPU reference: Morton codes, sorted
permutation, leaf boxes, the PLOC tree (topology and child boxes) and the
radix-tree topology bit-exact; boxes conservative."""

import numpy as np
import pytest
import torch

from synthetic import scenes
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _build(scene, Q=11.3449, lbvh=False):
    from tests._gpu import gaussians
    from paper_2501_19196_amd import renderer as R, _lib as L
    g = gaussians(scene)
    bvh = R.build_bvh(g, R.Params(Q=Q, flags=L.RS_BUILD_LBVH if lbvh else 0))
    torch.cuda.synchronize()
    return R.download(bvh), R.read_status(bvh)


def _chain(n):
    """Gaussians along x with slowly growing isotropic scale: each leaf's
    nearest cluster is its left neighbour, so clustering merges about one pair
    per iteration and reaches the pairing cap."""
    from synthetic.scenes import Scene
    rng = np.random.default_rng(n)
    mean = np.zeros((n, 3), np.float32)
    mean[:, 0] = np.arange(n)
    scale = np.repeat((0.3 + 0.001 * np.arange(n))[:, None], 3, 1).astype(np.float32)
    quat = np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1))
    return Scene(mean, scale, quat, np.full(n, 0.5, np.float32), rng.uniform(size=(n, 3)).astype(np.float32))


def _scene(which):
    if which == "config1":
        return scenes.scene_config1()
    if which == "clusters100k":
        return scenes.scene_config2(n=100_000)
    if which == "ragged":
        return scenes.random_scene(7, 2048 * 3 + 17)  # several sort tiles plus a ragged tail
    if which == "dups":
        sc = scenes.random_scene(8, 5000)
        sc.mean[::3] = sc.mean[0]  # many identical codes
        return sc
    if which == "equal_boxes":
        sc = scenes.random_scene(12, 4500)
        sc.mean[:] = sc.mean[0]
        sc.scale[:] = sc.scale[0]
        sc.quat[:] = sc.quat[0]
        return sc
    if which == "local_edge":
        return scenes.random_scene(13, 4097)  # one cluster more than the single-workgroup finish holds
    if which == "chain600":
        return _chain(600)
    if which == "chain20k":
        return _chain(20_000)  # leaves the finish kernel more clusters than fit in LDS
    if which == "scene1M":
        return scenes.scene_config4()  # the scene-scale workload's 1M Gaussians
    if which == "batch300k":
        return scenes.scene_config3()
    raise ValueError(which)


@pytest.mark.parametrize("which", ["config1", "clusters100k", "ragged", "dups", "equal_boxes", "local_edge",
                                   "chain600", "chain20k", "batch300k", "scene1M"])
def test_leaf_boxes_and_ploc_tree_bit_exact(which):
    print("case ploc", which, flush=True)
    sc = _scene(which)
    got, status = _build(sc)
    assert status == 0
    codes, _, _ = O.morton_codes(sc.mean)
    _, perm = O.sort_codes(codes)
    np.testing.assert_array_equal(got["perm"], perm)
    lb = O.leaf_boxes(sc.mean, sc.scale, sc.quat, perm)
    np.testing.assert_array_equal(got["leaf_boxes"], lb)
    child, boxes, _ = O.ploc(lb)
    np.testing.assert_array_equal(got["child"], child)
    np.testing.assert_array_equal(got["boxes"], boxes)


@pytest.mark.parametrize("which", ["config1", "clusters100k", "ragged", "dups", "scene1M"])
def test_morton_sort_topology_bit_exact(which):
    """The radix-tree builder (RS_BUILD_LBVH)."""
    print("case lbvh", which, flush=True)
    sc = _scene(which)
    got, status = _build(sc, lbvh=True)
    assert status == 0
    codes, lo, hi = O.morton_codes(sc.mean)
    np.testing.assert_array_equal(got["bounds"][:3], lo)
    np.testing.assert_array_equal(got["bounds"][3:], hi)
    s, perm = O.sort_codes(codes)
    np.testing.assert_array_equal(got["codes"], s)
    np.testing.assert_array_equal(got["perm"], perm)
    child, leaf = O.radix_tree(s)
    gc = got["child"]
    want = np.where(leaf, ~child, child)
    np.testing.assert_array_equal(gc, want)


@pytest.mark.parametrize("lbvh", [False, True])
def test_boxes_are_conservative(lbvh):
    sc = scenes.random_scene(9, 3000)
    got, _ = _build(sc, lbvh=lbvh)
    perm = got["perm"]
    lb = got["leaf_boxes"]
    Q = 11.3449
    rng = np.random.default_rng(0)
    # points on each confidence ellipsoid: m + R S sqrt(Q) u, |u| = 1
    u = rng.normal(size=(64, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for j in range(0, sc.n, 7):
        i = perm[j]
        R = O.rotation(sc.quat[i].astype(np.float64))
        pts = sc.mean[i].astype(np.float64) + (u * np.sqrt(Q) * sc.scale[i].astype(np.float64)) @ R.T
        assert np.all(pts >= lb[j, :3]) and np.all(pts <= lb[j, 3:]), j
    # every internal node's child boxes contain their subtrees
    child, boxes = got["child"], got["boxes"]
    n = sc.n

    def subtree_box(ref):
        if ref < 0:
            return lb[~ref]
        b = boxes[ref]
        return np.concatenate([np.minimum(b[0, :3], b[1, :3]), np.maximum(b[0, 3:], b[1, 3:])])

    for i in range(n - 1):
        for c in range(2):
            sb = subtree_box(child[i, c])
            assert np.all(boxes[i, c, :3] <= sb[:3]) and np.all(boxes[i, c, 3:] >= sb[3:])


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("lbvh", [False, True])
def test_tiny_scenes(n, lbvh):
    sc = scenes.random_scene(10, n)
    got, status = _build(sc, lbvh=lbvh)
    assert status == 0
    codes, _, _ = O.morton_codes(sc.mean)
    s, perm = O.sort_codes(codes)
    np.testing.assert_array_equal(got["perm"], perm)
    if n >= 2 and lbvh:
        child, leaf = O.radix_tree(s)
        np.testing.assert_array_equal(got["child"], np.where(leaf, ~child, child))
    elif n >= 2:
        child, _, _ = O.ploc(O.leaf_boxes(sc.mean, sc.scale, sc.quat, perm))
        np.testing.assert_array_equal(got["child"], child)


def test_nonfinite_input_sets_status():
    from paper_2501_19196_amd import _lib as L
    sc = scenes.random_scene(11, 100)
    sc.scale[5, 1] = np.nan
    _, status = _build(sc)
    assert status == L.RS_ERR_NONFINITE
