"""Pins of the BVH-builder reference in oracle/rs_oracle_bvh.c: the bit-exact
leaf boxes against the support function of the confidence ellipsoid, and the
PLOC tree against hand-worked cases, structural invariants, its tie rule, its
iteration cap and its surface-area cost. CPU only."""

import numpy as np
import pytest

from oracle import oracle as O
from synthetic import scenes


def _sorted_boxes(sc, Q=O.Q_DEFAULT):
    codes, _, _ = O.morton_codes(sc.mean)
    _, perm = O.sort_codes(codes)
    return O.leaf_boxes(sc.mean, sc.scale, sc.quat, perm, Q), perm


def _check_tree(child, boxes, lb):
    """Every leaf once, every internal node but the root once, boxes = exact unions."""
    n = lb.shape[0]
    seen_leaf = np.zeros(n, int)
    seen_node = np.zeros(n - 1, int)
    for refs in child:
        for r in refs:
            if r < 0:
                seen_leaf[~r] += 1
            else:
                seen_node[r] += 1
    assert np.all(seen_leaf == 1)
    assert seen_node[0] == 0 and np.all(seen_node[1:] == 1)
    sub = np.zeros((n - 1, 6), np.float32)
    # children are created before their parents: higher ids first
    for i in range(n - 2, -1, -1):
        parts = [lb[~r] if r < 0 else sub[r] for r in child[i]]
        for c in range(2):
            np.testing.assert_array_equal(boxes[i, c], parts[c])
        sub[i, :3] = np.minimum(parts[0][:3], parts[1][:3])
        sub[i, 3:] = np.maximum(parts[0][3:], parts[1][3:])
    depth = np.zeros(n - 1, int)
    for i in range(n - 1):
        for r in child[i]:
            if r >= 0:
                assert r > i  # reverse creation order
                depth[r] = depth[i] + 1
    return depth.max() + 1


def test_leaf_boxes_match_the_support_function():
    """max of x_k over the ellipsoid is m_k + sqrt(Q Sigma_kk), Sigma = R S^2 R^T
    (R from the independent rotation routine); the box adds 1e-5 relative and
    1e-7 (1 + |m|) absolute padding and rounds outward."""
    sc = scenes.random_scene(21, 500)
    lb, perm = _sorted_boxes(sc)
    Q = float(np.float32(O.Q_DEFAULT))  # the float32 knob
    for j in range(sc.n):
        i = perm[j]
        R = O.rotation(sc.quat[i].astype(np.float64))
        S2 = np.diag(sc.scale[i].astype(np.float64) ** 2)
        sig = R @ S2 @ R.T
        m = sc.mean[i].astype(np.float64)
        half = np.sqrt(Q * np.diag(sig)) * (1 + 1e-5) + 1e-7 * (1 + np.abs(m))
        lo, hi = lb[j, :3].astype(np.float64), lb[j, 3:].astype(np.float64)
        assert np.all(lo <= m - half * (1 - 1e-12)) and np.all(hi >= m + half * (1 - 1e-12)), j
        # outward rounding by at most one float32 step beyond the FP64 value
        ulp_lo = np.spacing(np.abs(m - half).astype(np.float32)).astype(np.float64)
        ulp_hi = np.spacing(np.abs(m + half).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(lo - (m - half)) <= 2 * ulp_lo)
        assert np.all(np.abs(hi - (m + half)) <= 2 * ulp_hi)


def test_leaf_boxes_contain_sampled_surface_points():
    sc = scenes.random_scene(22, 300)
    lb, perm = _sorted_boxes(sc)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for j in range(sc.n):
        i = perm[j]
        R = O.rotation(sc.quat[i].astype(np.float64))
        pts = sc.mean[i].astype(np.float64) + (u * np.sqrt(O.Q_DEFAULT) * sc.scale[i]) @ R.T
        assert np.all(pts >= lb[j, :3]) and np.all(pts <= lb[j, 3:])


def test_ploc_hand_worked_line():
    """Unit boxes at x = 0, 1.5, 10, 11.5: the two close pairs merge first
    (nodes 2 and 1, in position order), then the root joins them."""
    lb = np.array([[0, 0, 0, 1, 1, 1], [1.5, 0, 0, 2.5, 1, 1], [10, 0, 0, 11, 1, 1], [11.5, 0, 0, 12.5, 1, 1]],
                  np.float32)
    child, boxes, it = O.ploc(lb)
    np.testing.assert_array_equal(child, [[2, 1], [~2, ~3], [~0, ~1]])
    assert it == 2
    np.testing.assert_array_equal(boxes[0, 0], [0, 0, 0, 2.5, 1, 1])
    np.testing.assert_array_equal(boxes[0, 1], [10, 0, 0, 12.5, 1, 1])


def test_ploc_nearest_is_by_union_area_not_by_position():
    """A small box next to a large one pairs with the small box two positions
    away: union area decides, not adjacency."""
    lb = np.array([[0, 0, 0, 10, 10, 10],       # large
                   [10, 0, 0, 10.5, 0.5, 0.5],   # small, adjacent to both
                   [10.6, 0, 0, 11.1, 0.5, 0.5]], np.float32)
    child, _, _ = O.ploc(lb)
    # first merge (node 1): positions 1 and 2; then the root joins position 0 and node 1
    np.testing.assert_array_equal(child, [[~0, 1], [~1, ~2]])


@pytest.mark.parametrize("n", [2, 7, 8, 33])
def test_ploc_equal_boxes_pair_up(n):
    """Exact ties pair (0,1), (2,3), ...: a balanced tree of depth ceil(log2 n)."""
    lb = np.tile(np.array([[0, 0, 0, 1, 1, 1]], np.float32), (n, 1))
    child, boxes, it = O.ploc(lb)
    depth = _check_tree(child, boxes, lb)
    assert depth == int(np.ceil(np.log2(n)))
    assert it == int(np.ceil(np.log2(n)))
    # the first merge is leaves 0 and 1
    np.testing.assert_array_equal(child[n - 2], [~0, ~1])


@pytest.mark.parametrize("which", ["random", "clusters", "dups", "ragged"])
def test_ploc_tree_invariants(which):
    if which == "random":
        sc = scenes.random_scene(23, 3000)
    elif which == "clusters":
        sc = scenes.scene_config2(n=20_000)
    elif which == "dups":
        sc = scenes.random_scene(24, 2000)
        sc.mean[::3] = sc.mean[0]
        sc.scale[::3] = sc.scale[0]
        sc.quat[::3] = sc.quat[0]
    else:
        sc = scenes.random_scene(25, 4097)
    lb, _ = _sorted_boxes(sc)
    child, boxes, it = O.ploc(lb)
    _check_tree(child, boxes, lb)
    assert it < O.ploc_cap(sc.n)


def _sah(child, boxes, lb):
    def area(b):
        e = (b[..., 3:] - b[..., :3]).astype(np.float64)
        return 2 * (e[..., 0] * e[..., 1] + e[..., 1] * e[..., 2] + e[..., 2] * e[..., 0])
    # internal node areas: union of its two child boxes
    u = np.concatenate([np.minimum(boxes[:, 0, :3], boxes[:, 1, :3]), np.maximum(boxes[:, 0, 3:], boxes[:, 1, 3:])], 1)
    return (area(u).sum() + area(lb).sum()) / area(u[0])


def test_ploc_surface_area_cost_beats_the_radix_tree():
    """The clustering's purpose: a lower surface-area cost than the Morton
    radix tree over the same leaves (the same leaf order)."""
    sc = scenes.scene_config4(n=30_000)
    lb, _ = _sorted_boxes(sc)
    child, boxes, _ = O.ploc(lb)
    codes, _, _ = O.morton_codes(sc.mean)
    s, _ = O.sort_codes(codes)
    rc, leaf = O.radix_tree(s)
    rc = np.where(leaf, ~rc, rc)
    # boxes of the radix tree bottom-up
    n = sc.n
    rb = np.zeros((n - 1, 2, 6), np.float32)
    done = np.zeros(n - 1, bool)
    sub = np.zeros((n - 1, 6), np.float32)

    def box_of(r):
        return lb[~r] if r < 0 else sub[r]
    order = []
    stack = [0]
    while stack:
        i = stack.pop()
        order.append(i)
        stack.extend(r for r in rc[i] if r >= 0)
    for i in reversed(order):
        for c in range(2):
            rb[i, c] = box_of(rc[i, c])
        sub[i, :3] = np.minimum(rb[i, 0, :3], rb[i, 1, :3])
        sub[i, 3:] = np.maximum(rb[i, 0, 3:], rb[i, 1, 3:])
        done[i] = True
    assert done.all()
    assert _sah(child, boxes, lb) < 0.85 * _sah(rc, rb, lb)


def test_ploc_iteration_cap_forces_pairs():
    """A chain of slowly growing boxes merges about one pair per iteration (each
    box's nearest is its smaller left neighbour); past the cap the build pairs
    positions (0,1), (2,3), ... (halving the clusters) and still ends in one
    valid tree."""
    n = 600
    x = np.arange(n, dtype=np.float64) * 1.0
    w = 1.0 + 0.01 * np.arange(n)
    lb = np.zeros((n, 6), np.float32)
    lb[:, 0] = x
    lb[:, 3] = x + w
    lb[:, 4] = w
    lb[:, 5] = w
    child, boxes, it = O.ploc(lb)
    _check_tree(child, boxes, lb)
    cap = O.ploc_cap(n)
    assert cap == 256
    # the chain outlasts the cap; pairing then needs at most ceil(log2 n) more
    assert cap < it <= cap + int(np.ceil(np.log2(n)))
    # one pair per iteration: leaves (0, 1), then (2, 3), then (4, 5)
    np.testing.assert_array_equal(child[n - 2], [~0, ~1])
    np.testing.assert_array_equal(child[n - 3], [~2, ~3])
    np.testing.assert_array_equal(child[n - 4], [~4, ~5])
