"""Pins of the CPU BVH reference (Morton codes, stable sort, radix-tree
topology) against properties its definition fixes. CPU only."""

import numpy as np

from synthetic import scenes


def deinterleave(codes):
    q = np.zeros((codes.shape[0], 3), np.int64)
    for b in range(10):
        for k in range(3):
            q[:, k] |= ((codes.astype(np.int64) >> (3 * b + (2 - k))) & 1) << b
    return q


def test_morton_quantisation_and_interleave(orc):
    sc = scenes.scene_config1()
    codes, lo, hi = orc.morton_codes(sc.mean)
    assert codes.max() < (1 << 30)
    np.testing.assert_array_equal(lo, sc.mean.min(0))
    np.testing.assert_array_equal(hi, sc.mean.max(0))
    q = deinterleave(codes)
    # quantisation: q_k = floor((c - lo) * 1024 / (hi - lo)), clamped to 1023; the
    # float32 spec may differ from the exact value only where the exact product
    # is within float32 rounding of an integer
    exact = (sc.mean.astype(np.float64) - lo) * 1024.0 / (hi.astype(np.float64) - lo)
    fl = np.minimum(np.floor(exact), 1023).astype(np.int64)
    near_int = np.abs(exact - np.round(exact)) < 1e-3
    ok = (q == fl) | near_int
    assert ok.all()
    # the minimum per axis quantises to 0 and the maximum to 1023
    for k in range(3):
        assert q[np.argmin(sc.mean[:, k]), k] == 0
        assert q[np.argmax(sc.mean[:, k]), k] == 1023


def test_morton_order_is_lexicographic_on_bits():
    """Interleave property: comparing codes compares (x9 y9 z9 x8 ...) bit strings."""
    from oracle import oracle as O
    rng = np.random.default_rng(3)
    mean = np.float32(rng.uniform(-1, 1, (500, 3)))
    codes, _, _ = O.morton_codes(mean)
    q = deinterleave(codes)
    # rebuild each code from its quantised coordinates by string concatenation
    def code_str(v):
        bits = []
        for b in range(9, -1, -1):
            for k in range(3):
                bits.append(str((v[k] >> b) & 1))
        return int("".join(bits), 2)
    assert all(code_str(q[i]) == int(codes[i]) for i in range(500))


def test_degenerate_axis_gives_zero():
    from oracle import oracle as O
    mean = np.float32(np.stack([np.linspace(-1, 1, 100), np.zeros(100), np.full(100, 2.0)], 1))
    codes, _, _ = O.morton_codes(mean)
    q = deinterleave(codes)
    assert np.all(q[:, 1] == 0) and np.all(q[:, 2] == 0)


def test_sort_is_stable(orc):
    rng = np.random.default_rng(5)
    codes = rng.integers(0, 50, size=2000).astype(np.uint32)  # many ties
    s, perm = orc.sort_codes(codes)
    np.testing.assert_array_equal(perm, np.argsort(codes, kind="stable"))
    np.testing.assert_array_equal(s, codes[perm])


def _check_tree(orc, sorted_codes):
    n = sorted_codes.shape[0]
    child, leaf = orc.radix_tree(sorted_codes)
    assert child.shape == (n - 1, 2)
    key = (sorted_codes.astype(np.uint64) << np.uint64(32)) | np.arange(n, dtype=np.uint64)

    def prefix(i, j):
        x = int(key[i]) ^ int(key[j])
        return 64 if x == 0 else 64 - x.bit_length()

    # walk from the root and recover each node's range
    seen_leaf = np.zeros(n, bool)
    seen_int = np.zeros(n - 1, bool)
    stack = [(0, 0, n - 1)]
    while stack:
        node, f, l = stack.pop()
        assert not seen_int[node]
        seen_int[node] = True
        assert node in (f, l)  # an internal node sits at one end of its range
        common = prefix(f, l)
        g = child[node, 0]
        assert child[node, 1] == g + 1
        assert f <= g < l
        # every key of each half shares more than `common` bits; the halves differ at that bit
        assert prefix(f, g) > common and prefix(g + 1, l) > common
        for c, (a, b) in enumerate(((f, g), (g + 1, l))):
            if a == b:
                assert leaf[node, c] and child[node, c] == a
                assert not seen_leaf[a]
                seen_leaf[a] = True
            else:
                assert not leaf[node, c]
                stack.append((child[node, c], a, b))
    assert seen_leaf.all() and seen_int.all()


def test_radix_tree_structure(orc):
    rng = np.random.default_rng(6)
    for n in (2, 3, 7, 64, 1000):
        codes = np.sort(rng.integers(0, 1 << 30, size=n).astype(np.uint32))
        _check_tree(orc, codes)
    # heavy duplicates: the index bits separate equal codes
    codes = np.sort(rng.integers(0, 8, size=500).astype(np.uint32))
    _check_tree(orc, codes)
    _check_tree(orc, np.zeros(300, np.uint32))
