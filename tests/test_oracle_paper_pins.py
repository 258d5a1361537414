"""Pins of the oracle's paper-variant backward (second threshold eps2): it
reduces to the exact adjoint when no second phase runs, it counts the
second-phase hits the definition implies, and it is the gradient (by central
differences) of the extended composite E = plain render with K_max = J and no
eps1 stop, for the composited Gaussians. CPU only."""

import numpy as np
import pytest

from synthetic import scenes


def _rays(n, seed, spread=0.15):
    rng = np.random.default_rng(seed)
    o = np.tile([0.0, 0.0, -3.0], (n, 1)) + rng.normal(scale=0.02, size=(n, 3))
    d = np.column_stack([rng.normal(scale=spread, size=(n, 2)), np.ones(n)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.float32(o), np.float32(d)


def _opaque_scene(seed, n=80):
    sc = scenes.random_scene(seed, n, box=0.5, flat_frac=0.3, scale_lo=0.08, scale_hi=0.3)
    rng = np.random.default_rng(seed + 100)
    sc.opacity[:] = np.float32(rng.uniform(0.3, 0.9, size=n))
    return sc


def test_paper_variant_without_second_phase_is_the_exact_adjoint(orc):
    sc = _opaque_scene(60)
    o, d = _rays(64, 61)
    g = np.random.default_rng(62).normal(size=(64, 3))
    p = orc.Params(eps1=1e-2, max_hits=64, bg=(0.1, 0.2, 0.3))
    ref = orc.render_bwd(sc, o, d, g, p)
    got, extra, _ = orc.render_bwd_paper(sc, o, d, g, p, eps2=2.0)  # T2 = 1 < 2: nothing collected
    assert np.all(extra == 0)
    for k in ref:
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-12, atol=1e-15)


def test_second_phase_counts(orc):
    """eps2 = 0 collects every remaining hit up to K_max; the count follows
    the definition written out here from the sorted hits and alphas."""
    sc = _opaque_scene(63)
    o, d = _rays(40, 64)
    for max_hits in (0, 12):
        p = orc.Params(eps1=5e-2, max_hits=max_hits)
        _, extra0, _ = orc.render_bwd_paper(sc, o, d, np.ones((40, 3)), p, eps2=0.0)
        _, extra1, _ = orc.render_bwd_paper(sc, o, d, np.ones((40, 3)), p, eps2=0.05)
        for r in range(40):
            _, _, _, al = orc.ray_hits(sc, o, d, r, p)
            T, L, by_eps = 1.0, 0, False
            for a in al:
                if max_hits and L >= max_hits:
                    break
                T *= 1 - a
                L += 1
                if T < p.eps1:
                    by_eps = True
                    break
            rest = len(al) - L
            cap = (max_hits - L) if max_hits else rest
            want0 = min(rest, cap) if by_eps else 0
            assert extra0[r] == want0, (r, max_hits)
            x, T2 = 0, 1.0
            if by_eps:
                while x < min(rest, cap) and T2 >= 0.05:
                    T2 *= 1 - al[L + x]
                    x += 1
            assert extra1[r] == x, (r, max_hits)
        assert (extra0 > 0).sum() > 5


@pytest.mark.parametrize("which", [0, 1, 2])
def test_paper_variant_is_the_gradient_of_the_extended_composite(orc, which):
    """For one ray with L composited and J collected hits, the paper-variant
    gradient of each composited Gaussian equals the central difference of
    <g, plain render with K_max = J and eps1 = 0>; collected-only Gaussians
    get no gradient."""
    sc = _opaque_scene(65, n=120)
    o, d = _rays(48, 66, spread=0.08)
    g = np.float64([[0.7, -0.4, 1.1]])
    p = orc.Params(eps1=2e-2, max_hits=0, bg=(0.2, 0.3, 0.4))
    _, extra, near = orc.render_bwd_paper(sc, o, d, np.ones((48, 3)), p, eps2=1e-3)
    ray = np.nonzero((extra > 1) & ~near)[0][3 * which]
    o, d = o[ray:ray + 1], d[ray:ray + 1]
    grads, extra, near = orc.render_bwd_paper(sc, o, d, g, p, eps2=1e-3)
    _, _, L = orc.render_fwd(sc, o, d, p)
    L = int(L[0])
    idx, _, _, _ = orc.ray_hits(sc, o, d, 0, p)
    assert extra[0] > 0 and not near[0], (L, extra)
    J = L + int(extra[0])
    pe = orc.Params(eps1=0.0, max_hits=J, bg=p.bg)
    loss = lambda s2: float(np.sum(orc.render_fwd(s2, o, d, pe)[0] * g))
    for i in idx[J:J + 3]:  # beyond J: nothing
        assert np.all(grads["mean"][i] == 0)
    for i in idx[L:J]:  # collected only: no gradient
        assert np.all(grads["mean"][i] == 0) and grads["opacity"][i] == 0
    checked = 0
    for i in idx[:L]:
        for name, comp in (("mean", 0), ("mean", 2), ("opacity", None), ("scale", 1), ("quat", 3), ("rgb", 1)):
            base = getattr(sc, name)
            v0 = float(base[i] if comp is None else base[i, comp])
            if name == "scale" and base[i].min() < 1e-3:
                continue
            ests = []
            for h in (2.0 ** -16, 2.0 ** -17):
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
            an = grads[name][i] if comp is None else grads[name][i, comp]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-7), (name, i, comp)
            checked += 1
    assert checked >= 8


def test_paper_variant_differs_from_exact_on_the_last_hit(orc):
    """The reading matters: with a second phase, the last composited
    Gaussian's opacity gradient changes (c_L - R2 instead of c_L - bg)."""
    sc = _opaque_scene(67)
    o, d = _rays(32, 68)
    g = np.ones((32, 3))
    p = orc.Params(eps1=2e-2, max_hits=0)
    ex = orc.render_bwd(sc, o, d, g, p)
    pa, extra, _ = orc.render_bwd_paper(sc, o, d, g, p, eps2=1e-3)
    assert extra.sum() > 0
    assert np.abs(pa["opacity"] - ex["opacity"]).max() > 1e-3
