"""Pins of the loss oracle (oracle/loss.py): window moments against scipy's
Gaussian filter, SSIM of an image with itself, symmetry, the pure-L2 limit,
and central differences of the loss against the App. A.7 gradient. CPU only."""

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter

from oracle import loss as OL


def _pair(seed, h=23, w=31):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 1, size=(h, w, 3))
    b = np.clip(a + rng.normal(scale=0.1, size=(h, w, 3)), 0, 1)
    return a, b


def test_window_moments_match_scipy_gaussian_filter():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(19, 27))
    w = OL.window(5, 1.5)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    ref = gaussian_filter(img, sigma=1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
    np.testing.assert_allclose(OL.wsum(img, w), ref, atol=1e-14)


def test_ssim_of_identical_images():
    a, _ = _pair(1)
    assert OL.loss(a, a, lam=1.0) == pytest.approx(0.0, abs=1e-14)
    np.testing.assert_allclose(OL.loss_grad(a, a, lam=0.7), 0.0, atol=1e-14)


def test_symmetry_and_l2_limit():
    a, b = _pair(2)
    assert OL.loss(a, b, lam=0.6) == pytest.approx(OL.loss(b, a, lam=0.6), rel=1e-13)
    h, w, _ = a.shape
    np.testing.assert_allclose(OL.loss_grad(a, b, lam=0.0), 2 * (a - b) / (3 * h * w), rtol=1e-13)
    assert OL.loss(a, b, lam=0.0) == pytest.approx(((a - b) ** 2).mean(), rel=1e-13)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_matches_central_differences(lam):
    a, b = _pair(3, h=14, w=17)
    g = OL.loss_grad(a, b, lam=lam)
    rng = np.random.default_rng(4)
    for _ in range(40):
        i, j, c = rng.integers(0, 14), rng.integers(0, 17), rng.integers(0, 3)
        ests = []
        for hstep in (1e-4, 5e-5):
            ap, am = a.copy(), a.copy()
            ap[i, j, c] += hstep
            am[i, j, c] -= hstep
            ests.append((OL.loss(ap, b, lam) - OL.loss(am, b, lam)) / (2 * hstep))
        fd = (4 * ests[1] - ests[0]) / 3
        assert g[i, j, c] == pytest.approx(fd, rel=1e-6, abs=1e-12), (i, j, c)
