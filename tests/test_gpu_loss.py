"""Training-loss kernels (L2 + D-SSIM and the App. A.7 gradient) against the
FP64 oracle: small and ragged images element by element, a full 1920 x 1080
image on sampled pixels (each checked on a crop that holds its whole
dependency region) and against an independent FP64 separable filter for the
loss value."""

import numpy as np
import pytest
import torch
from scipy.ndimage import gaussian_filter

from oracle import loss as OL

pytestmark = pytest.mark.gpu


def _R():
    from paper_2501_19196_amd import renderer as R
    return R


def _pair(seed, h, w, noise=0.1):
    rng = np.random.default_rng(seed)
    a = np.float32(rng.uniform(0, 1, size=(h, w, 3)))
    b = np.float32(np.clip(a + rng.normal(scale=noise, size=(h, w, 3)), 0, 1))
    return a, b


def _gpu(a, b, lam=0.2, radius=5, sigma=1.5):
    R = _R()
    h, w, _ = a.shape
    loss, g = R.image_loss(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), w, h, lam, radius, sigma)
    torch.cuda.synchronize()
    return float(loss.cpu()[0]), g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("h,w,lam", [(29, 37, 0.2), (8, 64, 1.0), (1, 1, 0.2), (200, 5, 0.5), (33, 33, 0.0)])
def test_loss_matches_oracle(h, w, lam):
    print("case loss", h, w, lam, flush=True)
    a, b = _pair(h * 100 + w, h, w)
    lg, gg = _gpu(a, b, lam)
    lr = OL.loss(a, b, lam)
    gr = OL.loss_grad(a, b, lam)
    assert lg == pytest.approx(lr, rel=2e-5, abs=1e-7)
    scale = np.abs(gr).max()
    assert np.abs(gg - gr).max() <= 2e-4 * scale, (np.abs(gg - gr).max(), scale)
    assert np.linalg.norm(gg - gr) <= 1e-4 * np.linalg.norm(gr)


def test_window_radius_and_sigma_knobs():
    print("case loss knobs", flush=True)
    a, b = _pair(5, 40, 52)
    for radius, sigma in ((1, 0.8), (3, 1.0), (7, 2.5)):
        lg, gg = _gpu(a, b, 0.8, radius, sigma)
        assert lg == pytest.approx(OL.loss(a, b, 0.8, radius, sigma), rel=2e-5)
        gr = OL.loss_grad(a, b, 0.8, radius, sigma)
        assert np.linalg.norm(gg - gr) <= 1e-4 * np.linalg.norm(gr)


def test_identical_images():
    a, _ = _pair(6, 50, 70)
    lg, gg = _gpu(a, a, 0.5)
    assert abs(lg) < 1e-6
    assert np.abs(gg).max() < 1e-9


def test_full_hd_sampled_pixels_and_loss_value():
    """1920 x 1080: the gradient of sampled pixels (interior, edges, corners)
    from the oracle run on a crop with a 12-pixel margin (the gradient of a
    pixel depends on the image within 2r = 10 of it; the 1/(hw) factors are
    rescaled), and the loss against a separable FP64 Gaussian filter."""
    print("case loss full hd", flush=True)
    H, W = 1080, 1920
    rng = np.random.default_rng(7)
    yy, xx = np.mgrid[0:H, 0:W]
    base = 0.5 + 0.4 * np.sin(xx[..., None] / 37.0 + np.arange(3)) * np.cos(yy[..., None] / 23.0)
    a = np.float32(np.clip(base + rng.normal(scale=0.05, size=(H, W, 3)), 0, 1))
    b = np.float32(np.clip(base + rng.normal(scale=0.05, size=(H, W, 3)), 0, 1))
    lam = 0.2
    lg, gg = _gpu(a, b, lam)
    # loss value: FP64 separable filtering (zero outside the image)
    f = lambda x: gaussian_filter(x, sigma=1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
    tot = 0.0
    for ch in range(3):
        I, J = a[..., ch].astype(np.float64), b[..., ch].astype(np.float64)
        mu, mh = f(I), f(J)
        A = 2 * mu * mh + OL.C1
        B = 2 * (f(I * J) - mu * mh) + OL.C2
        C = mu * mu + mh * mh + OL.C1
        D = f(I * I) - mu * mu + f(J * J) - mh * mh + OL.C2
        tot += (1 - lam) * ((I - J) ** 2).mean() + lam * (1 - (A * B / (C * D)).mean()) / 2
    assert lg == pytest.approx(tot / 3, rel=1e-4)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (5, 700), (H - 3, 1200), (540, 0), (300, W - 7)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(24)]
    m = 12
    gscale = np.abs(gg).max()
    worst = 0.0
    for i, j in pts:
        y0, y1, x0, x1 = max(0, i - m), min(H, i + m + 1), max(0, j - m), min(W, j + m + 1)
        # crop edges inside the image are >= 12 from the pixel; edges on the image border are real
        ref = OL.loss_grad(a[y0:y1, x0:x1], b[y0:y1, x0:x1], lam)[i - y0, j - x0]
        ref = ref * ((y1 - y0) * (x1 - x0)) / (H * W)
        err = np.abs(gg[i, j] - ref).max() / max(np.abs(ref).max(), 1e-2 * gscale)
        worst = max(worst, err)
    print("full-hd sampled worst relative error", worst, flush=True)
    assert worst <= 1e-3
