"""FP64 oracle of the training loss (TEST INFRASTRUCTURE ONLY).

The paper's loss (Sec. 3, "Loss Function"; App. A.7) per colour channel is
    L_ch = (1 - lambda) * mean_pixels (I - I_hat)^2 + lambda * (1 - SSIM_ch) / 2,
with SSIM_ch the mean over pixels of the SSIM map, and the total loss is the
mean over the three channels (App. A.7 averages the channel gradients).
SSIM at pixel (k, l) uses window moments with a Gaussian window w of radius r
summing to 1: mu = w * I, sigma^2 = w * I^2 - mu^2, sigma_xy = w * (I I_hat) - mu mu_hat,
SSIM = (2 mu mu_hat + c1)(2 sigma_xy + c2) / ((mu^2 + mu_hat^2 + c1)(sigma^2 + sigma_hat^2 + c2)),
c1 = 0.01^2, c2 = 0.03^2 (intensities in [0, 1]).

Readings where the paper is silent: the window is 11 x 11 (r = 5) with sigma
1.5 (the usual SSIM window), the image is zero outside its borders (every map
position sums the full window), and lambda defaults to 0.2.

dL_SSIM/dI follows App. A.7: (1/hw) ((E * w) + I_hat (F * w) - I (G * w)) with
the E, F, G maps defined there; here the window sums are written out as
direct 2-D sums over the (2r+1)^2 offsets (no separable filtering).
"""

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(radius=5, sigma=1.5):
    """(2r+1)^2 Gaussian window normalised to sum 1."""
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-x ** 2 / (2.0 * sigma ** 2))
    w2 = np.outer(g, g)
    return w2 / w2.sum()


def wsum(img, w):
    """sum_{m,n} w[m,n] img[k+m, l+n] for every (k, l), zero outside the image."""
    r = w.shape[0] // 2
    h, wd = img.shape
    pad = np.zeros((h + 2 * r, wd + 2 * r))
    pad[r:r + h, r:r + wd] = img
    out = np.zeros((h, wd))
    for m in range(-r, r + 1):
        for n in range(-r, r + 1):
            out += w[m + r, n + r] * pad[r + m:r + m + h, r + n:r + n + wd]
    return out


def ssim_terms(I, J, w):
    mu, mu_h = wsum(I, w), wsum(J, w)
    s2 = wsum(I * I, w) - mu * mu
    s2_h = wsum(J * J, w) - mu_h * mu_h
    sxy = wsum(I * J, w) - mu * mu_h
    A = 2 * mu * mu_h + C1
    B = 2 * sxy + C2
    C = mu * mu + mu_h * mu_h + C1
    D = s2 + s2_h + C2
    return mu, mu_h, A, B, C, D


def loss(img, target, lam=0.2, radius=5, sigma=1.5):
    """img, target: [h, w, 3]. Returns the scalar loss."""
    img = np.asarray(img, np.float64)
    target = np.asarray(target, np.float64)
    h, wd, _ = img.shape
    w = window(radius, sigma)
    tot = 0.0
    for ch in range(3):
        I, J = img[:, :, ch], target[:, :, ch]
        _, _, A, B, C, D = ssim_terms(I, J, w)
        ssim = (A * B / (C * D)).mean()
        l2 = ((I - J) ** 2).mean()
        tot += (1 - lam) * l2 + lam * (1 - ssim) / 2
    return tot / 3.0


def loss_grad(img, target, lam=0.2, radius=5, sigma=1.5):
    """dL/d img ([h, w, 3]) by the App. A.7 formula."""
    img = np.asarray(img, np.float64)
    target = np.asarray(target, np.float64)
    h, wd, _ = img.shape
    w = window(radius, sigma)
    wf = w[::-1, ::-1]  # (E * w)_ij = sum_kl E_kl w_{i-k, j-l}: a correlation with the flipped window
    out = np.zeros_like(img)
    for ch in range(3):
        I, J = img[:, :, ch], target[:, :, ch]
        mu, mu_h, A, B, C, D = ssim_terms(I, J, w)
        k = 2.0 / (C * C * D * D)
        E = k * (C * D * mu_h * (B - A) - A * B * mu * (D - C))
        F = k * A * C * D
        G = k * A * B * C
        dssim = (wsum(E, wf) + J * wsum(F, wf) - I * wsum(G, wf)) / (h * wd)
        out[:, :, ch] = (2 * (1 - lam) / (h * wd)) * (I - J) - (lam / 2) * dssim
    return out / 3.0
