"""Seeded Gaussian scenes shaped like the paper's trained scenes.

The paper trains on Mip-NeRF360, Tanks & Temples and Deep Blending (Sec. 4,
Table 1); those datasets and trained scenes are not available, so these
generators stand in for them at the scene sizes of the measured workloads.

Every array is float32 and C-contiguous. Parameters are the *activated*
values the renderer consumes: world-space scales (> 0), opacity in [0, 1),
raw quaternions (r, i, j, k) that need not be unit length, RGB in [0, 1].
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Scene:
    mean: np.ndarray     # [n, 3] float32
    scale: np.ndarray    # [n, 3] float32, > 0
    quat: np.ndarray     # [n, 4] float32, (r, i, j, k), nonzero
    opacity: np.ndarray  # [n]    float32, in [0, 1)
    rgb: np.ndarray      # [n, 3] float32

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def arrays(self):
        return self.mean, self.scale, self.quat, self.opacity, self.rgb

    def copy(self) -> "Scene":
        return Scene(*(a.copy() for a in self.arrays()))

    def subset(self, idx) -> "Scene":
        return Scene(*(np.ascontiguousarray(a[idx]) for a in self.arrays()))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _attributes(rng, n, flat_frac, scale_kind="loguniform", opacity_kind="sigmoid01"):
    """Scales, quaternions, opacities and colours for n Gaussians."""
    if scale_kind == "loguniform":
        scale = np.exp(rng.uniform(np.log(0.01), np.log(0.1), size=(n, 3)))
    elif scale_kind == "lognormal":
        scale = np.exp(rng.normal(np.log(0.02), 0.7, size=(n, 3)))
    else:
        raise ValueError(scale_kind)
    flat = rng.random(n) < flat_frac
    axis = rng.integers(0, 3, size=n)
    scale[flat, axis[flat]] = 1e-5
    quat = rng.normal(size=(n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    if opacity_kind == "sigmoid01":
        opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    elif opacity_kind == "mixed":
        opaque = rng.random(n) < 0.2
        opacity = _sigmoid(rng.normal(-1.0, 1.0, size=n))
        opacity[opaque] = rng.uniform(0.95, 0.999, size=int(opaque.sum()))
    else:
        raise ValueError(opacity_kind)
    # float32 rounding of sigmoid(x) for large x can give exactly 1.0; keep < 1.
    opacity = np.minimum(opacity, 0.999)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    return scale, quat, opacity, rgb


def random_scene(seed, n, box=1.0, flat_frac=0.3, scale_lo=0.01, scale_hi=0.1):
    """Uniform means in [-box, box]^3 with the default attribute mix."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-box, box, size=(n, 3))
    scale = np.exp(rng.uniform(np.log(scale_lo), np.log(scale_hi), size=(n, 3)))
    flat = rng.random(n) < flat_frac
    axis = rng.integers(0, 3, size=n)
    scale[flat, axis[flat]] = 1e-5
    quat = rng.normal(size=(n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    opacity = np.minimum(_sigmoid(rng.normal(size=n)), 0.999)
    rgb = rng.uniform(size=(n, 3))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(rgb))


def scene_config1(seed=0, n=1000):
    """1k Gaussians, means uniform in [-1,1]^3, 30% flat."""
    return random_scene(seed, n, box=1.0, flat_frac=0.3)


def _clustered_means(rng, n, n_clusters=8, centre_box=1.4, sigma=0.3, bound=2.0):
    centres = rng.uniform(-centre_box, centre_box, size=(n_clusters, 3))
    out = np.empty((0, 3))
    while out.shape[0] < n:
        k = rng.integers(0, n_clusters, size=2 * n)
        pts = centres[k] + rng.normal(0.0, sigma, size=(2 * n, 3))
        pts = pts[np.all(np.abs(pts) <= bound, axis=1)]
        out = np.concatenate([out, pts])
    return out[:n]


def scene_config2(seed=1, n=100_000, flat_frac=0.3):
    """8 isotropic clusters (sigma 0.3) rejection-sampled into [-2,2]^3."""
    rng = np.random.default_rng(seed)
    mean = _clustered_means(rng, n)
    scale, quat, opacity, rgb = _attributes(rng, n, flat_frac)
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(rgb))


def jittered_target(scene, seed=2, sigma=0.01):
    """Copy of a scene with means moved by N(0, sigma^2) per coordinate."""
    rng = np.random.default_rng(seed)
    t = scene.copy()
    t.mean = _f32(scene.mean.astype(np.float64) + rng.normal(0.0, sigma, size=scene.mean.shape))
    return t


def scene_config3(seed=3, n=300_000):
    """Clustered layout with 40% flat Gaussians."""
    return scene_config2(seed=seed, n=n, flat_frac=0.4)


def _ground_and_clusters(rng, n):
    n_plane = n // 2
    plane = np.empty((n_plane, 3))
    plane[:, :2] = rng.uniform(-4.0, 4.0, size=(n_plane, 2))
    plane[:, 2] = rng.normal(0.0, 0.02, size=n_plane)
    n_cl = n - n_plane
    centres = np.empty((64, 3))
    centres[:, :2] = rng.uniform(-3.0, 3.0, size=(64, 2))
    centres[:, 2] = rng.uniform(0.2, 2.0, size=64)
    k = rng.integers(0, 64, size=n_cl)
    cl = centres[k] + rng.normal(0.0, 0.3, size=(n_cl, 3))
    mean = np.concatenate([plane, cl])
    return mean[rng.permutation(n)]


def scene_config4(seed=4, n=1_000_000):
    """Ground plane plus 64 clusters; log-normal scales; 20% near-opaque."""
    rng = np.random.default_rng(seed)
    mean = _ground_and_clusters(rng, n)
    scale, quat, opacity, rgb = _attributes(rng, n, 0.3, scale_kind="lognormal", opacity_kind="mixed")
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(rgb))


def scene_config5(seed=5, n=500_000):
    """The scene-scale distribution at 500k Gaussians (used with a mirror mesh)."""
    return scene_config4(seed=seed, n=n)
