"""A few training steps end to end: the paper's activations (sigmoid opacity
and scale, Sec. 5), the renderer's autograd Function (BVH rebuilt every step),
the L2 + D-SSIM loss kernels and torch's Adam with the paper's beta and eps.
The loss must fall, and both adjoint forms (exact, the paper's variant) must
train the same scene."""

import numpy as np
import pytest
import torch

from synthetic import scenes
from synthetic.cameras import look_at_camera, pinhole_rays

pytestmark = pytest.mark.gpu


def _logit(x):
    x = np.clip(x, 1e-4, 1 - 1e-4)
    return np.log(x / (1 - x))


@pytest.mark.parametrize("flags,hit_list", [(0, 0), (0, 512), (16, 512)])
def test_adam_steps_reduce_the_loss(flags, hit_list):
    print("case train", flags, hit_list, flush=True)
    from paper_2501_19196_amd import renderer as R
    W, H = 64, 48
    true = scenes.random_scene(80, 1500, box=0.8, scale_lo=0.03, scale_hi=0.12)
    cam = look_at_camera((0, 0, -3), (0, 0, 0), (0, 1, 0), W, H, fov_y_deg=45)
    o, d = pinhole_rays(cam)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    p = R.Params(flags=flags, hit_list=hit_list, max_hits=512, eps2=1e-3)
    views = [(0, W, H)]
    with torch.no_grad():
        target = R.render(*(dev(a) for a in true.arrays()), dev(o), dev(d), p, views)
    # start from a perturbed copy: means jittered, opacities and colours reset
    rng = np.random.default_rng(81)
    mean = dev(true.mean + np.float32(rng.normal(scale=0.03, size=true.mean.shape))).requires_grad_(True)
    scale_raw = dev(np.float32(_logit(true.scale))).requires_grad_(True)
    quat = dev(true.quat).requires_grad_(True)
    opac_raw = dev(np.float32(np.zeros(true.n))).requires_grad_(True)
    rgb = dev(np.float32(np.full((true.n, 3), 0.5))).requires_grad_(True)
    opt = torch.optim.Adam([mean, scale_raw, quat, opac_raw, rgb], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    losses = []
    for _ in range(40):
        opt.zero_grad()
        img = R.render(mean, torch.sigmoid(scale_raw), quat, torch.sigmoid(opac_raw), rgb, dev(o), dev(d), p, views)
        loss = R.ImageLoss.apply(img, target, W, H, 0.2)
        loss.backward()
        opt.step()
        losses.append(float(loss))
    print("loss", losses[0], "->", losses[-1], flush=True)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0]
