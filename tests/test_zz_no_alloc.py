"""rs_loss_noalloc (the loss without a workspace argument, for callers that
cannot allocate) against rs_loss with a caller workspace: two calls in a row,
the second on a smaller image, both through the C ABI."""

import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _images(w, h, seed):
    rng = np.random.default_rng(seed)
    a = np.float32(rng.uniform(0, 1, (h, w, 3)))
    b = np.float32(np.clip(a + rng.normal(scale=0.1, size=a.shape), 0, 1))
    return torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()


def test_noalloc_loss_equals_workspace_loss():
    from paper_2501_19196_amd import _lib as L
    lib = L.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lp = L.rs_loss_params()
    lib.rs_default_loss_params(C.byref(lp))
    p = lambda t: C.c_void_p(t.data_ptr())
    for w, h, seed in ((640, 480, 1), (200, 130, 2)):  # the second call smaller than the first
        print("case noalloc loss", w, h, flush=True)
        img, tgt = _images(w, h, seed)
        ws = torch.empty(int(lib.rs_loss_workspace_bytes(w, h)), dtype=torch.uint8, device="cuda")
        loss_ws, grad_ws = torch.empty(1, device="cuda"), torch.empty_like(img)
        loss_na, grad_na = torch.full((1,), float("nan"), device="cuda"), torch.full_like(img, float("nan"))
        assert lib.rs_loss(p(img), p(tgt), w, h, C.byref(lp), p(loss_ws), p(grad_ws), p(ws), stream) == 0
        assert lib.rs_loss_noalloc(p(img), p(tgt), w, h, C.byref(lp), p(loss_na), p(grad_na), stream) == 0
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical results
        np.testing.assert_array_equal(loss_na.cpu().numpy(), loss_ws.cpu().numpy())
        np.testing.assert_array_equal(grad_na.cpu().numpy(), grad_ws.cpu().numpy())
        assert np.isfinite(loss_na.cpu().numpy()).all() and float(loss_na) > 0


def test_noalloc_loss_rejects_images_beyond_its_scratch():
    from paper_2501_19196_amd import _lib as L
    lib = L.lib()
    lp = L.rs_loss_params()
    lib.rs_default_loss_params(C.byref(lp))
    img, tgt = _images(8, 8, 3)
    out = torch.empty(1, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    w = h = 4096  # 4096^2 pixels need 9 maps of 64 MiB, beyond the 96 MiB array
    assert lib.rs_loss_workspace_bytes(w, h) > lib.rs_loss_noalloc_max_bytes()
    assert lib.rs_loss_noalloc(p(img), p(tgt), w, h, C.byref(lp), p(out), None, None) == L.RS_ERR_UNSUPPORTED
