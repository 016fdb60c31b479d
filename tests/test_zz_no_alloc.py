"""msp_loss_noalloc (the entry point for callers that cannot allocate device
memory) against msp_loss, through the C ABI: every loss kind, two calls in a
row with the second on a smaller input (the fixed scratch keeps the first
call's contents), sizes beyond the fixed scratch rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _images(V, H, W, seed):
    import torch
    rng = np.random.default_rng(seed)
    img = torch.from_numpy(rng.uniform(0, 1, size=(V, 4, H, W)).astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.uniform(0, 1, size=(V, 3, H, W)).astype(np.float32)).cuda()
    return img, tgt


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_noalloc_loss_matches_msp_loss(gpu, kind):
    import torch
    for (V, H, W), seed in (((3, 96, 128), 1), ((1, 40, 33), 2)):
        img, tgt = _images(V, H, W, seed)
        ref_l, ref_g = gpu.loss(img, tgt, kind=kind, lam=0.6)
        out = torch.full((1,), float("nan"), device="cuda")
        dimg = torch.full_like(img, float("nan"))
        l, g = gpu.loss(img, tgt, kind=kind, lam=0.6, noalloc=True, out=out, dimg=dimg)
        torch.cuda.synchronize()
        assert torch.equal(l, ref_l), (kind, V, H, W, float(l), float(ref_l))
        assert torch.equal(g, ref_g), (kind, V, H, W)
        # loss only, no gradient
        l2, g2 = gpu.loss(img, tgt, kind=kind, lam=0.6, noalloc=True, want_grad=False)
        torch.cuda.synchronize()
        assert g2 is None and torch.equal(l2, ref_l)


def test_noalloc_loss_rejects_sizes_beyond_its_scratch(gpu):
    img, tgt = _images(8, 256, 256, 3)     # L1 + (1 - SSIM) needs ~66 MiB here
    with pytest.raises(gpu.MspError, match="fixed"):
        gpu.loss(img, tgt, kind=2, noalloc=True)
    l, _ = gpu.loss(img, tgt, kind=0, noalloc=True)   # MSE fits at any size
    r, _ = gpu.loss(img, tgt, kind=0)
    assert float(l) == float(r)
