"""Captured fwd+bwd steps (msp_step_graph) and the tile autotuner (msp_autotune)
against the eager calls."""
import numpy as np
import pytest

from oracle import convert as oc
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, to_gpu

pytestmark = pytest.mark.gpu


def _scene(sh=False, n=600, seed=21):
    g = scenes.gaussians(n, seed, 0.02, 0.12, flat=True, sh=sh)
    return to_gpu(faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0, sh=g.sh)))


@pytest.mark.parametrize("sh", [False, True])
def test_graph_replays_match_eager(gpu, sh):
    import torch
    f = _scene(sh)
    cams = scenes.ring_cameras(3, 96, 64)
    opts = gpu.RenderOptions(tile_w=16, tile_h=16, color_mode=1 if sh else 0)
    print("graph sh", sh, flush=True)
    step = gpu.GraphStep(f, cams, opts)
    for rep in range(4):
        dimg = torch.from_numpy(scenes.upstream_grad(3, 64, 96, seed=10 + rep)).cuda()
        img, grads = step(dimg)
        torch.cuda.synchronize()
        img = img.clone()
        grads = {k: v.clone() for k, v in grads.items()}
        # eager work between replays
        eimg, st = gpu.render(f, cams, opts)
        eg = gpu.render_backward(st, f, dimg)
        torch.cuda.synchronize()
        assert torch.equal(img, eimg), rep
        for k in eg:
            assert torch.allclose(grads[k], eg[k], rtol=1e-4, atol=1e-6 * float(eg[k].abs().max())), (rep, k)
    info = step.info()
    assert info["captures"] == 1 and info["replays"] == 3 and info["overflows"] == 0


def test_graph_recaptures_after_overflow(gpu):
    import torch
    f = _scene(n=300, seed=22)
    cams = scenes.ring_cameras(2, 64, 64)
    opts = gpu.RenderOptions(tile_w=8, tile_h=8)
    step = gpu.GraphStep(f, cams, opts)
    dimg = torch.from_numpy(scenes.upstream_grad(2, 64, 64, seed=1)).cuda()
    step(dimg)
    step(dimg)
    # grow every face threefold in place: the tile lists outgrow the captured capacity
    g = f["pos"].view(3, -1, 9)
    centre = g[:, :, :1].clone()
    g.copy_(centre + 3.0 * (g - centre))
    img, grads = step(dimg)
    torch.cuda.synchronize()
    img = img.clone()
    eimg, st = gpu.render(f, cams, opts)
    eg = gpu.render_backward(st, f, dimg)
    torch.cuda.synchronize()
    assert torch.equal(img, eimg)
    for k in eg:
        assert torch.allclose(grads[k], eg[k], rtol=1e-4, atol=1e-6 * float(eg[k].abs().max()))
    info = step.info()
    assert info["overflows"] == 1 and info["captures"] == 2


def test_autotune_choice_renders_identically(gpu):
    import torch
    f = _scene(n=800, seed=23)
    cams = scenes.ring_cameras(2, 128, 96)
    base = gpu.RenderOptions()
    dimg = torch.from_numpy(scenes.upstream_grad(2, 96, 128, seed=2)).cuda()
    best = gpu.autotune(f, cams, base, dimg)
    assert (best.tile_w, best.tile_h) in [(8, 8), (16, 16), (32, 16), (32, 32)] and best.kbuf in (8, 12, 16)
    a, _ = gpu.render(f, cams, best)
    b, _ = gpu.render(f, cams, gpu.RenderOptions(tile_w=8, tile_h=8, kbuf=8))
    c, _ = gpu.render(f, cams, gpu.RenderOptions())  # context default is now the tuned choice
    assert torch.equal(a, b) and torch.equal(a, c)


def test_graph_replays_are_timed(gpu):
    """Stage events captured into the graph are read back after every replay."""
    import torch

    from paper_2502_07754_amd import _lib
    f = _scene(n=400, seed=24)
    cams = scenes.ring_cameras(2, 64, 64)
    opts = gpu.RenderOptions(tile_w=16, tile_h=16)
    ctx = _lib.Context.get(0)
    ctx.timing(True)
    try:
        step = gpu.GraphStep(f, cams, opts)
        dimg = torch.from_numpy(scenes.upstream_grad(2, 64, 64, seed=3)).cuda()
        step(dimg)                     # eager run + capture
        torch.cuda.synchronize()
        ctx.read_timing()
        for _ in range(3):
            step(dimg)
        t = ctx.read_timing()
        assert step.info()["replays"] == 3
        assert t["composite"][1] == 3 and t["composite"][0] > 0.0
        assert t["bwd_grads"][1] == 3 and t["setup"][1] == 3
        assert ctx.read_timing()["composite"] == (0.0, 0)
    finally:
        ctx.timing(False)
        ctx.read_timing()
