"""GPU parity of the fine-tuning pieces (msp_loss, msp_adam_step, msp_prune,
msp_convert_rings) against the oracle, and the fine-tuning loop itself."""
import math

import numpy as np
import pytest

from oracle import convert as oc
from oracle import finetune as ft
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, gaussians_gpu, to_gpu

pytestmark = pytest.mark.gpu


def _imgs(seed, V=2, H=40, W=48):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (V, 4, H, W)).astype(np.float32)
    tgt = rng.uniform(0, 1, (V, 3, H, W)).astype(np.float32)
    return img, tgt


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_loss_parity(gpu, kind):
    import torch
    img, tgt = _imgs(kind)
    L, dimg = gpu.loss(torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda(), kind, 0.6)
    L = float(L.item())
    dimg = dimg.cpu().numpy().astype(np.float64)
    x = img[:, :3].astype(np.float64)
    y = tgt.astype(np.float64)
    if kind == 0:
        rl, rg = ft.mse(x, y)
    elif kind == 1:
        rl, rg = ft.l1(x, y)
    else:
        rl, rg = ft.paper_loss(x, y, 0.6)
    assert L == pytest.approx(rl, rel=1e-5)
    np.testing.assert_allclose(dimg[:, :3], rg, rtol=1e-3, atol=1e-4 * np.abs(rg).max())
    assert np.all(dimg[:, 3] == 0.0)


def test_loss_identical_images(gpu):
    import torch
    img, _ = _imgs(5)
    t = torch.from_numpy(img).cuda()
    L, _ = gpu.loss(t, t[:, :3].contiguous(), 2, 0.6)
    assert abs(float(L.item())) < 1e-6


def test_adam_parity(gpu):
    import torch
    rng = np.random.default_rng(3)
    p = rng.normal(size=1000).astype(np.float32)
    q = rng.uniform(0, 1, 300).astype(np.float32)
    pg, qg = torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda()
    state = {k: torch.zeros_like(v) for k, v in (("pm", pg), ("pv", pg), ("qm", qg), ("qv", qg))}
    rp, rq = p.astype(np.float64), q.astype(np.float64)
    rs = dict(pm=np.zeros(1000), pv=np.zeros(1000), qm=np.zeros(300), qv=np.zeros(300))
    for step in range(1, 4):
        g1 = rng.normal(size=1000).astype(np.float32)
        g2 = rng.normal(size=300).astype(np.float32)
        gpu.adam_step([dict(param=pg, grad=torch.from_numpy(g1).cuda(), m=state["pm"], v=state["pv"], lr=0.01),
                       dict(param=qg, grad=torch.from_numpy(g2).cuda(), m=state["qm"], v=state["qv"], lr=0.05,
                            clamp=(0.0, 1.0))], step)
        rp, rs["pm"], rs["pv"] = ft.adam_step(rp, g1, rs["pm"], rs["pv"], step, 0.01)
        rq, rs["qm"], rs["qv"] = ft.adam_step(rq, g2, rs["qm"], rs["qv"], step, 0.05, lo=0.0, hi=1.0)
        np.testing.assert_allclose(pg.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(qg.cpu().numpy(), rq, rtol=1e-5, atol=1e-6)
    assert float(qg.min()) >= 0.0 and float(qg.max()) <= 1.0


def test_prune_parity(gpu):
    import torch
    g = scenes.gaussians(400, 8, 0.01, 0.1, flat=True, sh=True)
    f = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0, sh=g.sh))
    rng = np.random.default_rng(1)
    # push a random third of the vertices below the threshold
    low = rng.uniform(0, 1, f["opacity"].shape) < 0.6
    f["opacity"] = np.where(low, np.float32(math.exp(-4) * 0.5), f["opacity"]).astype(np.float32)
    mom = rng.normal(size=(3, f["opacity"].shape[0])).astype(np.float32)
    ref, (rmom,) = ft.prune(f, math.exp(-4), [mom])
    fg = to_gpu(f)
    mg = torch.from_numpy(mom).cuda()
    out, (mo,) = gpu.prune(fg, math.exp(-4), [mg])
    assert out["idx"].shape[1] < f["idx"].shape[1] and out["pos"].shape[1] < f["pos"].shape[1]
    for k in ("pos", "opacity", "rgb", "idx", "gid", "sh"):
        np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].astype(out[k].cpu().numpy().dtype), err_msg=k)
    np.testing.assert_array_equal(mo.cpu().numpy(), rmom)


@pytest.mark.parametrize("K,rings", [(8, 3), (16, 4)])
def test_rings_parity(gpu, K, rings):
    g = scenes.gaussians(200, 6, 0.01, 0.1, flat=True)
    out = gpu.convert_rings(gaussians_gpu(g), K, rings, 3.0)
    ref = ft.ring_convert(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, rings)
    assert np.array_equal(out["idx"].cpu().numpy(), ref["idx"])
    assert np.array_equal(out["gid"].cpu().numpy(), ref["gid"])
    np.testing.assert_allclose(out["pos"].cpu().numpy(), ref["pos"], atol=4e-6)
    np.testing.assert_allclose(out["opacity"].cpu().numpy(), ref["opacity"], rtol=1e-6)


def test_finetune_reduces_error_and_resumes(gpu, tmp_path):
    """Fine-tuning with the paper's loss (the default) lowers the image MSE; in
    deterministic mode a run resumed from a checkpoint repeats the original
    run's next steps bit for bit (faces, moments and losses)."""
    import torch

    from paper_2502_07754_amd.finetune import FineTuneConfig, FineTuner
    g = scenes.gaussians(600, 30, 0.02, 0.12, flat=True)
    cams = scenes.ring_cameras(4, 64, 48)
    tgt_g = scenes.perturbed(g, 31)
    tf = gpu.convert_rings(gaussians_gpu(tgt_g), 16, 3, 3.0)
    timg, _ = gpu.render(tf, cams, gpu.RenderOptions())
    targets = timg[:, :3].contiguous()
    faces = gpu.convert(gaussians_gpu(g), 8, 2.0)
    cfg = FineTuneConfig(lr_color=1e-2, prune_every=5)
    assert cfg.loss_kind == gpu.MSP_LOSS_L1_DSSIM and cfg.lam == 0.6
    opts = gpu.RenderOptions(deterministic=1)
    ftn = FineTuner(faces, cams, targets, cfg, opts)
    e0 = ftn.mse()
    for _ in range(12):
        ftn.step()
    e1 = ftn.mse()
    assert e1 < 0.8 * e0, (e0, e1)
    path = str(tmp_path / "ck.npz")
    ftn.save(path)
    a = FineTuner(faces, cams, targets, cfg, opts)
    a.load(path)
    assert a.t == ftn.t
    for k in ("pos", "opacity", "rgb", "idx"):
        assert torch.equal(a.faces[k], ftn.faces[k])
    la = [float(a.step().item()) for _ in range(3)]
    lb = [float(ftn.step().item()) for _ in range(3)]
    assert la == lb, (la, lb)
    for k in ("pos", "opacity", "rgb", "idx"):
        assert torch.equal(a.faces[k], ftn.faces[k]), k
    for k in ("pos", "opacity", "rgb"):
        assert torch.equal(a.m[k], ftn.m[k]) and torch.equal(a.v[k], ftn.v[k]), k


def test_finetune_step_matches_oracle_chain(gpu):
    """One FineTuner step with the paper's loss (lambda = 0.6) on a small scene
    against the oracle chain: float64 render, Eq. loss and its gradient, the
    frozen-fragment adjoint over every pixel, Adam. Targets are seeded values
    above every image value, so the L1 term's sign never depends on rounding;
    every pixel must meet the image bar (no ambiguous pixel in this scene)."""
    import torch

    from oracle import render as orr
    from paper_2502_07754_amd.finetune import FineTuneConfig, FineTuner
    from tests.helpers import faces_f64, grad_close
    g = scenes.gaussians(150, 60, 0.03, 0.15, flat=True)
    f32 = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0))
    cams = scenes.ring_cameras(2, 40, 32)
    rng = np.random.default_rng(61)
    tgt = rng.uniform(1.1, 1.6, size=(2, 3, 32, 40)).astype(np.float32)
    fg = to_gpu(f32)
    opts = gpu.RenderOptions(t_eps=0.0)
    cfg = FineTuneConfig(lr_color=1e-2, prune_every=0)
    ftn = FineTuner(fg, cams, torch.from_numpy(tgt).cuda(), cfg, opts)
    # the image the step starts from (FineTuner works on its own copy of the faces)
    img, st = gpu.render(fg, cams, opts)
    L = float(ftn.step().item())
    f64 = faces_f64(f32)
    px = [(i, j) for j in range(32) for i in range(40)]
    ref_img = np.zeros((2, 3, 32, 40))
    gi = img.cpu().numpy().astype(np.float64)
    for v, cam in enumerate(cams):
        r = orr.render_pixels(f64, cam, px)
        got = np.stack([gi[v][:, j, i] for i, j in px])
        assert np.max(np.abs(got - r)) <= 1e-4, v
        for n, (i, j) in enumerate(px):
            ref_img[v, :, j, i] = r[n, :3]
    rl, rg = ft.paper_loss(ref_img, tgt.astype(np.float64), 0.6)
    assert L == pytest.approx(rl, rel=1e-5, abs=1e-6), (L, rl)
    dimg = np.zeros((2, 4, 32, 40))
    dimg[:, :3] = rg
    ref = dict(dpos=0.0, dop=0.0, drgb=0.0)
    for v, cam in enumerate(cams):
        r = orr.render_backward_pixels(f64, cam, px, [dimg[v, :, j, i] for i, j in px])
        for k in ref:
            ref[k] = ref[k] + r[k]
    lr = ft.lr_groups(1e-2)
    new = {}
    for key, gk, pk in (("pos", "dpos", "pos"), ("rgb", "drgb", "rgb"), ("opacity", "dop", "opacity")):
        clamp = (0.0, 1.0) if key == "opacity" else (None, None)
        p1, _, _ = ft.adam_step(f64[pk], ref[gk], 0.0, 0.0, 1, lr[key], lo=clamp[0], hi=clamp[1])
        new[key] = (p1, np.asarray(ref[gk]))
    for key, (p1, gref) in new.items():
        got = ftn.faces[key].cpu().numpy().astype(np.float64)
        step_ref = p1 - f64[key]
        step_got = got - f64[key]
        # where the gradient is well above its error bar the update is -lr sign(g) (Adam's first
        # step); elsewhere the sign may legitimately differ, and the step is bounded by lr
        firm = np.abs(gref) > 1e-2 * np.abs(gref).max()
        assert firm.sum() > 50, key
        np.testing.assert_allclose(step_got[firm], step_ref[firm], rtol=1e-3, atol=1e-7, err_msg=key)
        assert np.all(np.abs(step_got) <= lr[key] * (1 + 1e-5) + 1e-7), key
    # and the gradients themselves, from a backward of the GPU's own state
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg.astype(np.float32)).cuda())
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("drgb", "drgb")):
        ok, ex = grad_close(gr[k].cpu().numpy(), ref[rk])
        assert ok, (k, ex)


def test_finetune_tracks_mse_of_each_step(gpu):
    """FineTuner(track_mse=True) records, at every step, the image MSE of the
    render that step starts from (the training loss stays the paper's loss):
    it equals msp_loss's MSE of the same faces rendered before the step."""
    from paper_2502_07754_amd.finetune import FineTuneConfig, FineTuner
    g = scenes.gaussians(400, 32, 0.02, 0.12, flat=True)
    cams = scenes.ring_cameras(3, 48, 40)
    tf = gpu.convert_rings(gaussians_gpu(scenes.perturbed(g, 33)), 16, 3, 3.0)
    timg, _ = gpu.render(tf, cams, gpu.RenderOptions())
    targets = timg[:, :3].contiguous()
    faces = gpu.convert(gaussians_gpu(g), 8, 2.0)
    ftn = FineTuner(faces, cams, targets, FineTuneConfig(prune_every=0), gpu.RenderOptions(), track_mse=True)
    for _ in range(3):
        before = ftn.mse()
        L = ftn.step()
        assert float(ftn.last_mse.item()) == before
        assert float(L.item()) != before  # the step's loss is the L1 + (1 - SSIM) mix, not the MSE
