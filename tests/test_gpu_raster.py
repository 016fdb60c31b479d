"""GPU parity of conversion, binning, ordering, compositing and the adjoint
against the CPU oracle, through the C ABI (msp_convert, msp_render,
msp_render_backward)."""
import numpy as np
import pytest

from oracle import binning as ob
from oracle import convert as oc
from oracle import render as orr
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, faces_f64, gaussians_gpu, grad_close, to_gpu

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4          # per channel, float32 image against the float64 oracle
MAX_FLAGGED = 0.02      # fraction of covered pixels allowed to be ambiguous


def _say(*a):
    print(*a, flush=True)


def _oracle_faces(g, K, sigma):
    return faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, sigma))


# ---------------------------------------------------------------------------
# conversion
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,K,flat", [(1000, 8, True), (777, 16, True), (513, 8, False), (64, 3, True), (5, 64, False)])
def test_convert_parity(gpu, n, K, flat):
    import torch
    _say("convert", n, K, flat)
    g = scenes.gaussians(n, 17, 0.01, 0.1, flat=flat)
    out = gpu.convert(gaussians_gpu(g), K, 2.0)
    torch.cuda.synchronize()
    ref = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0)
    assert np.array_equal(out["idx"].cpu().numpy(), ref["idx"])
    assert np.array_equal(out["gid"].cpu().numpy(), ref["gid"])
    pos = out["pos"].cpu().numpy().astype(np.float64)
    # 4 ulp of the magnitude of the terms that make up each coordinate
    mag = np.abs(np.asarray(g.mean, np.float64)) + 2.0 * np.max(np.asarray(g.scale, np.float64), axis=0)
    mag = np.repeat(mag, K + 1, axis=1)
    ulp = np.spacing(mag.astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(pos - ref["pos"]) <= 4 * ulp)
    op = out["opacity"].cpu().numpy()
    assert np.all(np.abs(op - ref["opacity"]) <= np.spacing(np.float32(ref["opacity"]).astype(np.float32)))
    assert np.array_equal(out["rgb"].cpu().numpy(), ref["rgb"].astype(np.float32))


def test_convert_sh_and_empty(gpu):
    import torch
    g = scenes.gaussians(300, 3, 0.01, 0.1, flat=True, sh=True)
    out = gpu.convert(gaussians_gpu(g), 16, 2.0)
    torch.cuda.synchronize()
    ref = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 16, 2.0, sh=g.sh)
    assert np.array_equal(out["sh"].cpu().numpy(), ref["sh"].astype(np.float32))
    e = scenes.gaussians(0, 3, 0.01, 0.1, flat=True)
    out = gpu.convert(gaussians_gpu(e), 8, 2.0)
    assert out["pos"].shape == (3, 0) and out["idx"].shape == (3, 0)


@pytest.mark.parametrize("n,K", [(1, 4), (257, 8), (1000, 16)])
def test_convert_three_fans_parity(gpu, n, K):
    """3D-Gaussian conversion (three fans sharing their axis points) against the oracle."""
    import torch
    _say("convert three fans", n, K)
    g = scenes.gaussians(n, 19, 0.005, 0.05, flat=False, sh=True)
    out = gpu.convert(gaussians_gpu(g), K, 2.0, mode=gpu.MSP_FAN_3D)
    torch.cuda.synchronize()
    ref = oc.convert_three_fans(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0)
    assert np.array_equal(out["idx"].cpu().numpy(), ref["idx"])
    assert np.array_equal(out["gid"].cpu().numpy(), ref["gid"])
    per = 7 + 3 * (K - 4)
    mag = np.abs(np.asarray(g.mean, np.float64)) + 2.0 * np.max(np.asarray(g.scale, np.float64), axis=0)
    ulp = np.spacing(np.repeat(mag, per, axis=1).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(out["pos"].cpu().numpy().astype(np.float64) - ref["pos"]) <= 4 * ulp)
    np.testing.assert_allclose(out["opacity"].cpu().numpy(), ref["opacity"], rtol=1e-6)
    assert np.array_equal(out["rgb"].cpu().numpy(), ref["rgb"].astype(np.float32))
    sh = np.asarray(g.sh, np.float32)
    assert np.array_equal(out["sh"].cpu().numpy(), np.repeat(sh, 3 * K, axis=1))


def test_three_fan_image_parity(gpu):
    """A small 3D scene converted with three fans renders like the oracle."""
    g = scenes.gaussians(150, 23, 0.05, 0.2, flat=False)
    f = faces_f32(oc.convert_three_fans(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0))
    cam = scenes.ring_cameras(1, 48, 40)[0]
    img, _ = gpu.render(to_gpu(f), [cam], gpu.RenderOptions(t_eps=0.0))
    px = [(i, j) for j in range(40) for i in range(48)]
    unexplained, flagged, covered, worst = _check_image(img[0].cpu().numpy().astype(np.float64), f, cam, px)
    print("three fans:", worst, flagged, covered, flush=True)
    assert not unexplained and flagged <= 0.02 * covered


def test_convert_rejects_bad_sigma(gpu):
    g = scenes.gaussians(10, 3, 0.01, 0.1, flat=True)
    for s in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(gpu.MspError):
            gpu.convert(gaussians_gpu(g), 8, s)


# ---------------------------------------------------------------------------
# tile lists and their order: bit-exact against the float32 statement
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 16)])
def test_tile_lists_bit_exact_config1(gpu, tile):
    g, cams, p = scenes.config1()
    f = _oracle_faces(g, p["K"], p["sigma"])
    _say("tiles config1", tile)
    img, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=tile[0], tile_h=tile[1]))
    off, keys = st.tiles(0)
    roff, rkeys = ob.tile_lists(f["pos"], f["idx"], cams[0], *tile)
    assert np.array_equal(off, roff)
    assert np.array_equal(keys, rkeys)
    _, (px0, px1, py0, py1), _ = ob.face_ranges(f["pos"], f["idx"], cams[0])
    assert st.stats()["footprint_pixels"] == int(np.sum((px1 - px0 + 1) * (py1 - py0 + 1)))


def test_tile_lists_bit_exact_multiview_ragged(gpu):
    g = scenes.gaussians(3000, 9, 0.01, 0.1, flat=True)
    f = _oracle_faces(g, 8, 2.0)
    cams = scenes.ring_cameras(3, 100, 70)
    _say("tiles multiview ragged")
    _, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=16, tile_h=8))
    for v in range(3):
        off, keys = st.tiles(v)
        roff, rkeys = ob.tile_lists(f["pos"], f["idx"], cams[v], 16, 8)
        assert np.array_equal(off, roff) and np.array_equal(keys, rkeys), v


def test_tile_lists_bit_exact_config2(gpu):
    g, cams, p = scenes.config2()
    f = _oracle_faces(g, p["K"], p["sigma"])
    _say("tiles config2")
    _, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=16, tile_h=16))
    off, keys = st.tiles(0)
    roff, rkeys = ob.tile_lists(f["pos"], f["idx"], cams[0], 16, 16)
    assert np.array_equal(off, roff)
    assert np.array_equal(keys, rkeys)


@pytest.mark.parametrize("n,seed", [(2000, 41), (6000, 42), (9000, 43), (16000, 45)])
def test_tile_lists_bit_exact_long_lists(gpu, n, seed):
    """Large Gaussians over a small image: tile lists of ~9k to ~71k entries,
    longer than one sorting chunk, so they go through the pairwise merges
    (several passes, and odd run counts that carry a run through a pass
    unmerged)."""
    g = scenes.gaussians(n, seed, 0.3, 0.6, flat=True)
    f = _oracle_faces(g, 8, 2.0)
    cams = scenes.ring_cameras(1, 64, 48)
    _say("tiles long lists", n)
    _, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=32, tile_h=32))
    off, keys = st.tiles(0)
    roff, rkeys = ob.tile_lists(f["pos"], f["idx"], cams[0], 32, 32)
    assert np.diff(roff).max() > 8192
    assert np.array_equal(off, roff)
    assert np.array_equal(keys, rkeys)


# ---------------------------------------------------------------------------
# images
# ---------------------------------------------------------------------------
def _check_image(gpu_img, f, cam, pixels, bg=(0.0, 0.0, 0.0), view_col=None, processes=8):
    f64 = faces_f64(f)
    ref = orr.render_pixels(f64, cam, pixels, bg=bg, view_col=view_col)
    got = np.stack([gpu_img[:, j, i] for i, j in pixels])
    err = np.max(np.abs(got - ref), axis=1)
    bad = np.flatnonzero(err > IMG_TOL)
    flagged = np.zeros(len(pixels), dtype=bool)
    if len(bad):
        flagged[bad] = orr.ambiguous_pixels(f64, cam, [pixels[b] for b in bad], bg=bg, view_col=view_col)
    unexplained = [pixels[b] for b in bad if not flagged[b]]
    covered = max(1, int(np.sum(ref[:, 3] > 0)))
    return unexplained, int(flagged.sum()), covered, float(err.max()) if len(err) else 0.0


@pytest.mark.parametrize("tile,kbuf", [((16, 16), 16), ((8, 8), 8), ((32, 16), 16), ((32, 16), 12)])
def test_image_config1_all_pixels(gpu, tile, kbuf):
    g, cams, p = scenes.config1()
    f = _oracle_faces(g, p["K"], p["sigma"])
    _say("image config1", tile, kbuf)
    img, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=tile[0], tile_h=tile[1], kbuf=kbuf, t_eps=0.0))
    img = img[0].cpu().numpy().astype(np.float64)
    px = [(i, j) for j in range(128) for i in range(128)]
    unexplained, nflag, covered, worst = _check_image(img, f, cams[0], px)
    _say("worst", worst, "flagged", nflag, "covered", covered)
    assert not unexplained, unexplained[:10]
    assert nflag <= MAX_FLAGGED * covered


def test_image_early_stop_bound(gpu):
    """With t_eps = 1e-6 the image differs from the full composite by at most t_eps per channel."""
    g, cams, p = scenes.config1()
    f = to_gpu(_oracle_faces(g, p["K"], p["sigma"]))
    a, _ = gpu.render(f, cams, gpu.RenderOptions(t_eps=0.0))
    b, _ = gpu.render(f, cams, gpu.RenderOptions(t_eps=1e-6))
    assert float((a - b).abs().max()) <= 2e-6


def test_image_config2_sampled(gpu):
    g, cams, p = scenes.config2()
    f = _oracle_faces(g, p["K"], p["sigma"])
    _say("image config2")
    img, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(tile_w=16, tile_h=16, t_eps=0.0))
    img = img[0].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(2)
    px = [(int(i), int(j)) for i, j in rng.integers(250, 550, size=(24, 2))]
    unexplained, nflag, covered, worst = _check_image(img, f, cams[0], px)
    _say("worst", worst, "flagged", nflag)
    assert not unexplained, unexplained
    assert nflag <= 2
    s = st.stats()
    assert s["entries"] > 0 and s["fragments"] > 0


def test_image_deep_overlap_forces_rescans(gpu):
    """Many large overlapping faces at interleaved depths: the ordering buffer
    overflows, the rescans keep the exact order."""
    rng = np.random.default_rng(4)
    F = 120
    c = np.zeros((F, 1, 3)) + [0, 0, 3.0]
    tris = c + rng.normal(0, 0.5, (F, 3, 3)) * [1, 1, 0.4]
    f = dict(pos=tris.reshape(F * 3, 3).T.copy(), opacity=rng.uniform(0.02, 0.15, F * 3),
             rgb=rng.uniform(0, 1, (3, F * 3)), idx=np.arange(3 * F, dtype=np.int32).reshape(F, 3).T.copy())
    f = faces_f32(f)
    cam = scenes.Camera(world_to_cam=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32),
                        fx=30.0, fy=30.0, cx=16.0, cy=16.0, width=32, height=32)
    _say("deep overlap")
    img, st = gpu.render(to_gpu(f), [cam], gpu.RenderOptions(tile_w=8, tile_h=8, kbuf=8, t_eps=0.0))
    s = st.stats()
    assert s["restarts"] > 0
    img = img[0].cpu().numpy().astype(np.float64)
    px = [(i, j) for j in range(32) for i in range(32)]
    unexplained, nflag, covered, worst = _check_image(img, f, cam, px)
    _say("worst", worst, "restarts", s["restarts"])
    assert not unexplained, unexplained[:10]


def test_image_empty_and_culled(gpu):
    import torch
    cam = scenes.ring_cameras(1, 40, 24)[0]
    empty = dict(pos=np.zeros((3, 0), np.float32), opacity=np.zeros(0, np.float32), rgb=np.zeros((3, 0), np.float32),
                 idx=np.zeros((3, 0), np.int32))
    img, _ = gpu.render(to_gpu(empty), [cam], gpu.RenderOptions(bg=(0.25, 0.5, 0.75)))
    exp = torch.tensor([0.25, 0.5, 0.75, 0.0], device=img.device).view(1, 4, 1, 1).expand_as(img)
    assert torch.equal(img, exp)
    g = scenes.gaussians(200, 1, 0.01, 0.1, flat=True)
    f = _oracle_faces(g, 8, 2.0)
    # every corner ends up at z_c < 0: the whole scene is behind the camera
    behind = scenes.Camera(world_to_cam=np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, -10]], np.float32),
                           fx=20.0, fy=20.0, cx=20.0, cy=12.0, width=40, height=24)
    img, st = gpu.render(to_gpu(f), [behind], gpu.RenderOptions())
    assert float(img[:, 3].abs().max()) == 0.0 and st.stats()["entries"] == 0


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def test_backward_small_scene_all_pixels(gpu):
    import torch
    g = scenes.gaussians(200, 31, 0.02, 0.15, flat=True)
    f = _oracle_faces(g, 8, 2.0)
    cam = scenes.ring_cameras(1, 48, 40)[0]
    dimg = scenes.upstream_grad(1, 40, 48, seed=3)
    _say("backward small")
    fg = to_gpu(f)
    img, st = gpu.render(fg, [cam], gpu.RenderOptions(t_eps=0.0, bg=(0.1, 0.2, 0.3)))
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg).cuda())
    torch.cuda.synchronize()
    px = [(i, j) for j in range(40) for i in range(48)]
    f64 = faces_f64(f)
    # pixels where float32 may pick another fragment set are left out of the comparison
    ref_img = orr.render_pixels(f64, cam, px, bg=(0.1, 0.2, 0.3))
    gi = img[0].cpu().numpy().astype(np.float64)
    got = np.stack([gi[:, j, i] for i, j in px])
    bad = np.flatnonzero(np.max(np.abs(got - ref_img), axis=1) > IMG_TOL)
    keep = [p for n, p in enumerate(px) if n not in set(bad.tolist())]
    assert len(bad) <= 0.02 * len(px)
    if len(bad):
        # rerun the GPU backward with the gradient zeroed on the left-out pixels
        d2 = dimg.copy()
        for n in bad:
            i, j = px[n]
            d2[0, :, j, i] = 0.0
        gr = gpu.render_backward(st, fg, torch.from_numpy(d2).cuda())
        dimg = d2
    ref = orr.render_backward_pixels(f64, cam, keep, [dimg[0, :, j, i] for i, j in keep], bg=(0.1, 0.2, 0.3))
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("drgb", "drgb")):
        ok, ex = grad_close(gr[k].cpu().numpy(), ref[rk])
        assert ok, (k, ex)


def test_backward_config2_sampled_pixels(gpu):
    """Full config-2 scene; the upstream gradient is non-zero only on sampled
    pixels, so the GPU gradient is the sum of those pixels' contributions,
    which the oracle computes one by one."""
    import torch
    g, cams, p = scenes.config2()
    f = _oracle_faces(g, p["K"], p["sigma"])
    fg = to_gpu(f)
    _say("backward config2")
    img, st = gpu.render(fg, cams, gpu.RenderOptions(t_eps=0.0))
    rng = np.random.default_rng(8)
    px = [(int(i), int(j)) for i, j in rng.integers(300, 500, size=(12, 2))]
    f64 = faces_f64(f)
    ref_img = orr.render_pixels(f64, cams[0], px)
    gi = img[0].cpu().numpy().astype(np.float64)
    px = [p for n, p in enumerate(px) if np.max(np.abs(gi[:, p[1], p[0]] - ref_img[n])) <= IMG_TOL]
    assert len(px) >= 10
    full = scenes.upstream_grad(1, 800, 800, seed=3)
    dimg = np.zeros_like(full)
    for i, j in px:
        dimg[0, :, j, i] = full[0, :, j, i]
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg).cuda())
    ref = orr.render_backward_pixels(f64, cams[0], px, [dimg[0, :, j, i] for i, j in px])
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("drgb", "drgb")):
        a = gr[k].cpu().numpy()
        ok, ex = grad_close(a, ref[rk])
        assert ok, (k, ex)
        assert np.count_nonzero(ref[rk]) > 0


def test_backward_config2_finite_differences(gpu):
    """Central finite differences (h = 1e-3) of the loss sum(g * image) on the
    full 800x800 / 800k-face scene, for the opacity and the three colour
    channels of one vertex of each of 64 random faces, against the adjoint.
    These parameters change values, never coverage, so the difference quotient
    is the frozen-fragment derivative; positions move coverage at h = 1e-3
    (a quarter pixel here) and are checked against the oracle's gradient,
    which finite differences pin on the CPU."""
    import torch
    g, cams, p = scenes.config2()
    fg = to_gpu(_oracle_faces(g, p["K"], p["sigma"]))
    opts = gpu.RenderOptions(t_eps=0.0)
    img, st = gpu.render(fg, cams, opts)
    up = torch.from_numpy(scenes.upstream_grad(1, 800, 800, seed=9)).cuda()
    gr = gpu.render_backward(st, fg, up)
    gr = {k: v.cpu().numpy().astype(np.float64) for k, v in gr.items()}
    base = img.double()
    rng = np.random.default_rng(12)
    # 64 random faces among those with a visible vertex: a 1e-3 step of a hidden vertex changes
    # no pixel at float32 resolution, so finite differences cannot resolve its (tiny) gradient
    idx = fg["idx"].cpu().numpy()
    corner = rng.integers(0, 3, idx.shape[1])
    cand = np.flatnonzero(np.abs(gr["dopacity"][idx[corner, np.arange(idx.shape[1])]]) >= 1e-2)
    faces = rng.choice(cand, 64, replace=False)
    verts = idx[corner[faces], faces]
    h = 1e-3
    _say("finite differences config2")

    def loss_delta(param, index):
        """(L(+h) - L(-h)) / (actual step) with the float32 values actually rendered, and the
        rounding bound of that quotient: 8 ulp(1) per changed pixel channel, weighted by |g|."""
        x0 = float(param[index])
        vals, noise = [], 0.0
        for s in (+1, -1):
            param[index] = x0 + s * h
            xs = float(param[index])
            im, _ = gpu.render(fg, cams, opts)
            d = im.double() - base
            vals.append((float((d * up.double()).sum()), xs))
            noise += float(((d != 0).double() * up.double().abs()).sum()) * 8 * 2.0 ** -23
        param[index] = x0
        step = vals[0][1] - vals[1][1]
        return (vals[0][0] - vals[1][0]) / step, noise / abs(step)

    checked = 0
    for v in verts:
        v = int(v)
        cases = [] if not (h < float(fg["opacity"][v]) < 1 - h) else [(fg["opacity"], v, gr["dopacity"][v])]
        cases += [(fg["rgb"][c], v, gr["drgb"][c, v]) for c in range(3)]
        for param, index, want in cases:
            if abs(want) < 1e-3:
                continue
            fd, tol = loss_delta(param, index)
            assert abs(fd - want) <= 1e-3 * abs(want) + tol, (v, fd, want, tol)
            checked += 1
    _say("finite differences checked", checked)
    assert checked >= 128


def test_autograd_function(gpu):
    import torch
    g = scenes.gaussians(100, 5, 0.02, 0.15, flat=True)
    f = to_gpu(_oracle_faces(g, 8, 2.0))
    cam = scenes.ring_cameras(1, 32, 32)[0]
    pos = f["pos"].clone().requires_grad_(True)
    op = f["opacity"].clone().requires_grad_(True)
    rgb = f["rgb"].clone().requires_grad_(True)
    img = gpu.MeshRender.apply(pos, op, rgb, f["idx"], [cam], gpu.RenderOptions())
    w = torch.randn_like(img)
    (img * w).sum().backward()
    _, st = gpu.render(f, [cam], gpu.RenderOptions())
    ref = gpu.render_backward(st, f, w.contiguous())
    assert torch.allclose(pos.grad, ref["dpos"], rtol=1e-5, atol=1e-7)
    assert torch.allclose(op.grad, ref["dopacity"], rtol=1e-5, atol=1e-7)
    assert torch.allclose(rgb.grad, ref["drgb"], rtol=1e-5, atol=1e-7)


def test_render_rejects_bad_arguments(gpu):
    g = scenes.gaussians(10, 1, 0.01, 0.1, flat=True)
    f = to_gpu(_oracle_faces(g, 8, 2.0))
    cams = scenes.ring_cameras(2, 32, 32)
    with pytest.raises(gpu.MspError):
        gpu.render(f, cams, gpu.RenderOptions(tile_w=12))
    with pytest.raises(gpu.MspError):
        gpu.render(f, cams, gpu.RenderOptions(kbuf=5))
    bad = scenes.ring_cameras(1, 16, 32)
    with pytest.raises(gpu.MspError):
        gpu.render(f, [cams[0], bad[0]], gpu.RenderOptions())


# ---------------------------------------------------------------------------
# spherical-harmonics colour (per face, per view)
# ---------------------------------------------------------------------------
def _sh_scene(n=400, K=16, seed=12):
    g = scenes.gaussians(n, seed, 0.02, 0.15, flat=True, sh=True)
    f = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, sh=g.sh))
    return f


def test_sh_images_multiview(gpu):
    from oracle import sh as osh
    f = _sh_scene()
    cams = scenes.ring_cameras(3, 56, 40)
    _say("sh images")
    img, st = gpu.render(to_gpu(f), cams, gpu.RenderOptions(t_eps=0.0, color_mode=1, bg=(0.05, 0.1, 0.0)))
    img = img.cpu().numpy().astype(np.float64)
    f64 = faces_f64(f)
    for v, cam in enumerate(cams):
        col, _ = osh.face_colours(f64["sh"], f64["pos"], f64["idx"], cam)
        px = [(i, j) for j in range(40) for i in range(56)]
        unexplained, nflag, covered, worst = _check_image(img[v], f, cam, px, bg=(0.05, 0.1, 0.0), view_col=col)
        _say("view", v, "worst", worst, "flagged", nflag)
        assert not unexplained, unexplained[:10]
        assert nflag <= MAX_FLAGGED * covered


def test_sh_backward_multiview(gpu):
    import torch
    from oracle import sh as osh
    f = _sh_scene(n=150, K=16, seed=13)
    cams = scenes.ring_cameras(2, 40, 32)
    fg = to_gpu(f)
    _say("sh backward")
    img, st = gpu.render(fg, cams, gpu.RenderOptions(t_eps=0.0, color_mode=1))
    dimg = scenes.upstream_grad(2, 32, 40, seed=5)
    f64 = faces_f64(f)
    px = [(i, j) for j in range(32) for i in range(40)]
    gi = img.cpu().numpy().astype(np.float64)
    ref = dict(dpos=np.zeros_like(f64["pos"]), dop=np.zeros_like(f64["opacity"]), dsh=np.zeros_like(f64["sh"]))
    for v, cam in enumerate(cams):
        col, _ = osh.face_colours(f64["sh"], f64["pos"], f64["idx"], cam)
        rimg = orr.render_pixels(f64, cam, px, view_col=col)
        got = np.stack([gi[v][:, j, i] for i, j in px])
        for n in np.flatnonzero(np.max(np.abs(got - rimg), axis=1) > IMG_TOL):
            i, j = px[n]
            dimg[v, :, j, i] = 0.0
        r = orr.render_backward_pixels(f64, cam, px, [dimg[v, :, j, i] for i, j in px], view_col=col)
        dsh, dpos_dir = osh.face_colours_backward(f64["sh"], f64["pos"], f64["idx"], cam, r["dcol"])
        ref["dpos"] += r["dpos"] + dpos_dir
        ref["dop"] += r["dop"]
        ref["dsh"] += dsh
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg).cuda())
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("dsh", "dsh")):
        ok, ex = grad_close(gr[k].cpu().numpy(), ref[rk])
        assert ok, (k, ex)


@pytest.mark.parametrize("sh", [False, True])
def test_stored_lists_backward_matches_recompute(gpu, sh):
    """Lists stored by the forward give the same gradients as recomputed ones,
    also with row budgets that are not a multiple of the 8-row groups the lists
    are laid out in (the scene's longest list exactly, and 5 rows more); a row
    budget too small for the scene falls back to recomputation."""
    import torch
    f = to_gpu(_sh_scene(n=500, K=8, seed=40) if sh else _oracle_faces(scenes.gaussians(500, 40, 0.02, 0.15, True), 8, 2.0))
    cams = scenes.ring_cameras(2, 80, 64)
    dimg = torch.from_numpy(scenes.upstream_grad(2, 64, 80, seed=6)).cuda()
    cm = 1 if sh else 0
    base = gpu.RenderOptions(color_mode=cm)
    i0, s0 = gpu.render(f, cams, base)
    g0 = gpu.render_backward(s0, f, dimg)
    mx = int(s0.nfrag().max())
    assert mx > 8
    for rows in (64, mx, mx + 5, 1):
        o = gpu.RenderOptions(color_mode=cm, list_rows=rows)
        i1, s1 = gpu.render(f, cams, o)
        g1 = gpu.render_backward(s1, f, dimg)
        torch.cuda.synchronize()
        if rows >= mx:
            assert s1.status() == 0, rows     # the stored lists were used
        assert torch.equal(i0, i1)
        for k in g0:
            assert torch.allclose(g0[k], g1[k], rtol=1e-4, atol=1e-6 * float(g0[k].abs().max())), (rows, k)
    # the captured step with stored lists
    step = gpu.GraphStep(f, cams, gpu.RenderOptions(color_mode=cm, list_rows=64))
    for _ in range(3):
        img, gr = step(dimg)
    torch.cuda.synchronize()
    assert torch.equal(img, i0)
    for k in g0:
        assert torch.allclose(g0[k], gr[k], rtol=1e-4, atol=1e-6 * float(g0[k].abs().max()))
