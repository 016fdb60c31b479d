"""GPU parity of the render adjoint beyond the basic scenes: faces seen nearly
edge-on (the ray/triangle Jacobian is ill-conditioned there), the
deterministic (fixed-point) summation mode against the float-atomic one and
against the oracle, graphs discarded by uncaptured calls on their state, and
the capacity report of a state. All through the C ABI."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import convert as oc
from oracle import render as orr
from oracle import sh as osh
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, faces_f64, grad_close, to_gpu

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _say(*a):
    print(*a, flush=True)


def _frozen_images_and_mask(gpu, fg, f, cams, opts, view_col=None):
    """Renders on the GPU; returns (img, state, list of per-view pixel lists whose
    GPU value matches the oracle at the image bar)."""
    img, st = gpu.render(fg, cams, opts)
    gi = img.cpu().numpy().astype(np.float64)
    f64 = faces_f64(f)
    keep = []
    for v, cam in enumerate(cams):
        H, W = int(cam.height), int(cam.width)
        px = [(i, j) for j in range(H) for i in range(W)]
        col = None if view_col is None else view_col[v]
        ref = orr.render_pixels(f64, cam, px, bg=opts.bg, view_col=col)
        got = np.stack([gi[v][:, j, i] for i, j in px])
        ok = np.max(np.abs(got - ref), axis=1) <= IMG_TOL
        keep.append([p for n, p in enumerate(px) if ok[n]])
        _say("view", v, "pixels outside the image bar", int((~ok).sum()), "of", len(px))
        assert (~ok).sum() <= 0.02 * len(px)
    return img, st, keep


def _masked_upstream(shape, keep, seed):
    full = scenes.upstream_grad(*shape, seed=seed)
    d = np.zeros_like(full)
    for v, px in enumerate(keep):
        for i, j in px:
            d[v, :, j, i] = full[v, :, j, i]
    return d


# ---------------------------------------------------------------------------
# faces seen nearly edge-on
# ---------------------------------------------------------------------------
def _oblique_fans(n, seed, cam_pos, cos_lo, cos_hi, K=8):
    """n flat Gaussians whose fan plane makes |cos(normal, view ray)| in
    [cos_lo, cos_hi] with the ray from cam_pos to the Gaussian's mean."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-0.7, 0.7, size=(n, 3))
    scale = np.zeros((n, 3))
    scale[:, :2] = np.exp(rng.uniform(np.log(0.15), np.log(0.35), size=(n, 2)))
    quat = np.zeros((n, 4))
    cosv = np.zeros(n)
    for g in range(n):
        v = mean[g] - cam_pos
        v /= np.linalg.norm(v)
        u = np.cross(v, rng.normal(size=3))
        u /= np.linalg.norm(u)
        c = rng.uniform(cos_lo, cos_hi) * rng.choice([-1.0, 1.0])
        nrm = np.sqrt(1 - c * c) * u + c * v          # the fan's normal
        a1 = np.cross(nrm, rng.normal(size=3))
        a1 /= np.linalg.norm(a1)
        a2 = np.cross(nrm, a1)
        R = np.stack([a1, a2, nrm], axis=1)            # columns: fan axes, normal (third scale 0)
        q = Rotation.from_matrix(R).as_quat()          # (x, y, z, w)
        quat[g] = [q[3], q[0], q[1], q[2]]
        cosv[g] = abs(nrm @ v)
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    rgb = rng.uniform(0, 1, size=(n, 3))
    f = faces_f32(oc.convert_fan(mean.T.copy(), scale.T.copy(), quat.T.copy(), opacity, rgb.T.copy(), K, 2.0))
    return f, cosv


def _face_cos(f64, cam):
    P, I = f64["pos"], f64["idx"]
    Wm = np.asarray(cam.world_to_cam, np.float64)
    centre = -np.linalg.solve(Wm[:, :3], Wm[:, 3])
    p0, p1, p2 = P[:, I[0]], P[:, I[1]], P[:, I[2]]
    nrm = np.cross(p1 - p0, p2 - p0, axis=0)
    view = (p0 + p1 + p2) / 3 - centre[:, None]
    return np.abs((nrm * view).sum(0)) / (np.linalg.norm(nrm, axis=0) * np.linalg.norm(view, axis=0))


@pytest.mark.parametrize("cos_lo,cos_hi,n,det", [(0.005, 0.05, 150, 0), (0.002, 0.01, 400, 0), (0.005, 0.05, 150, 1)])
def test_oblique_fans_strict_gradient_bar(gpu, cos_lo, cos_hi, n, det):
    """Fans whose planes are within a few degrees of containing the view ray:
    positions, opacities and colours at |d| <= 1e-3 |g| + 1e-6 max |g| with
    no exception list."""
    import torch
    W = H = 160
    cam = scenes.ring_cameras(1, W, H)[0]
    Wm = np.asarray(cam.world_to_cam, np.float64)
    cpos = -np.linalg.solve(Wm[:, :3], Wm[:, 3])
    f, cosv = _oblique_fans(n, 77, cpos, cos_lo, cos_hi)
    f64 = faces_f64(f)
    fc = _face_cos(f64, cam)
    fg = to_gpu(f)
    opts = gpu.RenderOptions(t_eps=0.0, deterministic=det)
    _say("oblique fans", cos_lo, cos_hi, "face |cos| range", fc.min(), fc.max())
    img, st, keep = _frozen_images_and_mask(gpu, fg, f, [cam], opts)
    nfr = st.nfrag()
    assert nfr.sum() > 3000, nfr.sum()
    dimg = _masked_upstream((1, H, W), keep, seed=21)
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg).cuda())
    ref = orr.render_backward_pixels(f64, cam, keep[0], [dimg[0, :, j, i] for i, j in keep[0]])
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("drgb", "drgb")):
        got = gr[k].cpu().numpy()
        ok, ex = grad_close(got, ref[rk])
        if not ok:
            g = np.asarray(got, np.float64).reshape(-1, f64["opacity"].shape[0])
            r = np.asarray(ref[rk]).reshape(-1, f64["opacity"].shape[0])
            tol = 1e-3 * np.abs(r) + 1e-6 * np.abs(r).max()
            badv = np.flatnonzero((np.abs(g - r) > tol).any(axis=0))
            _say(k, "vertices outside the bar", len(badv), [(int(v), g[:, v], r[:, v]) for v in badv[:5]])
        assert ok, (k, ex)
        assert np.count_nonzero(ref[rk]) > 500


# ---------------------------------------------------------------------------
# deterministic summation
# ---------------------------------------------------------------------------
def _rgb_scene(n, seed):
    g = scenes.gaussians(n, seed, 0.02, 0.15, flat=True)
    return faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0))


def _sh_scene(n, seed, K=8):
    g = scenes.gaussians(n, seed, 0.02, 0.15, flat=True, sh=True)
    return faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, sh=g.sh))


@pytest.mark.parametrize("sh,rows", [(False, 0), (False, 64), (True, 0), (True, 64)])
def test_deterministic_backward_repeats_bitwise(gpu, sh, rows):
    """Two backwards of one render give identical bits in deterministic mode,
    and stay within 1e-5 |g| + 1e-7 max |g| of the float-atomic sums."""
    import torch
    f = to_gpu(_sh_scene(2000, 50) if sh else _rgb_scene(2000, 50))
    cams = scenes.ring_cameras(3, 96, 80)
    dimg = torch.from_numpy(scenes.upstream_grad(3, 80, 96, seed=9)).cuda()
    cm = 1 if sh else 0
    i_f, s_f = gpu.render(f, cams, gpu.RenderOptions(color_mode=cm, list_rows=rows))
    g_f = gpu.render_backward(s_f, f, dimg)
    i_d, s_d = gpu.render(f, cams, gpu.RenderOptions(color_mode=cm, list_rows=rows, deterministic=1))
    g1 = gpu.render_backward(s_d, f, dimg)
    g1 = {k: v.clone() for k, v in g1.items()}
    g2 = gpu.render_backward(s_d, f, dimg)
    # a second state, rendered anew: the same bits again
    i_e, s_e = gpu.render(f, cams, gpu.RenderOptions(color_mode=cm, list_rows=rows, deterministic=1))
    g3 = gpu.render_backward(s_e, f, dimg)
    torch.cuda.synchronize()
    assert torch.equal(i_f, i_d) and torch.equal(i_d, i_e)
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k
        assert torch.equal(g1[k], g3[k]), k
        a = g_f[k].double()
        d = g1[k].double()
        tol = 1e-5 * a.abs() + 1e-7 * float(a.abs().max())
        assert bool(((a - d).abs() <= tol).all()), (k, float(((a - d).abs() - tol).max()))


def test_deterministic_backward_matches_oracle_sh(gpu):
    """Deterministic mode against the oracle, SH colour over two views (the
    colour's view-direction term has its own fixed-point class)."""
    import torch
    f = _sh_scene(150, 13, K=16)
    cams = scenes.ring_cameras(2, 40, 32)
    fg = to_gpu(f)
    f64 = faces_f64(f)
    cols = [osh.face_colours(f64["sh"], f64["pos"], f64["idx"], c)[0] for c in cams]
    opts = gpu.RenderOptions(t_eps=0.0, color_mode=1, deterministic=1)
    img, st, keep = _frozen_images_and_mask(gpu, fg, f, cams, opts, view_col=cols)
    dimg = _masked_upstream((2, 32, 40), keep, seed=5)
    ref = dict(dpos=np.zeros_like(f64["pos"]), dop=np.zeros_like(f64["opacity"]), dsh=np.zeros_like(f64["sh"]))
    for v, cam in enumerate(cams):
        r = orr.render_backward_pixels(f64, cam, keep[v], [dimg[v, :, j, i] for i, j in keep[v]], view_col=cols[v])
        dsh, dpos_dir = osh.face_colours_backward(f64["sh"], f64["pos"], f64["idx"], cam, r["dcol"])
        ref["dpos"] += r["dpos"] + dpos_dir
        ref["dop"] += r["dop"]
        ref["dsh"] += dsh
    gr = gpu.render_backward(st, fg, torch.from_numpy(dimg).cuda())
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("dsh", "dsh")):
        ok, ex = grad_close(gr[k].cpu().numpy(), ref[rk])
        assert ok, (k, ex)


def test_deterministic_graph_step_repeats_bitwise(gpu):
    """The captured step in deterministic mode: every replay gives the same bits
    as the uncaptured deterministic backward."""
    import torch
    f = to_gpu(_rgb_scene(3000, 51))
    cams = scenes.ring_cameras(2, 128, 96)
    dimg = torch.from_numpy(scenes.upstream_grad(2, 96, 128, seed=10)).cuda()
    opts = gpu.RenderOptions(list_rows=64, deterministic=1)
    i0, s0 = gpu.render(f, cams, opts)
    g0 = gpu.render_backward(s0, f, dimg)
    step = gpu.GraphStep(f, cams, opts)
    for _ in range(4):
        img, gr = step(dimg)
        torch.cuda.synchronize()
        assert torch.equal(img, i0)
        for k in g0:
            assert torch.equal(gr[k], g0[k]), k
    assert step.info()["replays"] >= 3


# ---------------------------------------------------------------------------
# captured graphs and uncaptured calls on one state
# ---------------------------------------------------------------------------
def test_eager_calls_discard_the_captured_graph(gpu):
    """graph step on views A, an uncaptured render of other views B of the same
    size on the same state, graph step on A again: the result equals the
    uncaptured step on A (the cameras the graph would read were replaced)."""
    import torch
    f = to_gpu(_rgb_scene(2000, 52))
    camsA = scenes.ring_cameras(2, 96, 72)
    camsB = scenes.ring_cameras(2, 96, 72, radius=2.2, elevation_deg=25.0)
    dimg = torch.from_numpy(scenes.upstream_grad(2, 72, 96, seed=11)).cuda()
    opts = gpu.RenderOptions(list_rows=64, deterministic=1)
    iA, sA = gpu.render(f, camsA, opts)
    gA = gpu.render_backward(sA, f, dimg)
    iB, sB = gpu.render(f, camsB, opts)
    assert not torch.equal(iA, iB)
    step = gpu.GraphStep(f, camsA, opts)
    for _ in range(2):
        step(dimg)
    assert step.info()["captures"] == 1
    gpu.render(f, camsB, opts, state=step.state)       # uncaptured render, other cameras
    img, gr = step(dimg)
    torch.cuda.synchronize()
    assert torch.equal(img, iA)
    for k in gA:
        assert torch.equal(gr[k], gA[k]), k
    assert step.info()["captures"] == 2
    # an uncaptured backward on the state discards the graph too
    gpu.render_backward(step.state, f, dimg)
    img, gr = step(dimg)
    torch.cuda.synchronize()
    assert torch.equal(img, iA) and step.info()["captures"] == 3


def test_state_status_reports_short_lists(gpu):
    import torch
    f = to_gpu(_rgb_scene(2000, 53))
    cams = scenes.ring_cameras(1, 64, 64)
    dimg = torch.from_numpy(scenes.upstream_grad(1, 64, 64, seed=12)).cuda()
    _, st = gpu.render(f, cams, gpu.RenderOptions(list_rows=256))
    gpu.render_backward(st, f, dimg)
    assert st.status() == 0
    _, st = gpu.render(f, cams, gpu.RenderOptions(list_rows=1))
    g1 = gpu.render_backward(st, f, dimg)
    assert st.status() == -4          # MSP_EOVERFLOW: lists recomputed, results complete
    _, s0 = gpu.render(f, cams, gpu.RenderOptions())
    g0 = gpu.render_backward(s0, f, dimg)
    for k in g0:
        assert torch.allclose(g0[k], g1[k], rtol=1e-4, atol=1e-6 * float(g0[k].abs().max()))
