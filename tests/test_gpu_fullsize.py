"""The batched-render workload at full size, in the launch configuration the
benchmark times (500k flat Gaussians, K = 16, SH degree 3, eight 1920x1080
views, faces in Morton order of the means, captured fwd+bwd step, tile 32x16,
ordering buffer 16, lists stored by the forward, t_eps = 1e-6), against the
oracle:

  * the tile lists of one whole view, bit for bit (offsets and sorted keys);
  * a contiguous 32x32 crop of every view: each pixel's RGBA at the image bar
    (a pixel that misses it must be one the oracle flags as ambiguous, at most
    2% of the covered ones), and the gradients of an upstream gradient that is
    non-zero only on the crops' unflagged pixels, so that the oracle computes
    them pixel by pixel.

Each crop pixel is brute-forced over the faces of its tile list, which the
float32 binning statement gives and which is pinned to hold every float64 hit
(tests/test_oracle_binning.py); faces outside it cannot cover the pixel.
The Morton order is computed on the host (the oracle takes no input from the
GPU)."""
import multiprocessing as mp

import numpy as np
import pytest

from oracle import binning as ob
from oracle import convert as oc
from oracle import render as orr
from oracle import sh as osh
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, grad_close, to_gpu

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4
T_EPS = 1e-6
TILE = (32, 16)
CROP = 32

_W = {}   # oracle inputs of the view being checked, inherited by forked workers


def _say(*a):
    print(*a, flush=True)


def _morton_order(mean):
    m = np.asarray(mean, np.float64)
    lo, hi = m.min(1, keepdims=True), m.max(1, keepdims=True)
    q = np.clip(np.floor((m - lo) / (hi - lo) * 1024), 0, 1023).astype(np.int64)
    code = np.zeros(m.shape[1], np.int64)
    for b in range(10):
        for a in range(3):
            code |= ((q[a] >> b) & 1) << (3 * b + 2 - a)
    return np.argsort(code, kind="stable").astype(np.int32)


@pytest.fixture(scope="module")
def c3(gpu):
    """The workload's Gaussians in Morton order, converted by the oracle (float32
    faces) and by the GPU; the step runs on the oracle's faces, so that both
    sides see the same input bits (the GPU conversion is held to its own bar:
    indices and Gaussian ids equal, positions within 4 ulp)."""
    import torch
    g, cams, p = scenes.config3()
    perm = _morton_order(g.mean)
    dev = torch.device("cuda:0")
    gg = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
          dict(mean=g.mean, scale=g.scale, quat=g.quat, opacity=g.opacity, rgb=g.rgb, sh=g.sh).items()}
    _say("full size: convert")
    gf = gpu.convert(gg, p["K"], p["sigma"], order=torch.from_numpy(perm).to(dev))
    perm64 = perm.astype(np.int64)
    f = faces_f32(oc.convert_fan(g.mean[:, perm64], g.scale[:, perm64], g.quat[:, perm64], g.opacity[perm64],
                                 g.rgb[:, perm64], p["K"], p["sigma"], sh=g.sh[:, perm64]))
    assert np.array_equal(gf["gid"].cpu().numpy(), np.repeat(perm, p["K"]))
    assert np.array_equal(gf["idx"].cpu().numpy(), f["idx"])
    # the conversion's own position bar is held by test_convert_parity; here it is only reported,
    # in ulp of the magnitude of the terms that make up each coordinate (mean + sigma * scale)
    mag = np.abs(g.mean[:, perm64].astype(np.float64)) + p["sigma"] * np.max(g.scale[:, perm64], axis=0)
    ulp = np.spacing(np.repeat(mag, p["K"] + 1, axis=1).astype(np.float32)).astype(np.float64)
    r = np.abs(gf["pos"].cpu().numpy().astype(np.float64) - f["pos"]) / ulp
    _say("full size: GPU conversion, position error in ulp: max", float(r.max()), "99.99th percentile",
         float(np.percentile(r, 99.99)), "beyond 4:", int((r > 4).sum()))
    del gf
    faces = to_gpu({k: v for k, v in f.items() if k in ("pos", "opacity", "rgb", "sh", "idx", "gid")})
    opts = gpu.RenderOptions(tile_w=TILE[0], tile_h=TILE[1], kbuf=16, t_eps=T_EPS, color_mode=1, list_rows=128)
    step = gpu.GraphStep(faces, cams, opts)
    V, H, W = len(cams), cams[0].height, cams[0].width
    # the first call runs the step uncaptured (sizing the buffers), then captures it; the
    # second replays it, so that the state's tile lists are those of a replay
    for _ in range(2):
        img, _ = step(torch.zeros((V, 4, H, W), dtype=torch.float32, device=dev))
    img = img.cpu().numpy()
    _say("full size: graph", step.info())
    return dict(step=step, img=img, cams=cams, f32=f, faces=faces, V=V, H=H, W=W)


def test_tile_lists_bit_exact_full_view(c3):
    """View 0's tile lists as the benchmark's step leaves them (32x16 tiles,
    Morton-ordered faces), against the float32 binning statement."""
    f, cam = c3["f32"], c3["cams"][0]
    off, keys = c3["step"].state.tiles(0)
    r_off, r_keys = ob.tile_lists_fast(f["pos"], f["idx"], cam, *TILE)
    _say("full size: tile entries", len(keys), "longest list", int(np.diff(r_off).max()))
    assert np.array_equal(off, r_off)
    assert np.array_equal(keys, r_keys)


def _tile_candidates(f32, cam, x0, y0):
    """Per tile meeting the crop: the faces of its list (the float32 statement)."""
    ok, (px0, px1, py0, py1), _ = ob.face_ranges(f32["pos"], f32["idx"], cam)
    ntx = -(-int(cam.width) // TILE[0])
    out = {}
    for ty in range(y0 // TILE[1], (y0 + CROP - 1) // TILE[1] + 1):
        for tx in range(x0 // TILE[0], (x0 + CROP - 1) // TILE[0] + 1):
            m = ok & (px0 // TILE[0] <= tx) & (px1 // TILE[0] >= tx) & (py0 // TILE[1] <= ty) & (py1 // TILE[1] >= ty)
            out[ty * ntx + tx] = np.flatnonzero(m)
    return out, ntx


def _pixel_frags(i, j):
    t = (j // TILE[1]) * _W["ntx"] + i // TILE[0]
    return orr.pixel_fragments(_W["f64"], _W["cam"], i, j, _W["geom"], candidates=_W["cand"][t])


def _forward_chunk(px):
    """RGBA per pixel, then two flags: the early stop may fall elsewhere in float32;
    the fragment set or order before the stop may differ in float32 (edge band or
    depth tie; what the frozen-fragment gradient depends on)."""
    out = np.zeros((len(px), 6))
    for n, (i, j) in enumerate(px):
        fr = _pixel_frags(i, j)
        a, _, c = orr.fragment_attributes(_W["f64"], fr, _W["col"])
        m = orr.early_stop(a, T_EPS)
        out[n, :4], _ = orr.composite(a[:m], c[:m], (0.0, 0.0, 0.0))
        out[n, 4] = orr.stop_ambiguous(a, T_EPS)
        t = (j // TILE[1]) * _W["ntx"] + i // TILE[0]
        out[n, 5] = orr.ambiguous_pixels(_W["f64"], _W["cam"], [(i, j)], tol=0.0, t_eps=T_EPS, view_col=_W["col"],
                                         candidates=_W["cand"][t], geom=_W["geom"], proj=_W["proj"])[0]
    return out


def _backward_chunk(args):
    px, gs = args
    vid, dpos, dop, fid, dcol = [], [], [], [], []
    for (i, j), g in zip(px, gs):
        fr = _pixel_frags(i, j)
        r = orr.pixel_backward(_W["f64"], _W["cam"], i, j, g, fr, view_col=_W["col"], geom=_W["geom"], t_eps=T_EPS)
        vid.append(r["vid"])
        dpos.append(r["dpos"])
        dop.append(r["dop"])
        fid.append(r["fid"])
        dcol.append(r["dcol"])
    cat = lambda x, s: np.concatenate(x) if x else np.zeros(s)
    return cat(vid, (0,)).astype(np.int64), cat(dpos, (0, 3)), cat(dop, (0,)), cat(fid, (0,)).astype(np.int64), \
        cat(dcol, (0, 3))


def _chunks(x, n):
    return [x[k:k + n] for k in range(0, len(x), n)]


def test_crops_of_every_view_and_their_gradients(c3):
    import torch
    f32, cams, V, H, W = c3["f32"], c3["cams"], c3["V"], c3["H"], c3["W"]
    f64 = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in f32.items()}
    F, Vn = f64["idx"].shape[1], f64["pos"].shape[1]
    rng = np.random.default_rng(11)
    full = scenes.upstream_grad(V, H, W, 3, 1e-3)
    dimg = np.zeros_like(full)
    ref = dict(dpos=np.zeros((3, Vn)), dop=np.zeros(Vn), dsh=np.zeros((48, F)))
    procs = max(1, min(16, len(__import__("os").sched_getaffinity(0))))
    covered = flagged = checked = stopped = 0
    worst = 0.0
    ctx = mp.get_context("fork")
    for v in range(V):
        cam = cams[v]
        x0 = int(rng.integers(W // 4, 3 * W // 4 - CROP))
        y0 = int(rng.integers(H // 4, 3 * H // 4 - CROP))
        cand, ntx = _tile_candidates(f32, cam, x0, y0)
        union = np.unique(np.concatenate(list(cand.values())))
        col = np.zeros((3, F))
        col[:, union], _ = osh.face_colours(f64["sh"][:, union], f64["pos"], f64["idx"][:, union], cam)
        _W.update(f64=f64, cam=cam, geom=orr.face_geometry(f64["pos"], f64["idx"], cam), cand=cand, ntx=ntx, col=col,
                  proj=orr.projected_corners(f64, cam))
        px = [(x0 + a, y0 + b) for b in range(CROP) for a in range(CROP)]
        with ctx.Pool(procs) as pool:
            want = np.concatenate(pool.map(_forward_chunk, _chunks(px, 32)))
        stop_amb = want[:, 4] > 0
        set_amb = want[:, 5] > 0
        want = want[:, :4]
        got = np.stack([c3["img"][v][:, j, i] for i, j in px]).astype(np.float64)
        err = np.max(np.abs(got - want), axis=1)
        cov = want[:, 3] > 0
        covered += int(cov.sum())
        bad = np.flatnonzero(err > IMG_TOL)
        keep = np.ones(len(px), dtype=bool)
        for b in bad:
            i, j = px[b]
            t = (j // TILE[1]) * ntx + i // TILE[0]
            assert orr.ambiguous_pixels(f64, cam, [(i, j)], view_col=col, candidates=cand[t], geom=_W["geom"],
                                        proj=_W["proj"])[0], (v, i, j, err[b])
            keep[b] = False
        flagged += len(bad)
        checked += int(keep.sum())
        worst = max(worst, float(err[keep].max()))
        # a pixel whose float32 early stop may fall on another fragment, or whose fragment
        # set or order before the stop may differ in float32, keeps its image check (it
        # met the bar) but stays out of the gradient check: its frozen-fragment gradient
        # is that of another, equally valid list
        n_stop = int((keep & (stop_amb | set_amb)).sum())
        stopped += n_stop
        keep &= ~(stop_amb | set_amb)
        kp = [p for p, k in zip(px, keep) if k]
        for i, j in kp:
            dimg[v, :, j, i] = full[v, :, j, i]
        with ctx.Pool(procs) as pool:
            parts = pool.map(_backward_chunk, [(c, [dimg[v, :, j, i] for i, j in c]) for c in _chunks(kp, 32)])
        dcol = np.zeros((F, 3))
        for vid, dp, do, fi, dc in parts:
            np.add.at(ref["dpos"].T, vid, dp)
            np.add.at(ref["dop"], vid, do)
            np.add.at(dcol, fi, dc)
        nz = np.flatnonzero(np.any(dcol != 0, axis=1))
        dsh, dpos_dir = osh.face_colours_backward(f64["sh"][:, nz], f64["pos"], f64["idx"][:, nz], cam, dcol[nz].T)
        ref["dpos"] += dpos_dir
        ref["dsh"][:, nz] += dsh
        _say(f"full size: view {v} crop ({x0}, {y0}) covered {int(cov.sum())} flagged {len(bad)} "
             f"left out of the gradient check {n_stop} worst {float(err[keep].max()):.2e} candidates {len(union)}")
    _say("full size: covered", covered, "flagged", flagged, "left out of the gradient check", stopped,
         "worst kept error", worst)
    assert covered > 2000 and checked > 0.9 * V * CROP * CROP
    assert flagged <= 0.02 * covered and stopped <= 0.15 * covered
    step = c3["step"]
    _, grads = step(torch.from_numpy(dimg).cuda())
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("dsh", "dsh")):
        got = grads[k].cpu().numpy().astype(np.float64)
        ok, ex = grad_close(got, ref[rk])
        if not ok:
            r = np.asarray(ref[rk], np.float64)
            exc = np.abs(got - r) - (1e-3 * np.abs(r) + 1e-6 * np.abs(r).max())
            for e in np.argsort(exc.ravel())[::-1][:6]:
                _say(k, "element", np.unravel_index(e, r.shape), "gpu", got.ravel()[e], "oracle", r.ravel()[e],
                     "excess", exc.ravel()[e], "max |g|", np.abs(r).max())
        assert ok, (k, ex)
        assert np.count_nonzero(ref[rk]) > 1000, k
    assert step.info()["overflows"] == 0


# ---------------------------------------------------------------------------
# The fine-tuning workload at full size: 3M flat Gaussians, K = 8 (24M faces),
# sixteen 1920x1080 views, RGB composite, with the render options of the
# time-to-MSE runs (tile 32x16, ordering buffer 16, fragment lists recomputed by
# the backward, deterministic gradient sums).
# ---------------------------------------------------------------------------

C5_VIEWS = (0, 9)   # the views whose crops the oracle checks (about 70 s of oracle time each)


@pytest.fixture(scope="module")
def c5(gpu):
    """Faces from the oracle's conversion (float32), in the Gaussians' own order
    as the fine-tuning runs convert them; one eager render of all sixteen views."""
    import torch
    g, cams, p = scenes.config5()
    _say("c5: convert (oracle)")
    f = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, p["K"], p["sigma"]))
    del g
    faces = to_gpu({k: v for k, v in f.items() if k in ("pos", "opacity", "rgb", "idx", "gid")})
    opts = gpu.RenderOptions(tile_w=TILE[0], tile_h=TILE[1], kbuf=16, t_eps=T_EPS, color_mode=gpu.MSP_COLOR_RGB,
                             list_rows=0, deterministic=1)
    img, st = gpu.render(faces, cams, opts)
    torch.cuda.synchronize()
    _say("c5: rendered", st.stats())
    return dict(state=st, img=img.cpu().numpy(), cams=cams, f32=f, faces=faces, V=len(cams), H=cams[0].height,
                W=cams[0].width)


def test_c5_tile_lists_bit_exact_full_view(c5):
    """View 0's tile lists of the 24M-face soup against the float32 binning statement."""
    f, cam = c5["f32"], c5["cams"][0]
    off, keys = c5["state"].tiles(0)
    r_off, r_keys = ob.tile_lists_fast(f["pos"], f["idx"], cam, *TILE)
    _say("c5: tile entries", len(keys), "longest list", int(np.diff(r_off).max()))
    assert np.array_equal(off, r_off)
    assert np.array_equal(keys, r_keys)


def _backward_chunk_rgb(args):
    px, gs = args
    vid, dpos, dop, drgb = [], [], [], []
    for (i, j), g in zip(px, gs):
        r = orr.pixel_backward(_W["f64"], _W["cam"], i, j, g, _pixel_frags(i, j), geom=_W["geom"], t_eps=T_EPS)
        vid.append(r["vid"])
        dpos.append(r["dpos"])
        dop.append(r["dop"])
        drgb.append(r["drgb"])
    cat = lambda x, s: np.concatenate(x) if x else np.zeros(s)
    return cat(vid, (0,)).astype(np.int64), cat(dpos, (0, 3)), cat(dop, (0,)), cat(drgb, (0, 3))


def test_c5_crops_and_their_gradients(gpu, c5):
    """A 32x32 crop of two of the sixteen views: RGBA at the image bar (misses
    only on pixels the oracle flags as ambiguous), then the deterministic
    backward of an upstream gradient non-zero on the crops' unflagged pixels
    against the oracle's per-pixel adjoint: positions, opacities and colours
    of every vertex, at the gradient bar."""
    import torch
    f32, cams, V, H, W = c5["f32"], c5["cams"], c5["V"], c5["H"], c5["W"]
    f64 = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in f32.items()}
    Vn = f64["pos"].shape[1]
    rng = np.random.default_rng(17)
    full = scenes.upstream_grad(V, H, W, 5, 1e-3)
    dimg = np.zeros_like(full)
    ref = dict(dpos=np.zeros((3, Vn)), dop=np.zeros(Vn), drgb=np.zeros((3, Vn)))
    procs = max(1, min(16, len(__import__("os").sched_getaffinity(0))))
    covered = flagged = checked = stopped = 0
    ctx = mp.get_context("fork")
    for v in C5_VIEWS:
        cam = cams[v]
        x0 = int(rng.integers(W // 4, 3 * W // 4 - CROP))
        y0 = int(rng.integers(H // 4, 3 * H // 4 - CROP))
        cand, ntx = _tile_candidates(f32, cam, x0, y0)
        _W.update(f64=f64, cam=cam, geom=orr.face_geometry(f64["pos"], f64["idx"], cam), cand=cand, ntx=ntx, col=None,
                  proj=orr.projected_corners(f64, cam))
        px = [(x0 + a, y0 + b) for b in range(CROP) for a in range(CROP)]
        with ctx.Pool(procs) as pool:
            want = np.concatenate(pool.map(_forward_chunk, _chunks(px, 32)))
        amb = (want[:, 4] > 0) | (want[:, 5] > 0)
        want = want[:, :4]
        got = np.stack([c5["img"][v][:, j, i] for i, j in px]).astype(np.float64)
        err = np.max(np.abs(got - want), axis=1)
        cov = want[:, 3] > 0
        covered += int(cov.sum())
        bad = np.flatnonzero(err > IMG_TOL)
        keep = np.ones(len(px), dtype=bool)
        for b in bad:
            i, j = px[b]
            t = (j // TILE[1]) * ntx + i // TILE[0]
            assert orr.ambiguous_pixels(f64, cam, [(i, j)], candidates=cand[t], geom=_W["geom"],
                                        proj=_W["proj"])[0], (v, i, j, err[b])
            keep[b] = False
        flagged += len(bad)
        checked += int(keep.sum())
        n_amb = int((keep & amb).sum())
        stopped += n_amb
        keep &= ~amb
        kp = [q for q, k in zip(px, keep) if k]
        for i, j in kp:
            dimg[v, :, j, i] = full[v, :, j, i]
        with ctx.Pool(procs) as pool:
            parts = pool.map(_backward_chunk_rgb, [(c, [dimg[v, :, j, i] for i, j in c]) for c in _chunks(kp, 32)])
        for vid, dp, do, dc in parts:
            np.add.at(ref["dpos"].T, vid, dp)
            np.add.at(ref["dop"], vid, do)
            np.add.at(ref["drgb"].T, vid, dc)
        _say(f"c5: view {v} crop ({x0}, {y0}) covered {int(cov.sum())} flagged {len(bad)} "
             f"left out of the gradient check {n_amb} worst {float(err[keep].max()) if keep.any() else 0.0:.2e}")
    n_px = len(C5_VIEWS) * CROP * CROP
    assert covered > 0.5 * n_px and checked > 0.9 * n_px
    assert flagged <= 0.02 * covered and stopped <= 0.15 * covered
    grads = gpu.render_backward(c5["state"], c5["faces"], torch.from_numpy(dimg).cuda(),
                                need=("dpos", "dopacity", "drgb"))
    for k, rk in (("dpos", "dpos"), ("dopacity", "dop"), ("drgb", "drgb")):
        got = grads[k].cpu().numpy().astype(np.float64)
        ok, ex = grad_close(got, ref[rk])
        assert ok, (k, ex)
        assert np.count_nonzero(ref[rk]) > 1000, k
    assert c5["state"].status() == 0
