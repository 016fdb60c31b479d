"""Pins of the oracle renderer and its adjoint (rendering section: transform,
depth-ordered layers, interpolated vertex attributes, front-to-back blending
through alpha) against closed forms, invariants, an independent loop-only
renderer and finite differences."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import render as orr
from paper_2502_07754_amd import scenes


def cam_identity(W=16, H=16, f=20.0, znear=0.01):
    return scenes.Camera(world_to_cam=np.concatenate([np.eye(3), np.zeros((3, 1))], 1),
                         fx=f, fy=f, cx=W / 2, cy=H / 2, width=W, height=H, znear=znear)


def soup(tris, ops, cols):
    """tris [F][3][3] corner positions, ops [F][3], cols [F][3][3] -> face dict (unshared vertices)."""
    tris = np.asarray(tris, np.float64)
    F = tris.shape[0]
    return dict(pos=tris.reshape(F * 3, 3).T.copy(), opacity=np.asarray(ops, np.float64).reshape(F * 3),
                rgb=np.asarray(cols, np.float64).reshape(F * 3, 3).T.copy(),
                idx=np.arange(3 * F, dtype=np.int32).reshape(F, 3).T.copy())


def all_pixels(cam):
    return [(i, j) for j in range(cam.height) for i in range(cam.width)]


def test_empty_and_behind_camera():
    cam = cam_identity()
    empty = soup(np.zeros((0, 3, 3)), np.zeros((0, 3)), np.zeros((0, 3, 3)))
    out = orr.render_pixels(empty, cam, all_pixels(cam), bg=(0.1, 0.2, 0.3))
    np.testing.assert_array_equal(out, np.tile([0.1, 0.2, 0.3, 0.0], (256, 1)))
    behind = soup([[[-50, -50, -2], [50, -50, -2], [0, 50, -2]]], [[1, 1, 1]], [[[1, 0, 0]] * 3])
    out = orr.render_pixels(behind, cam, all_pixels(cam))
    assert np.all(out == 0.0)
    # a face with one corner at the near plane is dropped as a whole
    near = soup([[[-50, -50, 2], [50, -50, 2], [0, 50, 0.01]]], [[1, 1, 1]], [[[1, 0, 0]] * 3])
    assert np.all(orr.render_pixels(near, cam, all_pixels(cam)) == 0.0)


def test_parallel_face_matches_planar_barycentrics():
    cam = cam_identity()
    tri = np.array([[-3.0, -2.5, 2.0], [3.5, -2.0, 2.0], [0.2, 3.0, 2.0]])
    ops = [0.2, 0.5, 0.8]
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    f = soup([tri], [ops], [cols])
    px = all_pixels(cam)
    out = orr.render_pixels(f, cam, px)
    A = np.stack([tri[:, 0], tri[:, 1], np.ones(3)])
    for n, (i, j) in enumerate(px):
        P = 2.0 * orr.pixel_dir(cam, i, j)
        b = np.linalg.solve(A, [P[0], P[1], 1.0])
        if np.all(b >= 0):
            alpha = b @ ops
            np.testing.assert_allclose(out[n, 3], alpha, atol=1e-13)
            np.testing.assert_allclose(out[n, :3], alpha * (b @ np.asarray(cols, float)), atol=1e-13)
        else:
            assert np.all(out[n] == 0.0)


def test_tilted_face_is_perspective_correct():
    cam = cam_identity(W=24, H=24)
    tri = np.array([[-4.0, -4.0, 1.5], [4.0, -3.0, 3.5], [0.0, 4.0, 6.0]])
    ops = [0.1, 0.9, 0.4]
    f = soup([tri], [ops], [[[1, 1, 1]] * 3])
    px = all_pixels(cam)
    out = orr.render_pixels(f, cam, px)
    nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    M = np.vstack([tri.T, np.ones(3)])
    uv = np.stack([20 * tri[:, 0] / tri[:, 2] + 12, 20 * tri[:, 1] / tri[:, 2] + 12])
    max_affine_gap = 0.0
    for n, (i, j) in enumerate(px):
        d = orr.pixel_dir(cam, i, j)
        t = (nrm @ tri[0]) / (nrm @ d)
        b = np.linalg.lstsq(M, np.concatenate([t * d, [1.0]]), rcond=None)[0]
        if np.all(b >= 0):
            np.testing.assert_allclose(out[n, 3], b @ ops, atol=1e-12)
            # screen-space (affine) barycentrics differ for a tilted face
            lam = np.linalg.solve(np.vstack([uv, np.ones(3)]), [i + 0.5, j + 0.5, 1.0])
            max_affine_gap = max(max_affine_gap, abs(lam @ ops - b @ ops))
    assert max_affine_gap > 1e-2


def test_two_parallel_faces_closed_form():
    cam = cam_identity()
    big = np.array([[-50, -50, 0.0], [50, -50, 0.0], [0, 50, 0.0]])
    f = soup([big + [0, 0, 3.0], big + [0, 0, 2.0]], [[0.3] * 3, [0.6] * 3],
             [[[0.2, 0.4, 0.6]] * 3, [[0.9, 0.1, 0.5]] * 3])
    out = orr.render_pixels(f, cam, all_pixels(cam))
    a1, c1 = 0.6, np.array([0.9, 0.1, 0.5])     # nearer (z = 2) is face 1
    a2, c2 = 0.3, np.array([0.2, 0.4, 0.6])
    np.testing.assert_allclose(out[:, :3], np.tile(a1 * c1 + (1 - a1) * a2 * c2, (256, 1)), atol=1e-14)
    np.testing.assert_allclose(out[:, 3], 1 - (1 - a1) * (1 - a2), atol=1e-14)


def test_opaque_face_occludes():
    cam = cam_identity()
    rng = np.random.default_rng(5)
    big = np.array([[-50, -50, 0.0], [50, -50, 0.0], [0, 50, 0.0]])
    behind = [big + [rng.normal(), rng.normal(), 3.0 + k] for k in range(4)]
    front = big + [0, 0, 2.0]
    tris = behind + [front]
    ops = rng.uniform(0, 1, (5, 3))
    ops[4] = 1.0
    cols = rng.uniform(0, 1, (5, 3, 3))
    out = orr.render_pixels(soup(tris, ops, cols), cam, all_pixels(cam))
    alone = orr.render_pixels(soup([front], ops[4:], cols[4:]), cam, all_pixels(cam))
    np.testing.assert_array_equal(out[:, 3], 1.0)
    np.testing.assert_allclose(out, alone, atol=1e-15)


def _random_scene(rng, F, spread=1.0, z0=3.0):
    c = rng.uniform(-spread, spread, (F, 1, 3)) + [0, 0, z0]
    tris = c + rng.normal(0, 0.6, (F, 3, 3))
    return soup(tris, rng.uniform(0, 1, (F, 3)), rng.uniform(0, 1, (F, 3, 3)))


def test_transmittance_monotone_and_alpha_order_free():
    rng = np.random.default_rng(11)
    cam = cam_identity()
    f = _random_scene(rng, 30)
    px = all_pixels(cam)
    out, frs = orr.render_pixels(f, cam, px, return_frags=True)
    for fr in frs:
        a, _, c = orr.fragment_attributes(f, fr)
        _, T = orr.composite(a, c, (0, 0, 0))
        assert np.all(np.diff(T) <= 0.0)
    perm = rng.permutation(30)
    tris = f["pos"].T.reshape(30, 3, 3)[perm]
    g = soup(tris, f["opacity"].reshape(30, 3)[perm], f["rgb"].T.reshape(30, 3, 3)[perm])
    out2 = orr.render_pixels(g, cam, px)
    np.testing.assert_allclose(out2[:, 3], out[:, 3], atol=1e-14)
    np.testing.assert_allclose(out2, out, atol=1e-14)      # no exact depth ties in a random scene


def test_uniform_colour_scales_with_alpha():
    rng = np.random.default_rng(12)
    cam = cam_identity()
    f = _random_scene(rng, 25)
    f["rgb"][:] = np.array([[0.3], [0.7], [0.45]])
    out = orr.render_pixels(f, cam, all_pixels(cam))
    np.testing.assert_allclose(out[:, :3], out[:, 3:4] * [0.3, 0.7, 0.45], atol=1e-14)


def test_rigid_motion_invariance():
    rng = np.random.default_rng(13)
    cam = cam_identity()
    f = _random_scene(rng, 20)
    Q = Rotation.random(random_state=3).as_matrix()
    s = np.array([0.3, -1.2, 2.0])
    g = dict(f)
    g["pos"] = (Q @ f["pos"]) + s[:, None]
    W = np.asarray(cam.world_to_cam, np.float64)
    R2 = W[:, :3] @ Q.T
    cam2 = scenes.Camera(world_to_cam=np.concatenate([R2, (W[:, 3] - R2 @ s)[:, None]], 1),
                         fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy, width=cam.width, height=cam.height)
    np.testing.assert_allclose(orr.render_pixels(g, cam2, all_pixels(cam)),
                               orr.render_pixels(f, cam, all_pixels(cam)), atol=1e-12)


def _loop_renderer(faces, cam, i, j, bg=(0.0, 0.0, 0.0)):
    """Second, loop-only statement: ray/plane intersection and signed sub-area inside test."""
    d = orr.pixel_dir(cam, i, j)
    W = np.asarray(cam.world_to_cam, np.float64)
    P = faces["pos"].T @ W[:, :3].T + W[:, 3]
    hits = []
    for f in range(faces["idx"].shape[1]):
        ids = faces["idx"][:, f]
        v = [P[k] for k in ids]
        if min(x[2] for x in v) <= cam.znear:
            continue
        n = np.cross(v[1] - v[0], v[2] - v[0])
        den = n @ d
        if den == 0.0:
            continue
        t = (n @ v[0]) / den
        if t <= cam.znear:
            continue
        X = t * d
        nn = n @ n
        b = [np.cross(v[(k + 1) % 3] - X, v[(k + 2) % 3] - X) @ n / nn for k in range(3)]
        if min(b) < 0:
            continue
        a = min(1.0, max(0.0, sum(b[k] * faces["opacity"][ids[k]] for k in range(3))))
        c = sum(b[k] * faces["rgb"][:, ids[k]] for k in range(3))
        hits.append((t, f, a, c))
    hits.sort(key=lambda h: (h[0], h[1]))
    T, C = 1.0, np.zeros(3)
    for _, _, a, c in hits:
        C = C + T * a * c
        T *= 1 - a
    return np.concatenate([C + T * np.asarray(bg), [1 - T]])


@pytest.mark.parametrize("seed", range(5))
def test_tiny_scenes_against_loop_renderer(seed):
    rng = np.random.default_rng(100 + seed)
    cam = cam_identity(W=12, H=10)
    f = _random_scene(rng, int(rng.integers(1, 9)))
    px = all_pixels(cam)
    out = orr.render_pixels(f, cam, px, bg=(0.05, 0.1, 0.2))
    ref = np.array([_loop_renderer(f, cam, i, j, (0.05, 0.1, 0.2)) for i, j in px])
    np.testing.assert_allclose(out, ref, atol=1e-12)


def _fd_setup(seed=21, F=12):
    rng = np.random.default_rng(seed)
    cam = cam_identity(W=10, H=10)
    f = _random_scene(rng, F, spread=0.5)
    f["opacity"] = rng.uniform(0.05, 0.6, f["opacity"].shape)   # keep the clamp inactive
    px = all_pixels(cam)
    geom = orr.face_geometry(f["pos"], f["idx"], cam)
    frs = [orr.pixel_fragments(f, cam, i, j, geom) for i, j in px]
    g = rng.standard_normal((len(px), 4))
    return rng, cam, f, px, frs, g


def _frozen_loss(f, cam, px, frs, g, bg=(0.0, 0.0, 0.0)):
    return sum(g[n] @ orr.frozen_pixel_value(f, cam, i, j, frs[n]["fid"], bg) for n, (i, j) in enumerate(px)
               if len(frs[n]["fid"]) > 0)


def test_adjoint_against_finite_differences():
    rng, cam, f, px, frs, g = _fd_setup()
    bg = (0.2, 0.1, 0.05)
    gr = orr.render_backward_pixels(f, cam, px, g, bg=bg)
    h = 1e-6
    V = f["opacity"].shape[0]
    for v in rng.choice(V, 8, replace=False):
        for ax in range(3):
            fp = {k: np.array(x, copy=True) for k, x in f.items()}
            fm = {k: np.array(x, copy=True) for k, x in f.items()}
            fp["pos"][ax, v] += h
            fm["pos"][ax, v] -= h
            fd = (_frozen_loss(fp, cam, px, frs, g, bg) - _frozen_loss(fm, cam, px, frs, g, bg)) / (2 * h)
            np.testing.assert_allclose(gr["dpos"][ax, v], fd, rtol=1e-6, atol=1e-8)
            fp = {k: np.array(x, copy=True) for k, x in f.items()}
            fm = {k: np.array(x, copy=True) for k, x in f.items()}
            fp["rgb"][ax, v] += h
            fm["rgb"][ax, v] -= h
            fd = (_frozen_loss(fp, cam, px, frs, g, bg) - _frozen_loss(fm, cam, px, frs, g, bg)) / (2 * h)
            np.testing.assert_allclose(gr["drgb"][ax, v], fd, rtol=1e-6, atol=1e-8)
        fp = {k: np.array(x, copy=True) for k, x in f.items()}
        fm = {k: np.array(x, copy=True) for k, x in f.items()}
        fp["opacity"][v] += h
        fm["opacity"][v] -= h
        fd = (_frozen_loss(fp, cam, px, frs, g, bg) - _frozen_loss(fm, cam, px, frs, g, bg)) / (2 * h)
        np.testing.assert_allclose(gr["dop"][v], fd, rtol=1e-6, atol=1e-8)


def test_adjoint_against_torch_autograd():
    torch = pytest.importorskip("torch")
    rng, cam, f, px, frs, g = _fd_setup(seed=22)
    gr = orr.render_backward_pixels(f, cam, px, g)
    pos = torch.tensor(f["pos"], dtype=torch.float64, requires_grad=True)
    op = torch.tensor(f["opacity"], dtype=torch.float64, requires_grad=True)
    rgb = torch.tensor(f["rgb"], dtype=torch.float64, requires_grad=True)
    W = torch.tensor(np.asarray(cam.world_to_cam, np.float64))
    P = pos.T @ W[:, :3].T + W[:, 3]
    idx = torch.tensor(f["idx"].astype(np.int64))
    loss = torch.zeros((), dtype=torch.float64)
    for n, (i, j) in enumerate(px):
        d = torch.tensor(orr.pixel_dir(cam, i, j))
        T = torch.ones((), dtype=torch.float64)
        C = torch.zeros(3, dtype=torch.float64)
        for fid in frs[n]["fid"]:
            ids = idx[:, fid]
            v0, v1, v2 = P[ids[0]], P[ids[1]], P[ids[2]]
            M = torch.stack([-d, v1 - v0, v2 - v0], 1)
            x = torch.linalg.solve(M, -v0)
            b = torch.stack([1 - x[1] - x[2], x[1], x[2]])
            a = torch.clamp(b @ op[ids], 0, 1)
            c = rgb[:, ids] @ b
            C = C + T * a * c
            T = T * (1 - a)
        loss = loss + torch.tensor(g[n, :3]) @ C + g[n, 3] * (1 - T)
    loss.backward()
    np.testing.assert_allclose(gr["dpos"], pos.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gr["dop"], op.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gr["drgb"], rgb.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_adjoint_dot_product():
    """<w, J d> = <J^T w, d> for a random direction d in (pos, opacity, rgb)."""
    rng, cam, f, px, frs, g = _fd_setup(seed=23)
    gr = orr.render_backward_pixels(f, cam, px, g)
    dpos = rng.standard_normal(f["pos"].shape)
    dop = rng.standard_normal(f["opacity"].shape)
    drgb = rng.standard_normal(f["rgb"].shape)
    h = 1e-6
    fp = dict(f, pos=f["pos"] + h * dpos, opacity=f["opacity"] + h * dop, rgb=f["rgb"] + h * drgb)
    fm = dict(f, pos=f["pos"] - h * dpos, opacity=f["opacity"] - h * dop, rgb=f["rgb"] - h * drgb)
    lhs = (_frozen_loss(fp, cam, px, frs, g) - _frozen_loss(fm, cam, px, frs, g)) / (2 * h)
    rhs = np.sum(gr["dpos"] * dpos) + np.sum(gr["dop"] * dop) + np.sum(gr["drgb"] * drgb)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-6)


def test_early_stop_three_layers_closed_form():
    """A pixel stops once its transmittance falls below t_eps: with three layers of
    alpha 0.9 the transmittance before them is 1, 0.1, 0.01."""
    cam = cam_identity()
    big = np.array([[-50, -50, 0.0], [50, -50, 0.0], [0, 50, 0.0]])
    cols = [[[0.9, 0.1, 0.5]] * 3, [[0.2, 0.4, 0.6]] * 3, [[0.7, 0.7, 0.1]] * 3]
    f = soup([big + [0, 0, 2.0], big + [0, 0, 3.0], big + [0, 0, 4.0]], [[0.9] * 3] * 3, cols)
    c = [np.array(x[0]) for x in cols]
    px = [(8, 8)]
    for t_eps, layers in ((0.0, 3), (0.005, 3), (0.05, 2), (0.5, 1), (1.0, 1)):
        out = orr.render_pixels(f, cam, px, t_eps=t_eps)[0]
        T, C = 1.0, np.zeros(3)
        for k in range(layers):
            C += T * 0.9 * c[k]
            T *= 0.1
        np.testing.assert_allclose(out, np.concatenate([C, [1 - T]]), atol=1e-14)
    # just above the transmittance before the third layer: it is dropped; at it: kept
    assert orr.early_stop(np.array([0.9, 0.9, 0.9]), 0.01 + 1e-12) == 2
    assert orr.early_stop(np.array([0.9, 0.9, 0.9]), 0.01 - 1e-12) == 3


def test_early_stop_adjoint_against_finite_differences():
    """The adjoint with an early stop differentiates the truncated lists: finite
    differences of the frozen truncated fragments, and zero gradients for faces
    that only appear behind the stop."""
    rng, cam, f, px, frs, g = _fd_setup(seed=23, F=30)
    t_eps = 0.5
    _, cut = orr.render_pixels(f, cam, px, return_frags=True, t_eps=t_eps)
    assert sum(len(c["fid"]) < len(fr["fid"]) for c, fr in zip(cut, frs)) >= 5
    gr = orr.render_backward_pixels(f, cam, px, g, t_eps=t_eps)
    h = 1e-6
    seen = np.unique(np.concatenate([c["fid"] for c in cut]))
    used_v = np.unique(np.asarray(f["idx"])[:, seen])
    for v in rng.choice(used_v, 6, replace=False):
        for key, shape in (("pos", 3), ("rgb", 3), ("opacity", 1)):
            for ax in range(shape):
                fp = {k: np.array(x, copy=True) for k, x in f.items()}
                fm = {k: np.array(x, copy=True) for k, x in f.items()}
                if shape == 1:
                    fp[key][v] += h
                    fm[key][v] -= h
                    want = gr["dop"][v]
                else:
                    fp[key][ax, v] += h
                    fm[key][ax, v] -= h
                    want = gr["dpos" if key == "pos" else "drgb"][ax, v]
                fd = (_frozen_loss(fp, cam, px, cut, g) - _frozen_loss(fm, cam, px, cut, g)) / (2 * h)
                np.testing.assert_allclose(want, fd, rtol=1e-6, atol=1e-8)
    behind = np.setdiff1d(np.arange(f["opacity"].shape[0]), used_v)
    assert len(behind) > 0 and np.all(gr["dop"][behind] == 0) and np.all(gr["dpos"][:, behind] == 0)
