"""Pins of the two oracle helpers that decide which GPU results are excused
from the parity bars: `render.ambiguous_pixels` (rendering section: a pixel
whose float32 fragment set or order may legitimately differ from the float64
one) and `rays.near_boundary` (a ray whose float32 hit test may include or drop
a face). Each case is built by hand so that the expected flag follows from
the geometry alone: a pixel centre placed exactly on a projected edge, 0.3 px
inside a face, on two coplanar faces at one depth; a ray through a vertex, a
centroid, an interval end."""
import numpy as np
import pytest

from oracle import rays as ory
from oracle import render as orr
from paper_2502_07754_amd import scenes

W = H = 16
FOC = 20.0


def cam():
    return scenes.Camera(world_to_cam=np.concatenate([np.eye(3), np.zeros((3, 1))], 1),
                         fx=FOC, fy=FOC, cx=W / 2, cy=H / 2, width=W, height=H, znear=0.01)


def soup(tris, ops, cols):
    tris = np.asarray(tris, np.float64)
    F = tris.shape[0]
    return dict(pos=tris.reshape(F * 3, 3).T.copy(), opacity=np.asarray(ops, np.float64).reshape(F * 3),
                rgb=np.asarray(cols, np.float64).reshape(F * 3, 3).T.copy(),
                idx=np.arange(3 * F, dtype=np.int32).reshape(F, 3).T.copy())


def xw(u, z):
    """Camera-space x at depth z of the pixel-space column u (identity camera)."""
    return (u - W / 2) / FOC * z


def left_right(u_edge, zl, zr, rot=0):
    """Two faces whose projections meet along the vertical line u = u_edge: the
    left one at depth zl, the right one at depth zr (each parallel to the image
    plane). `rot` cycles the corner order of the left face, which moves the
    shared edge to each of its three edge slots."""
    yl, yh = -3.0, 3.0
    L = [[xw(-40, zl), yl * zl, zl], [xw(u_edge, zl), yl * zl, zl], [xw(u_edge, zl), yh * zl, zl]]
    R = [[xw(u_edge, zr), yl * zr, zr], [xw(60, zr), yh * zr, zr], [xw(u_edge, zr), yh * zr, zr]]
    L = L[rot:] + L[:rot]
    return [L, R]


@pytest.mark.parametrize("rot", [0, 1, 2])
def test_pixel_centre_on_a_shared_edge_is_flagged(rot):
    # pixel (8, 8) has its centre at u = 8.5; the faces meet exactly there, at
    # different depths (so the depth-tie rule cannot be what flags it)
    f = soup(left_right(8.5, 2.0, 3.0, rot), [[0.6] * 3, [0.6] * 3],
             [[[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]
    # the same geometry with the pixel 0.3 px inside the left face: not flagged
    f = soup(left_right(8.8, 2.0, 3.0, rot), [[0.6] * 3, [0.6] * 3],
             [[[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]
    # 0.3 px inside the right face: not flagged either
    f = soup(left_right(8.2, 2.0, 3.0, rot), [[0.6] * 3, [0.6] * 3],
             [[[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]


def test_edge_pixel_with_a_face_just_outside_is_flagged():
    # the right face's edge passes a hair (well inside the float32 band) to the
    # right of the centre: the float64 test misses it, a float32 test may not
    eps = 1e-6
    f = soup(left_right(8.5 + eps, 2.0, 3.0)[1:], [[0.7] * 3], [[[0, 1, 0]] * 3])
    fr = orr.pixel_fragments(f, cam(), 8, 8)
    assert len(fr["fid"]) == 0
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]
    # the same face 0.3 px away: nothing to flag
    f = soup(left_right(8.8, 2.0, 3.0)[1:], [[0.7] * 3], [[[0, 1, 0]] * 3])
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]


def test_edge_whose_toggle_changes_nothing_is_not_flagged():
    # two opaque coplanar faces of one colour meeting at the pixel centre: the
    # pixel is that colour whichever of them is kept
    f = soup(left_right(8.5, 2.0, 2.0), [[1.0] * 3, [1.0] * 3], [[[0.3, 0.5, 0.7]] * 3] * 2)
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]
    # the same with different colours: flagged
    f = soup(left_right(8.5, 2.0, 2.0), [[1.0] * 3, [1.0] * 3], [[[0.3, 0.5, 0.7]] * 3, [[0.7, 0.5, 0.3]] * 3])
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]


def big(z, col, op):
    """A face parallel to the image plane at depth z covering the whole view."""
    return [[xw(-100, z), -5 * z, z], [xw(100, z), -5 * z, z], [0.0, 5 * z, z]], [op] * 3, [col] * 3


def test_coplanar_faces_at_one_depth_are_flagged_by_the_tie_rule():
    t0, o0, c0 = big(2.0, [1, 0, 0], 0.5)
    t1, o1, c1 = big(2.0, [0, 0, 1], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    px = [(3, 4), (8, 8), (12, 2)]
    fr = orr.pixel_fragments(f, cam(), 8, 8)
    assert len(fr["fid"]) == 2 and fr["z"][0] == fr["z"][1]
    assert np.all(orr.ambiguous_pixels(f, cam(), px))
    # equal attributes: the order does not matter, nothing to flag
    t1, o1, c1 = big(2.0, [1, 0, 0], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert not np.any(orr.ambiguous_pixels(f, cam(), px))
    # different colours well apart in depth: the order is not ambiguous
    t1, o1, c1 = big(2.5, [0, 0, 1], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert not np.any(orr.ambiguous_pixels(f, cam(), px))
    # depths within the 1e-6 relative band: flagged; just outside it: not
    t1, o1, c1 = big(2.0 * (1 + 5e-7), [0, 0, 1], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert np.all(orr.ambiguous_pixels(f, cam(), px))
    t1, o1, c1 = big(2.0 * (1 + 5e-6), [0, 0, 1], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert not np.any(orr.ambiguous_pixels(f, cam(), px))


def test_flag_threshold_follows_tol():
    # swapping two layers of alpha 0.5 changes the pixel by 0.25 |c0 - c1|
    t0, o0, c0 = big(2.0, [0.5, 0.5, 0.5], 0.5)
    t1, o1, c1 = big(2.0, [0.5 + 4e-4, 0.5, 0.5], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.9e-4)[0]
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=1.1e-4)[0]


# ---- rays.near_boundary -----------------------------------------------------

TRI = np.array([[0.0, 0.0, 5.0], [2.0, 0.0, 5.0], [0.0, 2.0, 5.0]])


def one_face():
    return dict(pos=TRI.T.copy(), opacity=np.full(3, 0.5), rgb=np.zeros((3, 3)),
                idx=np.arange(3, dtype=np.int32).reshape(3, 1))


def rays_to(points):
    P = np.asarray(points, np.float64)
    O = np.zeros((3, len(P)))
    return O, P.T.copy()


@pytest.mark.parametrize("corner", [0, 1, 2])
def test_ray_through_a_vertex_is_listed(corner):
    O, D = rays_to([TRI[corner]])
    fl = ory.near_boundary(one_face(), O, D, np.zeros(1), np.full(1, np.inf))
    assert list(fl[0]) == [0]


def test_ray_through_the_centroid_is_not_listed():
    O, D = rays_to([TRI.mean(0)])
    fl = ory.near_boundary(one_face(), O, D, np.zeros(1), np.full(1, np.inf))
    assert len(fl[0]) == 0


def test_edge_band_and_interval_ends():
    mid01 = 0.5 * (TRI[0] + TRI[1])           # on the edge v = 0
    out = mid01 + np.array([0.0, -1e-3, 0.0])  # v = -5e-4: outside the band
    near = mid01 + np.array([0.0, -1e-5, 0.0])  # v = -5e-6: inside the band, a miss in float64
    inner = mid01 + np.array([0.0, 1e-3, 0.0])  # v = +5e-4: a clean hit
    O, D = rays_to([mid01, out, near, inner])
    fl = ory.near_boundary(one_face(), O, D, np.zeros(4), np.full(4, np.inf))
    assert [len(x) for x in fl] == [1, 0, 1, 0]
    # a clean hit at t = 1 (d reaches the face): listed when an interval end sits at it
    O, D = rays_to([TRI.mean(0)] * 4)
    t0 = np.array([0.0, 1.0 - 1e-6, 0.0, 0.5])
    t1 = np.array([np.inf, np.inf, 1.0 + 1e-6, 0.9])
    fl = ory.near_boundary(one_face(), O, D, t0, t1)
    assert [len(x) for x in fl] == [0, 1, 1, 0]


def test_candidate_restriction_changes_nothing_when_it_covers_the_pixel():
    # a random soup in front of the camera plus the shared-edge pair: restricting
    # each pixel to the faces whose projected box comes near it leaves its flag as it was
    from oracle import convert as oc
    g = scenes.gaussians(200, 9, 0.05, 0.4, flat=True)
    mean = g.mean + np.array([[0.0], [0.0], [3.0]])
    r = oc.convert_fan(mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0)
    e = soup(left_right(8.5, 2.0, 3.0), [[0.6] * 3, [0.6] * 3], [[[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    nv = r["pos"].shape[1]
    f = dict(pos=np.concatenate([r["pos"], e["pos"]], 1), opacity=np.concatenate([r["opacity"], e["opacity"]]),
             rgb=np.concatenate([r["rgb"], e["rgb"]], 1), idx=np.concatenate([r["idx"], e["idx"] + nv], 1))
    c = cam()
    px = [(8, 8)] + [(i, j) for j in range(0, 16, 3) for i in range(0, 16, 3)]
    full = orr.ambiguous_pixels(f, c, px)
    uv, keep = orr.projected_corners(f, c)
    lo, hi = uv.min(axis=1), uv.max(axis=1)
    for n, (i, j) in enumerate(px):
        cand = np.flatnonzero(keep & (lo[:, 0] <= i + 1.5) & (hi[:, 0] >= i - 0.5) & (lo[:, 1] <= j + 1.5)
                              & (hi[:, 1] >= j - 0.5))
        assert orr.ambiguous_pixels(f, c, [(i, j)], candidates=cand)[0] == full[n]
    assert full[0] and not full.all()


def test_stop_ambiguity():
    # three layers of alpha 0.9: T = 1, 0.1, 0.01, 0.001 before/after them
    a = [0.9, 0.9, 0.9]
    assert orr.stop_ambiguous(a, 0.01)            # T before the third layer is exactly t_eps
    assert orr.stop_ambiguous(a, 0.01 * (1 + 5e-6))
    assert not orr.stop_ambiguous(a, 0.01 * (1 + 5e-5))
    assert not orr.stop_ambiguous(a, 0.003)
    assert orr.stop_ambiguous(a, 0.001)           # the transmittance after the last layer
    assert not orr.stop_ambiguous(a, 0.0)
    # the early stop it guards: at t_eps just above 0.01 the third layer is dropped, just below it is kept
    assert orr.early_stop(a, 0.01 * (1 + 1e-9)) == 2 and orr.early_stop(a, 0.01 * (1 - 1e-9)) == 3


def test_with_an_early_stop_only_what_comes_before_it_counts():
    # an opaque front face (alpha 1) ends every pixel at once; a face sharing an edge
    # with the pixel centre behind it changes nothing once the composite stops there,
    # in front of it everything
    front = big(2.0, [0.2, 0.4, 0.6], 1.0)
    pair = left_right(8.5, 3.0, 3.5)
    f = soup([front[0]] + pair, [front[1], [0.6] * 3, [0.6] * 3], [front[2], [[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.0, t_eps=1e-6)[0]
    # without the stop the faces behind still change the (untruncated) value by 0: T = 0 after alpha 1
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.0)[0]
    # a translucent front face: the edge behind it now shows
    front = big(2.0, [0.2, 0.4, 0.6], 0.5)
    f = soup([front[0]] + pair, [front[1], [0.6] * 3, [0.6] * 3], [front[2], [[1, 0, 0]] * 3, [[0, 0, 1]] * 3])
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.0, t_eps=1e-6)[0]
    # the stop reached before the edge (t_eps above the transmittance behind the front face)
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.0, t_eps=0.6)[0]
    # with tol = 0, any tie among composited fragments with different attributes counts
    t0, o0, c0 = big(2.0, [0.5, 0.5, 0.5], 0.5)
    t1, o1, c1 = big(2.0, [0.5 + 1e-7, 0.5, 0.5], 0.5)
    f = soup([t0, t1], [o0, o1], [c0, c1])
    assert orr.ambiguous_pixels(f, cam(), [(8, 8)], tol=0.0)[0]
    assert not orr.ambiguous_pixels(f, cam(), [(8, 8)])[0]
