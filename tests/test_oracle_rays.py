"""Pins of the ray oracle: a hand-computed hit (t, barycentrics, alpha),
stacked opaque-ish squares in closed form (products over intervals, nearest
hit, alpha threshold, ties to the smaller face id), agreement with the
rasteriser oracle (a primary ray's transmittance is 1 - A of its pixel), and
invariance under a rigid motion of faces and rays."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import convert as oc
from oracle import rays as ory
from oracle import render as orr
from paper_2502_07754_amd import scenes


def _tri():
    return dict(pos=np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0]]), idx=np.array([[0], [1], [2]]),
                opacity=np.array([0.1, 0.5, 0.9]))


def test_single_triangle_by_hand():
    f = _tri()
    t, u, v, hit = ory.intersect(f["pos"], f["idx"], [0.2, 0.3, 1.0], [0.0, 0.0, -1.0])
    assert hit[0] and np.isclose(t[0], 1.0) and np.isclose(u[0], 0.2) and np.isclose(v[0], 0.3)
    a = ory.hit_alpha(f["opacity"], f["idx"], u, v)
    assert np.isclose(a[0], 0.5 * 0.1 + 0.2 * 0.5 + 0.3 * 0.9)
    O = np.array([[0.2, 0.2, 0.8], [0.3, 0.3, 0.8], [1.0, 1.0, 1.0]])
    D = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [-1.0, -2.0, -1.0]])
    T = ory.transmittance(f, O, D, np.zeros(3), np.array([np.inf, 0.4, np.inf]))
    # first ray hits; second has t = 0.5 outside (0, 0.4); third passes outside the triangle (u + v = 1.6)
    assert np.allclose(T, [1 - 0.42, 1.0, 1.0])
    # the closed edge counts, a ray in the plane does not
    _, _, _, h = ory.intersect(f["pos"], f["idx"], [0.5, 0.5, 1.0], [0.0, 0.0, -1.0])
    assert h[0]
    _, _, _, h = ory.intersect(f["pos"], f["idx"], [-1.0, 0.2, 0.0], [1.0, 0.0, 0.0])
    assert not h[0]


def _squares(zs, ops):
    """Squares [-1, 1]^2 at heights zs, two triangles each, uniform opacity per square."""
    pos, idx, op = [], [], []
    for k, (z, o) in enumerate(zip(zs, ops)):
        pos += [[-1, -1, z], [1, -1, z], [1, 1, z], [-1, 1, z]]
        b = 4 * k
        idx += [[b, b + 1, b + 2], [b, b + 2, b + 3]]
        op += [o] * 4
    return dict(pos=np.array(pos, float).T, idx=np.array(idx).T, opacity=np.array(op, float))


def test_stacked_squares_closed_form():
    zs = [0.5, 1.0, 2.0, 3.5]
    ops = [0.3, 0.05, 0.6, 0.9]
    f = _squares(zs, ops)
    rng = np.random.default_rng(0)
    O = np.vstack([rng.uniform(-0.7, 0.7, (2, 50)), np.zeros((1, 50))])   # stays inside every square
    D = np.vstack([rng.uniform(-0.05, 0.05, (2, 50)), np.ones((1, 50))])
    T = ory.transmittance(f, O, D, np.zeros(50), np.full(50, np.inf))
    assert np.allclose(T, np.prod(1 - np.array(ops)))
    T = ory.transmittance(f, O, D, np.full(50, 0.75), np.full(50, 2.5))     # only z = 1 and z = 2
    assert np.allclose(T, (1 - 0.05) * (1 - 0.6))
    t, fid, u, v = ory.closest_hit(f, O, D, np.zeros(50), np.full(50, np.inf), 0.0)
    assert np.allclose(t, 0.5) and np.all(fid // 2 == 0)
    t, fid, u, v = ory.closest_hit(f, O, D, np.zeros(50), np.full(50, np.inf), 0.1)   # skips 0.05
    assert np.allclose(t, 0.5)
    t, fid, u, v = ory.closest_hit(f, O, D, np.full(50, 0.6), np.full(50, np.inf), 0.1)
    assert np.allclose(t, 2.0) and np.all(fid // 2 == 2)
    t, fid, u, v = ory.closest_hit(f, O, D, np.zeros(50), np.full(50, 0.4), 0.0)
    assert np.all(fid == -1) and np.all(np.isinf(t))
    # a duplicated square: equal t, the smaller face id wins
    g = _squares([1.0, 1.0], [0.5, 0.5])
    t, fid, _, _ = ory.closest_hit(g, O, D, np.zeros(50), np.full(50, np.inf), 0.0)
    assert np.all(fid < 2)


def test_primary_rays_match_the_rasteriser():
    g = scenes.gaussians(60, 11, 0.05, 0.3, flat=True)
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0)
    cam = scenes.ring_cameras(1, 24, 20)[0]
    W = np.asarray(cam.world_to_cam, np.float64)
    Rm, tt = W[:, :3], W[:, 3]
    centre = -Rm.T @ tt
    px = [(i, j) for j in range(20) for i in range(24)]
    dc = np.array([[(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, 1.0] for i, j in px]).T
    D = Rm.T @ dc
    O = np.repeat(centre[:, None], len(px), axis=1)
    T = ory.transmittance(f, O, D, np.zeros(len(px)), np.full(len(px), np.inf))
    A = orr.render_pixels(f, cam, px)[:, 3]
    flags = ory.near_boundary(f, O, D, np.zeros(len(px)), np.full(len(px), np.inf))
    clean = np.array([len(fl) == 0 for fl in flags])
    assert clean.sum() > 0.9 * len(px) and np.sum(A[clean] > 0) > 100
    assert np.allclose(T[clean], 1 - A[clean], atol=1e-12)


def test_rigid_motion_invariance():
    g = scenes.gaussians(80, 12, 0.05, 0.3, flat=True)
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 6, 2.0)
    rng = np.random.default_rng(3)
    O = rng.uniform(-1, 1, (3, 64))
    D = rng.normal(size=(3, 64))
    t0, t1 = np.full(64, 1e-3), np.full(64, np.inf)
    Rm = Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()
    sh = np.array([[0.4], [-2.0], [1.5]])
    f2 = dict(f, pos=Rm @ f["pos"] + sh)
    T1 = ory.transmittance(f, O, D, t0, t1)
    T2 = ory.transmittance(f2, Rm @ O + sh, Rm @ D, t0, t1)
    assert np.allclose(T1, T2, atol=1e-12) and np.any(T1 < 1)
    a = ory.closest_hit(f, O, D, t0, t1, 0.0)
    b = ory.closest_hit(f2, Rm @ O + sh, Rm @ D, t0, t1, 0.0)
    assert np.array_equal(a[1], b[1]) and np.allclose(a[0][a[1] >= 0], b[0][b[1] >= 0])
