"""Pins of the mesh-prior oracle: the subdivision tiles the face (brute force
over random points, equal areas), the n = 2 case equals the midpoint split
written out by hand, secondary vertices lie inside their mesh face with
barycentric coordinates equal to scipy's softmax of the logits, closed-form
limits (equal logits -> centroid, one dominant logit -> that corner), and the
adjoint against central finite differences and the softmax shift invariance."""
import numpy as np
import pytest
from scipy.special import softmax as sp_softmax

from oracle import prior as op
from paper_2502_07754_amd import scenes


@pytest.fixture(scope="module")
def mesh():
    return scenes.icosphere(1, seed=3)


def _bary2(p, tri):
    """2D barycentric coordinates of points p [N][2] in triangle tri [3][2]."""
    a, b, c = tri
    M = np.array([b - a, c - a]).T
    uv = np.linalg.solve(M, (p - a).T).T
    return np.column_stack([1 - uv.sum(1), uv])


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_subdivision_tiles_the_face(n):
    sub = op.subdivision(n)
    assert sub.shape == (n * n, 3, 3)
    assert np.allclose(sub.sum(axis=2), 1.0)
    assert np.allclose(sub * n, np.round(sub * n))          # corners on the grid k / n
    tri2 = sub[:, :, 1:]                                     # (w2, w3) plane; the face is (0,0), (1,0), (0,1)
    e1, e2 = tri2[:, 1] - tri2[:, 0], tri2[:, 2] - tri2[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    assert np.allclose(area, 0.5 / (n * n))
    pts = np.random.default_rng(0).dirichlet([1, 1, 1], size=4000)[:, 1:]
    hits = np.zeros(len(pts), dtype=int)
    for t in tri2:
        hits += (_bary2(pts, t) > 1e-12).all(axis=1)
    assert np.all(hits == 1)


def test_n2_is_the_midpoint_split():
    m = np.array([[0.3, -0.2, 1.1], [1.4, 0.1, 0.9], [0.2, 1.3, 1.2]]).T   # [3][3], columns m1..m3
    idx = np.array([[0], [1], [2]])
    logits, fidx = op.prior_init(1, 2, 1e-12)
    pos = op.prior_vertices(m, idx, 2, logits)
    tris = [pos[:, fidx[:, f]].T for f in range(4)]
    m1, m2, m3 = m.T
    want = [[m1, (m1 + m2) / 2, (m1 + m3) / 2], [m2, (m2 + m1) / 2, (m2 + m3) / 2],
            [m3, (m3 + m1) / 2, (m3 + m2) / 2], [(m1 + m2) / 2, (m2 + m3) / 2, (m1 + m3) / 2]]

    def key(tri):
        return sorted(tuple(np.round(p, 9)) for p in tri)
    assert sorted(key(t) for t in tris) == sorted(key(w) for w in want)


def test_vertices_inside_their_face(mesh):
    n = 3
    Fm = mesh.n_faces
    rng = np.random.default_rng(1)
    logits = rng.normal(0, 2, size=(3, 3 * n * n * Fm))
    pos = op.prior_vertices(mesh.pos, mesh.idx, n, logits)
    want = sp_softmax(logits, axis=0)
    p = mesh.pos.astype(np.float64)
    for v in range(0, logits.shape[1], 7):
        f = v // (3 * n * n)
        M = p[:, mesh.idx[:, f]]                              # columns m1..m3; the face misses the origin
        w = np.linalg.solve(M, pos[:, v])
        assert np.all(w > 0) and abs(w.sum() - 1) < 1e-9
        assert np.allclose(w, want[:, v], atol=1e-9)


def test_closed_form_limits(mesh):
    n = 2
    V = 3 * n * n * mesh.n_faces
    p = mesh.pos.astype(np.float64)
    f = np.arange(V) // (3 * n * n)
    cen = op.prior_vertices(mesh.pos, mesh.idx, n, np.full((3, V), 0.7))
    assert np.allclose(cen, (p[:, mesh.idx[0, f]] + p[:, mesh.idx[1, f]] + p[:, mesh.idx[2, f]]) / 3, atol=1e-12)
    for j in range(3):
        th = np.zeros((3, V))
        th[j] = 60.0
        assert np.allclose(op.prior_vertices(mesh.pos, mesh.idx, n, th), p[:, mesh.idx[j, f]], atol=1e-12)


def test_initial_layout(mesh):
    n, shrink = 3, 0.05
    T, Fm = n * n, mesh.n_faces
    logits, idx = op.prior_init(Fm, n, shrink)
    assert logits.shape == (3, 3 * T * Fm) and idx.shape == (3, T * Fm)
    assert np.array_equal(idx, np.arange(3 * T * Fm).reshape(-1, 3).T)
    a = sp_softmax(logits, axis=0)
    assert np.allclose(a.T.reshape(Fm, T, 3, 3), op.initial_weights(n, shrink)[None], atol=1e-12)
    sub = op.subdivision(n)
    # each corner moved exactly `shrink` of the way to its sub-triangle's centroid
    d0 = np.linalg.norm(sub - sub.mean(1, keepdims=True), axis=2)
    d1 = np.linalg.norm(op.initial_weights(n, shrink) - sub.mean(1, keepdims=True), axis=2)
    assert np.allclose(d1, (1 - shrink) * d0)
    # shrunk sub-triangles are disjoint: no corner of one lies inside another
    w = op.initial_weights(n, shrink)[:, :, 1:]
    for s in range(T):
        for t in range(T):
            if s != t:
                assert not (_bary2(w[s], w[t]) > 0).all(axis=1).any()


def test_backward_finite_differences(mesh):
    n = 2
    rng = np.random.default_rng(2)
    V = 3 * n * n * mesh.n_faces
    logits = rng.normal(0, 1, size=(3, V))
    dpos = rng.normal(0, 1, size=(3, V))
    g = op.prior_backward(mesh.pos, mesh.idx, n, logits, dpos)
    h = 1e-6
    for j in range(3):
        e = np.zeros_like(logits)
        e[j] = h
        fd = ((op.prior_vertices(mesh.pos, mesh.idx, n, logits + e) -
               op.prior_vertices(mesh.pos, mesh.idx, n, logits - e)) * dpos).sum(axis=0) / (2 * h)
        assert np.allclose(g[j], fd, rtol=1e-6, atol=1e-8)


def test_shift_invariance(mesh):
    n = 1
    rng = np.random.default_rng(4)
    V = 3 * mesh.n_faces
    logits = rng.normal(0, 1, size=(3, V))
    c = rng.normal(0, 5, size=V)
    assert np.allclose(op.prior_vertices(mesh.pos, mesh.idx, n, logits),
                       op.prior_vertices(mesh.pos, mesh.idx, n, logits + c), atol=1e-12)
    g = op.prior_backward(mesh.pos, mesh.idx, n, logits, rng.normal(size=(3, V)))
    assert np.allclose(g.sum(axis=0), 0.0, atol=1e-12)
