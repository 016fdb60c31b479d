"""Mesh-prior mode, float64 (oracle; test infrastructure only).

Follows the paper's section "MeshSplats with Mesh Prior": on top of a
geometry mesh, every mesh face M = {m_1, m_2, m_3} carries a fixed number of
secondary, disjoint triangles; each secondary vertex is a convex combination
v = a_1 m_1 + a_2 m_2 + a_3 m_3 with a on the probability simplex, and the
weights a are what training moves (with the vertices' colours and opacities),
so the secondary triangles stay on the mesh face.

Readings where the paper is silent:
  * the simplex constraint is kept by a softmax over three free logits per
    secondary vertex (a = softmax(theta));
  * the fixed number of secondary triangles per mesh face is T = n^2, the
    regular subdivision with n segments per edge; the grid point (a, b)
    (0 <= a, b, a + b <= n) has weights ((n - a - b)/n, a/n, b/n) on
    (m_1, m_2, m_3); sub-triangle order: for a = 0..n-1, b = 0..n-1-a, the
    upward triangle ((a,b), (a+1,b), (a,b+1)) and then, when a + b <= n - 2,
    the downward one ((a+1,b), (a+1,b+1), (a,b+1));
  * initial weights: each corner's grid weights moved a fraction `shrink`
    (0 < shrink < 1) towards its sub-triangle's centroid, so every weight is
    positive and theta = log(weight) is finite; secondary triangles start as
    slightly shrunk copies of the subdivision, disjoint as the paper asks;
  * layout: secondary face f = mesh_face * T + t owns vertices 3f, 3f+1, 3f+2
    in corner order; logits are [3][V] with row j the logit of mesh corner j;
  * the geometry mesh is fixed (it comes from an external tool); gradients
    stop at the logits;
  * initial colours are the mesh's vertex colours interpolated with the
    initial weights when the mesh has colours, else a constant.
"""
from __future__ import annotations

import numpy as np


def subdivision(n: int) -> np.ndarray:
    """Barycentric corners of the n^2 sub-triangles: [T][3 corners][3 weights on m_1..m_3]."""
    def w(a, b):
        return [(n - a - b) / n, a / n, b / n]

    tris = []
    for a in range(n):
        for b in range(n - a):
            tris.append([w(a, b), w(a + 1, b), w(a, b + 1)])
            if a + b <= n - 2:
                tris.append([w(a + 1, b), w(a + 1, b + 1), w(a, b + 1)])
    return np.asarray(tris, dtype=np.float64)


def initial_weights(n: int, shrink: float) -> np.ndarray:
    """[T][3][3]: subdivision corners moved `shrink` of the way to their sub-triangle's centroid."""
    sub = subdivision(n)
    cen = sub.mean(axis=1, keepdims=True)
    return (1.0 - shrink) * sub + shrink * cen


def prior_init(n_mesh_faces: int, n: int, shrink: float):
    """Initial logits [3][V] and face indices [3][F] for V = 3 T Fm, F = T Fm."""
    T = n * n
    a0 = initial_weights(n, shrink)                               # [T][corner][j]
    F = n_mesh_faces * T
    alpha = np.tile(a0.reshape(T * 3, 3), (n_mesh_faces, 1))      # [V][j]
    logits = np.log(alpha).T.copy()
    idx = np.arange(3 * F, dtype=np.int64).reshape(F, 3).T.copy()
    return logits, idx


def softmax(theta):
    """Softmax over axis 0 (the three mesh corners), shifted by the maximum."""
    theta = np.asarray(theta, dtype=np.float64)
    e = np.exp(theta - theta.max(axis=0, keepdims=True))
    return e / e.sum(axis=0, keepdims=True)


def _corners(mesh_pos, mesh_idx, n, V):
    """Per secondary vertex, the positions of its mesh face's corners: [3 corners][3 xyz][V]."""
    T = n * n
    mf = np.arange(V) // (3 * T)
    mp = np.asarray(mesh_pos, dtype=np.float64)
    mi = np.asarray(mesh_idx)
    return np.stack([mp[:, mi[j, mf]] for j in range(3)])


def prior_vertices(mesh_pos, mesh_idx, n: int, logits):
    """Secondary vertex positions [3][V]: v = sum_j softmax(theta)_j m_j of the vertex's mesh face."""
    logits = np.asarray(logits, dtype=np.float64)
    V = logits.shape[1]
    a = softmax(logits)
    m = _corners(mesh_pos, mesh_idx, n, V)
    return sum(a[j] * m[j] for j in range(3))


def prior_backward(mesh_pos, mesh_idx, n: int, logits, dpos):
    """dL/dtheta [3][V] from dL/dv [3][V] through v = sum_j a_j m_j, a = softmax(theta):
    with g_j = dL/dv . m_j, dL/dtheta_j = a_j (g_j - sum_k a_k g_k)."""
    logits = np.asarray(logits, dtype=np.float64)
    dpos = np.asarray(dpos, dtype=np.float64)
    V = logits.shape[1]
    a = softmax(logits)
    m = _corners(mesh_pos, mesh_idx, n, V)
    g = np.stack([(dpos * m[j]).sum(axis=0) for j in range(3)])
    return a * (g - (a * g).sum(axis=0, keepdims=True))


def prior_colors(mesh_rgb, mesh_idx, n: int, logits):
    """Initial secondary colours [3][V]: the mesh vertex colours mixed with the same weights."""
    return prior_vertices(mesh_rgb, mesh_idx, n, logits)
