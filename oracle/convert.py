"""Gaussian -> triangle-fan conversion, float64 (oracle; test infrastructure only).

Follows the paper's section "Transformation for Flat Gaussians": two scaled
principal axes (Eq. 2d_scaledrot), K evenly spaced angles on [-pi, pi), boundary
vertices v = m + cos(theta) A + sin(theta) B (the vertex equation), a fan of K
triangles sharing the centre, per-vertex colour copied from the Gaussian and
per-vertex opacity equal to the Gaussian's at the centre and opac_mul times it
on the boundary (the opacity paragraph of the same section).

Readings where the paper is silent or garbled:
  * scales are linear (already exponentiated) and `sigma` is the multiplier, so
    sigma = 2.7 with scale = exp(s) is the paper's literal formula;
  * the two axes are those of the two largest scales (ties to the lower index),
    taken in increasing index order as (A, B);
  * angles theta_k = -pi + 2 pi k / K (half-open, so no zero-area face);
  * vertex layout: Gaussian g owns vertices g(K+1) (centre) and g(K+1)+1+k
    (boundary k); face gK+k = (centre, boundary k, boundary (k+1) mod K).

The 3D variant of the section "Transformation for 3D Gaussians" (three fans
on the planes (1,2), (1,3), (2,3) with shared intersection points) is
`convert_three_fans`.
"""
from __future__ import annotations

import numpy as np


def quat_to_rot(q):
    """Unit quaternion (w, x, y, z) rows -> rotation matrices [N][3][3] (columns r1, r2, r3)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def top2_axes(scale):
    """Indices (a, b), a < b, of the two largest scales per Gaussian; ties go to the lower index."""
    s = np.asarray(scale, dtype=np.float64)          # [N][3]
    n = s.shape[0]
    a = np.empty(n, dtype=np.int64)
    b = np.empty(n, dtype=np.int64)
    for g in range(n):
        # the dropped axis is the smallest scale; among equal smallest, the highest index
        order = sorted(range(3), key=lambda i: (s[g, i], -i))
        drop = order[0]
        keep = [i for i in range(3) if i != drop]
        a[g], b[g] = keep[0], keep[1]
    return a, b


def fan_angles(K):
    """theta_k = -pi + 2 pi k / K, k = 0..K-1."""
    return -np.pi + 2.0 * np.pi * np.arange(K) / K


def convert_fan(mean, scale, quat, opacity, rgb, K, sigma, opac_mul=0.2, sh=None):
    """Flat-fan conversion.

    Inputs use the scene layout ([3][N] etc.) as float32 or float64; outputs are
    float64 in the face-buffer layout: pos [3][V], opacity [V], rgb [3][V],
    idx [3][F] int32, gid [F] int32, and sh [48][F] when `sh` is given
    (each face carries its Gaussian's coefficients).
    """
    m = np.asarray(mean, np.float64).T
    s = np.asarray(scale, np.float64).T
    q = np.asarray(quat, np.float64).T
    o = np.asarray(opacity, np.float64)
    c = np.asarray(rgb, np.float64).T
    n = m.shape[0]
    R = quat_to_rot(q)
    a, b = top2_axes(s)
    gi = np.arange(n)
    A = (sigma * s[gi, a])[:, None] * R[gi, :, a]    # scaled_rot_1
    B = (sigma * s[gi, b])[:, None] * R[gi, :, b]    # scaled_rot_2
    th = fan_angles(K)
    V = n * (K + 1)
    pos = np.empty((V, 3))
    op = np.empty(V)
    col = np.empty((V, 3))
    centre = gi * (K + 1)
    pos[centre] = m
    op[centre] = o
    col[centre] = c
    for k in range(K):
        vid = centre + 1 + k
        pos[vid] = m + np.cos(th[k]) * A + np.sin(th[k]) * B
        op[vid] = opac_mul * o
        col[vid] = c
    F = n * K
    idx = np.empty((F, 3), dtype=np.int32)
    gid = np.empty(F, dtype=np.int32)
    for k in range(K):
        f = gi * K + k
        idx[f, 0] = centre
        idx[f, 1] = centre + 1 + k
        idx[f, 2] = centre + 1 + (k + 1) % K
        gid[f] = gi
    out = dict(pos=pos.T.copy(), opacity=op, rgb=col.T.copy(), idx=idx.T.copy(), gid=gid)
    if sh is not None:
        shg = np.asarray(sh, np.float64)              # [48][N]
        out["sh"] = shg[:, gid].copy()
    return out


def convert_three_fans(mean, scale, quat, opacity, rgb, K, sigma, opac_mul=0.2):
    """3D-Gaussian conversion: one fan on each of the planes (1,2), (1,3), (2,3).

    Section "Transformation for 3D Gaussians" (Eq. 3d_scaledrot and the plane
    pairs). Points at plane intersections are shared: each plane (i, j) has the
    boundary points m + cos(t) A_i + sin(t) A_j; the points at t = -pi, -pi/2, 0,
    pi/2 lie on the axes +-A_i, +-A_j and are merged when K is a multiple of 4.
    Vertex layout per Gaussian: centre, then the 6 axis points
    (+A1, -A1, +A2, -A2, +A3, -A3), then the remaining boundary points plane by
    plane in angle order. Faces: plane p (0:(1,2), 1:(1,3), 2:(2,3)) face k =
    (centre, b_p(k), b_p((k+1) mod K)), face id g*3K + p*K + k.
    """
    m = np.asarray(mean, np.float64).T
    s = np.asarray(scale, np.float64).T
    q = np.asarray(quat, np.float64).T
    o = np.asarray(opacity, np.float64)
    c = np.asarray(rgb, np.float64).T
    n = m.shape[0]
    if K % 4 != 0:
        raise ValueError("three-fan conversion shares axis points only for K divisible by 4")
    R = quat_to_rot(q)
    th = fan_angles(K)
    planes = [(0, 1), (0, 2), (1, 2)]
    per = 1 + 6 + 3 * (K - 4)
    V = n * per
    pos = np.empty((V, 3))
    op = np.empty(V)
    col = np.empty((V, 3))
    F = n * 3 * K
    idx = np.empty((F, 3), dtype=np.int32)
    gid = np.empty(F, dtype=np.int32)
    for g in range(n):
        base = g * per
        ax = [sigma * s[g, i] * R[g, :, i] for i in range(3)]
        pos[base] = m[g]
        op[base] = o[g]
        col[base] = c[g]
        for i in range(3):
            pos[base + 1 + 2 * i] = m[g] + ax[i]
            pos[base + 2 + 2 * i] = m[g] - ax[i]
        op[base + 1: base + 7] = opac_mul * o[g]
        col[base + 1: base + 7] = c[g]
        nxt = base + 7
        for p, (i, j) in enumerate(planes):
            ring = []
            for k in range(K):
                # exact quarter turns land on the shared axis points
                quarter = (4 * k) % K == 0
                if quarter:
                    step = (4 * k) // K          # 0:-pi, 1:-pi/2, 2:0, 3:pi/2
                    vid = {0: base + 2 + 2 * i, 1: base + 2 + 2 * j,
                           2: base + 1 + 2 * i, 3: base + 1 + 2 * j}[step]
                else:
                    vid = nxt
                    pos[vid] = m[g] + np.cos(th[k]) * ax[i] + np.sin(th[k]) * ax[j]
                    op[vid] = opac_mul * o[g]
                    col[vid] = c[g]
                    nxt += 1
                ring.append(vid)
            for k in range(K):
                f = g * 3 * K + p * K + k
                idx[f] = (base, ring[k], ring[(k + 1) % K])
                gid[f] = g
        assert nxt == base + per
    return dict(pos=pos.T.copy(), opacity=op, rgb=col.T.copy(), idx=idx.T.copy(), gid=gid)
