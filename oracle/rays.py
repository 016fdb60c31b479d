"""Secondary rays through the face soup, float64 (oracle; test infrastructure only).

The paper's motivation (abstract and introduction) is that the converted soup
can be ray traced: shadow rays and incoherent secondary rays see the same
semi-transparent faces the rasteriser composites. Two queries over a set of
rays (origin o, direction d, parameter interval (t0, t1)):

  * transmittance: the product of (1 - alpha) over every face the ray hits
    inside the interval (order-free, so no sorting is needed);
  * closest hit: the hit with the smallest t among those with
    alpha >= alpha_min (ties to the smaller face id), with its barycentrics.

Readings (the paper names the use, not the arithmetic):
  * ray/triangle test of Moller and Trumbore: with e1 = p1 - p0,
    e2 = p2 - p0, det = e1 . (d x e2); det = 0 (ray parallel to the plane)
    is a miss; u, v are the barycentric weights of p1 and p2, the triangle is
    closed (u >= 0, v >= 0, u + v <= 1) and the interval open (t0 < t < t1);
  * opacity at a hit: alpha = clamp((1 - u - v) o0 + u o1 + v o2, 0, 1), the
    renderer's interpolation at the same point (the barycentrics of a 3D point
    on the face are what perspective-correct interpolation recovers);
  * faces are double-sided.
"""
from __future__ import annotations

import numpy as np


def intersect(pos, idx, o, d):
    """One ray against every face: (t, u, v, hit) arrays over faces (hit ignores the interval)."""
    P = np.asarray(pos, np.float64)
    I = np.asarray(idx, np.int64)
    p0, p1, p2 = P[:, I[0]], P[:, I[1]], P[:, I[2]]                # [3][F]
    o = np.asarray(o, np.float64).reshape(3, 1)
    d = np.asarray(d, np.float64).reshape(3, 1)
    e1, e2 = p1 - p0, p2 - p0
    pv = np.cross(d, e2, axis=0)
    det = (e1 * pv).sum(axis=0)
    ok = det != 0.0
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    tv = o - p0
    u = (tv * pv).sum(axis=0) * inv
    qv = np.cross(tv, e1, axis=0)
    v = (d * qv).sum(axis=0) * inv
    t = (e2 * qv).sum(axis=0) * inv
    hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1)
    return t, u, v, hit


def hit_alpha(opacity, idx, u, v):
    """alpha = clamp((1-u-v) o0 + u o1 + v o2, 0, 1) per face."""
    op = np.asarray(opacity, np.float64)
    I = np.asarray(idx, np.int64)
    return np.clip((1 - u - v) * op[I[0]] + u * op[I[1]] + v * op[I[2]], 0.0, 1.0)


def transmittance(faces, origins, dirs, t0, t1):
    """T per ray [R]: product of (1 - alpha) over hits with t0 < t < t1."""
    O = np.asarray(origins, np.float64)
    D = np.asarray(dirs, np.float64)
    R = O.shape[1]
    out = np.ones(R)
    for r in range(R):
        t, u, v, hit = intersect(faces["pos"], faces["idx"], O[:, r], D[:, r])
        sel = hit & (t > t0[r]) & (t < t1[r])
        a = hit_alpha(faces["opacity"], faces["idx"], u, v)
        out[r] = np.prod(1.0 - a[sel])
    return out


def closest_hit(faces, origins, dirs, t0, t1, alpha_min):
    """(t, face, u, v) per ray: the smallest t with t0 < t < t1 and alpha >= alpha_min, ties to the
    smaller face id; face -1 and t = inf when there is none."""
    O = np.asarray(origins, np.float64)
    D = np.asarray(dirs, np.float64)
    R = O.shape[1]
    T = np.full(R, np.inf)
    Fid = np.full(R, -1, np.int64)
    U = np.zeros(R)
    V = np.zeros(R)
    for r in range(R):
        t, u, v, hit = intersect(faces["pos"], faces["idx"], O[:, r], D[:, r])
        a = hit_alpha(faces["opacity"], faces["idx"], u, v)
        sel = np.flatnonzero(hit & (t > t0[r]) & (t < t1[r]) & (a >= alpha_min))
        if len(sel):
            k = sel[np.lexsort((sel, t[sel]))[0]]
            T[r], Fid[r], U[r], V[r] = t[k], k, u[k], v[k]
    return T, Fid, U, V


def near_boundary(faces, origins, dirs, t0, t1, eps_b=1e-4, eps_t=1e-5):
    """Per ray, whether some face's test is within a float32 decision margin:
    a barycentric within eps_b of its bound, or t within eps_t (relative) of an
    interval end, on a face whose plane the ray meets. A float32 test may
    include or drop such a face; returns the indices of those faces per ray."""
    O = np.asarray(origins, np.float64)
    D = np.asarray(dirs, np.float64)
    R = O.shape[1]
    flags = []
    for r in range(R):
        t, u, v, _ = intersect(faces["pos"], faces["idx"], O[:, r], D[:, r])
        inside = (u >= -eps_b) & (v >= -eps_b) & (u + v <= 1 + eps_b)
        edge = inside & ((np.abs(u) < eps_b) | (np.abs(v) < eps_b) | (np.abs(1 - u - v) < eps_b))
        scale = np.maximum(1.0, np.abs(t))
        tb = inside & ((np.abs(t - t0[r]) < eps_t * scale) | (np.abs(t - t1[r]) < eps_t * scale))
        flags.append(np.flatnonzero(edge | tb))
    return flags
