"""Brute-force renderer of a triangle soup and its adjoint, float64 (oracle; test infrastructure only).

What is computed (rendering section: MVP transform, layers peeled in depth
order, per-vertex attributes interpolated across each triangle, layers blended
front to back through the alpha channel, final RGB and alpha read out):

  * camera coordinates x_c = R x + t with the camera's 3x4 world-to-camera
    matrix; pixel (i, j) looks along d = ((i+1/2-cx)/fx, (j+1/2-cy)/fy, 1), so the
    ray parameter of a hit equals its camera-space depth z;
  * faces with any vertex at z <= znear are dropped (no clipping);
  * every remaining face is intersected with every pixel ray
    (Moller-Trumbore, double sided, closed edges); a hit needs det != 0,
    u >= 0, v >= 0, u + v <= 1 and t > znear, with barycentrics (1-u-v, u, v),
    which are the perspective-correct ones;
  * alpha = clamp(sum_k b_k o_k, 0, 1), colour = sum_k b_k c_k (or the face's
    per-view colour when colours come from spherical harmonics);
  * all hits are sorted by (depth, face id) and composited front to back:
    C = sum_i T_i a_i c_i, T_{i+1} = T_i (1 - a_i), RGB = C + T_{n+1} bg,
    A = 1 - T_{n+1}; by default with no early stop, and with t_eps > 0 only the
    fragments whose transmittance before them is at least t_eps (the pixel
    stops once it falls below; a list truncated there is composited as if it
    ended there, and the adjoint differentiates that truncated list).

The adjoint freezes the set and order of fragments (the derivative of an
unantialiased rasteriser) and differentiates the rest exactly:
  back to front with S_{n+1} = bg, P_{n+1} = 1:
    dc_i = g T_i a_i
    da_i = T_i (g . (c_i - S_{i+1})) + gA T_i P_{i+1}
    S_i = a_i c_i + (1 - a_i) S_{i+1},  P_i = (1 - a_i) P_{i+1}
  per vertex k of the fragment's face: do_k += b_k da_i (zero where the clamp
  is active), dc_k += b_k dc_i, dL/db_k = o_k da_i + c_k . dc_i, and through the
  intersection: with M = [-d, e1, e2] and x = (t, u, v) solving M x = -v0,
  dL/dv_k = -b_k M^{-T} (0, dL/du, dL/dv) in camera space, then R^T back to world.
"""
from __future__ import annotations

import numpy as np


def cam_arrays(cam):
    W = np.asarray(cam.world_to_cam, np.float64)
    return dict(R=W[:, :3], t=W[:, 3], fx=float(cam.fx), fy=float(cam.fy), cx=float(cam.cx),
                cy=float(cam.cy), W=int(cam.width), H=int(cam.height), znear=float(cam.znear))


def to_camera(pos, cam):
    """World positions [3][V] -> camera coordinates [V][3] (float64)."""
    c = cam_arrays(cam)
    p = np.asarray(pos, np.float64).T
    return p @ c["R"].T + c["t"]


def pixel_dir(cam, i, j):
    c = cam_arrays(cam)
    return np.array([(i + 0.5 - c["cx"]) / c["fx"], (j + 0.5 - c["cy"]) / c["fy"], 1.0])


def face_geometry(pos, idx, cam):
    """Camera-space corners and the near-plane mask of every face."""
    pc = to_camera(pos, cam)
    I = np.asarray(idx, np.int64)
    v0, v1, v2 = pc[I[0]], pc[I[1]], pc[I[2]]
    zn = cam_arrays(cam)["znear"]
    keep = (v0[:, 2] > zn) & (v1[:, 2] > zn) & (v2[:, 2] > zn)
    return v0, v1, v2, keep


def intersect(d, v0, v1, v2, znear):
    """Moller-Trumbore of one ray (origin 0, direction d) against many triangles.

    Returns (hit mask, t, b0, b1, b2) arrays over the triangles.
    """
    e1 = v1 - v0
    e2 = v2 - v0
    p = np.cross(d[None, :], e2)
    det = np.einsum("ij,ij->i", e1, p)
    ok = det != 0.0
    inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
    s = -v0
    u = np.einsum("ij,ij->i", s, p) * inv
    q = np.cross(s, e1)
    v = (q @ d) * inv
    t = np.einsum("ij,ij->i", e2, q) * inv
    hit = ok & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > znear)
    return hit, t, 1.0 - u - v, u, v


def pixel_fragments(faces, cam, i, j, geom=None, candidates=None):
    """All fragments of pixel (i, j), sorted by (depth, face id).

    Returns a dict of arrays: fid, z, b [n][3]. `candidates` optionally limits the
    faces tested (used only where the caller can prove the others cannot hit).
    """
    v0, v1, v2, keep = geom if geom is not None else face_geometry(faces["pos"], faces["idx"], cam)
    fids = np.flatnonzero(keep) if candidates is None else np.asarray(candidates)[keep[candidates]]
    d = pixel_dir(cam, i, j)
    hit, t, b0, b1, b2 = intersect(d, v0[fids], v1[fids], v2[fids], cam_arrays(cam)["znear"])
    f = fids[hit]
    z = t[hit]
    b = np.stack([b0[hit], b1[hit], b2[hit]], axis=1)
    order = np.lexsort((f, z))
    return dict(fid=f[order], z=z[order], b=b[order])


def fragment_attributes(faces, frags, view_col=None):
    """alpha (clamped), raw alpha and colour of each fragment."""
    I = np.asarray(faces["idx"], np.int64)[:, frags["fid"]]      # [3][n]
    o = np.asarray(faces["opacity"], np.float64)[I]              # [3][n]
    raw = np.einsum("nk,kn->n", frags["b"], o)
    alpha = np.clip(raw, 0.0, 1.0)
    if view_col is None:
        C = np.asarray(faces["rgb"], np.float64)[:, I]           # [3 ch][3 k][n]
        col = np.einsum("nk,ckn->nc", frags["b"], C)
    else:
        col = np.asarray(view_col, np.float64)[:, frags["fid"]].T  # [n][3]
    return alpha, raw, col


def composite(alpha, col, bg):
    """Front-to-back over-compositing of an ordered list; returns (rgba, T list with T_1..T_{n+1})."""
    n = len(alpha)
    T = np.empty(n + 1)
    T[0] = 1.0
    C = np.zeros(3)
    for k in range(n):
        C += T[k] * alpha[k] * col[k]
        T[k + 1] = T[k] * (1.0 - alpha[k])
    rgba = np.concatenate([C + T[n] * np.asarray(bg, np.float64), [1.0 - T[n]]])
    return rgba, T


def early_stop(alpha, t_eps):
    """Number of leading fragments composited when a pixel stops once its
    transmittance falls below t_eps: fragment k is composited iff the
    transmittance before it is >= t_eps (t_eps = 0: all of them)."""
    T = 1.0
    for k, a in enumerate(alpha):
        if T < t_eps:
            return k
        T *= 1.0 - a
    return len(alpha)


def stop_ambiguous(alpha, t_eps, rel=1e-5):
    """Whether the early stop of a pixel may fall on another fragment in float32:
    some transmittance before a fragment, T_k = prod_{j<k} (1 - a_j), lies within
    rel * t_eps of t_eps (the float32 running product carries a relative error of
    a few 1e-7 per fragment, so the test T_k >= t_eps can go either way)."""
    if t_eps <= 0:
        return False
    T = 1.0
    for a in alpha:
        if abs(T - t_eps) <= rel * t_eps:
            return True
        T *= 1.0 - a
    return abs(T - t_eps) <= rel * t_eps


def _head(frags, n):
    return {k: (None if v is None else v[:n]) for k, v in frags.items()}


def render_pixels(faces, cam, pixels, bg=(0.0, 0.0, 0.0), view_col=None, return_frags=False, t_eps=0.0):
    """RGBA at the listed pixels [(i, j), ...]; optionally the fragment lists (as composited)."""
    geom = face_geometry(faces["pos"], faces["idx"], cam)
    out = np.zeros((len(pixels), 4))
    frs = []
    for n, (i, j) in enumerate(pixels):
        fr = pixel_fragments(faces, cam, i, j, geom)
        a, _, c = fragment_attributes(faces, fr, view_col)
        m = early_stop(a, t_eps)
        fr = _head(fr, m)
        out[n], _ = composite(a[:m], c[:m], bg)
        frs.append(fr)
    return (out, frs) if return_frags else out


def _render_rows(args):
    faces, cam, rows, bg, view_col = args
    W = int(cam.width)
    geom = face_geometry(faces["pos"], faces["idx"], cam)
    res = np.zeros((len(rows), 4, W))
    nfr = np.zeros((len(rows), W), dtype=np.int64)
    for r, j in enumerate(rows):
        for i in range(W):
            fr = pixel_fragments(faces, cam, i, j, geom)
            a, _, c = fragment_attributes(faces, fr, view_col)
            res[r, :, i], _ = composite(a, c, bg)
            nfr[r, i] = len(a)
    return rows, res, nfr


def render_image(faces, cam, bg=(0.0, 0.0, 0.0), view_col=None, processes=1):
    """Full RGBA image [4][H][W] and fragment counts [H][W] of one view."""
    H, W = int(cam.height), int(cam.width)
    img = np.zeros((4, H, W))
    nfrag = np.zeros((H, W), dtype=np.int64)
    chunks = [list(range(r, min(H, r + 4))) for r in range(0, H, 4)]
    jobs = [(faces, cam, rows, bg, view_col) for rows in chunks]
    if processes > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            results = pool.map(_render_rows, jobs)
    else:
        results = [_render_rows(j) for j in jobs]
    for rows, res, nfr in results:
        for r, j in enumerate(rows):
            img[:, j, :] = res[r]
            nfrag[j, :] = nfr[r]
    return img, nfrag


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------

def pixel_backward(faces, cam, i, j, g_rgba, frags, bg=(0.0, 0.0, 0.0), view_col=None, geom=None, t_eps=0.0):
    """Gradient contributions of one pixel with a frozen fragment list (truncated
    by the early stop when t_eps > 0).

    Returns dict: vid [m] vertex ids, dpos [m][3] (world), dop [m], drgb [m][3],
    and, in per-view-colour mode, fid [n] with dcol [n][3].
    """
    c = cam_arrays(cam)
    v0, v1, v2, _ = geom if geom is not None else face_geometry(faces["pos"], faces["idx"], cam)
    alpha, raw, col = fragment_attributes(faces, frags, view_col)
    n = early_stop(alpha, t_eps)
    frags = _head(frags, n)
    alpha, raw, col = alpha[:n], raw[:n], col[:n]
    _, T = composite(alpha, col, bg)
    g = np.asarray(g_rgba[:3], np.float64)
    gA = float(g_rgba[3])
    S = np.asarray(bg, np.float64).copy()
    P = 1.0
    I = np.asarray(faces["idx"], np.int64)
    o_all = np.asarray(faces["opacity"], np.float64)
    rgb_all = np.asarray(faces["rgb"], np.float64)
    d = pixel_dir(cam, i, j)
    vids, dpos, dop, drgb = [], [], [], []
    dcol = np.zeros((n, 3))
    for k in range(n - 1, -1, -1):
        f = frags["fid"][k]
        b = frags["b"][k]
        dc = g * T[k] * alpha[k]
        da = T[k] * float(g @ (col[k] - S)) + gA * T[k] * P
        S = alpha[k] * col[k] + (1.0 - alpha[k]) * S
        P = (1.0 - alpha[k]) * P
        da_raw = da if (0.0 < raw[k] < 1.0) else 0.0
        vk = I[:, f]
        ok = o_all[vk]
        if view_col is None:
            ck = rgb_all[:, vk].T                    # [3 k][3 ch]
            dLdb = ok * da_raw + ck @ dc
        else:
            dLdb = ok * da_raw
            dcol[k] = dc
        gx = np.array([0.0, dLdb[1] - dLdb[0], dLdb[2] - dLdb[0]])
        e1 = v1[f] - v0[f]
        e2 = v2[f] - v0[f]
        M = np.stack([-d, e1, e2], axis=1)
        w = np.linalg.solve(M.T, gx)
        for kk in range(3):
            vids.append(vk[kk])
            dpos.append(c["R"].T @ (-b[kk] * w))
            dop.append(b[kk] * da_raw)
            drgb.append(b[kk] * dc if view_col is None else np.zeros(3))
    out = dict(vid=np.asarray(vids, np.int64), dpos=np.asarray(dpos).reshape(-1, 3),
               dop=np.asarray(dop), drgb=np.asarray(drgb).reshape(-1, 3))
    if view_col is not None:
        out["fid"] = frags["fid"].copy()
        out["dcol"] = dcol
    return out


def render_backward_pixels(faces, cam, pixels, g_pixels, bg=(0.0, 0.0, 0.0), view_col=None, t_eps=0.0):
    """Sum of pixel_backward over the listed pixels -> per-vertex gradients (and per-face dcol)."""
    geom = face_geometry(faces["pos"], faces["idx"], cam)
    V = np.asarray(faces["opacity"]).shape[0]
    F = np.asarray(faces["idx"]).shape[1]
    dpos = np.zeros((V, 3))
    dop = np.zeros(V)
    drgb = np.zeros((V, 3))
    dcol = np.zeros((F, 3))
    for (i, j), g in zip(pixels, g_pixels):
        fr = pixel_fragments(faces, cam, i, j, geom)
        r = pixel_backward(faces, cam, i, j, g, fr, bg, view_col, geom, t_eps)
        np.add.at(dpos, r["vid"], r["dpos"])
        np.add.at(dop, r["vid"], r["dop"])
        np.add.at(drgb, r["vid"], r["drgb"])
        if view_col is not None:
            np.add.at(dcol, r["fid"], r["dcol"])
    out = dict(dpos=dpos.T.copy(), dop=dop, drgb=drgb.T.copy())
    if view_col is not None:
        out["dcol"] = dcol.T.copy()
    return out


def frozen_pixel_value(faces, cam, i, j, fids, bg=(0.0, 0.0, 0.0), view_col=None):
    """Pixel RGBA for a fixed ordered list of faces, re-intersecting each face's
    plane (barycentrics may fall outside the triangle). Used for finite differences
    of the frozen-fragment derivative."""
    v0, v1, v2, _ = face_geometry(faces["pos"], faces["idx"], cam)
    d = pixel_dir(cam, i, j)
    fids = np.asarray(fids, np.int64)
    e1 = v1[fids] - v0[fids]
    e2 = v2[fids] - v0[fids]
    p = np.cross(d[None, :], e2)
    det = np.einsum("ij,ij->i", e1, p)
    s = -v0[fids]
    u = np.einsum("ij,ij->i", s, p) / det
    q = np.cross(s, e1)
    v = (q @ d) / det
    fr = dict(fid=fids, z=None, b=np.stack([1 - u - v, u, v], axis=1))
    a, _, c = fragment_attributes(faces, fr, view_col)
    rgba, _ = composite(a, c, bg)
    return rgba


# ---------------------------------------------------------------------------
# Pixels where float32 arithmetic may legitimately pick a different fragment set
# or order than this float64 statement.
# ---------------------------------------------------------------------------

def projected_corners(faces, cam):
    """Pixel coordinates (u, v) of every face corner, float64: [F][3][2], plus near mask."""
    c = cam_arrays(cam)
    v0, v1, v2, keep = face_geometry(faces["pos"], faces["idx"], cam)
    P = np.stack([v0, v1, v2], axis=1)               # [F][3][3]
    z = np.where(P[..., 2] > 0, P[..., 2], 1.0)
    uv = np.stack([c["fx"] * P[..., 0] / z + c["cx"], c["fy"] * P[..., 1] / z + c["cy"]], axis=-1)
    return uv, keep


def ambiguous_pixels(faces, cam, pixels, tol=1e-4, edge_px=None, ztol=1e-6, bg=(0.0, 0.0, 0.0),
                     view_col=None, candidates=None, t_eps=0.0, geom=None, proj=None):
    """Flags pixels whose value depends on float32 rounding of coverage or order.

    A pixel is flagged when (i) some face has a screen-space edge within
    `edge_px` pixels of the pixel centre and toggling that face changes the
    pixel by more than `tol`, or (ii) two of its fragments have depths within
    `ztol` relative and swapping them changes the pixel by more than `tol`.
    The pixel's value is composited with the early stop t_eps (0: every
    fragment), so with tol = 0 a pixel is flagged exactly when its fragment set
    or order before the stop may differ in float32 (what the frozen-fragment
    gradient depends on). `candidates` optionally limits the faces examined
    (used only where the caller can prove that no other face comes within
    edge_px of the pixels). `geom` (face_geometry) and `proj`
    (projected_corners) may be passed to reuse them across calls.
    """
    c = cam_arrays(cam)
    if edge_px is None:
        edge_px = 16.0 * float(np.spacing(np.float32(max(c["W"], c["H"]))))
    uv_all, keep_all = proj if proj is not None else projected_corners(faces, cam)
    sub = np.flatnonzero(keep_all) if candidates is None else np.asarray(candidates, np.int64)
    sub = sub[keep_all[sub]]
    uv = uv_all[sub]
    if geom is None:
        geom = face_geometry(faces["pos"], faces["idx"], cam)

    def value(a, co):
        m = early_stop(a, t_eps)
        v, _ = composite(a[:m], co[:m], bg)
        return v

    flags = np.zeros(len(pixels), dtype=bool)
    for n, (i, j) in enumerate(pixels):
        p = np.array([i + 0.5, j + 0.5])
        near = np.zeros(len(sub), dtype=bool)
        for a, b in ((0, 1), (1, 2), (2, 0)):
            A = uv[:, a]
            B = uv[:, b]
            AB = B - A
            L2 = np.einsum("ij,ij->i", AB, AB)
            tt = np.clip(np.einsum("ij,ij->i", p - A, AB) / np.where(L2 > 0, L2, 1.0), 0.0, 1.0)
            Q = A + tt[:, None] * AB
            dist = np.linalg.norm(p - Q, axis=1)
            near |= dist <= edge_px
        fr = pixel_fragments(faces, cam, i, j, geom, candidates=candidates)
        al, _, co = fragment_attributes(faces, fr, view_col)
        base = value(al, co)
        bad = False
        for f in sub[near]:
            if f in set(fr["fid"].tolist()):
                m = fr["fid"] != f
                fr2 = dict(fid=fr["fid"][m], z=fr["z"][m], b=fr["b"][m])
            else:
                # include it with its (slightly outside) barycentrics, in depth order
                d = pixel_dir(cam, i, j)
                hit, t, b0, b1, b2 = intersect(d, geom[0][[f]], geom[1][[f]], geom[2][[f]], -np.inf)
                if not np.isfinite(t[0]) or t[0] <= c["znear"]:
                    continue
                fid = np.concatenate([fr["fid"], [f]])
                z = np.concatenate([fr["z"], t])
                b = np.concatenate([fr["b"], np.clip(np.stack([b0, b1, b2], 1), 0.0, 1.0)])
                o = np.lexsort((fid, z))
                fr2 = dict(fid=fid[o], z=z[o], b=b[o])
            a2, _, c2 = fragment_attributes(faces, fr2, view_col)
            if np.max(np.abs(value(a2, c2) - base)) > tol:
                bad = True
                break
        if not bad and len(fr["z"]) > 1:
            z = fr["z"]
            close = np.flatnonzero(np.abs(np.diff(z)) <= ztol * np.maximum(np.abs(z[1:]), 1e-30))
            for k in close:
                o = np.arange(len(z))
                o[k], o[k + 1] = k + 1, k
                if np.max(np.abs(value(al[o], co[o]) - base)) > tol:
                    bad = True
                    break
        flags[n] = bad
    return flags
