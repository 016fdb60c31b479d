"""Tile binning and per-tile depth order, stated in float32 (oracle; test infrastructure only).

The paper renders through a rasteriser that orders layers by depth (rendering
section); how faces reach tiles is internal to that rasteriser and is not in
the paper. The HIP path bins faces to screen tiles and orders each tile's list
by its faces' nearest depth. This module states that binning rule as an exact
float32 formula, evaluated with numpy float32 scalars/arrays (every operation
is one IEEE-754 binary32 op, no fused multiply-add), so tile lists and their
order can be compared bit for bit:

  camera coordinates  x_c = ((W00 x + W01 y) + W02 z) + W03 (same for y_c, z_c)
  pixel coordinates   u = fx (x_c / z_c) + cx,  v = fy (y_c / z_c) + cy
  near cull           the face is dropped if any corner has z_c <= znear
  pixel range         px0 = max(0, ceil((min u - 1/2) - 2^-8)),
                      px1 = min(W-1, floor((max u - 1/2) + 2^-8)); same for rows
  tiles               tx = px // tile_w, ty = py // tile_h over the pixel range;
                      a face with an empty range has no tile
  key                 (bits(min z_c) << 32) | face id, sorted ascending per tile

Its link to the float64 renderer is a pin: every float64 hit (pixel, face)
has the face in that pixel's tile list.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
MARGIN = F32(2.0 ** -8)


def project_f32(pos, cam):
    """pos [3][V] float32 -> (xc, yc, zc, u, v) float32 arrays, fixed operation order."""
    P = np.asarray(pos, dtype=np.float32)
    W = np.asarray(cam.world_to_cam, dtype=np.float32)
    x, y, z = P[0], P[1], P[2]
    xc = ((W[0, 0] * x + W[0, 1] * y) + W[0, 2] * z) + W[0, 3]
    yc = ((W[1, 0] * x + W[1, 1] * y) + W[1, 2] * z) + W[1, 3]
    zc = ((W[2, 0] * x + W[2, 1] * y) + W[2, 2] * z) + W[2, 3]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = F32(cam.fx) * (xc / zc) + F32(cam.cx)
        v = F32(cam.fy) * (yc / zc) + F32(cam.cy)
    return xc, yc, zc, u, v


def face_ranges(pos, idx, cam):
    """Per face: visible flag, pixel range (px0, px1, py0, py1) and zmin (float32)."""
    _, _, zc, u, v = project_f32(pos, cam)
    I = np.asarray(idx, np.int64)
    zf = zc[I]                                    # [3][F]
    uf = u[I]
    vf = v[I]
    zn = F32(cam.znear)
    vis = np.all(zf > zn, axis=0)
    zmin = np.min(zf, axis=0)
    with np.errstate(invalid="ignore", over="ignore"):
        umin = np.min(uf, axis=0)
        umax = np.max(uf, axis=0)
        vmin = np.min(vf, axis=0)
        vmax = np.max(vf, axis=0)
        half = F32(0.5)
        fx0 = np.ceil((umin - half) - MARGIN)
        fx1 = np.floor((umax - half) + MARGIN)
        fy0 = np.ceil((vmin - half) - MARGIN)
        fy1 = np.floor((vmax - half) + MARGIN)
    Wm1 = F32(cam.width - 1)
    Hm1 = F32(cam.height - 1)
    fx0 = np.maximum(fx0, F32(0))
    fy0 = np.maximum(fy0, F32(0))
    fx1 = np.minimum(fx1, Wm1)
    fy1 = np.minimum(fy1, Hm1)
    ok = vis & np.isfinite(umin) & np.isfinite(umax) & np.isfinite(vmin) & np.isfinite(vmax)
    ok &= (fx0 <= fx1) & (fy0 <= fy1)
    px0 = np.where(ok, fx0, 0).astype(np.int64)
    px1 = np.where(ok, fx1, -1).astype(np.int64)
    py0 = np.where(ok, fy0, 0).astype(np.int64)
    py1 = np.where(ok, fy1, -1).astype(np.int64)
    return ok, (px0, px1, py0, py1), zmin.astype(np.float32)


def tile_lists(pos, idx, cam, tile_w, tile_h):
    """(offsets [n_tiles+1] int64, keys [E] uint64) for one view, each tile sorted ascending."""
    ok, (px0, px1, py0, py1), zmin = face_ranges(pos, idx, cam)
    ntx = -(-int(cam.width) // tile_w)
    nty = -(-int(cam.height) // tile_h)
    zbits = zmin.view(np.uint32).astype(np.uint64)
    per_tile = [[] for _ in range(ntx * nty)]
    for f in np.flatnonzero(ok):
        key = (int(zbits[f]) << 32) | int(f)
        for ty in range(py0[f] // tile_h, py1[f] // tile_h + 1):
            for tx in range(px0[f] // tile_w, px1[f] // tile_w + 1):
                per_tile[ty * ntx + tx].append(key)
    offsets = np.zeros(ntx * nty + 1, dtype=np.int64)
    keys = []
    for t, lst in enumerate(per_tile):
        lst.sort()
        keys.extend(lst)
        offsets[t + 1] = offsets[t] + len(lst)
    return offsets, np.asarray(keys, dtype=np.uint64)


def tile_lists_fast(pos, idx, cam, tile_w, tile_h):
    """tile_lists for large scenes: the same statement with the (face, tile)
    pairs enumerated by array operations instead of Python loops (pinned equal
    to tile_lists); the lists are ordered by sorting (tile, key) pairs."""
    ok, (px0, px1, py0, py1), zmin = face_ranges(pos, idx, cam)
    ntx = -(-int(cam.width) // tile_w)
    nty = -(-int(cam.height) // tile_h)
    f = np.flatnonzero(ok)
    tx0, tx1 = px0[f] // tile_w, px1[f] // tile_w
    ty0, ty1 = py0[f] // tile_h, py1[f] // tile_h
    nx = tx1 - tx0 + 1
    cnt = nx * (ty1 - ty0 + 1)
    owner = np.repeat(np.arange(len(f)), cnt)                     # which drawn face each pair belongs to
    first = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    k = np.arange(int(cnt.sum())) - first[owner]                  # the pair's rank within its face
    tile = (ty0[owner] + k // nx[owner]) * ntx + (tx0[owner] + k % nx[owner])
    key = (zmin.view(np.uint32).astype(np.uint64)[f[owner]] << np.uint64(32)) | f[owner].astype(np.uint64)
    order = np.lexsort((key, tile))
    counts = np.bincount(tile, minlength=ntx * nty)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return offsets, key[order]
