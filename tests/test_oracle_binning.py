"""Pins of the float32 tile-binning statement: it is conservative with respect
to the float64 renderer (no hit is ever missing from its pixel's tile list),
each tile list is strictly sorted by (nearest depth, face id), and a hand-placed
face lands exactly on the tiles its pixel footprint covers."""
import numpy as np
import pytest

from oracle import binning as ob
from oracle import convert as oc
from oracle import render as orr
from paper_2502_07754_amd import scenes


def _faces32(g, K, sigma):
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, sigma)
    return {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in f.items()}


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 16)])
def test_conservative_and_sorted(tile):
    g = scenes.gaussians(1000, 5, 0.01, 0.1, flat=True)
    cam = scenes.ring_cameras(3, 48, 40)[1]
    f32 = _faces32(g, 8, 2.0)
    off, keys = ob.tile_lists(f32["pos"], f32["idx"], cam, *tile)
    tw, th = tile
    ntx = -(-cam.width // tw)
    f64 = {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in f32.items()}
    geom = orr.face_geometry(f64["pos"], f64["idx"], cam)
    misses = 0
    hits = 0
    for j in range(cam.height):
        for i in range(cam.width):
            fr = orr.pixel_fragments(f64, cam, i, j, geom)
            t = (j // th) * ntx + i // tw
            fids = set((keys[off[t]:off[t + 1]] & np.uint64(0xFFFFFFFF)).astype(np.int64).tolist())
            hits += len(fr["fid"])
            misses += sum(int(f) not in fids for f in fr["fid"])
    assert hits > 1000
    assert misses == 0
    for t in range(len(off) - 1):
        seg = keys[off[t]:off[t + 1]]
        assert np.all(seg[1:] > seg[:-1])


def test_hand_placed_face_tiles():
    # identity camera, fx = fy = 10, centre (16, 16): a face at z = 1 with corners
    # projecting to pixel coordinates (4.2, 5.0), (20.7, 6.0), (9.0, 17.3)
    cam = scenes.Camera(world_to_cam=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32),
                        fx=10.0, fy=10.0, cx=16.0, cy=16.0, width=32, height=32)
    uv = np.array([[4.2, 5.0], [20.7, 6.0], [9.0, 17.3]])
    pos = np.stack([(uv[:, 0] - 16) / 10, (uv[:, 1] - 16) / 10, np.ones(3)]).astype(np.float32)
    idx = np.array([[0], [1], [2]], dtype=np.int32)
    ok, (px0, px1, py0, py1), zmin = ob.face_ranges(pos, idx, cam)
    # pixel centres i + 1/2 inside [4.2, 20.7] are i = 4..20; rows j + 1/2 in [5, 17.3] are j = 5..16
    assert ok[0] and (px0[0], px1[0], py0[0], py1[0]) == (4, 20, 5, 16)
    assert zmin[0] == np.float32(1.0)
    off, keys = ob.tile_lists(pos, idx, cam, 8, 8)
    counts = np.diff(off).reshape(4, 4)
    expect = np.zeros((4, 4), int)
    expect[0:3, 0:3] = 1          # tile columns 0..2 (pixels 0..23), rows 0..2 (pixels 0..23)
    assert np.array_equal(counts, expect)
    assert np.all(keys == (np.uint64(np.float32(1.0).view(np.uint32)) << np.uint64(32)))


def test_near_cull_and_offscreen():
    cam = scenes.Camera(world_to_cam=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32),
                        fx=10.0, fy=10.0, cx=16.0, cy=16.0, width=32, height=32)
    pos = np.array([[0, 0.1, 0, 100, 101, 100], [0, 0, 0.1, 0, 0, 1], [0.01, 1, 1, 1, 1, 1]], np.float32)
    idx = np.array([[0, 3], [1, 4], [2, 5]], np.int32)
    ok, _, _ = ob.face_ranges(pos, idx, cam)
    assert not ok[0]          # one corner at z = znear
    assert not ok[1]          # projects far right of the image


@pytest.mark.parametrize("n,seed,tile,W,H", [(1000, 5, (8, 8), 48, 40), (3000, 6, (32, 16), 100, 70),
                                             (500, 7, (16, 16), 33, 65), (0, 8, (16, 16), 32, 32)])
def test_fast_tile_lists_equal_the_loop_statement(n, seed, tile, W, H):
    g = scenes.gaussians(max(n, 1), seed, 0.01, 0.3, flat=True)
    cam = scenes.ring_cameras(3, W, H)[seed % 3]
    f32 = _faces32(g, 8, 2.0)
    if n == 0:
        f32["idx"] = f32["idx"][:, :0]
    a_off, a_keys = ob.tile_lists(f32["pos"], f32["idx"], cam, *tile)
    b_off, b_keys = ob.tile_lists_fast(f32["pos"], f32["idx"], cam, *tile)
    assert np.array_equal(a_off, b_off)
    assert np.array_equal(a_keys, b_keys)
    assert n == 0 or len(a_keys) > n
