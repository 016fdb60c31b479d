"""Mesh export: a converted fan soup written as PLY reads back unchanged, with
the layout a PLY reader expects (header counts, byte size)."""
import os

import numpy as np

from oracle import convert as oc
from paper_2502_07754_amd import scenes
from paper_2502_07754_amd.export import read_ply, write_ply
from tests.helpers import faces_f32


def test_ply_round_trip(tmp_path):
    g = scenes.gaussians(50, 4, 0.01, 0.1, flat=True)
    f = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0))
    path = str(tmp_path / "fans.ply")
    write_ply(path, f)
    back = read_ply(path)
    assert np.array_equal(back["pos"], f["pos"])
    assert np.array_equal(back["rgb"], f["rgb"])
    assert np.array_equal(back["opacity"], f["opacity"])
    assert np.array_equal(back["idx"], f["idx"])
    assert np.all(back["nvert"] == 3)
    V, F = f["pos"].shape[1], f["idx"].shape[1]
    with open(path, "rb") as fh:
        head = fh.read(400).split(b"end_header\n")[0].decode()
    assert f"element vertex {V}" in head and f"element face {F}" in head
    hdr = len(head) + len("end_header\n")
    assert os.path.getsize(path) == hdr + V * 7 * 4 + F * (1 + 3 * 4)
