"""Export of a face soup to a standard mesh format.

The point of the conversion (introduction and conclusion of the paper) is a
mesh that ordinary mesh tools and renderers can load. This writes the faces
as binary little-endian PLY: per vertex x, y, z, red, green, blue and alpha
(float32; alpha is the vertex opacity), per face its three vertex indices.
Faces that reference no vertex are impossible by construction; vertices no
face references are written as they are (pruned soups contain none).

    from paper_2502_07754_amd.export import write_ply
    write_ply("scene.ply", faces)       # dict of tensors or arrays: pos [3][V], rgb [3][V], opacity [V], idx [3][F]
"""
from __future__ import annotations

import numpy as np


def _host(a):
    if a is None:
        return None
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a)


def write_ply(path: str, faces: dict) -> None:
    """Binary PLY with per-vertex colour and opacity (alpha)."""
    pos = _host(faces["pos"]).astype(np.float32)
    rgb = _host(faces.get("rgb"))
    op = _host(faces["opacity"]).astype(np.float32)
    idx = _host(faces["idx"]).astype(np.int32)
    V, F = pos.shape[1], idx.shape[1]
    if rgb is None:
        rgb = np.full((3, V), 0.5, np.float32)
    rgb = rgb.astype(np.float32)
    if idx.size and (idx.min() < 0 or idx.max() >= V):
        raise ValueError("face indices out of range")
    vert = np.empty(V, dtype=[("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("red", "<f4"), ("green", "<f4"),
                              ("blue", "<f4"), ("alpha", "<f4")])
    vert["x"], vert["y"], vert["z"] = pos
    vert["red"], vert["green"], vert["blue"] = rgb
    vert["alpha"] = op
    face = np.empty(F, dtype=[("n", "u1"), ("v", "<i4", (3,))])
    face["n"] = 3
    face["v"] = idx.T
    header = ("ply\nformat binary_little_endian 1.0\n"
              f"element vertex {V}\n"
              "property float x\nproperty float y\nproperty float z\n"
              "property float red\nproperty float green\nproperty float blue\nproperty float alpha\n"
              f"element face {F}\n"
              "property list uchar int vertex_indices\n"
              "end_header\n")
    with open(path, "wb") as fh:
        fh.write(header.encode("ascii"))
        fh.write(vert.tobytes())
        fh.write(face.tobytes())


def read_ply(path: str) -> dict:
    """Reads back what write_ply writes (same header layout only)."""
    with open(path, "rb") as fh:
        data = fh.read()
    end = data.index(b"end_header\n") + len(b"end_header\n")
    lines = data[:end].decode("ascii").splitlines()
    V = int(next(l for l in lines if l.startswith("element vertex")).split()[2])
    F = int(next(l for l in lines if l.startswith("element face")).split()[2])
    vt = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("red", "<f4"), ("green", "<f4"), ("blue", "<f4"),
                   ("alpha", "<f4")])
    ft = np.dtype([("n", "u1"), ("v", "<i4", (3,))])
    vert = np.frombuffer(data, dtype=vt, count=V, offset=end)
    face = np.frombuffer(data, dtype=ft, count=F, offset=end + V * vt.itemsize)
    return dict(pos=np.stack([vert["x"], vert["y"], vert["z"]]), rgb=np.stack([vert["red"], vert["green"], vert["blue"]]),
                opacity=vert["alpha"].copy(), idx=face["v"].T.copy(), nvert=face["n"].copy())
