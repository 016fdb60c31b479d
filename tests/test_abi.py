"""The C ABI library loads, exports every function include/msp.h declares, and
its struct layouts match the Python binding (CPU only: no compute call)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2502_07754_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(libmsp_path):
    lib = C.CDLL(libmsp_path)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS), "binding and header disagree"


def test_version_and_sizing(libmsp_path):
    lib = _lib.load()
    assert lib.msp_version() == 10000
    nv, nf = C.c_int64(), C.c_int64()
    assert lib.msp_convert_size(1000, 8, 0, C.byref(nv), C.byref(nf)) == 0
    assert (nv.value, nf.value) == (9000, 8000)
    assert lib.msp_convert_size(500_000, 16, 0, C.byref(nv), C.byref(nf)) == 0
    assert (nv.value, nf.value) == (8_500_000, 8_000_000)
    assert lib.msp_convert_size(0, 8, 0, C.byref(nv), C.byref(nf)) == 0 and nf.value == 0
    for n, K, mode in [(-1, 8, 0), (10, 2, 0), (10, 65, 0), (10, 8, 7), (300_000_000, 8, 0), (10, 6, 1)]:
        assert lib.msp_convert_size(n, K, mode, C.byref(nv), C.byref(nf)) == -1
    # three fans: centre + 6 shared axis points + 3 (K - 4) others; 3K faces (19 vertices for K = 8)
    assert lib.msp_convert_size(100, 8, 1, C.byref(nv), C.byref(nf)) == 0
    assert (nv.value, nf.value) == (1900, 2400)
    assert lib.msp_convert_size(10, 4, 1, C.byref(nv), C.byref(nf)) == 0
    assert (nv.value, nf.value) == (70, 120)


def test_prior_sizing(libmsp_path):
    lib = _lib.load()
    nv, nf = C.c_int64(), C.c_int64()
    assert lib.msp_prior_size(327_680, 2, C.byref(nv), C.byref(nf)) == 0
    assert (nv.value, nf.value) == (3 * 4 * 327_680, 4 * 327_680)
    assert lib.msp_prior_size(0, 1, C.byref(nv), C.byref(nf)) == 0 and nv.value == 0
    for Fm, n in [(-1, 1), (10, 0), (10, 17), (200_000_000, 2)]:
        assert lib.msp_prior_size(Fm, n, C.byref(nv), C.byref(nf)) == -1
    assert lib.msp_prior_init(None, None, 1, 0.05, 0.5, None, None, None) == -1


def test_null_context_is_rejected(libmsp_path):
    lib = _lib.load()
    assert lib.msp_destroy(None) == -1
    assert lib.msp_set_stream(None, None) == -1
    assert lib.msp_last_error(None) == b"null context"
    assert lib.msp_convert(None, None, 8, 2.0, 0.2, 0, None) == -1
    assert lib.msp_render(None, None, None, 1, None, None, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of every ABI struct, compiled with gcc against msp.h, equal the ctypes layouts."""
    structs = {"msp_gaussians": _lib.Gaussians, "msp_faces": _lib.Faces, "msp_camera": _lib.Camera,
               "msp_render_opts": _lib.RenderOpts, "msp_face_grads": _lib.FaceGrads,
               "msp_render_stats": _lib.RenderStats, "msp_mesh": _lib.Mesh, "msp_adam_group": _lib.AdamGroup,
               "msp_rays": _lib.Rays}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "msp.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, f"{cname}.{fname}"
