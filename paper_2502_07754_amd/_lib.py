"""ctypes binding of libmsp.so (include/msp.h). Argument marshalling only.

Every computation runs in the HIP library; there is no Python or CPU fallback.
If the library is missing or the device is not a GPU, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")


class MspError(RuntimeError):
    pass


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p), ("sh", C.c_void_p)]


class Faces(C.Structure):
    _fields_ = [("n_verts", C.c_int64), ("n_faces", C.c_int64), ("pos", C.c_void_p), ("opacity", C.c_void_p),
                ("rgb", C.c_void_p), ("sh", C.c_void_p), ("idx", C.c_void_p), ("gid", C.c_void_p)]


class Mesh(C.Structure):
    _fields_ = [("n_verts", C.c_int64), ("n_faces", C.c_int64), ("pos", C.c_void_p), ("idx", C.c_void_p),
                ("rgb", C.c_void_p)]


class Rays(C.Structure):
    _fields_ = [("n", C.c_int64), ("origin", C.c_void_p), ("dir", C.c_void_p), ("tmin", C.c_void_p),
                ("tmax", C.c_void_p), ("order", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("world_to_cam", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("znear", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class RenderOpts(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("kbuf", C.c_int32), ("color_mode", C.c_int32),
                ("t_eps", C.c_float), ("bg", C.c_float * 3), ("list_rows", C.c_int32), ("deterministic", C.c_int32)]


class FaceGrads(C.Structure):
    _fields_ = [("dpos", C.c_void_p), ("dopacity", C.c_void_p), ("drgb", C.c_void_p), ("dsh", C.c_void_p)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float), ("lo", C.c_float), ("hi", C.c_float), ("clamp", C.c_int32)]


class RenderStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_views", "width", "height", "tile_w", "tile_h", "entries",
                                         "max_tile_entries", "fragments", "restarts",
                                         "footprint_pixels")]


EXPORTS = {
    # name: (restype, argtypes)
    "msp_version": (C.c_int, []),
    "msp_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "msp_destroy": (C.c_int, [C.c_void_p]),
    "msp_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "msp_last_error": (C.c_char_p, [C.c_void_p]),
    "msp_convert_size": (C.c_int, [C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "msp_convert": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float, C.c_int,
                              C.POINTER(Faces)]),
    "msp_state_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "msp_state_free": (C.c_int, [C.c_void_p, C.c_void_p]),
    "msp_render": (C.c_int, [C.c_void_p, C.POINTER(Faces), C.POINTER(Camera), C.c_int, C.POINTER(RenderOpts),
                             C.c_void_p, C.c_void_p]),
    "msp_render_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Faces), C.c_void_p, C.POINTER(FaceGrads)]),
    "msp_state_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RenderStats)]),
    "msp_debug_tiles": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "msp_debug_nfrag": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "msp_step_graph": (C.c_int, [C.c_void_p, C.POINTER(Faces), C.POINTER(Camera), C.c_int, C.POINTER(RenderOpts),
                                 C.c_void_p, C.c_void_p, C.POINTER(FaceGrads), C.c_void_p]),
    "msp_state_status": (C.c_int, [C.c_void_p, C.c_void_p]),
    "msp_graph_info": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64)]),
    "msp_autotune": (C.c_int, [C.c_void_p, C.POINTER(Faces), C.POINTER(Camera), C.c_int, C.POINTER(RenderOpts),
                               C.c_void_p, C.c_void_p, C.POINTER(FaceGrads), C.POINTER(RenderOpts)]),
    "msp_loss": (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                           C.c_void_p, C.c_void_p]),
    "msp_loss_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                   C.c_int, C.c_void_p, C.c_void_p]),
    "msp_adam_step": (C.c_int, [C.c_void_p, C.POINTER(AdamGroup), C.c_int, C.c_int, C.c_float, C.c_float,
                                C.c_float]),
    "msp_prune": (C.c_int, [C.c_void_p, C.POINTER(Faces), C.c_float, C.POINTER(C.c_void_p), C.POINTER(C.c_int),
                            C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "msp_rings_size": (C.c_int, [C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "msp_convert_rings": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_int, C.c_float,
                                    C.POINTER(Faces)]),
    "msp_prior_size": (C.c_int, [C.c_int64, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "msp_prior_init": (C.c_int, [C.c_void_p, C.POINTER(Mesh), C.c_int, C.c_float, C.c_float, C.c_void_p, C.c_void_p,
                                 C.POINTER(Faces)]),
    "msp_prior_vertices": (C.c_int, [C.c_void_p, C.POINTER(Mesh), C.c_int, C.c_void_p, C.c_void_p]),
    "msp_prior_backward": (C.c_int, [C.c_void_p, C.POINTER(Mesh), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "msp_spatial_order": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_void_p]),
    "msp_point_order": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "msp_convert_ordered": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float, C.c_int,
                                      C.c_void_p, C.POINTER(Faces)]),
    "msp_bvh_build": (C.c_int, [C.c_void_p, C.POINTER(Faces), C.POINTER(C.c_void_p)]),
    "msp_bvh_free": (C.c_int, [C.c_void_p, C.c_void_p]),
    "msp_bvh_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "msp_bvh_status": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "msp_trace_transmittance": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Rays), C.c_float, C.c_void_p]),
    "msp_trace_closest": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Rays), C.c_float, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "msp_refiner_create": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "msp_refiner_free": (C.c_int, [C.c_void_p, C.c_void_p]),
    "msp_refiner_set_weights": (C.c_int, [C.c_void_p, C.c_void_p] + [C.c_void_p] * 6),
    "msp_refiner_features": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_void_p]),
    "msp_refiner_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "msp_refiner_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64] + [C.c_void_p] * 7),
    "msp_refiner_apply": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float, C.c_void_p,
                                    C.POINTER(Faces)]),
    "msp_refiner_targets": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float,
                                      C.POINTER(Faces), C.c_void_p]),
    "msp_refiner_apply_backward": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float,
                                             C.c_void_p, C.POINTER(FaceGrads), C.c_void_p]),
    "msp_refiner_weights": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.c_int, C.c_float, C.c_float,
                                      C.c_void_p]),
    "msp_refiner_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.c_void_p, C.c_void_p]),
    "msp_timing_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "msp_timing_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
}

STAGES = ["convert", "sh_eval", "setup", "scan", "emit", "sort", "composite", "block_max", "bwd_lists",
          "bwd_grads", "sh_bwd", "other"]

_lib = None
_lock = threading.Lock()


def load():
    """Loads libmsp.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise MspError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_07754_amd.build`")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in EXPORTS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


class Context:
    """One msp_ctx per device; each call binds it to torch's current stream."""

    _by_device: dict = {}

    def __init__(self, device: int):
        import torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        rc = self.lib.msp_create(device, C.c_void_p(stream), C.byref(h))
        if rc != 0:
            raise MspError(f"msp_create failed ({rc})")
        self.h = h

    @classmethod
    def get(cls, device: int) -> "Context":
        ctx = cls._by_device.get(device)
        if ctx is None:
            ctx = cls._by_device[device] = Context(device)
        return ctx

    def bind_stream(self):
        import torch
        self.lib.msp_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def timing(self, on: bool):
        self.check(self.lib.msp_timing_enable(self.h, 1 if on else 0), "msp_timing_enable")

    def read_timing(self) -> dict:
        import numpy as np
        ms = np.zeros(len(STAGES), dtype=np.float64)
        calls = np.zeros(len(STAGES), dtype=np.int64)
        self.check(self.lib.msp_timing_read(self.h, ms.ctypes.data_as(C.c_void_p), calls.ctypes.data_as(C.c_void_p),
                                            len(STAGES)), "msp_timing_read")
        return {n: (float(ms[i]), int(calls[i])) for i, n in enumerate(STAGES)}

    def check(self, rc: int, what: str):
        if rc != 0:
            msg = self.lib.msp_last_error(self.h)
            raise MspError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")
