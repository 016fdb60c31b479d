"""MeshSplats hot path for AMD Instinct MI355X (gfx950).

Thin Python layer over libmsp.so (include/msp.h): torch tensors supply device
memory and the stream; every step of conversion, binning, sorting,
compositing and the adjoint runs in the library's HIP kernels.

    faces = convert(gaussians, K=8, sigma=2.0)
    img, state = render(faces, cameras)
    grads = render_backward(state, faces, dimg)
    img = MeshRender.apply(pos, opacity, rgb, faces, cameras, options)  # autograd
"""
from __future__ import annotations

import ctypes as C
import dataclasses

from . import _lib
from ._lib import MspError

__all__ = ["convert", "render", "render_backward", "RenderOptions", "RenderState", "MeshRender", "MspError",
           "camera_struct", "load_library", "GraphStep", "autotune", "loss", "adam_step", "prune", "convert_rings",
           "Refiner", "refiner_features", "refiner_apply", "refiner_targets", "refiner_weights",
           "refiner_apply_backward", "refiner_loss", "MSP_FAN_FLAT", "MSP_FAN_3D", "prior_init", "prior_vertices",
           "prior_backward", "Bvh", "spatial_order", "point_order"]

MSP_COLOR_RGB = 0
MSP_COLOR_SH3 = 1
MSP_FAN_FLAT = 0
MSP_FAN_3D = 1


def load_library():
    return _lib.load()


def _dev_ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, name):
    import torch
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ctx(t):
    return _lib.Context.get(t.device.index if t.device.index is not None else 0)


def spatial_order(g: dict):
    """msp_spatial_order: int32 [N] order of the Gaussians along the Morton curve of their means."""
    import torch
    mean = _need(g["mean"], torch.float32, "mean")
    if mean.dim() != 2 or mean.shape[0] != 3:
        raise ValueError("mean must be [3][N]")
    ctx = _ctx(mean)
    ctx.bind_stream()
    order = torch.empty((mean.shape[1],), dtype=torch.int32, device=mean.device)
    G = _lib.Gaussians(mean.shape[1], _dev_ptr(mean), None, None, None, None, None)
    ctx.check(ctx.lib.msp_spatial_order(ctx.h, C.byref(G), _dev_ptr(order)), "msp_spatial_order")
    return order


def point_order(points):
    """msp_point_order: int32 [n] order of points [3][n] along their Morton curve (e.g. ray origins)."""
    import torch
    p = _need(points, torch.float32, "points")
    if p.dim() != 2 or p.shape[0] != 3:
        raise ValueError("points must be [3][n]")
    ctx = _ctx(p)
    ctx.bind_stream()
    order = torch.empty((p.shape[1],), dtype=torch.int32, device=p.device)
    ctx.check(ctx.lib.msp_point_order(ctx.h, _dev_ptr(p), p.shape[1], _dev_ptr(order)), "msp_point_order")
    return order


def convert(g: dict, K: int, sigma: float, opac_mul: float = 0.2, mode: int = 0, order=None) -> dict:
    """Gaussian -> triangle fans (msp_convert). `g` holds GPU float32 tensors
    mean [3,N], scale [3,N], quat [4,N], opacity [N], rgb [3,N] and optionally sh [48,N].
    mode MSP_FAN_FLAT (one fan over the two largest axes) or MSP_FAN_3D (three fans).
    With `order` (int32 [N], e.g. from spatial_order) output block i is converted
    from Gaussian order[i] and gid records it (msp_convert_ordered)."""
    import torch
    mean = _need(g["mean"], torch.float32, "mean")
    ctx = _ctx(mean)
    ctx.bind_stream()
    n = mean.shape[1]
    nv, nf = C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.msp_convert_size(n, K, int(mode), C.byref(nv), C.byref(nf)), "msp_convert_size")
    dev = mean.device
    sh = g.get("sh")
    out = dict(pos=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               opacity=torch.empty((nv.value,), dtype=torch.float32, device=dev),
               rgb=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               idx=torch.empty((3, nf.value), dtype=torch.int32, device=dev),
               gid=torch.empty((nf.value,), dtype=torch.int32, device=dev),
               sh=None if sh is None else torch.empty((48, nf.value), dtype=torch.float32, device=dev))
    G = _lib.Gaussians(n, _dev_ptr(mean), _dev_ptr(_need(g["scale"], torch.float32, "scale")),
                       _dev_ptr(_need(g["quat"], torch.float32, "quat")),
                       _dev_ptr(_need(g["opacity"], torch.float32, "opacity")),
                       _dev_ptr(_need(g["rgb"], torch.float32, "rgb")),
                       None if sh is None else _dev_ptr(_need(sh, torch.float32, "sh")))
    Fc = _faces_struct(out)
    if order is None:
        ctx.check(ctx.lib.msp_convert(ctx.h, C.byref(G), K, float(sigma), float(opac_mul), int(mode), C.byref(Fc)),
                  "msp_convert")
    else:
        _need(order, torch.int32, "order")
        if order.numel() != n:
            raise ValueError(f"order must have {n} entries")
        ctx.check(ctx.lib.msp_convert_ordered(ctx.h, C.byref(G), K, float(sigma), float(opac_mul), int(mode),
                                              _dev_ptr(order), C.byref(Fc)), "msp_convert_ordered")
    return out


def _faces_struct(f: dict) -> _lib.Faces:
    return _lib.Faces(f["pos"].shape[1], f["idx"].shape[1], _dev_ptr(f["pos"]), _dev_ptr(f["opacity"]),
                      _dev_ptr(f.get("rgb")), _dev_ptr(f.get("sh")), _dev_ptr(f["idx"]), _dev_ptr(f.get("gid")))


def camera_struct(cam) -> _lib.Camera:
    """scenes.Camera (or any object with the same fields) -> msp_camera."""
    import numpy as np
    W = np.asarray(cam.world_to_cam, dtype=np.float32).reshape(12)
    return _lib.Camera((C.c_float * 12)(*W.tolist()), cam.fx, cam.fy, cam.cx, cam.cy, cam.znear,
                       int(cam.width), int(cam.height))


@dataclasses.dataclass
class RenderOptions:
    tile_w: int = 0        # 0: the context's autotuned (or default 16) tile
    tile_h: int = 0
    kbuf: int = 0          # 0: default 16
    t_eps: float = 1e-6
    bg: tuple = (0.0, 0.0, 0.0)
    color_mode: int = MSP_COLOR_RGB
    list_rows: int = 0     # > 0: the forward stores fragment lists for the backward (0: recomputed)
    deterministic: int = 0  # 1: fixed-point gradient sums, identical bits on every run

    def struct(self) -> _lib.RenderOpts:
        return _lib.RenderOpts(self.tile_w, self.tile_h, self.kbuf, self.color_mode, self.t_eps,
                               (C.c_float * 3)(*self.bg), self.list_rows, int(self.deterministic))


class RenderState:
    """Library-owned tile lists and per-pixel counts of one render."""

    def __init__(self, ctx):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(ctx.lib.msp_state_create(ctx.h, C.byref(h)), "msp_state_create")
        self.h = h
        self.n_views = self.height = self.width = 0
        self.color_mode = MSP_COLOR_RGB

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.msp_state_free(self.ctx.h, self.h)
                self.h = None
        except Exception:
            pass

    def status(self) -> int:
        """MSP_OK (0), or MSP_EOVERFLOW (-4) when a bounded buffer of this state fell
        short and the library recovered (results complete either way)."""
        return int(self.ctx.lib.msp_state_status(self.ctx.h, self.h))

    def stats(self) -> dict:
        s = _lib.RenderStats()
        self.ctx.check(self.ctx.lib.msp_state_stats(self.ctx.h, self.h, C.byref(s)), "msp_state_stats")
        return {n: getattr(s, n) for n, _ in s._fields_}

    def tiles(self, view: int):
        import numpy as np
        st = self.stats()
        nt = -(-st["width"] // st["tile_w"]) * -(-st["height"] // st["tile_h"])
        off = np.zeros(nt + 1, dtype=np.int64)
        self.ctx.check(self.ctx.lib.msp_debug_tiles(self.ctx.h, self.h, view, off.ctypes.data_as(C.c_void_p), None),
                       "msp_debug_tiles")
        keys = np.zeros(max(1, int(off[-1])), dtype=np.uint64)
        self.ctx.check(self.ctx.lib.msp_debug_tiles(self.ctx.h, self.h, view, off.ctypes.data_as(C.c_void_p),
                                                    keys.ctypes.data_as(C.c_void_p)), "msp_debug_tiles")
        return off, keys[:int(off[-1])]

    def nfrag(self):
        import numpy as np
        out = np.zeros((self.n_views, self.height, self.width), dtype=np.int32)
        self.ctx.check(self.ctx.lib.msp_debug_nfrag(self.ctx.h, self.h, out.ctypes.data_as(C.c_void_p)),
                       "msp_debug_nfrag")
        return out


def render(faces: dict, cams, opts: RenderOptions | None = None, state: RenderState | None = None):
    """msp_render: returns (img [V,4,H,W] float32 on the faces' device, state)."""
    import torch
    opts = opts or RenderOptions()
    pos = _need(faces["pos"], torch.float32, "pos")
    _need(faces["opacity"], torch.float32, "opacity")
    _need(faces["idx"], torch.int32, "idx")
    if opts.color_mode == MSP_COLOR_RGB:
        _need(faces["rgb"], torch.float32, "rgb")
    else:
        _need(faces.get("sh"), torch.float32, "sh")
    ctx = _ctx(pos)
    ctx.bind_stream()
    V = len(cams)
    arr = (_lib.Camera * V)(*[camera_struct(c) for c in cams])
    H, W = int(cams[0].height), int(cams[0].width)
    img = torch.empty((V, 4, H, W), dtype=torch.float32, device=pos.device)
    state = state or RenderState(ctx)
    Fc = _faces_struct(faces)
    o = opts.struct()
    ctx.check(ctx.lib.msp_render(ctx.h, C.byref(Fc), arr, V, C.byref(o), _dev_ptr(img), state.h), "msp_render")
    state.n_views, state.height, state.width = V, H, W
    state.color_mode = opts.color_mode
    return img, state


def render_backward(state: RenderState, faces: dict, dimg, need=("dpos", "dopacity", "drgb", "dsh")) -> dict:
    """msp_render_backward: gradients of the last render on `state` (drgb in RGB
    mode, dsh in SH mode)."""
    import torch
    ctx = state.ctx
    ctx.bind_stream()
    dimg = _need(dimg, torch.float32, "dimg")
    nv = faces["pos"].shape[1]
    dev = faces["pos"].device
    out = {}
    if "dpos" in need:
        out["dpos"] = torch.empty((3, nv), dtype=torch.float32, device=dev)
    if "dopacity" in need:
        out["dopacity"] = torch.empty((nv,), dtype=torch.float32, device=dev)
    sh_mode = getattr(state, "color_mode", MSP_COLOR_RGB) == MSP_COLOR_SH3
    if "drgb" in need and not sh_mode:
        out["drgb"] = torch.empty((3, nv), dtype=torch.float32, device=dev)
    if "dsh" in need and sh_mode:
        out["dsh"] = torch.empty((48, faces["idx"].shape[1]), dtype=torch.float32, device=dev)
    G = _lib.FaceGrads(_dev_ptr(out.get("dpos")), _dev_ptr(out.get("dopacity")), _dev_ptr(out.get("drgb")),
                       _dev_ptr(out.get("dsh")))
    Fc = _faces_struct(faces)
    ctx.check(ctx.lib.msp_render_backward(ctx.h, state.h, C.byref(Fc), _dev_ptr(dimg), C.byref(G)),
              "msp_render_backward")
    return out


def _grads_for(state, faces, sh_mode, need=("dpos", "dopacity", "drgb", "dsh")) -> dict:
    import torch
    nv = faces["pos"].shape[1]
    dev = faces["pos"].device
    out = {}
    if "dpos" in need:
        out["dpos"] = torch.empty((3, nv), dtype=torch.float32, device=dev)
    if "dopacity" in need:
        out["dopacity"] = torch.empty((nv,), dtype=torch.float32, device=dev)
    if "drgb" in need and not sh_mode:
        out["drgb"] = torch.empty((3, nv), dtype=torch.float32, device=dev)
    if "dsh" in need and sh_mode:
        out["dsh"] = torch.empty((48, faces["idx"].shape[1]), dtype=torch.float32, device=dev)
    return out


class GraphStep:
    """A forward + backward step replayed as a captured HIP graph (msp_step_graph).

    The image and gradient buffers are owned by this object and reused by every
    call (the graph is bound to their addresses)."""

    def __init__(self, faces: dict, cams, opts: "RenderOptions", dimg_shape=None):
        import torch
        pos = _need(faces["pos"], torch.float32, "pos")
        self.ctx = _ctx(pos)
        self.faces = faces
        self.cams = cams
        self.opts = opts
        V, H, W = len(cams), int(cams[0].height), int(cams[0].width)
        self.img = torch.empty((V, 4, H, W), dtype=torch.float32, device=pos.device)
        self.dimg = torch.zeros((V, 4, H, W), dtype=torch.float32, device=pos.device)
        self.state = RenderState(self.ctx)
        self.state.n_views, self.state.height, self.state.width = V, H, W
        self.state.color_mode = opts.color_mode
        self.grads = _grads_for(self.state, faces, opts.color_mode == MSP_COLOR_SH3)
        self._arr = (_lib.Camera * V)(*[camera_struct(c) for c in cams])
        self._F = _faces_struct(faces)
        self._G = _lib.FaceGrads(_dev_ptr(self.grads.get("dpos")), _dev_ptr(self.grads.get("dopacity")),
                                 _dev_ptr(self.grads.get("drgb")), _dev_ptr(self.grads.get("dsh")))
        self._o = opts.struct()

    def __call__(self, dimg=None):
        """Runs one step; `dimg` (if given) is copied into the bound upstream-gradient buffer first."""
        if dimg is not None:
            self.dimg.copy_(dimg)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_step_graph(self.ctx.h, C.byref(self._F), self._arr, len(self.cams),
                                                   C.byref(self._o), _dev_ptr(self.img), _dev_ptr(self.dimg),
                                                   C.byref(self._G), self.state.h), "msp_step_graph")
        return self.img, self.grads

    def info(self) -> dict:
        c, r, o = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx.check(self.ctx.lib.msp_graph_info(self.ctx.h, self.state.h, C.byref(c), C.byref(r), C.byref(o)),
                       "msp_graph_info")
        return dict(captures=c.value, replays=r.value, overflows=o.value)


def autotune(faces: dict, cams, base: "RenderOptions", dimg=None) -> "RenderOptions":
    """msp_autotune: the fastest tile size / buffer depth for this scene and view set."""
    import torch
    pos = _need(faces["pos"], torch.float32, "pos")
    ctx = _ctx(pos)
    ctx.bind_stream()
    V, H, W = len(cams), int(cams[0].height), int(cams[0].width)
    img = torch.empty((V, 4, H, W), dtype=torch.float32, device=pos.device)
    sh_mode = base.color_mode == MSP_COLOR_SH3
    grads = _grads_for(None, faces, sh_mode) if dimg is not None else {}
    G = _lib.FaceGrads(_dev_ptr(grads.get("dpos")), _dev_ptr(grads.get("dopacity")), _dev_ptr(grads.get("drgb")),
                       _dev_ptr(grads.get("dsh")))
    arr = (_lib.Camera * V)(*[camera_struct(c) for c in cams])
    out = _lib.RenderOpts()
    Fc = _faces_struct(faces)
    b = base.struct()
    ctx.check(ctx.lib.msp_autotune(ctx.h, C.byref(Fc), arr, V, C.byref(b), _dev_ptr(img),
                                   None if dimg is None else _dev_ptr(_need(dimg, torch.float32, "dimg")),
                                   C.byref(G), C.byref(out)), "msp_autotune")
    return RenderOptions(tile_w=out.tile_w, tile_h=out.tile_h, kbuf=out.kbuf, t_eps=out.t_eps,
                         bg=tuple(out.bg), color_mode=out.color_mode, list_rows=out.list_rows,
                         deterministic=out.deterministic)


MSP_LOSS_MSE, MSP_LOSS_L1, MSP_LOSS_L1_DSSIM = 0, 1, 2


def loss(img, tgt, kind=MSP_LOSS_MSE, lam=0.6, want_grad=True, noalloc=False, out=None, dimg=None):
    """msp_loss (or msp_loss_noalloc, which uses the library's fixed per-GPU
    scratch and allocates nothing): (loss as a 1-element GPU tensor, dL/dimg
    [V,4,H,W] or None). `out` and `dimg` may be given to write into."""
    import torch
    _need(img, torch.float32, "img")
    _need(tgt, torch.float32, "tgt")
    ctx = _ctx(img)
    ctx.bind_stream()
    V, _, H, W = img.shape
    if out is None:
        out = torch.empty((1,), dtype=torch.float32, device=img.device)
    if dimg is None and want_grad:
        dimg = torch.empty_like(img)
    fn = ctx.lib.msp_loss_noalloc if noalloc else ctx.lib.msp_loss
    ctx.check(fn(ctx.h, kind, float(lam), _dev_ptr(img), _dev_ptr(tgt), V, H, W, _dev_ptr(out),
                 _dev_ptr(dimg if want_grad else None)), "msp_loss_noalloc" if noalloc else "msp_loss")
    return out, (dimg if want_grad else None)


def adam_step(groups: list, step: int, beta1=0.9, beta2=0.999, eps=1e-8):
    """msp_adam_step; each group: dict(param, grad, m, v, lr, clamp=(lo, hi) or None)."""
    import torch
    if not groups:
        return
    ctx = _ctx(groups[0]["param"])
    ctx.bind_stream()
    arr = (_lib.AdamGroup * len(groups))()
    for i, g in enumerate(groups):
        for k in ("param", "grad", "m", "v"):
            _need(g[k], torch.float32, k)
            if g[k].numel() != g["param"].numel():
                raise ValueError(f"adam group {i}: {k} has {g[k].numel()} elements, param {g['param'].numel()}")
        cl = g.get("clamp")
        arr[i] = _lib.AdamGroup(_dev_ptr(g["param"]), _dev_ptr(g["grad"]), _dev_ptr(g["m"]), _dev_ptr(g["v"]),
                                g["param"].numel(), float(g["lr"]), float(cl[0]) if cl else 0.0,
                                float(cl[1]) if cl else 0.0, 1 if cl else 0)
    ctx.check(ctx.lib.msp_adam_step(ctx.h, arr, len(groups), int(step), beta1, beta2, eps), "msp_adam_step")


def prune(faces: dict, thresh: float, vstate: list = ()):
    """msp_prune in place; returns (faces dict, vstate list) as views sized for the survivors."""
    import torch
    pos = _need(faces["pos"], torch.float32, "pos")
    ctx = _ctx(pos)
    ctx.bind_stream()
    Fc = _faces_struct(faces)
    n = len(vstate)
    ptrs = (C.c_void_p * max(1, n))(*[t.data_ptr() for t in vstate])
    rows = (C.c_int * max(1, n))(*[int(t.shape[0]) if t.dim() == 2 else 1 for t in vstate])
    nv, nf = C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.msp_prune(ctx.h, C.byref(Fc), float(thresh), ptrs, rows, n, C.byref(nv), C.byref(nf)),
              "msp_prune")
    V2, F2 = nv.value, nf.value

    def pack(t, r, m):
        flat = t.view(-1)[: r * m]
        return flat.view(r, m) if t.dim() == 2 else flat

    out = dict(faces)
    out["pos"] = pack(faces["pos"], 3, V2)
    out["opacity"] = pack(faces["opacity"], 1, V2)
    if faces.get("rgb") is not None:
        out["rgb"] = pack(faces["rgb"], 3, V2)
    out["idx"] = pack(faces["idx"], 3, F2)
    if faces.get("gid") is not None:
        out["gid"] = pack(faces["gid"], 1, F2)
    if faces.get("sh") is not None:
        out["sh"] = pack(faces["sh"], 48, F2)
    vs = [pack(t, int(t.shape[0]) if t.dim() == 2 else 1, V2) for t in vstate]
    return out, vs


def convert_rings(g: dict, K: int, rings: int, sigma_max: float = 3.0) -> dict:
    """msp_convert_rings: the multi-ring conversion used for fine-tuning targets."""
    import torch
    mean = _need(g["mean"], torch.float32, "mean")
    ctx = _ctx(mean)
    ctx.bind_stream()
    n = mean.shape[1]
    nv, nf = C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.msp_rings_size(n, K, rings, C.byref(nv), C.byref(nf)), "msp_rings_size")
    dev = mean.device
    out = dict(pos=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               opacity=torch.empty((nv.value,), dtype=torch.float32, device=dev),
               rgb=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               idx=torch.empty((3, nf.value), dtype=torch.int32, device=dev),
               gid=torch.empty((nf.value,), dtype=torch.int32, device=dev), sh=None)
    G = _lib.Gaussians(n, _dev_ptr(mean), _dev_ptr(_need(g["scale"], torch.float32, "scale")),
                       _dev_ptr(_need(g["quat"], torch.float32, "quat")),
                       _dev_ptr(_need(g["opacity"], torch.float32, "opacity")),
                       _dev_ptr(_need(g["rgb"], torch.float32, "rgb")), None)
    Fc = _faces_struct(out)
    ctx.check(ctx.lib.msp_convert_rings(ctx.h, C.byref(G), K, rings, float(sigma_max), C.byref(Fc)),
              "msp_convert_rings")
    return out


def _mesh_struct(mesh: dict) -> _lib.Mesh:
    import torch
    pos = _need(mesh["pos"], torch.float32, "mesh pos")
    idx = _need(mesh["idx"], torch.int32, "mesh idx")
    rgb = mesh.get("rgb")
    return _lib.Mesh(pos.shape[1], idx.shape[1], _dev_ptr(pos), _dev_ptr(idx),
                     None if rgb is None else _dev_ptr(_need(rgb, torch.float32, "mesh rgb")))


def prior_init(mesh: dict, n: int, shrink: float = 0.05, opacity0: float = 0.5, rgb0=(0.5, 0.5, 0.5)):
    """msp_prior_init: n^2 secondary triangles per face of the geometry mesh
    (dict of GPU tensors pos [3][Vm], idx [3][Fm] int32, optional rgb [3][Vm]).
    Returns (faces, logits [3][V])."""
    import torch
    M = _mesh_struct(mesh)
    ctx = _ctx(mesh["pos"])
    ctx.bind_stream()
    nv, nf = C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.msp_prior_size(M.n_faces, n, C.byref(nv), C.byref(nf)), "msp_prior_size")
    dev = mesh["pos"].device
    out = dict(pos=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               opacity=torch.empty((nv.value,), dtype=torch.float32, device=dev),
               rgb=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               idx=torch.empty((3, nf.value), dtype=torch.int32, device=dev),
               gid=torch.empty((nf.value,), dtype=torch.int32, device=dev), sh=None)
    logits = torch.empty((3, nv.value), dtype=torch.float32, device=dev)
    c0 = (C.c_float * 3)(*[float(x) for x in rgb0])
    Fc = _faces_struct(out)
    ctx.check(ctx.lib.msp_prior_init(ctx.h, C.byref(M), n, float(shrink), float(opacity0), c0, _dev_ptr(logits),
                                     C.byref(Fc)), "msp_prior_init")
    return out, logits


def prior_vertices(mesh: dict, n: int, logits, out=None):
    """msp_prior_vertices: secondary vertex positions [3][V] from the logits."""
    import torch
    M = _mesh_struct(mesh)
    logits = _need(logits, torch.float32, "logits")
    if tuple(logits.shape) != (3, 3 * n * n * M.n_faces):
        raise ValueError(f"logits must be [3][3 n^2 n_mesh_faces] = [3][{3 * n * n * M.n_faces}]")
    if out is None:
        out = torch.empty_like(logits)
    _need(out, torch.float32, "pos")
    if out.shape != logits.shape:
        raise ValueError("pos must have the logits' shape [3][V]")
    ctx = _ctx(logits)
    ctx.bind_stream()
    ctx.check(ctx.lib.msp_prior_vertices(ctx.h, C.byref(M), n, _dev_ptr(logits), _dev_ptr(out)), "msp_prior_vertices")
    return out


def prior_backward(mesh: dict, n: int, logits, dpos, out=None):
    """msp_prior_backward: dL/dlogits [3][V] from dL/dpos [3][V]."""
    import torch
    M = _mesh_struct(mesh)
    logits = _need(logits, torch.float32, "logits")
    if tuple(logits.shape) != (3, 3 * n * n * M.n_faces):
        raise ValueError(f"logits must be [3][3 n^2 n_mesh_faces] = [3][{3 * n * n * M.n_faces}]")
    dpos = _need(dpos, torch.float32, "dpos")
    if dpos.shape != logits.shape:
        raise ValueError("dpos must have the logits' shape [3][V]")
    if out is None:
        out = torch.empty_like(logits)
    _need(out, torch.float32, "dlogits")
    if out.shape != logits.shape:
        raise ValueError("dlogits must have the logits' shape [3][V]")
    ctx = _ctx(logits)
    ctx.bind_stream()
    ctx.check(ctx.lib.msp_prior_backward(ctx.h, C.byref(M), n, _dev_ptr(logits), _dev_ptr(dpos), _dev_ptr(out)),
              "msp_prior_backward")
    return out


class Bvh:
    """msp_bvh_build and the ray queries (secondary rays through the soup).

    The hierarchy holds a copy of the faces' corners and opacities taken when
    it is built; rebuild it after the faces change."""

    def __init__(self, faces: dict):
        import torch
        pos = _need(faces["pos"], torch.float32, "pos")
        _need(faces["opacity"], torch.float32, "opacity")
        _need(faces["idx"], torch.int32, "idx")
        self.ctx = _ctx(pos)
        self.ctx.bind_stream()
        self.n_leaves = int(faces["idx"].shape[1])
        self.device = pos.device
        F = _faces_struct(faces)
        h = C.c_void_p()
        self.ctx.check(self.ctx.lib.msp_bvh_build(self.ctx.h, C.byref(F), C.byref(h)), "msp_bvh_build")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                self.ctx.lib.msp_bvh_free(self.ctx.h, h)
            except Exception:
                pass
            self.h = None

    @staticmethod
    def _rays(origin, direction, tmin, tmax, order=None):
        import torch
        o = _need(origin, torch.float32, "origin")
        d = _need(direction, torch.float32, "dir")
        n = o.shape[1]
        if o.dim() != 2 or o.shape[0] != 3 or tuple(d.shape) != (3, n):
            raise ValueError("origin and dir must be [3][n]")
        t0 = _need(tmin, torch.float32, "tmin")
        t1 = _need(tmax, torch.float32, "tmax")
        if t0.numel() != n or t1.numel() != n:
            raise ValueError("tmin and tmax must have n entries")
        if order is not None:
            _need(order, torch.int32, "order")
            if order.numel() != n:
                raise ValueError("order must have n entries")
        return _lib.Rays(n, _dev_ptr(o), _dev_ptr(d), _dev_ptr(t0), _dev_ptr(t1), _dev_ptr(order)), n

    def transmittance(self, origin, direction, tmin, tmax, t_eps: float = 0.0, order=None):
        """msp_trace_transmittance: T [n]. `order` (int32 [n], e.g. point_order(origin)) is the
        order in which the rays are traced; results stay at each ray's index."""
        import torch
        R, n = self._rays(origin, direction, tmin, tmax, order)
        T = torch.empty((n,), dtype=torch.float32, device=self.device)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_trace_transmittance(self.ctx.h, self.h, C.byref(R), float(t_eps),
                                                            _dev_ptr(T)), "msp_trace_transmittance")
        return T

    def closest(self, origin, direction, tmin, tmax, alpha_min: float = 0.0, order=None):
        """msp_trace_closest: (t, face, u, v), each [n]; `order` as for transmittance."""
        import torch
        R, n = self._rays(origin, direction, tmin, tmax, order)
        e = lambda dt: torch.empty((n,), dtype=dt, device=self.device)
        t, f, u, v = e(torch.float32), e(torch.int32), e(torch.float32), e(torch.float32)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_trace_closest(self.ctx.h, self.h, C.byref(R), float(alpha_min), _dev_ptr(t),
                                                      _dev_ptr(f), _dev_ptr(u), _dev_ptr(v)), "msp_trace_closest")
        return t, f, u, v

    def export(self):
        """(nodes [n-1][16], leaves [n][16], root_box [6]) as float32 GPU tensors."""
        import torch
        n = self.n_leaves
        nodes = torch.empty((max(n - 1, 0), 16), dtype=torch.float32, device=self.device)
        leaves = torch.empty((n, 16), dtype=torch.float32, device=self.device)
        box = torch.empty((6,), dtype=torch.float32, device=self.device)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_bvh_export(self.ctx.h, self.h, _dev_ptr(nodes) if n > 1 else None,
                                                   _dev_ptr(leaves) if n > 0 else None, _dev_ptr(box)),
                       "msp_bvh_export")
        return nodes, leaves, box

    def status(self) -> dict:
        nl, ov, nn, nt = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
        self.ctx.check(self.ctx.lib.msp_bvh_status(self.ctx.h, self.h, C.byref(nl), C.byref(ov), C.byref(nn),
                                                   C.byref(nt)), "msp_bvh_status")
        return dict(n_leaves=nl.value, overflowed=bool(ov.value), node_visits=nn.value, leaf_tests=nt.value)


def _gauss_struct(g: dict) -> _lib.Gaussians:
    import torch
    mean = _need(g["mean"], torch.float32, "mean")
    sh = g.get("sh")
    return _lib.Gaussians(mean.shape[1], _dev_ptr(mean), _dev_ptr(_need(g["scale"], torch.float32, "scale")),
                          _dev_ptr(_need(g["quat"], torch.float32, "quat")),
                          _dev_ptr(_need(g["opacity"], torch.float32, "opacity")),
                          _dev_ptr(_need(g["rgb"], torch.float32, "rgb")),
                          None if sh is None else _dev_ptr(_need(sh, torch.float32, "sh")))


class Refiner:
    """The BF16-MFMA refiner MLP (msp_refiner_*): 15 -> 256 -> 256 -> n_out."""

    def __init__(self, n_out: int, device: int = 0):
        self.ctx = _lib.Context.get(device)
        h = C.c_void_p()
        self.ctx.check(self.ctx.lib.msp_refiner_create(self.ctx.h, int(n_out), C.byref(h)), "msp_refiner_create")
        self.h = h
        self.n_out = n_out

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.msp_refiner_free(self.ctx.h, self.h)
                self.h = None
        except Exception:
            pass

    def set_weights(self, p: dict):
        import torch
        args = [_dev_ptr(_need(p[k], torch.float32, k)) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_refiner_set_weights(self.ctx.h, self.h, *args), "msp_refiner_set_weights")

    def forward(self, x):
        import torch
        _need(x, torch.float32, "x")
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_refiner_forward(self.ctx.h, self.h, _dev_ptr(x), x.shape[0], _dev_ptr(y)),
                       "msp_refiner_forward")
        return y

    def backward(self, x, dy, want_dx: bool = False) -> dict:
        """Weight and bias gradients of sum(y * dy); with want_dx also "x", the
        input gradient [n][16] (column 15 zero)."""
        import torch
        _need(x, torch.float32, "x")
        _need(dy, torch.float32, "dy")
        dev = x.device
        g = dict(W1=torch.empty((256, 15), device=dev), b1=torch.empty(256, device=dev),
                 W2=torch.empty((256, 256), device=dev), b2=torch.empty(256, device=dev),
                 W3=torch.empty((self.n_out, 256), device=dev), b3=torch.empty(self.n_out, device=dev))
        if want_dx:
            g["x"] = torch.empty((x.shape[0], 16), device=dev)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.msp_refiner_backward(self.ctx.h, self.h, _dev_ptr(x), _dev_ptr(dy), x.shape[0],
                                                         *[_dev_ptr(g[k]) for k in ("W1", "b1", "W2", "b2", "W3",
                                                                                    "b3")],
                                                         _dev_ptr(g["x"]) if want_dx else None),
                       "msp_refiner_backward")
        return g


def refiner_targets(g: dict, K: int, sigma: float, tuned: dict, opac_mul: float = 0.2):
    """Least-squares refiner targets from a fine-tuned copy of the plain fan (msp_refiner_targets)."""
    import torch
    G = _gauss_struct(g)
    G.sh = None
    ctx = _ctx(g["mean"])
    ctx.bind_stream()
    y = torch.empty((G.n, 3 * K + 4), dtype=torch.float32, device=g["mean"].device)
    Fc = _faces_struct(tuned)
    ctx.check(ctx.lib.msp_refiner_targets(ctx.h, C.byref(G), int(K), float(sigma), float(opac_mul), C.byref(Fc),
                                          _dev_ptr(y)), "msp_refiner_targets")
    return y


def refiner_apply_backward(g: dict, K: int, sigma: float, y, grads: dict, opac_mul: float = 0.2):
    """dL/dy [N, 3K+4] from the gradients of the refined fan (msp_refiner_apply_backward)."""
    import torch
    G = _gauss_struct(g)
    G.sh = None
    ctx = _ctx(g["mean"])
    ctx.bind_stream()
    _need(y, torch.float32, "y")
    dy = torch.empty_like(y)
    gr = _lib.FaceGrads(_dev_ptr(grads.get("dpos")), _dev_ptr(grads.get("dopacity")), _dev_ptr(grads.get("drgb")),
                        None)
    ctx.check(ctx.lib.msp_refiner_apply_backward(ctx.h, C.byref(G), int(K), float(sigma), float(opac_mul),
                                                 _dev_ptr(y), C.byref(gr), _dev_ptr(dy)), "msp_refiner_apply_backward")
    return dy


def refiner_weights(g: dict, K: int, sigma: float, ref_len: float = 0.1):
    """Per-output loss weights [N, 3K+4] (msp_refiner_weights)."""
    import torch
    G = _gauss_struct(g)
    ctx = _ctx(g["mean"])
    ctx.bind_stream()
    w = torch.empty((G.n, 3 * K + 4), dtype=torch.float32, device=g["mean"].device)
    ctx.check(ctx.lib.msp_refiner_weights(ctx.h, C.byref(G), int(K), float(sigma), float(ref_len), _dev_ptr(w)),
              "msp_refiner_weights")
    return w


def refiner_loss(refiner: "Refiner", y, target, weight=None, want_grad=True):
    """(Weighted) mean squared error and its gradient (msp_refiner_loss)."""
    import torch
    _need(y, torch.float32, "y")
    _need(target, torch.float32, "target")
    if weight is not None:
        _need(weight, torch.float32, "weight")
    out = torch.empty((1,), dtype=torch.float32, device=y.device)
    dy = torch.empty_like(y) if want_grad else None
    refiner.ctx.bind_stream()
    refiner.ctx.check(refiner.ctx.lib.msp_refiner_loss(refiner.ctx.h, refiner.h, _dev_ptr(y), _dev_ptr(target),
                                                       _dev_ptr(weight), y.shape[0], _dev_ptr(out), _dev_ptr(dy)),
                      "msp_refiner_loss")
    return out, dy


def refiner_features(g: dict, K: int):
    import torch
    G = _gauss_struct(g)
    ctx = _ctx(g["mean"])
    ctx.bind_stream()
    x = torch.empty((G.n, 16), dtype=torch.float32, device=g["mean"].device)
    ctx.check(ctx.lib.msp_refiner_features(ctx.h, C.byref(G), int(K), _dev_ptr(x)), "msp_refiner_features")
    return x


def refiner_apply(g: dict, K: int, sigma: float, y, opac_mul: float = 0.2) -> dict:
    """Fan conversion with refiner outputs y [N, 3K+4] applied (msp_refiner_apply)."""
    import torch
    G = _gauss_struct(g)
    ctx = _ctx(g["mean"])
    ctx.bind_stream()
    _need(y, torch.float32, "y")
    nv, nf = C.c_int64(), C.c_int64()
    ctx.check(ctx.lib.msp_convert_size(G.n, K, 0, C.byref(nv), C.byref(nf)), "msp_convert_size")
    dev = g["mean"].device
    out = dict(pos=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               opacity=torch.empty((nv.value,), dtype=torch.float32, device=dev),
               rgb=torch.empty((3, nv.value), dtype=torch.float32, device=dev),
               idx=torch.empty((3, nf.value), dtype=torch.int32, device=dev),
               gid=torch.empty((nf.value,), dtype=torch.int32, device=dev), sh=None)
    G.sh = None
    Fc = _faces_struct(out)
    ctx.check(ctx.lib.msp_refiner_apply(ctx.h, C.byref(G), int(K), float(sigma), float(opac_mul), _dev_ptr(y),
                                        C.byref(Fc)), "msp_refiner_apply")
    return out


def _autograd():
    import torch

    class _MeshRender(torch.autograd.Function):
        """Differentiable render of a triangle soup: forward msp_render, backward
        msp_render_backward (fragment lists recomputed, not stored)."""

        @staticmethod
        def forward(ctx, pos, opacity, rgb, idx, cams, opts):
            faces = dict(pos=pos.contiguous(), opacity=opacity.contiguous(), rgb=rgb.contiguous(), idx=idx)
            img, state = render(faces, cams, opts)
            ctx.faces = faces
            ctx.state = state
            return img

        @staticmethod
        def backward(ctx, gimg):
            g = render_backward(ctx.state, ctx.faces, gimg.contiguous())
            return g["dpos"], g["dopacity"], g["drgb"], None, None, None

    return _MeshRender


class _LazyFunction:
    _fn = None

    def apply(self, *args):
        if _LazyFunction._fn is None:
            _LazyFunction._fn = _autograd()
        return _LazyFunction._fn.apply(*args)


MeshRender = _LazyFunction()
