"""Face-level fine-tuning loop (fine-tuning section of the paper).

Each step renders every training view, takes the image loss against the
targets (by default the paper's Eq. loss, 0.6 L1 + 0.4 (1 - SSIM); the
progress metric `mse()` stays the image MSE), runs the adjoint, and applies
Adam with the paper's two
learning rates (colours and opacities at lr_color, positions at
exp(-3) lr_color; opacities projected to [0, 1]). Every `prune_every` steps
(one step = one epoch over all views) faces whose vertex opacities are all
below exp(-4) are removed, with the vertices no face uses. All arithmetic runs
in libmsp; this module only sequences the calls and keeps the optimiser state.
"""
from __future__ import annotations

import dataclasses
import math

from . import (MSP_LOSS_L1_DSSIM, MSP_LOSS_MSE, RenderOptions, RenderState, adam_step, loss as msp_loss, prior_backward, prior_init,
               prior_vertices, prune as msp_prune, render, render_backward)
from . import _lib


@dataclasses.dataclass
class FineTuneConfig:
    lr_color: float = 1e-2
    loss_kind: int = MSP_LOSS_L1_DSSIM     # Eq. loss: lam L1 + (1 - lam) (1 - SSIM)
    lam: float = 0.6
    prune_every: int = 10
    prune_thresh: float = math.exp(-4.0)
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


class FineTuner:
    """Adam over per-vertex positions, colours and opacities of a face soup."""

    def __init__(self, faces: dict, cams, targets, cfg: FineTuneConfig | None = None,
                 opts: RenderOptions | None = None, track_mse: bool = False):
        import torch
        self.cfg = cfg or FineTuneConfig()
        # track_mse: also take the image MSE of every step's render (before its
        # update) into `last_mse`, whatever the training loss is
        self.track_mse = track_mse
        self.last_mse = None
        self.opts = opts or RenderOptions()
        self.cams = cams
        self.targets = targets
        self.faces = {k: (None if v is None else v.clone()) for k, v in faces.items()}
        z = torch.zeros_like
        self.m = dict(pos=z(self.faces["pos"]), opacity=z(self.faces["opacity"]), rgb=z(self.faces["rgb"]))
        self.v = dict(pos=z(self.faces["pos"]), opacity=z(self.faces["opacity"]), rgb=z(self.faces["rgb"]))
        self.t = 0
        self.history = []
        # tile lists, fragment lists and scratch are reused from step to step
        self.state = RenderState(_lib.Context.get(self.faces["pos"].device.index or 0))

    def lr(self):
        c = self.cfg.lr_color
        return dict(rgb=c, opacity=c, pos=math.exp(-3.0) * c)

    def step(self):
        """One epoch: render all views, loss, adjoint, Adam, prune on schedule. Returns the loss tensor."""
        img, st = render(self.faces, self.cams, self.opts, state=self.state)
        L, dimg = msp_loss(img, self.targets, self.cfg.loss_kind, self.cfg.lam)
        if self.track_mse:
            self.last_mse = L if self.cfg.loss_kind == MSP_LOSS_MSE else \
                msp_loss(img, self.targets, MSP_LOSS_MSE, want_grad=False)[0]
        g = render_backward(st, self.faces, dimg, need=("dpos", "dopacity", "drgb"))
        self.t += 1
        lr = self.lr()
        groups = [dict(param=self.faces["pos"], grad=g["dpos"], m=self.m["pos"], v=self.v["pos"], lr=lr["pos"]),
                  dict(param=self.faces["rgb"], grad=g["drgb"], m=self.m["rgb"], v=self.v["rgb"], lr=lr["rgb"]),
                  dict(param=self.faces["opacity"], grad=g["dopacity"], m=self.m["opacity"], v=self.v["opacity"],
                       lr=lr["opacity"], clamp=(0.0, 1.0))]
        adam_step(groups, self.t, self.cfg.beta1, self.cfg.beta2, self.cfg.eps)
        if self.cfg.prune_every and self.t % self.cfg.prune_every == 0:
            self.prune()
        self.history.append(L)
        return L

    def prune(self):
        vs = [self.m["pos"], self.v["pos"], self.m["rgb"], self.v["rgb"], self.m["opacity"], self.v["opacity"]]
        self.faces, vs = msp_prune(self.faces, self.cfg.prune_thresh, vs)
        self.m["pos"], self.v["pos"], self.m["rgb"], self.v["rgb"], self.m["opacity"], self.v["opacity"] = vs

    def mse(self) -> float:
        img, _ = render(self.faces, self.cams, self.opts, state=self.state)
        L, _ = msp_loss(img, self.targets, MSP_LOSS_MSE, want_grad=False)
        return float(L.item())

    # ---- checkpoint / resume ----
    def state_dict(self) -> dict:
        d = {f"face_{k}": v.detach().cpu().numpy() for k, v in self.faces.items() if v is not None}
        d.update({f"m_{k}": v.cpu().numpy() for k, v in self.m.items()})
        d.update({f"v_{k}": v.cpu().numpy() for k, v in self.v.items()})
        d["t"] = self.t
        return d

    def save(self, path: str):
        import numpy as np
        np.savez(path, **self.state_dict())

    def load(self, path: str):
        import numpy as np
        import torch
        d = np.load(path)
        dev = self.faces["pos"].device
        self.faces = {k[5:]: torch.from_numpy(d[k]).to(dev) for k in d.files if k.startswith("face_")}
        self.faces.setdefault("sh", None)
        for k in ("pos", "opacity", "rgb"):
            self.m[k] = torch.from_numpy(d[f"m_{k}"]).to(dev)
            self.v[k] = torch.from_numpy(d[f"v_{k}"]).to(dev)
        self.t = int(d["t"])


@dataclasses.dataclass
class PriorTuneConfig:
    lr_color: float = 1e-2
    lr_logits: float = math.exp(-3.0) * 1e-2   # the paper's position rate, exp(-3) lr_color
    loss_kind: int = MSP_LOSS_L1_DSSIM
    lam: float = 0.6
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


class PriorTuner:
    """Mesh-prior fine-tuning (mesh-prior section): secondary triangles on a
    fixed geometry mesh, n^2 per mesh face, whose vertices are softmax-weighted
    convex combinations of the face's corners. Each step sets the vertex
    positions from the logits, renders all views, takes the loss, runs the
    render adjoint, carries the position gradient to the logits, and applies
    Adam to logits (lr_logits, by default the paper's position rate
    exp(-3) lr_color), colours and opacities (lr_color; opacities
    projected to [0, 1]). The number of triangles per mesh face stays fixed,
    so there is no pruning."""

    def __init__(self, mesh: dict, n: int, cams, targets, cfg: PriorTuneConfig | None = None,
                 opts: RenderOptions | None = None, shrink: float = 0.05, opacity0: float = 0.5, init=None):
        import torch
        self.cfg = cfg or PriorTuneConfig()
        self.opts = opts or RenderOptions()
        self.mesh, self.n, self.cams, self.targets = mesh, n, cams, targets
        if init is None:
            self.faces, self.logits = prior_init(mesh, n, shrink, opacity0)
        else:
            self.faces, self.logits = ({k: (None if v is None else v.clone()) for k, v in init[0].items()},
                                       init[1].clone())
        self.dlogits = torch.empty_like(self.logits)
        z = torch.zeros_like
        self.m = dict(logits=z(self.logits), opacity=z(self.faces["opacity"]), rgb=z(self.faces["rgb"]))
        self.v = dict(logits=z(self.logits), opacity=z(self.faces["opacity"]), rgb=z(self.faces["rgb"]))
        self.t = 0
        self.history = []
        self.state = RenderState(_lib.Context.get(self.logits.device.index or 0))

    def step(self):
        """One epoch over all views. Returns the loss tensor."""
        c = self.cfg
        prior_vertices(self.mesh, self.n, self.logits, out=self.faces["pos"])
        img, st = render(self.faces, self.cams, self.opts, state=self.state)
        L, dimg = msp_loss(img, self.targets, c.loss_kind, c.lam)
        g = render_backward(st, self.faces, dimg, need=("dpos", "dopacity", "drgb"))
        prior_backward(self.mesh, self.n, self.logits, g["dpos"], out=self.dlogits)
        self.t += 1
        groups = [dict(param=self.logits, grad=self.dlogits, m=self.m["logits"], v=self.v["logits"], lr=c.lr_logits),
                  dict(param=self.faces["rgb"], grad=g["drgb"], m=self.m["rgb"], v=self.v["rgb"], lr=c.lr_color),
                  dict(param=self.faces["opacity"], grad=g["dopacity"], m=self.m["opacity"], v=self.v["opacity"],
                       lr=c.lr_color, clamp=(0.0, 1.0))]
        adam_step(groups, self.t, c.beta1, c.beta2, c.eps)
        self.history.append(L)
        return L

    def mse(self) -> float:
        prior_vertices(self.mesh, self.n, self.logits, out=self.faces["pos"])
        img, _ = render(self.faces, self.cams, self.opts, state=self.state)
        L, _ = msp_loss(img, self.targets, MSP_LOSS_MSE, want_grad=False)
        return float(L.item())
