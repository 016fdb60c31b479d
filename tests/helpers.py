"""Test-side helpers: move seeded inputs to the GPU and compare against the oracle."""
from __future__ import annotations

import numpy as np


def faces_f32(f: dict) -> dict:
    """Rounds an oracle face dict to the float32 values the GPU receives."""
    return {k: (np.ascontiguousarray(v.astype(np.float32)) if v.dtype == np.float64 else v) for k, v in f.items()}


def faces_f64(f: dict) -> dict:
    return {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in f.items()}


def to_gpu(d: dict, device="cuda:0") -> dict:
    import torch
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(device)) for k, v in d.items()}


def gaussians_gpu(g, device="cuda:0") -> dict:
    return to_gpu(dict(mean=g.mean, scale=g.scale, quat=g.quat, opacity=g.opacity, rgb=g.rgb, sh=g.sh), device)


def grad_close(gpu, ref, rel=1e-3, floor=1e-6):
    """|gpu - ref| <= rel |ref| + floor * max |ref| elementwise; returns (ok, worst excess)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = rel * np.abs(ref) + floor * np.max(np.abs(ref))
    ex = np.abs(gpu - ref) - tol
    return bool(np.all(ex <= 0)), float(np.max(ex))
