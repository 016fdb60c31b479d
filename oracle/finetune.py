"""Fine-tuning pieces, float64 (oracle; test infrastructure only).

Fine-tuning section of the paper: a loss mixing L1 and SSIM with lambda = 0.6
(Eq. loss), colours and opacities updated with lr_color and positions with
lr_verts = exp(-3) lr_color, and every 10 epochs the faces whose three vertex
opacities are all below exp(-4) removed together with vertices no face uses.

Readings:
  * the loss is 0.6 L1 + 0.4 (1 - SSIM) (minimising SSIM itself would be
    wrong); SSIM is that of Wang et al. (2004): 11x11 Gaussian window with
    sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, data range 1, valid windows only,
    averaged over windows and the three colour channels of every view;
  * MSE and L1 are means over views x 3 channels x pixels;
  * the optimiser is Adam (Kingma & Ba 2015) with bias correction; opacity is
    projected to [0, 1] after each step;
  * pruning keeps a face iff some vertex opacity is >= the threshold, keeps a
    vertex iff a kept face uses it, and compacts both stably (ids in order),
    remapping face indices and per-vertex optimiser state.

Also here: the multi-ring conversion used to make fine-tuning targets (a
denser, smoother stand-in for a Gaussian than the paper's fan), see ring_convert.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import correlate2d

from . import convert as oc

SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def gaussian_window(size=11, sigma=1.5):
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x ** 2 / (2 * sigma ** 2))
    g /= g.sum()
    return np.outer(g, g)


def mse(img, tgt):
    """img, tgt [V][3][H][W] -> (loss, dL/dimg)."""
    d = np.asarray(img, np.float64) - np.asarray(tgt, np.float64)
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


def l1(img, tgt):
    d = np.asarray(img, np.float64) - np.asarray(tgt, np.float64)
    n = d.size
    return float(np.sum(np.abs(d)) / n), np.sign(d) / n


def _ssim_plane(x, y, w):
    mx = correlate2d(x, w, mode="valid")
    my = correlate2d(y, w, mode="valid")
    sxx = correlate2d(x * x, w, mode="valid") - mx * mx
    syy = correlate2d(y * y, w, mode="valid") - my * my
    sxy = correlate2d(x * y, w, mode="valid") - mx * my
    A1 = 2 * mx * my + SSIM_C1
    A2 = 2 * sxy + SSIM_C2
    B1 = mx * mx + my * my + SSIM_C1
    B2 = sxx + syy + SSIM_C2
    S = A1 * A2 / (B1 * B2)
    return S, (mx, my, A1, A2, B1, B2)


def ssim(img, tgt, with_grad=True):
    """Mean SSIM over all valid windows, channels and views, and d mean / d img."""
    X = np.asarray(img, np.float64)
    Y = np.asarray(tgt, np.float64)
    w = gaussian_window()
    V, C, H, W = X.shape
    total = 0.0
    count = 0
    grad = np.zeros_like(X)
    for v in range(V):
        for c in range(C):
            S, (mx, my, A1, A2, B1, B2) = _ssim_plane(X[v, c], Y[v, c], w)
            total += S.sum()
            count += S.size
            if with_grad:
                # dS/d mu_x, dS/d E[x^2], dS/d E[xy] per window, then the adjoint of the window sums
                dS_dA1, dS_dA2 = A2 / (B1 * B2), A1 / (B1 * B2)
                dS_dB1 = -A1 * A2 / (B1 * B1 * B2)
                dS_dB2 = -A1 * A2 / (B1 * B2 * B2)
                # A1 = 2 mx my + C1; A2 = 2 (Exy - mx my) + C2; B1 = mx^2 + my^2 + C1; B2 = Exx - mx^2 + Eyy - my^2 + C2
                g_mx = dS_dA1 * 2 * my + dS_dA2 * (-2 * my) + dS_dB1 * 2 * mx + dS_dB2 * (-2 * mx)
                g_exx = dS_dB2
                g_exy = dS_dA2 * 2
                full = lambda m: correlate2d(m, w[::-1, ::-1], mode="full")
                grad[v, c] = full(g_mx) + 2 * X[v, c] * full(g_exx) + Y[v, c] * full(g_exy)
    grad /= count
    return total / count, grad


def paper_loss(img, tgt, lam=0.6):
    """lam L1 + (1 - lam) (1 - SSIM) and its gradient."""
    a, ga = l1(img, tgt)
    s, gs = ssim(img, tgt)
    return lam * a + (1 - lam) * (1 - s), lam * ga - (1 - lam) * gs


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=None, hi=None):
    """One Adam update (step counts from 1); returns new (param, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    p = param - lr * mh / (np.sqrt(vh) + eps)
    if lo is not None:
        p = np.clip(p, lo, hi)
    return p, m, v


def lr_groups(lr_color):
    """Per-group learning rates: colours and opacities lr_color, positions exp(-3) lr_color."""
    return dict(rgb=lr_color, opacity=lr_color, pos=math.exp(-3.0) * lr_color)


def prune(faces, thresh=math.exp(-4.0), vertex_state=()):
    """Removes faces whose three vertex opacities are all < thresh, then unused vertices.

    Returns (new faces dict, list of compacted vertex-state arrays [..][V']).
    """
    I = np.asarray(faces["idx"], np.int64)
    op = np.asarray(faces["opacity"])
    keep_f = np.any(op[I] >= thresh, axis=0)
    used = np.zeros(op.shape[0], dtype=bool)
    used[I[:, keep_f].ravel()] = True
    new_id = np.full(op.shape[0], -1, dtype=np.int64)
    kept_v = np.flatnonzero(used)
    new_id[kept_v] = np.arange(kept_v.size)
    kept_f = np.flatnonzero(keep_f)
    out = dict(faces)
    out["pos"] = np.asarray(faces["pos"])[:, kept_v]
    out["opacity"] = op[kept_v]
    if faces.get("rgb") is not None:
        out["rgb"] = np.asarray(faces["rgb"])[:, kept_v]
    out["idx"] = new_id[I[:, kept_f]].astype(np.int32)
    if faces.get("gid") is not None:
        out["gid"] = np.asarray(faces["gid"])[kept_f]
    if faces.get("sh") is not None:
        out["sh"] = np.asarray(faces["sh"])[:, kept_f]
    states = [np.asarray(s)[..., kept_v] for s in vertex_state]
    return out, states


def ring_convert(mean, scale, quat, opacity, rgb, K, rings, sigma_max=3.0):
    """Multi-ring fan used to render fine-tuning targets.

    Per Gaussian: a centre vertex and `rings` concentric rings of K vertices at
    radii r_j = sigma_max j / rings (j = 1..rings, in units of the scales) on
    the plane of the two largest axes (same axes and angles as the fan); vertex
    opacity is opacity * exp(-r^2 / 2) (the Gaussian's own fall-off, linearly
    interpolated across each triangle); faces: the centre fan to ring 1, then
    two triangles per quad between consecutive rings.
    Layout per Gaussian: centre, then ring 1 vertices k = 0..K-1, ring 2, ...
    Faces: K centre faces (c, r1_k, r1_{k+1}), then for j = 1..rings-1 and each
    k: (rj_k, r(j+1)_k, r(j+1)_{k+1}) and (rj_k, r(j+1)_{k+1}, rj_{k+1}).
    """
    m = np.asarray(mean, np.float64).T
    s = np.asarray(scale, np.float64).T
    q = np.asarray(quat, np.float64).T
    o = np.asarray(opacity, np.float64)
    c = np.asarray(rgb, np.float64).T
    n = m.shape[0]
    R = oc.quat_to_rot(q)
    a, b = oc.top2_axes(s)
    gi = np.arange(n)
    A = s[gi, a][:, None] * R[gi, :, a]
    B = s[gi, b][:, None] * R[gi, :, b]
    th = oc.fan_angles(K)
    per = 1 + rings * K
    pos = np.empty((n, per, 3))
    op = np.empty((n, per))
    pos[:, 0] = m
    op[:, 0] = o
    for j in range(1, rings + 1):
        r = sigma_max * j / rings
        for k in range(K):
            pos[:, 1 + (j - 1) * K + k] = m + r * (np.cos(th[k]) * A + np.sin(th[k]) * B)
            op[:, 1 + (j - 1) * K + k] = o * math.exp(-r * r / 2)
    col = np.repeat(c[:, None, :], per, axis=1)
    faces = []
    for k in range(K):
        faces.append((0, 1 + k, 1 + (k + 1) % K))
    for j in range(1, rings):
        for k in range(K):
            a0 = 1 + (j - 1) * K + k
            a1 = 1 + (j - 1) * K + (k + 1) % K
            b0 = 1 + j * K + k
            b1 = 1 + j * K + (k + 1) % K
            faces.append((a0, b0, b1))
            faces.append((a0, b1, a1))
    fl = np.asarray(faces, np.int64)
    idx = (gi[:, None, None] * per + fl[None]).reshape(-1, 3)
    return dict(pos=pos.reshape(-1, 3).T.copy(), opacity=op.reshape(-1), rgb=col.reshape(-1, 3).T.copy(),
                idx=idx.T.astype(np.int32).copy(), gid=np.repeat(gi, len(faces)).astype(np.int32))
