"""Refiner MLP with bfloat16 rounding points, float64 (oracle; test infrastructure only).

Not in the paper (which converts and fine-tunes only). A small network maps
each Gaussian to corrections of its fan so that fine-tuning starts closer to
its optimum; plain conversion stays the fallback (an untrained refiner with a
zero last layer reproduces it exactly).

  x  = (m (3), s / 0.1 (3), q normalised with w >= 0 (4), opacity (1), rgb (3), K / 16 (1))
  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,  widths 15 -> 256 -> 256 -> 3K + 4
  y  = (3K boundary offsets in the fan's local frame, opacity delta, rgb delta (3))

Rounding points (the GPU multiplies bfloat16 operands with float32
accumulation): x, W1, W2, W3, h1, h2 are rounded to bfloat16 before each
product; in the backward pass dy, dh2 and dh1 are. Biases, activations and
sums stay float64 here (float32 on the GPU). bfloat16 rounding is float32 ->
bfloat16 round-to-nearest-even on the bit pattern.

Applying y (refined_fan): boundary vertex k moves by
d_k0 a A^ + d_k1 b B^ + d_k2 sqrt(a b) n^ from its plain position, with a, b
the fan's semi-axes (sigma s_a, sigma s_b), A^, B^ their unit directions and
n^ = A^ x B^; the opacity becomes clamp(o + y_op, 0, 1) (boundary opac_mul of
that); colours rgb + y_rgb. The centre stays at the mean.
"""
from __future__ import annotations

import math

import numpy as np

from . import convert as oc

HIDDEN = 256
N_IN = 15


def bf16_round(x):
    """float64/float32 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    r = np.where(nan, (u | 0x00400000) & 0xFFFF0000, r)      # quiet NaN, sign kept
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(mean, scale, quat, opacity, rgb, K):
    """x [N][15] float64 from the scene layout."""
    m = np.asarray(mean, np.float64).T
    s = np.asarray(scale, np.float64).T / 0.1
    q = np.asarray(quat, np.float64).T
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    q = np.where(q[:, :1] < 0, -q, q)
    o = np.asarray(opacity, np.float64)[:, None]
    c = np.asarray(rgb, np.float64).T
    k = np.full((m.shape[0], 1), K / 16.0)
    return np.concatenate([m, s, q, o, c, k], axis=1)


def init_params(n_out, seed=0, zero_last=True):
    """He-initialised weights (float32 values), zero biases; W3 = 0 makes the refiner the identity."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2 / N_IN), (HIDDEN, N_IN)).astype(np.float32)
    W2 = rng.normal(0, math.sqrt(2 / HIDDEN), (HIDDEN, HIDDEN)).astype(np.float32)
    W3 = (np.zeros((n_out, HIDDEN)) if zero_last else rng.normal(0, math.sqrt(1 / HIDDEN), (n_out, HIDDEN)))
    return dict(W1=W1, b1=np.zeros(HIDDEN, np.float32), W2=W2, b2=np.zeros(HIDDEN, np.float32),
                W3=W3.astype(np.float32), b3=np.zeros(n_out, np.float32))


def forward(p, x, rounding=True):
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    h1 = np.maximum(r(x) @ r(p["W1"]).T + p["b1"], 0.0)
    h2 = np.maximum(r(h1) @ r(p["W2"]).T + p["b2"], 0.0)
    y = r(h2) @ r(p["W3"]).T + p["b3"]
    return y, (x, h1, h2)


def preactivations(p, x, rounding=True):
    """The two hidden layers before their ReLU, z1 and z2, as forward computes
    them (h1 = max(z1, 0), h2 = max(z2, 0)). A unit whose z lies within float32
    rounding of 0 may be on the other side of its ReLU in a float32 evaluation."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    z1 = r(x) @ r(p["W1"]).T + p["b1"]
    z2 = r(np.maximum(z1, 0.0)) @ r(p["W2"]).T + p["b2"]
    return z1, z2


def backward(p, cache, dy, rounding=True):
    """Gradients of sum(y * dy) w.r.t. W1, b1, W2, b2, W3, b3 and the input x."""
    r = bf16_round if rounding else (lambda a: np.asarray(a, np.float64))
    x, h1, h2 = cache
    dy = np.asarray(dy, np.float64)
    g = {}
    g["W3"] = r(dy).T @ r(h2)
    g["b3"] = dy.sum(0)
    dh2 = (r(dy) @ r(p["W3"])) * (h2 > 0)
    g["W2"] = r(dh2).T @ r(h1)
    g["b2"] = dh2.sum(0)
    dh1 = (r(dh2) @ r(p["W2"])) * (h1 > 0)
    g["W1"] = r(dh1).T @ r(x)
    g["b1"] = dh1.sum(0)
    g["x"] = r(dh1) @ r(p["W1"])  # input gradient [N][15], dh1 and W1 rounded like the other products
    return g


def refined_fan(mean, scale, quat, opacity, rgb, K, sigma, y, opac_mul=0.2):
    """Fan conversion with the refiner's corrections applied (see module docstring)."""
    base = oc.convert_fan(mean, scale, quat, opacity, rgb, K, sigma, opac_mul)
    s = np.asarray(scale, np.float64).T
    n = s.shape[0]
    R = oc.quat_to_rot(np.asarray(quat, np.float64).T)
    a_i, b_i = oc.top2_axes(s)
    gi = np.arange(n)
    Ah = R[gi, :, a_i]
    Bh = R[gi, :, b_i]
    Nh = np.cross(Ah, Bh)
    a = sigma * s[gi, a_i]
    b = sigma * s[gi, b_i]
    y = np.asarray(y, np.float64)
    pos = base["pos"].T.reshape(n, K + 1, 3).copy()
    for k in range(K):
        d = y[:, 3 * k: 3 * k + 3]
        pos[:, 1 + k] += (d[:, 0] * a)[:, None] * Ah + (d[:, 1] * b)[:, None] * Bh + \
            (d[:, 2] * np.sqrt(a * b))[:, None] * Nh
    o = np.clip(np.asarray(opacity, np.float64) + y[:, 3 * K], 0.0, 1.0)
    op = np.concatenate([o[:, None], np.repeat((opac_mul * o)[:, None], K, 1)], axis=1)
    c = np.asarray(rgb, np.float64).T + y[:, 3 * K + 1: 3 * K + 4]
    col = np.repeat(c[:, None, :], K + 1, axis=1)
    out = dict(base)
    out["pos"] = pos.reshape(-1, 3).T.copy()
    out["opacity"] = op.reshape(-1)
    out["rgb"] = col.reshape(-1, 3).T.copy()
    return out


def fit_targets(mean, scale, quat, opacity, rgb, K, sigma, tuned, opac_mul=0.2):
    """Per-Gaussian least-squares y* such that refined_fan(y*) best matches fine-tuned faces
    `tuned` (same vertex layout as the plain fan: no pruning)."""
    s = np.asarray(scale, np.float64).T
    n = s.shape[0]
    R = oc.quat_to_rot(np.asarray(quat, np.float64).T)
    a_i, b_i = oc.top2_axes(s)
    gi = np.arange(n)
    Ah, Bh = R[gi, :, a_i], R[gi, :, b_i]
    Nh = np.cross(Ah, Bh)
    a = sigma * s[gi, a_i]
    b = sigma * s[gi, b_i]
    base = oc.convert_fan(mean, scale, quat, opacity, rgb, K, sigma, opac_mul)
    P0 = base["pos"].T.reshape(n, K + 1, 3)
    P1 = np.asarray(tuned["pos"], np.float64).T.reshape(n, K + 1, 3)
    y = np.zeros((n, 3 * K + 4))
    for k in range(K):
        d = P1[:, 1 + k] - P0[:, 1 + k]
        y[:, 3 * k] = np.einsum("ij,ij->i", d, Ah) / np.maximum(a, 1e-12)
        y[:, 3 * k + 1] = np.einsum("ij,ij->i", d, Bh) / np.maximum(b, 1e-12)
        y[:, 3 * k + 2] = np.einsum("ij,ij->i", d, Nh) / np.maximum(np.sqrt(a * b), 1e-12)
    o0 = np.asarray(opacity, np.float64)
    ot = np.asarray(tuned["opacity"], np.float64).reshape(n, K + 1)
    # least squares over the centre (weight 1) and the boundary (opac_mul each)
    y[:, 3 * K] = ((ot[:, 0] - o0) + opac_mul * (ot[:, 1:] - opac_mul * o0[:, None]).sum(1)) / (1 + opac_mul ** 2 * K)
    ct = np.asarray(tuned["rgb"], np.float64).T.reshape(n, K + 1, 3)
    y[:, 3 * K + 1: 3 * K + 4] = ct.mean(1) - np.asarray(rgb, np.float64).T
    return y


def loss_weights(scale, K, sigma, ref_len=0.1):
    """Per-output weights [N][3K+4] for training the refiner: offset coordinate
    k along A^, B^, n^ weighs (a^2, b^2, a b) / ref^2 (its squared world-space
    length per unit), the opacity and colour deltas a b / ref^2 (fan area over
    the area of the same K-gon of radius ref)."""
    s = np.asarray(scale, np.float64).T
    n = s.shape[0]
    a_i, b_i = oc.top2_axes(s)
    gi = np.arange(n)
    a = sigma * s[gi, a_i]
    b = sigma * s[gi, b_i]
    w = np.empty((n, 3 * K + 4))
    w[:, 0:3 * K:3] = (a * a / ref_len ** 2)[:, None]
    w[:, 1:3 * K:3] = (b * b / ref_len ** 2)[:, None]
    w[:, 2:3 * K:3] = (a * b / ref_len ** 2)[:, None]
    w[:, 3 * K:] = (a * b / ref_len ** 2)[:, None]
    return w


def weighted_mse(y, t, w=None):
    """sum w (y - t)^2 / numel and its gradient with respect to y."""
    y = np.asarray(y, np.float64)
    d = y - np.asarray(t, np.float64)
    w = np.ones_like(d) if w is None else np.asarray(w, np.float64)
    return float(np.sum(w * d * d) / d.size), 2.0 * w * d / d.size


def refined_fan_backward(mean, scale, quat, opacity, rgb, K, sigma, y, dpos, dop, drgb, opac_mul=0.2):
    """dL/dy for L with gradients dpos [3][V], dop [V], drgb [3][V] at refined_fan(y).
    Boundary offset k: (a A^, b B^, sqrt(ab) n^) . dpos of vertex k; opacity:
    dop(centre) + opac_mul * sum dop(boundary) where 0 < o + y_op < 1; colour:
    sum of the fan's vertex colour gradients."""
    s = np.asarray(scale, np.float64).T
    n = s.shape[0]
    R = oc.quat_to_rot(np.asarray(quat, np.float64).T)
    a_i, b_i = oc.top2_axes(s)
    gi = np.arange(n)
    Ah, Bh = R[gi, :, a_i], R[gi, :, b_i]
    Nh = np.cross(Ah, Bh)
    a = sigma * s[gi, a_i]
    b = sigma * s[gi, b_i]
    y = np.asarray(y, np.float64)
    gp = np.asarray(dpos, np.float64).T.reshape(n, K + 1, 3)
    go = np.asarray(dop, np.float64).reshape(n, K + 1)
    gc = np.asarray(drgb, np.float64).T.reshape(n, K + 1, 3)
    dy = np.zeros((n, 3 * K + 4))
    for k in range(K):
        d = gp[:, 1 + k]
        dy[:, 3 * k] = a * np.einsum("ij,ij->i", d, Ah)
        dy[:, 3 * k + 1] = b * np.einsum("ij,ij->i", d, Bh)
        dy[:, 3 * k + 2] = np.sqrt(a * b) * np.einsum("ij,ij->i", d, Nh)
    u = np.asarray(opacity, np.float64) + y[:, 3 * K]
    dy[:, 3 * K] = np.where((u > 0) & (u < 1), go[:, 0] + opac_mul * go[:, 1:].sum(1), 0.0)
    dy[:, 3 * K + 1:] = gc.sum(1)
    return dy
