"""Pins of the oracle's fine-tuning pieces: losses (closed forms, SSIM
identities, finite differences), Adam against torch.optim.Adam, pruning on a
hand-built case, and the multi-ring target conversion against closed forms."""
import math

import numpy as np
import pytest
from scipy.ndimage import uniform_filter  # noqa: F401  (scipy present)
from scipy.spatial.transform import Rotation

from oracle import finetune as ft
from paper_2502_07754_amd import scenes


def _imgs(seed, V=2, H=20, W=23):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (V, 3, H, W)), rng.uniform(0, 1, (V, 3, H, W))


def test_mse_l1_closed_form_and_grad():
    x, y = _imgs(1)
    m, gm = ft.mse(x, y)
    assert m == pytest.approx(np.mean((x - y) ** 2), rel=1e-14)
    a, ga = ft.l1(x, y)
    assert a == pytest.approx(np.mean(np.abs(x - y)), rel=1e-14)
    i = (1, 2, 5, 7)
    h = 1e-6
    xp = x.copy(); xp[i] += h
    xm = x.copy(); xm[i] -= h
    assert gm[i] == pytest.approx((ft.mse(xp, y)[0] - ft.mse(xm, y)[0]) / (2 * h), rel=1e-6)
    assert ga[i] == pytest.approx((ft.l1(xp, y)[0] - ft.l1(xm, y)[0]) / (2 * h), rel=1e-6)


def test_ssim_identities():
    x, _ = _imgs(2)
    assert ft.ssim(x, x, with_grad=False)[0] == pytest.approx(1.0, abs=1e-14)
    # constant images: only the luminance term remains
    a, b = 0.3, 0.7
    X = np.full((1, 3, 15, 15), a)
    Y = np.full((1, 3, 15, 15), b)
    assert ft.ssim(X, Y, with_grad=False)[0] == pytest.approx((2 * a * b + ft.SSIM_C1) / (a * a + b * b + ft.SSIM_C1))
    # a constant shift leaves contrast-structure at 1: mean of the luminance term
    c = 0.1
    Y = x + c
    w = ft.gaussian_window()
    from scipy.signal import correlate2d
    want = []
    for v in range(x.shape[0]):
        for ch in range(3):
            mx = correlate2d(x[v, ch], w, mode="valid")
            my = mx + c
            want.append(((2 * mx * my + ft.SSIM_C1) / (mx * mx + my * my + ft.SSIM_C1)).ravel())
    assert ft.ssim(x, Y, with_grad=False)[0] == pytest.approx(np.mean(np.concatenate(want)), rel=1e-12)
    # window: normalised separable Gaussian with sigma 1.5
    g1 = np.exp(-np.arange(-5, 6) ** 2 / 4.5)
    np.testing.assert_allclose(w, np.outer(g1, g1) / g1.sum() ** 2, rtol=1e-14)


def test_ssim_gradient_by_finite_differences():
    x, y = _imgs(3, V=1, H=16, W=14)
    s, g = ft.ssim(x, y)
    h = 1e-4
    gmax = np.abs(g).max()
    for i in [(0, 0, 0, 0), (0, 1, 7, 6), (0, 2, 15, 13), (0, 0, 5, 10)]:
        xp = x.copy(); xp[i] += h
        xm = x.copy(); xm[i] -= h
        fd = (ft.ssim(xp, y, False)[0] - ft.ssim(xm, y, False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-4, abs=1e-6 * gmax)
    # directional derivative along a random direction
    d = np.random.default_rng(9).standard_normal(x.shape)
    fd = (ft.ssim(x + h * d, y, False)[0] - ft.ssim(x - h * d, y, False)[0]) / (2 * h)
    assert np.sum(g * d) == pytest.approx(fd, rel=1e-6)
    L, gL = ft.paper_loss(x, y)
    assert L == pytest.approx(0.6 * np.mean(np.abs(x - y)) + 0.4 * (1 - s), rel=1e-14)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads):
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = ft.adam_step(p, g, m, v, k + 1, 0.01)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-13, atol=1e-15)
    # step 1 closed form: -lr g / (|g| + eps)
    p1, _, _ = ft.adam_step(p0, grads[0], np.zeros(50), np.zeros(50), 1, 0.01)
    np.testing.assert_allclose(p1 - p0, -0.01 * grads[0] / (np.abs(grads[0]) + 1e-8), rtol=1e-12)
    # projection
    p2, _, _ = ft.adam_step(np.array([0.0, 1.0]), np.array([1.0, -1.0]), np.zeros(2), np.zeros(2), 1, 0.5, lo=0.0, hi=1.0)
    assert np.all(p2 == [0.0, 1.0])
    assert ft.lr_groups(0.01)["pos"] == pytest.approx(0.01 * math.exp(-3))


def test_prune_hand_case():
    t = math.exp(-4)
    # 6 vertices, 4 faces:
    # f0 (0,1,2): v0 above threshold -> kept
    # f1 (1,2,3): all below -> dropped (v1, v2 stay through f0; v3 only here -> removed)
    # f2 (4,5,2): v4 exactly at threshold -> kept ("below" is strict)
    # f3 (3,3,3): all below -> dropped
    op = np.array([0.5, t / 2, t / 3, t / 4, t, 0.0])
    faces = dict(pos=np.arange(18.0).reshape(3, 6), opacity=op, rgb=np.ones((3, 6)),
                 idx=np.array([[0, 1, 4, 3], [1, 2, 5, 3], [2, 3, 2, 3]], np.int32), gid=np.array([0, 0, 1, 1]))
    mom = np.arange(6.0)[None].repeat(2, 0)
    out, (m2,) = ft.prune(faces, t, [mom])
    assert out["idx"].T.tolist() == [[0, 1, 2], [3, 4, 2]]
    assert out["gid"].tolist() == [0, 1]
    np.testing.assert_array_equal(out["opacity"], op[[0, 1, 2, 4, 5]])
    np.testing.assert_array_equal(out["pos"], faces["pos"][:, [0, 1, 2, 4, 5]])
    np.testing.assert_array_equal(m2, mom[:, [0, 1, 2, 4, 5]])


@pytest.mark.parametrize("K,rings", [(8, 3), (16, 4)])
def test_ring_convert(K, rings):
    g = scenes.gaussians(30, 5, 0.01, 0.1, flat=True)
    out = ft.ring_convert(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, rings)
    per = 1 + rings * K
    nf = K * (2 * rings - 1)
    assert out["pos"].shape == (3, 30 * per) and out["idx"].shape == (3, 30 * nf)
    R = Rotation.from_quat(np.asarray(g.quat, np.float64).T[:, [1, 2, 3, 0]]).as_matrix()
    s = np.asarray(g.scale, np.float64).T
    m = np.asarray(g.mean, np.float64).T
    P = out["pos"].T.reshape(30, per, 3)
    op = out["opacity"].reshape(30, per)
    for n in range(30):
        for j in range(1, rings + 1):
            r = 3.0 * j / rings
            dv = P[n, 1 + (j - 1) * K: 1 + j * K] - m[n]
            e = (dv @ R[n][:, 0] / (r * s[n, 0])) ** 2 + (dv @ R[n][:, 1] / (r * s[n, 1])) ** 2
            np.testing.assert_allclose(e, 1.0, atol=1e-12)
            np.testing.assert_allclose(op[n, 1 + (j - 1) * K: 1 + j * K], g.opacity[n] * math.exp(-r * r / 2),
                                       rtol=1e-7)
        I = out["idx"].T[n * nf:(n + 1) * nf].astype(np.int64)
        Pg = out["pos"].T
        area = 0.5 * np.linalg.norm(np.cross(Pg[I[:, 1]] - Pg[I[:, 0]], Pg[I[:, 2]] - Pg[I[:, 0]]), axis=1).sum()
        np.testing.assert_allclose(area, 0.5 * K * math.sin(2 * math.pi / K) * 9.0 * s[n, 0] * s[n, 1], rtol=1e-12)
