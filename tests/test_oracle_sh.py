"""Pins of the oracle's real spherical harmonics and per-view face colour:
scipy's associated Legendre functions, orthonormality by quadrature, the
addition theorem, and finite differences of the colour adjoint."""
import math

import numpy as np
import pytest
from scipy.special import lpmv

from oracle import sh as osh
from paper_2502_07754_amd import scenes


def _scipy_basis(d):
    d = np.asarray(d, np.float64)
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    out = np.empty((len(d), 16))
    for b in range(16):
        l, m = osh.lm_of(b)
        am = abs(m)
        K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
        P = lpmv(am, l, np.cos(th))
        if m == 0:
            out[:, b] = K * P
        elif m > 0:
            out[:, b] = math.sqrt(2) * K * P * np.cos(m * ph)
        else:
            out[:, b] = math.sqrt(2) * K * P * np.sin(am * ph)
    return out


def _dirs(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_basis_matches_scipy_legendre():
    d = _dirs(500, 1)
    np.testing.assert_allclose(osh.basis(d), _scipy_basis(d), atol=1e-13)


def test_orthonormal_by_quadrature():
    zq, wq = np.polynomial.legendre.leggauss(16)
    nphi = 32
    ph = 2 * np.pi * np.arange(nphi) / nphi
    Z, PH = np.meshgrid(zq, ph, indexing="ij")
    S = np.sqrt(1 - Z ** 2)
    d = np.stack([S * np.cos(PH), S * np.sin(PH), Z], -1).reshape(-1, 3)
    w = (wq[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = osh.basis(d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_addition_theorem_and_dc():
    d = _dirs(200, 2)
    Y = osh.basis(d)
    for l in range(4):
        np.testing.assert_allclose((Y[:, l * l:(l + 1) ** 2] ** 2).sum(1), (2 * l + 1) / (4 * np.pi), rtol=1e-13)
    np.testing.assert_allclose(Y[:, 0], 0.5 / math.sqrt(math.pi), rtol=1e-15)


def test_basis_gradient_by_finite_differences():
    d = _dirs(50, 3)
    G = osh.basis_grad(d)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (osh.basis(d + e) - osh.basis(d - e)) / (2 * h)   # polynomial extension off the sphere
        np.testing.assert_allclose(G[:, :, j], fd, atol=1e-8)


def test_face_colour_adjoint_by_finite_differences():
    g = scenes.gaussians(20, 4, 0.05, 0.2, flat=True, sh=True)
    from oracle import convert as oc
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 4, 2.0, sh=g.sh)
    cam = scenes.ring_cameras(3, 32, 32)[1]
    rng = np.random.default_rng(5)
    dcol = rng.standard_normal((3, f["idx"].shape[1]))
    dsh, dpos = osh.face_colours_backward(f["sh"], f["pos"], f["idx"], cam, dcol)

    def L(shv, posv):
        c, _ = osh.face_colours(shv, posv, f["idx"], cam)
        return float(np.sum(c * dcol))

    h = 1e-6
    for r, c in [(0, 3), (5, 10), (47, 79), (20, 40)]:
        sp = f["sh"].copy(); sp[r, c] += h
        sm = f["sh"].copy(); sm[r, c] -= h
        np.testing.assert_allclose(dsh[r, c], (L(sp, f["pos"]) - L(sm, f["pos"])) / (2 * h), rtol=1e-6, atol=1e-9)
    for a, v in [(0, 0), (1, 7), (2, 30), (0, 99)]:
        pp = f["pos"].copy(); pp[a, v] += h
        pm = f["pos"].copy(); pm[a, v] -= h
        np.testing.assert_allclose(dpos[a, v], (L(f["sh"], pp) - L(f["sh"], pm)) / (2 * h), rtol=1e-5, atol=1e-8)


def test_dc_only_colour():
    """Only the l = 0 coefficients set: every view sees 1/2 + k0 / (2 sqrt(pi))."""
    g = scenes.gaussians(5, 6, 0.05, 0.2, flat=True, sh=True)
    sh = np.zeros((48, 5))
    sh[0:3] = [[0.3], [-0.1], [-2.0]]
    from oracle import convert as oc
    f = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0, sh=sh)
    for cam in scenes.ring_cameras(4, 16, 16):
        c, pre = osh.face_colours(f["sh"], f["pos"], f["idx"], cam)
        np.testing.assert_allclose(pre[:, 0], 0.5 + np.array([0.3, -0.1, -2.0]) * 0.5 / math.sqrt(math.pi))
        assert np.all(c[2] == 0.0)
