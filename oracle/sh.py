"""Real spherical harmonics up to degree 3 and view-dependent face colour, float64
(oracle; test infrastructure only).

The paper uses plain RGB per vertex (Gaussian-splatting paragraph: SH can be
replaced by RGB). The batched-render workload of this build colours each face
with degree-3 SH evaluated per view, read as follows:

  basis b = l^2 + l + m for l = 0..3, m = -l..l (16 functions), orthonormal on
  the sphere, with the associated Legendre functions P_l^m including the
  Condon-Shortley phase (-1)^m:
     Y_l0  = K_l0 P_l^0(cos t)
     Y_lm  = sqrt(2) K_lm P_l^m(cos t) cos(m p)        m > 0
     Y_l-m = sqrt(2) K_lm P_l^m(cos t) sin(m p)        m > 0
     K_lm  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
  where t is the polar angle from +z and p the azimuth from +x in the x-y
  plane of the world frame;
  face colour for a view: d = normalize(centroid - camera centre),
  colour_c = max(0, 1/2 + sum_b k[3 b + c] Y_b(d)), with centroid the mean of
  the face's three corners and coefficients laid out [48][F] (row 3 b + c).

The Cartesian form used here, Y_lm = c_lm P_l^(m)(z) Re/Im((x + i y)^m) with
P_l^(m) the m-th derivative of the Legendre polynomial, follows from
(1 - z^2)^(m/2) e^{i m p} = (x + i y)^m on the unit sphere; it is pinned
against scipy's associated Legendre functions.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg

LMAX = 3
NB = (LMAX + 1) ** 2


def lm_of(b):
    l = int(math.isqrt(b))
    return l, b - l * l - l


def k_lm(l, m):
    m = abs(m)
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def _poly(l, m):
    """Coefficients (ascending powers of z) of c_lm * d^m P_l / dz^m, with c_lm including sqrt(2), K_lm and (-1)^m."""
    P = npleg.leg2poly(npleg.Legendre.basis(l).coef)
    D = np.polynomial.polynomial.polyder(P, abs(m)) if abs(m) > 0 else P
    c = k_lm(l, m) * (1.0 if m == 0 else math.sqrt(2.0) * (-1.0) ** abs(m))
    return c * np.atleast_1d(D)


def basis(d):
    """Y_b(d) for unit directions d [n][3] -> [n][16]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    w = x + 1j * y
    out = np.empty((d.shape[0], NB))
    for b in range(NB):
        l, m = lm_of(b)
        p = np.polynomial.polynomial.polyval(z, _poly(l, m))
        if m == 0:
            out[:, b] = p
        elif m > 0:
            out[:, b] = p * np.real(w ** m)
        else:
            out[:, b] = p * np.imag(w ** (-m))
    return out


def basis_grad(d):
    """d Y_b / d(x, y, z) of the polynomial extension, [n][16][3]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    w = x + 1j * y
    out = np.zeros((d.shape[0], NB, 3))
    for b in range(NB):
        l, m = lm_of(b)
        pc = _poly(l, m)
        p = np.polynomial.polynomial.polyval(z, pc)
        dp = np.polynomial.polynomial.polyval(z, np.polynomial.polynomial.polyder(pc)) if len(pc) > 1 else 0.0 * z
        am = abs(m)
        if m == 0:
            out[:, b, 2] = dp
            continue
        q = w ** am
        dq = am * w ** (am - 1)              # d/dx (x+iy)^m ; d/dy = i * dq
        if m > 0:
            out[:, b, 0] = p * np.real(dq)
            out[:, b, 1] = p * np.real(1j * dq)
            out[:, b, 2] = dp * np.real(q)
        else:
            out[:, b, 0] = p * np.imag(dq)
            out[:, b, 1] = p * np.imag(1j * dq)
            out[:, b, 2] = dp * np.imag(q)
    return out


def camera_centre(cam):
    W = np.asarray(cam.world_to_cam, np.float64)
    return -np.linalg.solve(W[:, :3], W[:, 3])


def face_dirs(pos, idx, cam):
    """Unnormalised and unit view directions centroid - centre per face, [F][3] each."""
    P = np.asarray(pos, np.float64).T
    I = np.asarray(idx, np.int64)
    cen = (P[I[0]] + P[I[1]] + P[I[2]]) / 3.0
    v = cen - camera_centre(cam)
    return v, v / np.linalg.norm(v, axis=1, keepdims=True)


def face_colours(sh, pos, idx, cam):
    """[3][F] colour of every face for one view; also the pre-clamp values."""
    _, d = face_dirs(pos, idx, cam)
    Y = basis(d)                                            # [F][16]
    k = np.asarray(sh, np.float64).reshape(NB, 3, -1)       # [16][3][F]
    pre = 0.5 + np.einsum("fb,bcf->cf", Y, k)
    return np.maximum(pre, 0.0), pre


def face_colours_backward(sh, pos, idx, cam, dcol):
    """Adjoint of face_colours for one view: dL/dsh [48][F] and dL/dpos [3][V]."""
    v, d = face_dirs(pos, idx, cam)
    Y = basis(d)
    G = basis_grad(d)                                       # [F][16][3]
    k = np.asarray(sh, np.float64).reshape(NB, 3, -1)
    pre = 0.5 + np.einsum("fb,bcf->cf", Y, k)
    g = np.asarray(dcol, np.float64) * (pre > 0.0)          # [3][F]
    dsh = np.einsum("fb,cf->bcf", Y, g).reshape(48, -1)
    # dL/dd = sum_c g_c sum_b k_bc dY_b/dd, then through d = v/|v| and the centroid
    dd = np.einsum("cf,bcf,fbj->fj", g, k, G)
    nv = np.linalg.norm(v, axis=1, keepdims=True)
    dv = (dd - np.sum(dd * d, axis=1, keepdims=True) * d) / nv
    P = np.asarray(pos, np.float64)
    dpos = np.zeros_like(P)
    I = np.asarray(idx, np.int64)
    for c in range(3):
        np.add.at(dpos.T, I[c], dv / 3.0)
    return dsh, dpos
