"""Pair basis: Chebyshev radial functions x smooth cutoff x real spherical harmonics.

The paper builds B2 descriptors from "an equivariant basis of spherical harmonics and
radial functions" (Section V.B, Fig. 3) without fixing the radial set or the cutoff.
Readings used here:
  * radial functions T_n(x), x = 2r/r_c - 1, n = 0..n_rad-1 (Chebyshev polynomials of
    the first kind), multiplied by the cutoff f_c(r) = (r_c - r)^2 for r < r_c and 0
    beyond, which is continuous with a continuous first derivative at r_c;
  * orthonormal real spherical harmonics Y_lm (integral of Y^2 over the sphere = 1),
    flat index l^2 + l + m. Only the per-l normalisation matters for B2; the sign
    convention of each (l, m) cancels in the products of equal m.
"""
from __future__ import annotations

import math

import numpy as np


def chebyshev(x, n):
    """T_0..T_{n-1} at x by the three-term recurrence T_{k+1} = 2x T_k - T_{k-1}."""
    x = np.asarray(x, np.float64)
    t = np.empty(x.shape + (n,))
    t[..., 0] = 1.0
    if n > 1:
        t[..., 1] = x
    for k in range(1, n - 1):
        t[..., k + 1] = 2.0 * x * t[..., k] - t[..., k - 1]
    return t


def chebyshev_deriv(x, n):
    """dT_k/dx by differentiating the recurrence: T'_{k+1} = 2 T_k + 2x T'_k - T'_{k-1}."""
    x = np.asarray(x, np.float64)
    t = chebyshev(x, n)
    d = np.zeros(x.shape + (n,))
    if n > 1:
        d[..., 1] = 1.0
    for k in range(1, n - 1):
        d[..., k + 1] = 2.0 * t[..., k] + 2.0 * x * d[..., k] - d[..., k - 1]
    return d


def cutoff(r, rc):
    r = np.asarray(r, np.float64)
    return np.where(r < rc, (rc - r) ** 2, 0.0)


def cutoff_deriv(r, rc):
    r = np.asarray(r, np.float64)
    return np.where(r < rc, -2.0 * (rc - r), 0.0)


def radial(r, rc, n):
    """R_n(r) = T_n(2r/rc - 1) f_c(r)  ->  [..., n]."""
    x = 2.0 * np.asarray(r, np.float64) / rc - 1.0
    return chebyshev(x, n) * cutoff(r, rc)[..., None]


def radial_deriv(r, rc, n):
    """dR_n/dr = T_n'(x) (2/rc) f_c + T_n f_c'."""
    r = np.asarray(r, np.float64)
    x = 2.0 * r / rc - 1.0
    return (chebyshev_deriv(x, n) * (2.0 / rc) * cutoff(r, rc)[..., None]
            + chebyshev(x, n) * cutoff_deriv(r, rc)[..., None])


_PI = math.pi


def real_sph_harm(u, l_max=3):
    """Orthonormal real Y_lm of unit vectors u [..., 3] for l <= 3, textbook Cartesian forms."""
    if l_max > 3:
        raise NotImplementedError("closed forms are written out for l <= 3")
    u = np.asarray(u, np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    out = np.empty(u.shape[:-1] + ((l_max + 1) ** 2,))
    out[..., 0] = 0.5 * math.sqrt(1.0 / _PI)
    if l_max >= 1:
        c1 = math.sqrt(3.0 / (4.0 * _PI))
        out[..., 1] = c1 * y
        out[..., 2] = c1 * z
        out[..., 3] = c1 * x
    if l_max >= 2:
        c = 0.5 * math.sqrt(15.0 / _PI)
        out[..., 4] = c * x * y
        out[..., 5] = c * y * z
        out[..., 6] = 0.25 * math.sqrt(5.0 / _PI) * (3.0 * z * z - 1.0)
        out[..., 7] = c * x * z
        out[..., 8] = 0.25 * math.sqrt(15.0 / _PI) * (x * x - y * y)
    if l_max >= 3:
        out[..., 9] = 0.25 * math.sqrt(35.0 / (2 * _PI)) * y * (3.0 * x * x - y * y)
        out[..., 10] = 0.5 * math.sqrt(105.0 / _PI) * x * y * z
        out[..., 11] = 0.25 * math.sqrt(21.0 / (2 * _PI)) * y * (5.0 * z * z - 1.0)
        out[..., 12] = 0.25 * math.sqrt(7.0 / _PI) * z * (5.0 * z * z - 3.0)
        out[..., 13] = 0.25 * math.sqrt(21.0 / (2 * _PI)) * x * (5.0 * z * z - 1.0)
        out[..., 14] = 0.25 * math.sqrt(105.0 / _PI) * z * (x * x - y * y)
        out[..., 15] = 0.25 * math.sqrt(35.0 / (2 * _PI)) * x * (x * x - 3.0 * y * y)
    return out


def _grad_forms(u, l_max=3):
    """Gradient of the textbook forms above as functions on R^3 (not yet projected)."""
    u = np.asarray(u, np.float64)
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    zero = np.zeros_like(x)
    g = np.zeros(u.shape[:-1] + ((l_max + 1) ** 2, 3))
    if l_max >= 1:
        c1 = math.sqrt(3.0 / (4.0 * _PI))
        g[..., 1, 1] = c1
        g[..., 2, 2] = c1
        g[..., 3, 0] = c1
    if l_max >= 2:
        c = 0.5 * math.sqrt(15.0 / _PI)
        g[..., 4, :] = np.stack([c * y, c * x, zero], -1)
        g[..., 5, :] = np.stack([zero, c * z, c * y], -1)
        g[..., 6, :] = np.stack([zero, zero, 0.25 * math.sqrt(5.0 / _PI) * 6.0 * z], -1)
        g[..., 7, :] = np.stack([c * z, zero, c * x], -1)
        c22 = 0.25 * math.sqrt(15.0 / _PI)
        g[..., 8, :] = np.stack([2 * c22 * x, -2 * c22 * y, zero], -1)
    if l_max >= 3:
        a = 0.25 * math.sqrt(35.0 / (2 * _PI))
        g[..., 9, :] = np.stack([a * 6 * x * y, a * (3 * x * x - 3 * y * y), zero], -1)
        b = 0.5 * math.sqrt(105.0 / _PI)
        g[..., 10, :] = np.stack([b * y * z, b * x * z, b * x * y], -1)
        c = 0.25 * math.sqrt(21.0 / (2 * _PI))
        g[..., 11, :] = np.stack([zero, c * (5 * z * z - 1), c * 10 * y * z], -1)
        d = 0.25 * math.sqrt(7.0 / _PI)
        g[..., 12, :] = np.stack([zero, zero, d * (15 * z * z - 3)], -1)
        g[..., 13, :] = np.stack([c * (5 * z * z - 1), zero, c * 10 * x * z], -1)
        e = 0.25 * math.sqrt(105.0 / _PI)
        g[..., 14, :] = np.stack([e * 2 * x * z, -e * 2 * y * z, e * (x * x - y * y)], -1)
        g[..., 15, :] = np.stack([a * (3 * x * x - 3 * y * y), -a * 6 * x * y, zero], -1)
    return g


def real_sph_harm_grad(delta, l_max=3):
    """d/d(delta) of Y_lm(delta/|delta|) -> [..., n_lm, 3].

    Chain rule through the unit vector: (I - u u^T) grad_u F(u) / r, which is the
    same for any smooth extension F of Y_lm off the sphere.
    """
    delta = np.asarray(delta, np.float64)
    r = np.sqrt((delta * delta).sum(-1))
    u = delta / r[..., None]
    g = _grad_forms(u, l_max)
    radial_part = (g * u[..., None, :]).sum(-1)
    return (g - radial_part[..., None] * u[..., None, :]) / r[..., None, None]
