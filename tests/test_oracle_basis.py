"""Pins for the oracle's pair basis against closed forms and library routines."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy import special

from oracle import basis


def test_chebyshev_is_cos_n_theta():
    th = np.linspace(0.01, math.pi - 0.01, 57)
    t = basis.chebyshev(np.cos(th), 9)
    for n in range(9):
        np.testing.assert_allclose(t[:, n], np.cos(n * th), atol=1e-13)


def test_chebyshev_matches_numpy_chebval():
    x = np.linspace(-1, 1, 41)
    t = basis.chebyshev(x, 8)
    for n in range(8):
        c = np.zeros(n + 1)
        c[n] = 1
        np.testing.assert_allclose(t[:, n], npcheb.chebval(x, c), atol=1e-13)


def test_chebyshev_derivative_is_n_U():
    # T_n'(cos th) = n U_{n-1}(cos th) = n sin(n th) / sin th
    th = np.linspace(0.05, math.pi - 0.05, 33)
    d = basis.chebyshev_deriv(np.cos(th), 8)
    for n in range(8):
        np.testing.assert_allclose(d[:, n], n * np.sin(n * th) / np.sin(th), atol=1e-11)


def test_cutoff_shape():
    rc = 4.5
    r = np.array([0.0, 1.0, 4.4, 4.5, 5.0])
    np.testing.assert_allclose(basis.cutoff(r, rc), [20.25, 12.25, 0.01, 0.0, 0.0], atol=1e-14)
    np.testing.assert_allclose(basis.cutoff_deriv(r, rc), [-9.0, -7.0, -0.2, 0.0, 0.0], atol=1e-14)


def test_radial_derivative_fd():
    r = np.linspace(0.6, 4.49, 23)
    h = 1e-6
    fd = (basis.radial(r + h, 4.5, 8) - basis.radial(r - h, 4.5, 8)) / (2 * h)
    np.testing.assert_allclose(basis.radial_deriv(r, 4.5, 8), fd, atol=1e-7)


def _sphere_quadrature(n_theta=12, n_phi=24):
    x, w = np.polynomial.legendre.leggauss(n_theta)            # nodes in cos(theta)
    phi = np.arange(n_phi) * 2 * math.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    u = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).ravel()
    return u, wt


def test_real_sph_harm_orthonormal():
    u, wt = _sphere_quadrature()
    y = basis.real_sph_harm(u)
    gram = (y * wt[:, None]).T @ y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


def test_real_sph_harm_matches_scipy_up_to_sign():
    rng = np.random.default_rng(5)
    u = rng.standard_normal((200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    theta = np.arccos(u[:, 2])
    phi = np.arctan2(u[:, 1], u[:, 0])
    y = basis.real_sph_harm(u)
    for l in range(4):
        for m in range(-l, l + 1):
            c = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * c.real
            elif m < 0:
                ref = math.sqrt(2) * c.imag
            else:
                ref = c.real
            got = y[:, l * l + l + m]
            sign = np.sign((got * ref).sum())
            np.testing.assert_allclose(got, sign * ref, atol=1e-12, err_msg=f"l={l} m={m}")


def test_addition_theorem():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((50, 3))
    b = rng.standard_normal((50, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    ya, yb = basis.real_sph_harm(a), basis.real_sph_harm(b)
    cos = (a * b).sum(1)
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (ya[:, sl] * yb[:, sl]).sum(1)
        rhs = (2 * l + 1) / (4 * math.pi) * special.eval_legendre(l, cos)
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_sph_harm_gradient_fd():
    rng = np.random.default_rng(7)
    d = rng.standard_normal((20, 3)) * 2.0
    g = basis.real_sph_harm_grad(d)
    h = 1e-6
    for x in range(3):
        e = np.zeros(3)
        e[x] = h
        yp = basis.real_sph_harm((d + e) / np.linalg.norm(d + e, axis=1, keepdims=True))
        ym = basis.real_sph_harm((d - e) / np.linalg.norm(d - e, axis=1, keepdims=True))
        np.testing.assert_allclose(g[:, :, x], (yp - ym) / (2 * h), atol=1e-8)
