"""Sparse-GP mean and variance, unmapped and mapped (Eq. 1, Eq. 2, Section V.B).

With the normalised inner-product kernel k_xi(rho_1, rho_2) = sigma^2 (d_1 . d_2)^xi:
  mean      eps(d)  = sum_s k_2(d, d_s) alpha_s = d^T beta d,   beta = sigma^2 sum_s alpha_s d_s d_s^T
  variance  V(d)    = sigma^2 k1(d, d) - sigma^4 k1(d, D_S)^T K_SS^{-1} k1(D_S, d) = d^T gamma d,
            gamma   = sigma^2 I - sigma^4 D_S^T K_SS^{-1} D_S
Reading for Eq. 2: the k_1 factors inside it are the unscaled dot products d . d_s (the
sigma^2 and sigma^4 printed in front carry the signal variance), and K_SS is the sparse-set
kernel matrix sigma^2 D_S D_S^T plus a noise term on its diagonal. For d close to the span
of the sparse set V is a small difference of two terms of size sigma^2 (|d| = 1): the
near-cancelling form the split-precision path evaluates as a sum of squares.
"""
from __future__ import annotations

import numpy as np


def kernel_matrix(ds, sigma2, noise):
    """K_SS = sigma^2 D_S D_S^T + noise I  (xi = 1)."""
    return sigma2 * ds @ ds.T + noise * np.eye(len(ds))


def mean_unmapped(d, ds, alpha, sigma2):
    """eps(d) = sum_s sigma^2 (d . d_s)^2 alpha_s."""
    return (sigma2 * (d @ ds.T) ** 2) @ alpha


def beta_mapped(ds, alpha, sigma2):
    return sigma2 * (ds.T * alpha) @ ds


def variance_unmapped(d, ds, sigma2, noise):
    """sigma^2 (d . d) - sigma^4 k^T K_SS^{-1} k with k_s = d . d_s."""
    k = d @ ds.T
    kss = kernel_matrix(ds, sigma2, noise)
    sol = np.linalg.solve(kss, k.T).T
    return sigma2 * (d * d).sum(-1) - sigma2 ** 2 * (k * sol).sum(-1)


def gamma_mapped(ds, sigma2, noise):
    kss = kernel_matrix(ds, sigma2, noise)
    g = sigma2 * np.eye(ds.shape[1]) - sigma2 ** 2 * ds.T @ np.linalg.solve(kss, ds)
    return 0.5 * (g + g.T)
