"""Mapped quadratic models (Eq. 1, Eq. 2) and their gradient in the unnormalised descriptor.

Readings: one (beta, gamma) pair per central-atom species, each a full n_d x n_d
symmetric matrix; the outer sum over sparse points printed in Eq. 1 is already folded
into beta (the mapping's purpose, Section V.B), so e_i = d_i^T beta_{s_i} d_i and
V_i = d_i^T gamma_{s_i} d_i. The uncertainty is sqrt(V), with V clamped at 0.
"""
from __future__ import annotations

import math

import numpy as np


def energies(d, species, beta):
    """e_i = d_i^T beta_{s_i} d_i."""
    e = np.empty(len(d))
    for s in range(beta.shape[0]):
        m = species == s
        e[m] = np.einsum("ik,kl,il->i", d[m], beta[s], d[m])
    return e


def variances(d, species, gamma):
    """V_i = d_i^T gamma_{s_i} d_i."""
    return energies(d, species, gamma)


def uncertainties(v):
    return np.sqrt(np.maximum(v, 0.0))


def total_energy(e):
    """Exactly rounded sum (math.fsum)."""
    return math.fsum(np.asarray(e, np.float64).tolist())


def energy_grad_dtilde(d, norm, species, beta):
    """g_i = de_i/dd~_i = (2/|d~|) (beta d - e d) for symmetric beta (0 where |d~| = 0).

    d = d~/|d~| has Jacobian (I - d d^T)/|d~|, and d(d^T beta d)/dd = 2 beta d.
    """
    g = np.zeros_like(d)
    for s in range(beta.shape[0]):
        m = (species == s) & (norm > 0)
        if not m.any():
            continue
        y = d[m] @ (0.5 * (beta[s] + beta[s].T))
        e = (y * d[m]).sum(-1)
        g[m] = (2.0 / norm[m])[:, None] * (y - e[:, None] * d[m])
    return g
