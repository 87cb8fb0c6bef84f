"""Per-atom densities, B2 power spectrum and normalisation (Section V.B, Fig. 3).

c_{i,(s,n),l,m} = sum over neighbours j of species s with r_ij < r_c of R_n(r_ij) Y_lm(r^_ij)
d~_{(a,b),l}    = sum_m c_{a,l,m} c_{b,l,m}        for channel pairs a <= b
d_i             = d~_i / |d~_i|                     (the normalised descriptor)

With no neighbour inside the cutoff, |d~| = 0 and d is taken as 0.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .hyper import Hyper


def lm_l(h: Hyper):
    """l of each flat (l, m) index."""
    return np.concatenate([[l] * (2 * l + 1) for l in range(h.l_max + 1)])


def densities(n_atoms, species, i, j, delta, h: Hyper, rows=None):
    """c [n_rows, S*n_rad, n_lm] from list entries (i, j, delta) with any radius >= r_c.

    rows: which atoms to return (default all); pairs of other atoms are skipped.
    """
    rows = np.arange(n_atoms) if rows is None else np.asarray(rows)
    where = -np.ones(n_atoms, np.int64)
    where[rows] = np.arange(len(rows))
    r = np.sqrt((delta * delta).sum(-1))
    keep = (r < h.r_cut) & (where[i] >= 0)
    i, j, delta, r = i[keep], j[keep], delta[keep], r[keep]
    c = np.zeros((len(rows), h.n_channels, h.n_lm))
    if len(i) == 0:
        return c
    rad = basis.radial(r, h.r_cut, h.n_rad)                 # [P, n_rad]
    y = basis.real_sph_harm(delta / r[:, None], h.l_max)    # [P, n_lm]
    prod = rad[:, :, None] * y[:, None, :]                  # [P, n_rad, n_lm]
    sj = species[j]
    for s in range(h.n_species):
        m = sj == s
        if not m.any():
            continue
        blk = np.zeros((len(rows), h.n_rad, h.n_lm))
        np.add.at(blk, where[i[m]], prod[m])
        c[:, s * h.n_rad:(s + 1) * h.n_rad, :] += blk
    return c


def b2(c, h: Hyper):
    """Packed B2 vector d~ [N, n_desc] from densities c [N, channels, n_lm]."""
    lml = lm_l(h)
    out = np.empty((c.shape[0], h.n_desc))
    k = 0
    for a, b in h.pairs():
        prod = c[:, a, :] * c[:, b, :]
        for l in range(h.l_max + 1):
            out[:, k] = prod[:, lml == l].sum(-1)
            k += 1
    return out


def normalise(dt):
    norm = np.sqrt((dt * dt).sum(-1))
    safe = np.where(norm > 0, norm, 1.0)
    d = np.where(norm[:, None] > 0, dt / safe[:, None], 0.0)
    return d, norm
