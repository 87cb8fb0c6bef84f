"""Forces F = -dE/dr, E = sum_i e_i, by two routes that share nothing with the HIP path.

1. Explicit descriptor gradient (the direct route; Section V.B says the force
   reordering avoids forming it). For every list entry p = (i, j, s) inside the cutoff,
   with Delta_p = r_j + s L - r_i:
       dc_i[(s_j, n), lm] / dDelta_p = R_n'(r) r^ Y_lm + R_n grad Y_lm
       dd~_i[(a,b), l] / dDelta_p    = sum_m (dc_a/dDelta c_b + c_a dc_b/dDelta)
       h_p = de_i/dDelta_p          = g_i . dd~_i/dDelta_p
   then dE/dr_j += h_p and dE/dr_i -= h_p.
2. Central finite differences of the total energy, step h (FP64).

Virial (the stress the paper's model predicts, Section VI): under a homogeneous strain
x -> (I + eps) x of positions and cell, every pair vector becomes (I + eps) Delta_p, so
    W_ab = -dE/deps_ab = -sum_p h_p,a Delta_p,b
(symmetric for a rotation-invariant energy). For a free cluster this is sum_i r_i,a F_i,b.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .hyper import Hyper


def pair_basis_grad(delta, h: Hyper):
    """grad_Delta [R_n(r) Y_lm(r^)] -> [P, n_rad, n_lm, 3]."""
    r = np.sqrt((delta * delta).sum(-1))
    u = delta / r[:, None]
    rad = basis.radial(r, h.r_cut, h.n_rad)
    drad = basis.radial_deriv(r, h.r_cut, h.n_rad)
    y = basis.real_sph_harm(u, h.l_max)
    dy = basis.real_sph_harm_grad(delta, h.l_max)
    return (drad[:, :, None, None] * y[:, None, :, None] * u[:, None, None, :]
            + rad[:, :, None, None] * dy[:, None, :, :])


def descriptor_grad(c_i, sj, delta, h: Hyper):
    """Explicit dd~_i/dDelta_p for a chunk of pairs -> [P, n_desc, 3].

    c_i: [P, channels, n_lm] densities of each pair's centre atom; sj: neighbour species.
    """
    p = len(delta)
    grad = pair_basis_grad(delta, h)                                  # [P, n_rad, n_lm, 3]
    dc = np.zeros((p, h.n_channels, h.n_lm, 3))
    for s in range(h.n_species):
        m = sj == s
        dc[m, s * h.n_rad:(s + 1) * h.n_rad] = grad[m]
    bounds = [l * l for l in range(h.l_max + 1)]
    # t[p, a, b, l, x] = sum_{m in l} dc[p, a, lm, x] c[p, b, lm]
    prod = dc[:, :, None, :, :] * c_i[:, None, :, :, None]            # [P, a, b, lm, 3]
    t = np.add.reduceat(prod, bounds, axis=3)                         # [P, a, b, l, 3]
    jac = t + t.transpose(0, 2, 1, 3, 4)
    pairs = np.array(h.pairs())
    return jac[:, pairs[:, 0], pairs[:, 1]].reshape(p, h.n_desc, 3)


def forces_explicit(n_atoms, species, i, j, delta, c_rows, g_rows, where, h: Hyper,
                    targets=None, chunk=512):
    """F for `targets` (default all) from list entries (i, j, delta).

    c_rows, g_rows: densities and de/dd~ for the atoms that index into them via
    `where` (atom -> row, -1 if absent). Every centre i that owns a pair touching a
    target must have a row.
    """
    r = np.sqrt((delta * delta).sum(-1))
    keep = r < h.r_cut
    if targets is not None:
        tmask = np.zeros(n_atoms, bool)
        tmask[targets] = True
        keep &= tmask[i] | tmask[j]
    i, j, delta = i[keep], j[keep], delta[keep]
    if np.any(where[i] < 0):
        raise ValueError("a pair's centre atom has no descriptor row")
    grad_e = np.zeros((n_atoms, 3))
    for a in range(0, len(i), chunk):
        ii, jj, dd = i[a:a + chunk], j[a:a + chunk], delta[a:a + chunk]
        jac = descriptor_grad(c_rows[where[ii]], species[jj], dd, h)
        hp = np.einsum("pk,pkx->px", g_rows[where[ii]], jac)
        np.add.at(grad_e, jj, hp)
        np.add.at(grad_e, ii, -hp)
    f = -grad_e
    return f if targets is None else f[targets]


def virial_explicit(species, i, j, delta, c_rows, g_rows, where, h: Hyper, chunk=512):
    """W = -sum_p h_p (x) Delta_p over all list entries inside the cutoff (FP64 3x3)."""
    r = np.sqrt((delta * delta).sum(-1))
    keep = r < h.r_cut
    i, j, delta = i[keep], j[keep], delta[keep]
    w = np.zeros((3, 3))
    for a in range(0, len(i), chunk):
        ii, jj, dd = i[a:a + chunk], j[a:a + chunk], delta[a:a + chunk]
        jac = descriptor_grad(c_rows[where[ii]], species[jj], dd, h)
        hp = np.einsum("pk,pkx->px", g_rows[where[ii]], jac)
        w -= hp.T @ dd
    return w


def virial_fd(energy_fn, pos, box, axis, step=1e-5):
    """-dE/deps_aa by central differences of a uniaxial strain of positions and box."""
    pos = np.array(pos, np.float64)
    box = np.array(box, np.float64)
    out = []
    for sgn in (1.0, -1.0):
        f = np.ones(3)
        f[axis] += sgn * step
        out.append(energy_fn(pos * f, box * f))
    return -(out[0] - out[1]) / (2 * step)


def forces_fd(energy_fn, pos, atoms=None, step=1e-4):
    """Central differences -(E(x + h) - E(x - h)) / 2h for the listed atoms (default all)."""
    pos = np.array(pos, np.float64)
    atoms = np.arange(len(pos)) if atoms is None else np.asarray(atoms)
    f = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for x in range(3):
            p = pos.copy()
            p[a, x] += step
            ep = energy_fn(p)
            p[a, x] -= 2 * step
            em = energy_fn(p)
            f[k, x] = -(ep - em) / (2 * step)
    return f
