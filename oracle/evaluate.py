"""One force-field evaluation: e_i, V_i, sigma_i, F_i and E for a periodic cell.

`targets` restricts the outputs to a subset of atoms (a sample of a large cell): the
descriptors are then formed for the targets and their neighbours, which is what the
forces on the targets need.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import descriptors, forces, model, neighbors
from .hyper import DEFAULT, Hyper


@dataclasses.dataclass
class Result:
    rows: np.ndarray          # atom index of each row of d, e, V, sigma
    d: np.ndarray             # normalised descriptors [rows, n_desc]
    norm: np.ndarray          # |d~|
    e: np.ndarray             # per-atom energy
    v: np.ndarray             # per-atom variance
    sigma: np.ndarray         # per-atom uncertainty
    targets: np.ndarray       # atoms whose forces are in f
    f: np.ndarray | None      # forces [targets, 3]
    energy: float | None      # total energy (full evaluations only)
    c: np.ndarray | None = None
    virial: np.ndarray | None = None   # W = -dE/d(strain), 3x3 (full evaluations, on request)

    def row_of(self, atoms):
        where = {int(a): k for k, a in enumerate(self.rows)}
        return np.array([where[int(a)] for a in atoms])


def evaluate(pos, species, box, beta, gamma, h: Hyper = DEFAULT, targets=None,
             want_forces=True, keep_c=False, want_virial=False):
    pos = np.asarray(pos, np.float64)
    species = np.asarray(species)
    n = len(pos)
    if targets is None:
        rows = np.arange(n)
        i, j, s = neighbors.neighbor_list(pos, box, h.r_cut)
        tg = rows
    else:
        tg = np.asarray(targets, np.int64)
        _, jt, _ = neighbors.neighbor_list(pos, box, h.r_cut, rows=tg)
        rows = np.union1d(tg, jt)
        i, j, s = neighbors.neighbor_list(pos, box, h.r_cut, rows=rows)
    delta = neighbors.pair_vectors(pos, box, i, j, s)
    c = descriptors.densities(n, species, i, j, delta, h, rows)
    dt = descriptors.b2(c, h)
    d, norm = descriptors.normalise(dt)
    sp = species[rows]
    e = model.energies(d, sp, beta)
    v = model.variances(d, sp, gamma)
    f = None
    vir = None
    if want_forces or want_virial:
        g = model.energy_grad_dtilde(d, norm, sp, beta)
        where = -np.ones(n, np.int64)
        where[rows] = np.arange(len(rows))
        if want_forces:
            f = forces.forces_explicit(n, species, i, j, delta, c, g, where, h,
                                       targets=None if targets is None else tg)
        if want_virial:
            if targets is not None:
                raise ValueError("the virial is a whole-cell quantity")
            vir = forces.virial_explicit(species, i, j, delta, c, g, where, h)
    energy = model.total_energy(e) if targets is None else None
    return Result(rows, d, norm, e, v, model.uncertainties(v), tg, f, energy,
                  c if keep_c else None, vir)


def total_energy(pos, species, box, beta, h: Hyper = DEFAULT):
    zero = np.zeros_like(beta)
    return evaluate(pos, species, box, beta, zero, h, want_forces=False).energy
