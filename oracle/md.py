"""Velocity-Verlet NVE in FP64 (the integrator of the short MD checks).

Units: A, fs, amu, eV. Acceleration a = KAPPA * F / m with
KAPPA = 1 eV / (A amu) in A/fs^2 = 9.648533212e-3.
  v <- v + dt/2 a(x);  x <- x + dt v;  v <- v + dt/2 a(x_new)
"""
from __future__ import annotations

import numpy as np

KAPPA = 9.648533212e-3
MASS = {0: 1.008, 1: 195.084}


def masses(species):
    return np.array([MASS[int(s)] for s in species])


def kinetic(v, m):
    return 0.5 * float((m[:, None] * v * v).sum()) / KAPPA


def nve(pos, vel, species, dt, n_steps, force_fn):
    """force_fn(pos) -> (E_pot, F). Returns per-step arrays of (E_pot, E_kin) and final x, v."""
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    m = masses(species)
    ep, f = force_fn(x)
    epot, ekin = [ep], [kinetic(v, m)]
    for _ in range(n_steps):
        v = v + 0.5 * dt * KAPPA * f / m[:, None]
        x = x + dt * v
        ep, f = force_fn(x)
        v = v + 0.5 * dt * KAPPA * f / m[:, None]
        epot.append(ep)
        ekin.append(kinetic(v, m))
    return np.array(epot), np.array(ekin), x, v
