"""Velocity-Verlet NVE and Nose-Hoover NVT in FP64 (the integrators of the short MD
checks), hydrogen coordination numbers and reaction events. Test infrastructure.

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


# ---- Nose-Hoover NVT (the paper's production runs, Section VI.A: 450 K) ----
# One thermostat variable zeta per cell (no chain; readings: N_f = 3N - 3, damping time
# tau). Equations of motion: dx/dt = v, dv/dt = KAPPA F/m - zeta v,
# dzeta/dt = G(K) = (2K / (N_f k_B T0) - 1) / tau^2, deta/dt = zeta. Time-reversible
# splitting of one step dt (Trotter factorisation of the Liouville operator):
#   zeta += dt/2 G(K); v *= exp(-zeta dt/2); eta += zeta dt/2;       (thermostat half)
#   v += dt/2 a(x); x += dt v; v += dt/2 a(x_new)                    (velocity Verlet)
#   v *= exp(-zeta dt/2); eta += zeta dt/2; zeta += dt/2 G(K_new)    (thermostat half)
# Conserved: H' = E_pot + K + Q zeta^2 / 2 + N_f k_B T0 eta with Q = N_f k_B T0 tau^2.
KB = 8.617333262e-5        # eV / K


def n_free(n_atoms):
    return max(3 * n_atoms - 3, 1)


def nvt(pos, vel, species, dt, n_steps, force_fn, t0, tau, zeta0=0.0):
    """Returns per-step arrays of (E_pot, E_kin, zeta, eta) (step 0 = initial state) and
    the final x, v."""
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    m = masses(species)
    nf = n_free(len(m))
    g = lambda k: (2.0 * k / (nf * KB * t0) - 1.0) / (tau * tau)
    ep, f = force_fn(x)
    zeta, eta = zeta0, 0.0
    k = kinetic(v, m)
    out = [(ep, k, zeta, eta)]
    for _ in range(n_steps):
        zeta += 0.5 * dt * g(k)
        v = v * np.exp(-0.5 * dt * zeta)
        eta += 0.5 * dt * zeta
        v = v + 0.5 * dt * KAPPA * f / m[:, None]
        x = x + dt * v
        ep, f = force_fn(x)
        v = v + 0.5 * dt * KAPPA * f / m[:, None]
        v = v * np.exp(-0.5 * dt * zeta)
        eta += 0.5 * dt * zeta
        k = kinetic(v, m)
        zeta += 0.5 * dt * g(k)
        out.append((ep, k, zeta, eta))
    return np.array(out), x, v


def extended_energy(rec, n_atoms, t0, tau):
    """H' of each record row (E_pot, E_kin, zeta, eta) of nvt()."""
    nf = n_free(n_atoms)
    q = nf * KB * t0 * tau * tau
    return rec[:, 0] + rec[:, 1] + 0.5 * q * rec[:, 2] ** 2 + nf * KB * t0 * rec[:, 3]


# ---- hydrogen coordination and reaction events (Section VI.A) ----
# An H atom has coordination 1 when another H atom is within 1 A (squared distance < 1 in
# FP64 over all periodic images), else 0; other species are reported as 0. A change
# 1 -> 0 between two snapshots is a dissociation, 0 -> 1 a recombination.
R_COORD = 1.0


def coordination(pos, species, box):
    from . import neighbors
    i, j, s = neighbors.brute_force(pos, box, R_COORD)
    species = np.asarray(species)
    c = np.zeros(len(species), np.int32)
    hh = (species[i] == 0) & (species[j] == 0)
    c[i[hh]] = 1
    return c


def reaction_events(c_prev, c_now):
    """(dissociations, recombinations) between two coordination snapshots."""
    c_prev, c_now = np.asarray(c_prev), np.asarray(c_now)
    return int(np.sum((c_prev == 1) & (c_now == 0))), int(np.sum((c_prev == 0) & (c_now == 1)))
