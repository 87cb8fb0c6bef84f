"""FP64 oracle work for the GPU tests, spread over worker processes.

The workers import numpy and `oracle/` only (never torch or the HIP library) and are
started with the "spawn" method, so they share nothing with the process that holds the
GPU. At most 16 workers (the CPU share of one GPU on the test machines), each with one
BLAS thread.
"""
from __future__ import annotations

import os

import numpy as np


def _init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:  # pragma: no cover
        pass


def n_workers(n_jobs):
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cpus = os.cpu_count() or 1
    return max(1, min(16, cpus, n_jobs))


def run(fn, jobs):
    """[fn(job) for job in jobs] on a spawn pool (in order)."""
    import multiprocessing as mp
    if len(jobs) <= 1:
        return [fn(j) for j in jobs]
    with mp.get_context("spawn").Pool(n_workers(len(jobs)), initializer=_init) as pool:
        return pool.map(fn, jobs, chunksize=1)


def cell_energy_forces(job):
    """(E, F[n, 3]) of one periodic cell: job = (pos, species, box, beta, sigma)."""
    from oracle import evaluate as oev
    pos, species, box, beta, sigma = job
    r = oev.evaluate(pos, species, box, beta, sigma)
    return r.energy, r.f


def local_fd_forces(job):
    """Central differences -(E(x + h e) - E(x - h e)) / 2h of the oracle energy of one
    cell for the listed atoms and all three components. Moving atom a changes only the
    energies of a and of the atoms within r_cut of it, so each difference is taken over
    those atoms' energies (the same number as the difference of the cell totals, with less
    rounding); atoms are taken within r_cut + 0.01 A of the unmoved position, which covers
    both displaced positions for h << 0.01 A. job = (pos, species, box, beta, h, atoms)."""
    from oracle import evaluate as oev, neighbors as onl
    from oracle.hyper import DEFAULT
    pos, species, box, beta, h, atoms = job
    pos = np.asarray(pos, np.float64)
    zero = np.zeros_like(beta)
    f = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        _, j, _ = onl.neighbor_list(pos, box, DEFAULT.r_cut + 0.01, rows=np.array([a]))
        tg = np.union1d([a], j)
        for x in range(3):
            e = []
            for sgn in (1.0, -1.0):
                p = pos.copy()
                p[a, x] += sgn * h
                r = oev.evaluate(p, species, box, beta, zero, targets=tg, want_forces=False)
                e.append(r.e[r.row_of(tg)].sum())
            f[k, x] = -(e[0] - e[1]) / (2 * h)
    return f
