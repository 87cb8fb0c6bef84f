"""Seeded synthetic inputs: H2 gas over Pt(111) slabs, and the random mapped models.

This module only builds inputs. It holds none of the force field's arithmetic, so
both the FP64 oracle (tests) and the HIP path draw their inputs from here.

The geometry follows the paper's application (Section VI.A: H2 gas interacting
with a Pt(111) slab, H coverage on the surface). Sizes follow the workloads:
a 4x4x4 slab with 8 molecules (80 atoms), a 100x100x24 slab under a 1.14 kA gas
column (~1.0 M atoms), a 400x400x24 slab (~16 M atoms), batches of 6x6x4 cells,
and served slabs of random size with adsorbed H.

Units: Angstrom, amu. Species index: H = 0, Pt = 1 (sorted by atomic number).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

H, PT = 0, 1
MASS = np.array([1.008, 195.084])          # amu
A_PT = 3.92                                 # fcc Pt lattice constant
A_NN = A_PT / math.sqrt(2.0)                # in-plane spacing of Pt(111)
ROW = A_NN * math.sqrt(3.0) / 2.0           # spacing between close-packed rows
DZ = A_PT / math.sqrt(3.0)                  # (111) layer spacing
H2_BOND = 0.74
GAS_DENSITY = 1.0 / 200.0                   # molecules per cubic Angstrom


@dataclasses.dataclass
class Structure:
    pos: np.ndarray        # [N, 3] float64, wrapped into [0, L)
    species: np.ndarray    # [N] int32
    box: np.ndarray        # [3] float64 orthorhombic, periodic on all axes

    @property
    def n(self) -> int:
        return len(self.species)


@dataclasses.dataclass
class Batch:
    """Several independent periodic cells laid end to end in one atom array."""
    pos: np.ndarray        # [N, 3]
    species: np.ndarray    # [N]
    offsets: np.ndarray    # [n_struct + 1] int32 atom ranges
    boxes: np.ndarray      # [n_struct, 3]

    @property
    def n(self) -> int:
        return len(self.species)

    def structure(self, k: int) -> Structure:
        a, b = self.offsets[k], self.offsets[k + 1]
        return Structure(self.pos[a:b].copy(), self.species[a:b].copy(), self.boxes[k].copy())


def _wrap(pos, box):
    return pos - box * np.floor(pos / box)


def pt111_slab(nx: int, ny: int, nlayers: int):
    """Orthorhombic fcc(111) slab, ABC stacking, bottom layer at z = 0.

    Returns (positions [nx*ny*nlayers, 3], lateral box (Lx, Ly), z of the top layer).
    ny must be even so that the centred-rectangular cell is periodic.
    """
    if ny % 2:
        raise ValueError("ny must be even for an orthorhombic (111) cell")
    lx, ly = nx * A_NN, ny * ROW
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x0 = (i + 0.5 * (j % 2)) * A_NN
    y0 = j * ROW
    layers = []
    for k in range(nlayers):
        s = k % 3
        x = x0 + s * 0.5 * A_NN
        y = y0 + s * ROW / 3.0
        z = np.full_like(x, k * DZ)
        layers.append(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    pos = np.concatenate(layers)
    pos[:, 0] %= lx
    pos[:, 1] %= ly
    return pos, (lx, ly), (nlayers - 1) * DZ


def _place_h2(rng, n_mol, box, z_lo, z_hi, pt_pos, min_hh=1.5, min_hpt=2.0):
    """Place n_mol H2 molecules with centres uniform in [0,Lx)x[0,Ly)x[z_lo,z_hi).

    Axis uniform on the sphere, bond 0.74 A. A candidate is rejected if one of its
    atoms is closer than min_hh to an H of another molecule or closer than min_hpt
    to any Pt (minimum image). Proposals are drawn in batches; conflicts inside a
    batch are resolved in draw order, so the result depends only on the seed.
    """
    if n_mol == 0:
        return np.zeros((0, 3))
    box = np.asarray(box, dtype=np.float64)
    pt_tree = cKDTree(_wrap(pt_pos, box), boxsize=box) if len(pt_pos) else None
    acc = np.zeros((0, 3))
    while len(acc) // 2 < n_mol:
        need = n_mol - len(acc) // 2
        m = max(64, int(need * 1.6))
        c = np.empty((m, 3))
        c[:, 0] = rng.uniform(0.0, box[0], m)
        c[:, 1] = rng.uniform(0.0, box[1], m)
        c[:, 2] = rng.uniform(z_lo, z_hi, m)
        ax = rng.standard_normal((m, 3))
        ax /= np.linalg.norm(ax, axis=1, keepdims=True)
        hp = np.empty((2 * m, 3))
        hp[0::2] = c + 0.5 * H2_BOND * ax
        hp[1::2] = c - 0.5 * H2_BOND * ax
        hp = _wrap(hp, box)
        ok = np.ones(m, dtype=bool)
        if pt_tree is not None:
            d, _ = pt_tree.query(hp, k=1, distance_upper_bound=min_hpt)
            ok &= np.isinf(d).reshape(m, 2).all(axis=1)
        if len(acc):
            t = cKDTree(acc, boxsize=box)
            d, _ = t.query(hp, k=1, distance_upper_bound=min_hh)
            ok &= np.isinf(d).reshape(m, 2).all(axis=1)
        # conflicts among this batch's candidates, resolved in draw order
        cand = np.nonzero(ok)[0]
        if len(cand) > 1:
            sub = hp.reshape(m, 2, 3)[cand].reshape(-1, 3)
            pairs = cKDTree(sub, boxsize=box).query_pairs(min_hh, output_type="ndarray")
            if len(pairs):
                a, b = pairs[:, 0] // 2, pairs[:, 1] // 2
                keep = a != b
                a, b = np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])
                order = np.lexsort((b, a))
                a, b = a[order], b[order]
                dead = np.zeros(len(cand), dtype=bool)
                for u, v in zip(a.tolist(), b.tolist()):
                    if not dead[u]:
                        dead[v] = True
                cand = cand[~dead]
        cand = cand[:need]
        acc = np.concatenate([acc, hp.reshape(m, 2, 3)[cand].reshape(-1, 3)])
    return acc


def h2_over_pt111(nx, ny, nlayers, *, vacuum=None, gas_height=None, n_mol=None,
                  jitter=0.05, seed=0, density=GAS_DENSITY) -> Structure:
    """Pt(111) slab with an H2 gas in the gap above it (periodic along z as well).

    Exactly one of `vacuum` / `gas_height` gives the gap between the top layer and
    the periodic image of the bottom layer. `n_mol` defaults to density x gap volume.
    Gaussian jitter of standard deviation `jitter` is added to every coordinate.
    """
    rng = np.random.default_rng(seed)
    pt, (lx, ly), ztop = pt111_slab(nx, ny, nlayers)
    gap = vacuum if vacuum is not None else gas_height
    lz = ztop + gap
    box = np.array([lx, ly, lz])
    if n_mol is None:
        n_mol = int(round(density * lx * ly * gap))
    hpos = _place_h2(rng, n_mol, box, ztop, lz, pt)
    pos = np.concatenate([pt, hpos])
    species = np.concatenate([np.full(len(pt), PT, np.int32), np.full(len(hpos), H, np.int32)])
    pos = pos + rng.normal(0.0, jitter, pos.shape)
    return Structure(_wrap(pos, box), species, box)


def config_tiny(seed=0) -> Structure:
    """4x4x4 Pt(111) (64 Pt) + 8 H2 in 15 A of vacuum, 0.05 A jitter: 80 atoms."""
    return h2_over_pt111(4, 4, 4, vacuum=15.0, n_mol=8, jitter=0.05, seed=seed)


def config_large(seed=0) -> Structure:
    """100x100x24 Pt(111) (240 k Pt) + H2 gas at 1/200 A^3 in a 1142.2 A column: ~1.0 M atoms."""
    return h2_over_pt111(100, 100, 24, gas_height=1142.2, jitter=0.05, seed=seed)


def config_huge(seed=0) -> Structure:
    """400x400x24 Pt(111) (3.84 M Pt) + H2 gas at 1/200 A^3 in the same column: ~16 M atoms."""
    return h2_over_pt111(400, 400, 24, gas_height=1142.2, jitter=0.05, seed=seed)


def tiled(st: Structure, nx: int, ny: int) -> Structure:
    """The cell repeated nx x ny times laterally (a larger periodic cell). Every atom's
    environment is its original's translated by whole box lengths, so a quantity of the
    small cell holds for each of its copies; copy c = a + nx*b holds atoms [c*n, (c+1)*n)."""
    shifts = [(a, b) for b in range(ny) for a in range(nx)]
    pos = np.concatenate([st.pos + np.array([a * st.box[0], b * st.box[1], 0.0]) for a, b in shifts])
    return Structure(pos=pos, species=np.tile(st.species, len(shifts)),
                     box=np.array([nx * st.box[0], ny * st.box[1], st.box[2]]))


def concat(structs) -> Batch:
    pos = np.concatenate([s.pos for s in structs])
    species = np.concatenate([s.species for s in structs]).astype(np.int32)
    offsets = np.zeros(len(structs) + 1, np.int32)
    offsets[1:] = np.cumsum([s.n for s in structs])
    boxes = np.stack([s.box for s in structs])
    return Batch(pos, species, offsets, boxes)


def config_cells(n_cells=256, seed=0) -> Batch:
    """Batch of independent cells: 6x6x4 Pt(111) (144 Pt) + U{4..32} H2, 0.1 A jitter."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(4, 33, size=n_cells)
    cells = [h2_over_pt111(6, 6, 4, vacuum=15.0, n_mol=int(k), jitter=0.1, seed=seed * 100003 + 17 + c)
             for c, k in enumerate(counts)]
    return concat(cells)


def adsorbed_slab(n_target: int, coverage: float, seed: int, vacuum=15.0, jitter=0.05) -> Structure:
    """4-layer Pt(111) slab of about n_target atoms with coverage*n_surface H atoms.

    H sit at distinct random fcc-hollow sites 0.9 A above the top layer. The lateral
    size nx x ny (ny even) is chosen so that the atom count is close to n_target.
    """
    rng = np.random.default_rng(seed)
    nl = 4
    per_layer = max(4.0, n_target / (nl * (1.0 + coverage / nl)))
    # aspect: keep the cell roughly square (Lx ~ Ly)
    nx = max(2, int(round(math.sqrt(per_layer * ROW / A_NN))))
    ny = max(2, int(round(per_layer / nx / 2.0)) * 2)
    pt, (lx, ly), ztop = pt111_slab(nx, ny, nl)
    box = np.array([lx, ly, ztop + vacuum])
    top = pt[-nx * ny:]
    # fcc hollow above layer k sits where layer k+1 would be in ABC stacking
    s = nl % 3
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    hx = (i + 0.5 * (j % 2)) * A_NN + s * 0.5 * A_NN
    hy = j * ROW + s * ROW / 3.0
    sites = np.stack([hx.ravel() % lx, hy.ravel() % ly, np.full(nx * ny, ztop + 0.9)], axis=1)
    n_h = int(round(coverage * len(top)))
    pick = rng.choice(len(sites), size=n_h, replace=False)
    hpos = sites[np.sort(pick)]
    pos = np.concatenate([pt, hpos])
    species = np.concatenate([np.full(len(pt), PT, np.int32), np.full(n_h, H, np.int32)])
    pos = pos + rng.normal(0.0, jitter, pos.shape)
    return Structure(_wrap(pos, box), species, box)


def serving_requests(n_requests, rate=2000.0, lo=100, hi=50000, seed=0):
    """Poisson arrivals (rate per second) of slabs with log-uniform sizes in [lo, hi].

    Returns a list of (arrival_time_s, Structure). Coverage ~ U[0, 1] monolayer.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))
    cov = rng.uniform(0.0, 1.0, n_requests)
    seeds = rng.integers(0, 2**31 - 1, n_requests)
    return [(float(t[k]), adsorbed_slab(int(sizes[k]), float(cov[k]), int(seeds[k])))
            for k in range(n_requests)]


def random_psd(n: int, seed: int, scale: float = 1e-3) -> np.ndarray:
    """scale * A A^T / n with A ~ N(0,1)^{n x n}: a random symmetric PSD matrix (FP64)."""
    a = np.random.default_rng(seed).standard_normal((n, n))
    m = scale * (a @ a.T) / n
    return 0.5 * (m + m.T)


def random_model(n_d: int, n_species: int = 2, scale: float = 1e-3):
    """Per-species (beta, Sigma), seeds beta_s = 1 + s, Sigma_s = 1 + S + s."""
    beta = np.stack([random_psd(n_d, 1 + s, scale) for s in range(n_species)])
    sigma = np.stack([random_psd(n_d, 1 + n_species + s, scale) for s in range(n_species)])
    return beta, sigma


def maxwell_boltzmann(species, temperature, seed):
    """Velocities in A/fs at `temperature` K with zero centre-of-mass momentum."""
    kb = 8.617333262e-5          # eV/K
    kappa = 9.648533212e-3       # (eV/amu) -> A^2/fs^2
    m = MASS[species]
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((len(species), 3)) * np.sqrt(kb * temperature * kappa / m)[:, None]
    p = (m[:, None] * v).sum(0)
    v -= p / m.sum()
    return v
