"""Neighbour lists by definition: every periodic image within the list radius.

The local environment of atom i is every atom (and periodic image) closer than the
cutoff (Section V.B). A list entry is (i, j, sx, sy, sz): atom j shifted by the
integer image vector s, kept when |w_j - w_i + s*L|^2 < r^2 (strict), excluding
(i, i, 0). w = x - L*floor(x/L) is the wrapped position. The squared distance is
dx*dx + dy*dy + dz*dz evaluated left to right in FP64 with no fused multiply-add
(numpy never fuses), so an integer-exact comparison with another implementation of
the same expression is meaningful. Canonical order per atom: (j, sx, sy, sz).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree


def wrap(pos, box):
    pos = np.asarray(pos, np.float64)
    box = np.asarray(box, np.float64)
    return pos - box * np.floor(pos / box)


def _sq(dx, dy, dz):
    return dx * dx + dy * dy + dz * dz


def _canonical(i, j, s):
    order = np.lexsort((s[:, 2], s[:, 1], s[:, 0], j, i))
    return i[order].astype(np.int64), j[order].astype(np.int64), s[order].astype(np.int64)


def brute_force(pos, box, r):
    """O(N^2 * images) search over every image within reach. Any orthorhombic box.

    Returns (i, j, shifts[P, 3]) in canonical order.
    """
    w = wrap(pos, box)
    box = np.asarray(box, np.float64)
    r2 = r * r
    k = [int(math.ceil(r / box[a])) + 1 for a in range(3)]
    n = len(w)
    ii, jj, ss = [], [], []
    base = [w[None, :, a] - w[:, None, a] for a in range(3)]     # [i, j] = w_j - w_i
    for sx in range(-k[0], k[0] + 1):
        dx = base[0] + sx * box[0]
        for sy in range(-k[1], k[1] + 1):
            dy = base[1] + sy * box[1]
            for sz in range(-k[2], k[2] + 1):
                dz = base[2] + sz * box[2]
                m = _sq(dx, dy, dz) < r2
                if sx == 0 and sy == 0 and sz == 0:
                    m[np.arange(n), np.arange(n)] = False
                a, b = np.nonzero(m)
                if len(a):
                    ii.append(a)
                    jj.append(b)
                    ss.append(np.tile([sx, sy, sz], (len(a), 1)))
    if not ii:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros((0, 3), np.int64)
    return _canonical(np.concatenate(ii), np.concatenate(jj), np.concatenate(ss))


def brute_force_rows(pos, box, r, rows):
    """Brute force over all j for the atoms in `rows` only (same rule, same order).

    Per axis only the images that can come within r are kept, so a large box costs
    a few vector passes over all atoms per row.
    """
    w = wrap(pos, box)
    box = np.asarray(box, np.float64)
    r2 = r * r
    k = [int(math.ceil(r / box[a])) + 1 for a in range(3)]
    out_i, out_j, out_s = [], [], []
    for i in np.asarray(rows, np.int64):
        d0 = w - w[i]
        cand = []
        for a in range(3):
            svals = np.arange(-k[a], k[a] + 1)
            ok = np.abs(d0[:, a][None, :] + svals[:, None] * box[a]) < r       # [S, N]
            cand.append((svals, ok))
        anyok = cand[0][1].any(0) & cand[1][1].any(0) & cand[2][1].any(0)
        js = np.nonzero(anyok)[0]
        for j in js:
            for sx in cand[0][0][cand[0][1][:, j]]:
                dx = (w[j, 0] - w[i, 0]) + sx * box[0]
                for sy in cand[1][0][cand[1][1][:, j]]:
                    dy = (w[j, 1] - w[i, 1]) + sy * box[1]
                    for sz in cand[2][0][cand[2][1][:, j]]:
                        if j == i and sx == 0 and sy == 0 and sz == 0:
                            continue
                        dz = (w[j, 2] - w[i, 2]) + sz * box[2]
                        if _sq(dx, dy, dz) < r2:
                            out_i.append(i)
                            out_j.append(j)
                            out_s.append((sx, sy, sz))
    if not out_i:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros((0, 3), np.int64)
    return _canonical(np.array(out_i), np.array(out_j), np.array(out_s).reshape(-1, 3))


def kdtree(pos, box, r, rows=None):
    """Same list via a periodic k-d tree prefilter, for boxes wider than 2r per axis.

    The tree only proposes candidates (radius r plus a margin); each candidate is
    then kept or dropped by the exact rule. With L > 2r at most one image per axis
    can be within r, namely s = -round((w_j - w_i) / L).
    """
    box = np.asarray(box, np.float64)
    if np.any(box <= 2.0 * r):
        raise ValueError("kdtree neighbour search needs every box side > 2r")
    w = wrap(pos, box)
    wt = np.where(w >= box, w - box, w)          # the tree wants [0, L); exact test uses w
    tree = cKDTree(wt, boxsize=box)
    rows = np.arange(len(w)) if rows is None else np.asarray(rows, np.int64)
    cands = tree.query_ball_point(wt[rows], r + 1e-6)
    cnt = np.array([len(c) for c in cands])
    i = np.repeat(rows, cnt)
    j = np.concatenate([np.asarray(c, np.int64) for c in cands]) if len(cands) else np.zeros(0, np.int64)
    d0 = w[j] - w[i]
    s = -np.round(d0 / box).astype(np.int64)
    dx = (w[j, 0] - w[i, 0]) + s[:, 0] * box[0]
    dy = (w[j, 1] - w[i, 1]) + s[:, 1] * box[1]
    dz = (w[j, 2] - w[i, 2]) + s[:, 2] * box[2]
    keep = (_sq(dx, dy, dz) < r * r) & ~((i == j) & (s == 0).all(1))
    return _canonical(i[keep], j[keep], s[keep])


def neighbor_list(pos, box, r, rows=None):
    """Exact list at radius r: k-d tree route for wide boxes, brute force otherwise."""
    box = np.asarray(box, np.float64)
    if np.all(box > 2.0 * r):
        return kdtree(pos, box, r, rows)
    if rows is None:
        return brute_force(pos, box, r)
    return brute_force_rows(pos, box, r, rows)


def pair_vectors(pos, box, i, j, s):
    """Delta_ij = (w_j - w_i) + s*L for each list entry, FP64 [P, 3]."""
    w = wrap(pos, box)
    box = np.asarray(box, np.float64)
    return (w[j] - w[i]) + s * box
