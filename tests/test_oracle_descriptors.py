"""Pins for densities and B2: paper's dimensions, Legendre route, dimer closed form,
species blocks and invariances."""
import math
import os

import numpy as np
from scipy import special

from oracle import descriptors, neighbors
from oracle.hyper import DEFAULT, Hyper
from paper_2204_12573_amd import structures as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_dimensions_match_paper():
    rows = np.loadtxt(os.path.join(GOLDEN, "descriptor_dims.txt"), ndmin=2)
    for ns, nr, lm, full, single in rows.astype(int):
        h = Hyper(n_species=ns, n_rad=nr, l_max=lm)
        assert h.n_desc == full
        assert h.block_slice(0, 0).stop - h.block_slice(0, 0).start == single
    assert DEFAULT.n_desc == 544
    assert DEFAULT.block_slice(0, 0) == slice(0, 144)
    assert DEFAULT.block_slice(1, 1) == slice(400, 544)
    assert DEFAULT.block_slice(0, 1) == slice(144, 400)


def _env(pos, species, box, h=DEFAULT):
    i, j, s = neighbors.brute_force(pos, box, h.r_cut)
    d = neighbors.pair_vectors(pos, box, i, j, s)
    return i, j, d


def _cheb_cos(x, n):
    return math.cos(n * math.acos(x))


def test_dimer_closed_form():
    # one neighbour at distance r along a random direction: sum_m Y_lm Y_lm = (2l+1)/4pi,
    # so d~_{(a,b),l} = R_a(r) R_b(r) (2l+1)/(4 pi) with R_{(s,n)} = 0 unless s = s_j
    h = DEFAULT
    box = np.array([40.0, 40.0, 40.0])
    r = 2.3
    u = np.array([0.36, -0.48, 0.8])
    for sj in (0, 1):
        pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0] + r * u])
        species = np.array([1, sj])
        i, j, d = _env(pos, species, box)
        c = descriptors.densities(2, species, i, j, d, h)
        dt = descriptors.b2(c, h)[0]
        x = 2 * r / h.r_cut - 1
        rad = np.zeros(h.n_channels)
        for n in range(h.n_rad):
            rad[sj * h.n_rad + n] = _cheb_cos(x, n) * (h.r_cut - r) ** 2
        want = np.array([rad[a] * rad[b] * (2 * l + 1) / (4 * math.pi)
                         for a, b in h.pairs() for l in range(h.l_max + 1)])
        np.testing.assert_allclose(dt, want, rtol=1e-12, atol=1e-14)


def test_b2_by_legendre_route():
    # d~_{(a,b),l} = sum_{j,k} R_a(r_j) R_b(r_k) (2l+1)/(4pi) P_l(u_j . u_k): no spherical
    # harmonics and no densities involved
    h = DEFAULT
    st = S.config_tiny()
    i, j, d = _env(st.pos, st.species, st.box)
    c = descriptors.densities(st.n, st.species, i, j, d, h)
    dt = descriptors.b2(c, h)
    for atom in [0, 20, 63, 64, 71]:
        m = i == atom
        dd = d[m]
        r = np.linalg.norm(dd, axis=1)
        u = dd / r[:, None]
        sj = st.species[j[m]]
        x = 2 * r / h.r_cut - 1
        w = np.zeros((len(r), h.n_channels))
        for p in range(len(r)):
            for n in range(h.n_rad):
                w[p, sj[p] * h.n_rad + n] = _cheb_cos(x[p], n) * (h.r_cut - r[p]) ** 2
        cosm = np.clip(u @ u.T, -1, 1)
        want = []
        for a, b in h.pairs():
            for l in range(h.l_max + 1):
                pl = special.eval_legendre(l, cosm)
                want.append((2 * l + 1) / (4 * math.pi) * (w[:, a][:, None] * w[:, b][None, :] * pl).sum())
        np.testing.assert_allclose(dt[atom], want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_single_species_blocks_are_exact():
    h = DEFAULT
    st = S.config_tiny()
    i, j, d = _env(st.pos, st.species, st.box)
    dt = descriptors.b2(descriptors.densities(st.n, st.species, i, j, d, h), h)
    r = np.linalg.norm(d, axis=1)
    seen = np.zeros((st.n, 2), bool)
    seen[i[r < h.r_cut], st.species[j[r < h.r_cut]]] = True
    only_h = seen[:, 0] & ~seen[:, 1]
    only_pt = seen[:, 1] & ~seen[:, 0]
    assert only_h.any() and only_pt.any()
    hh, pp = h.block_slice(0, 0), h.block_slice(1, 1)
    assert np.all(dt[only_h][:, hh.stop:] == 0.0)
    assert np.all(dt[only_pt][:, :pp.start] == 0.0)
    assert np.all(np.abs(dt[only_h][:, hh]).sum(1) > 0)


def _cluster(seed=11):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-3.5, 3.5, (24, 3))
    keep = [0]
    for k in range(1, len(pos)):
        if np.min(np.linalg.norm(pos[keep] - pos[k], axis=1)) > 1.2:
            keep.append(k)
    pos = pos[keep]
    species = rng.integers(0, 2, len(pos))
    return pos, species


def _desc(pos, species, box):
    h = DEFAULT
    i, j, d = _env(pos, species, box)
    return descriptors.normalise(descriptors.b2(descriptors.densities(len(pos), species, i, j, d, h), h))[0]


def test_rotation_translation_permutation_invariance():
    pos, species = _cluster()
    box = np.array([60.0, 60.0, 60.0])
    base = _desc(pos + 30.0, species, box)
    q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    rot = _desc(pos @ q.T + 30.0, species, box)
    np.testing.assert_allclose(rot, base, atol=1e-12)
    tr = _desc(pos + np.array([31.7, 22.1, 40.3]), species, box)
    np.testing.assert_allclose(tr, base, atol=1e-12)
    perm = np.random.default_rng(4).permutation(len(pos))
    pm = _desc(pos[perm] + 30.0, species[perm], box)
    np.testing.assert_allclose(pm, base[perm], atol=1e-12)


def test_species_channel_assignment():
    # the H neighbour feeds only H channels, the Pt neighbour only Pt channels
    h = DEFAULT
    box = np.array([40.0, 40.0, 40.0])
    pos = np.array([[10.0, 10, 10], [11.5, 10, 10], [10, 12.0, 10]])
    species = np.array([1, 0, 1])
    i, j, d = _env(pos, species, box)
    c = descriptors.densities(3, species, i, j, d, h)[0]
    x_h = 2 * 1.5 / h.r_cut - 1
    x_pt = 2 * 2.0 / h.r_cut - 1
    y00 = 0.5 / math.sqrt(math.pi)
    for n in range(h.n_rad):
        np.testing.assert_allclose(c[n, 0], _cheb_cos(x_h, n) * (h.r_cut - 1.5) ** 2 * y00, atol=1e-13)
        np.testing.assert_allclose(c[h.n_rad + n, 0], _cheb_cos(x_pt, n) * (h.r_cut - 2.0) ** 2 * y00, atol=1e-13)
