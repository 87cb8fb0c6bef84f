"""Pins for the oracle's neighbour lists: lattice counts, symmetry, two routes agree."""
import numpy as np
import pytest

from oracle import neighbors
from paper_2204_12573_amd import structures as S


def _as_set(i, j, s):
    return set(zip(i.tolist(), j.tolist(), map(tuple, s.tolist())))


def test_simple_cubic_single_atom_counts():
    # one atom in a cube of side a: the list is every lattice vector a*s, s != 0, with
    # |a s| < r. Number of integer vectors with |s|^2 = n is r3(n): 6, 12, 8, 6, 24, 24
    # for n = 1..6 (sums of three squares).
    pos = np.array([[0.3, 0.7, 1.1]])
    r3 = {1: 6, 2: 12, 3: 8, 4: 6, 5: 24, 6: 24}
    for a, r in [(2.0, 4.7), (1.9, 4.0), (3.0, 4.7)]:
        i, j, s = neighbors.brute_force(pos, [a, a, a], r)
        want = sum(v for n, v in r3.items() if n * a * a < r * r)
        assert len(i) == want
        assert np.all((s * s).sum(1) * a * a < r * r)


def test_fcc_bulk_shell_counts():
    # perfect fcc, ABC stacking periodic along z (layers multiple of 3):
    # 12 neighbours at a/sqrt2 = 2.772, 6 at a = 3.92, next shell at 4.801
    pt, (lx, ly), _ = S.pt111_slab(6, 6, 6)
    box = np.array([lx, ly, 6 * S.DZ])
    for r, want in [(3.0, 12), (4.7, 18)]:
        i, j, s = neighbors.brute_force(pt, box, r)
        assert np.all(np.bincount(i, minlength=len(pt)) == want)


def test_list_is_symmetric_and_canonical():
    st = S.config_tiny()
    i, j, s = neighbors.brute_force(st.pos, st.box, 4.7)
    fwd = _as_set(i, j, s)
    rev = _as_set(j, i, -s)
    assert fwd == rev
    key = np.stack([i, j, s[:, 0], s[:, 1], s[:, 2]], 1)
    assert np.all(np.diff(np.lexsort(key.T[::-1])) > 0)   # already sorted
    assert not np.any((i == j) & (s == 0).all(1))


def test_small_box_has_repeated_images():
    # Ly = 4.8 A < 2 * 4.7: atoms see several images of the same neighbour (and of
    # themselves), each with its own shift
    st = S.h2_over_pt111(3, 2, 3, vacuum=8.0, n_mol=2, seed=1)
    i5, j5, s5 = neighbors.brute_force(st.pos, st.box, 5.0)
    assert np.any((i5 == j5) & (s5 != 0).any(1))
    i, j, s = neighbors.brute_force(st.pos, st.box, 4.7)
    pairs = set()
    dup = 0
    for a, b in zip(i.tolist(), j.tolist()):
        if (a, b) in pairs:
            dup += 1
        pairs.add((a, b))
    assert dup > 0


def test_kdtree_route_matches_brute_force():
    st = S.h2_over_pt111(8, 8, 4, vacuum=12.0, jitter=0.05, seed=3)
    assert np.all(st.box > 9.4)
    a = neighbors.brute_force(st.pos, st.box, 4.7)
    b = neighbors.kdtree(st.pos, st.box, 4.7)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_rows_route_matches_brute_force():
    st = S.config_tiny()
    rows = [0, 5, 64, 79]
    i, j, s = neighbors.brute_force(st.pos, st.box, 4.7)
    m = np.isin(i, rows)
    i2, j2, s2 = neighbors.brute_force_rows(st.pos, st.box, 4.7, rows)
    np.testing.assert_array_equal(i[m], i2)
    np.testing.assert_array_equal(j[m], j2)
    np.testing.assert_array_equal(s[m], s2)


def test_wrap_range_and_pair_vectors():
    st = S.config_tiny()
    shifted = st.pos + np.array([3, -2, 5]) * st.box
    w = neighbors.wrap(shifted, st.box)
    assert np.all(w >= 0) and np.all(w <= st.box)
    np.testing.assert_allclose(w, st.pos, atol=1e-12)
    i, j, s = neighbors.brute_force(st.pos, st.box, 4.7)
    d = neighbors.pair_vectors(st.pos, st.box, i, j, s)
    assert np.all(np.sqrt((d * d).sum(1)) < 4.7)
