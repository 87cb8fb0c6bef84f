"""HIP path vs the FP64 oracle through the C ABI: neighbour lists bit-exact, descriptors,
energies, variances, uncertainties and forces within the FP32 bound."""
import math

import numpy as np
import pytest
import torch

from oracle import evaluate as oev, neighbors as onl
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import structures as S

from .gpu_util import TOL, gpu_eval, rel_max, rel_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    return S.random_model(DEFAULT.n_desc)


def _list_equal(res, pos, box, r_list, rows=None):
    off, j, s = res["ev"].export_list()
    if rows is None:
        i0, j0, s0 = onl.brute_force(pos, box, r_list)
        n = len(pos)
        off0 = np.concatenate([[0], np.cumsum(np.bincount(i0, minlength=n))])
        np.testing.assert_array_equal(off, off0)
        np.testing.assert_array_equal(j, j0)
        np.testing.assert_array_equal(s, s0)
    else:
        i0, j0, s0 = onl.brute_force_rows(pos, box, r_list, rows)
        for a in rows:
            m = i0 == a
            np.testing.assert_array_equal(j[off[a]:off[a + 1]], j0[m], err_msg=f"atom {a}")
            np.testing.assert_array_equal(s[off[a]:off[a + 1]], s0[m], err_msg=f"atom {a}")


def _compare(res, ref, atoms=None, tol=TOL):
    atoms = np.arange(len(res["e"])) if atoms is None else np.asarray(atoms)
    rows = ref.row_of(atoms)
    errs = {
        "e": rel_max(res["e"][atoms], ref.e[rows]),
        "sigma": rel_max(res["sigma"][atoms], ref.sigma[rows]),
        "var": rel_max(res["var"][atoms], ref.v[rows]),
        "f": rel_vec(res["f"][atoms], ref.f),
        "norm": rel_max(res["norm"][atoms], ref.norm[rows]),
    }
    for k, v in errs.items():
        assert v <= tol, (k, v, errs)
    return errs


def test_tiny_cell_list_descriptors_energy_forces(model):
    beta, sigma = model
    st = S.config_tiny()
    print("case: tiny cell, 80 atoms", flush=True)
    res = gpu_eval(st.pos, st.species, st.box, beta, sigma, want_d=True)
    assert res["status"] == 0
    _list_equal(res, st.pos, st.box, 4.7)
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    assert np.abs(res["d"] - ref.d).max() <= 1e-6
    _compare(res, ref)
    assert abs(res["E"][0] - ref.energy) <= TOL * abs(ref.energy)
    np.testing.assert_allclose(res["var2"], res["var"], rtol=1e-6, atol=0)
    assert abs(res["sigma_max"][0] - ref.sigma.max()) <= TOL * ref.sigma.max()
    # net force vanishes (translation invariance) to FP32 rounding of the pair terms
    assert np.abs(res["f"].sum(0)).max() <= 1e-6 * np.abs(res["f"]).sum(0).max()


def test_small_box_repeated_images(model):
    # Ly = 4.8 A < 2 r_list: the same neighbour appears with several image shifts
    beta, sigma = model
    st = S.h2_over_pt111(3, 2, 3, vacuum=8.0, n_mol=2, seed=1)
    print("case: small box 3x2x3", flush=True)
    res = gpu_eval(st.pos, st.species, st.box, beta, sigma)
    _list_equal(res, st.pos, st.box, 4.7)
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    _compare(res, ref)


def test_tiny_box_below_list_radius(model):
    # a box side shorter than r_list (2.9 A < 4.7 A): stencil wider than one bin
    beta, sigma = model
    rng = np.random.default_rng(4)
    box = np.array([2.9, 6.0, 7.5])
    pos = rng.uniform(0, 1, (5, 3)) * box
    species = np.array([1, 0, 1, 0, 0], np.int32)
    print("case: box below list radius", flush=True)
    res = gpu_eval(pos, species, box, beta, sigma)
    _list_equal(res, pos, box, 4.7)
    ref = oev.evaluate(pos, species, box, beta, sigma)
    _compare(res, ref)


def test_list_radius_decisions_in_a_tall_box(model):
    # pairs placed at the list radius to within 1e-15 .. 1e-4 relative, in a cell 1000 A tall
    # (large coordinates: the largest FP32 rounding of positions, which the search's first
    # test works with), some reaching across the periodic faces: every decision must be the
    # FP64 one, as the oracle takes it
    beta, sigma = model
    rng = np.random.default_rng(31)
    box = np.array([24.0, 21.0, 1000.0])
    deltas = [0.0] + [sg * 10.0 ** -e for e in (15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4) for sg in (1, -1)]
    a = rng.uniform(0, 1, (3 * len(deltas), 3)) * box
    u = rng.standard_normal(a.shape)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    d = np.tile(deltas, 3)
    b = a + (4.7 * (1.0 + d))[:, None] * u
    pos = np.concatenate([a, b])
    species = rng.integers(0, 2, len(pos)).astype(np.int32)
    print(f"case: {len(a)} pairs at the list radius, 1000 A cell", flush=True)
    res = gpu_eval(pos, species, box, beta, sigma)
    _list_equal(res, pos, box, 4.7)


def test_batch_of_cells(model):
    beta, sigma = model
    b = S.config_cells(n_cells=12, seed=2)
    print("case: 12 cells", flush=True)
    res = gpu_eval(b.pos, b.species, b.boxes, beta, sigma, offsets=b.offsets)
    off, j, s = res["ev"].export_list()
    for k in range(12):
        st = b.structure(k)
        lo, hi = b.offsets[k], b.offsets[k + 1]
        i0, j0, s0 = onl.brute_force(st.pos, st.box, 4.7)
        np.testing.assert_array_equal(j[off[lo]:off[hi]], j0 + lo)
        np.testing.assert_array_equal(s[off[lo]:off[hi]], s0)
        ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
        sub = {key: (res[key][lo:hi] if isinstance(res[key], np.ndarray) and res[key].ndim >= 1
                     and len(res[key]) == len(b.species) else res[key]) for key in res}
        _compare(sub, ref)
        assert abs(res["E"][k] - ref.energy) <= TOL * abs(ref.energy)


def test_lists_of_all_256_cells(model):
    """The list of the 256-cell batch (the differentiation workload), every cell entirely,
    against brute force: offsets, neighbours, image shifts and order."""
    from paper_2204_12573_amd import engine
    beta, sigma = model
    b = S.config_cells(n_cells=256, seed=0)
    print(f"case: lists of 256 cells, {b.n} atoms", flush=True)
    ev = engine.Evaluator(engine.Model(beta, sigma), max_atoms=b.n, max_pairs=64 * b.n)
    p, s = engine.to_device(b.pos, b.species)
    ev.neighbors(p, s, b.offsets, b.boxes, 0.2)
    off, j, sh = ev.export_list()
    assert ev.status() == 0
    for k in range(256):
        st = b.structure(k)
        lo, hi = b.offsets[k], b.offsets[k + 1]
        i0, j0, s0 = onl.brute_force(st.pos, st.box, 4.7)
        off0 = np.concatenate([[0], np.cumsum(np.bincount(i0, minlength=st.n))])
        np.testing.assert_array_equal(off[lo:hi + 1] - off[lo], off0, err_msg=f"cell {k}")
        np.testing.assert_array_equal(j[off[lo]:off[hi]], j0 + lo, err_msg=f"cell {k}")
        np.testing.assert_array_equal(sh[off[lo]:off[hi]], s0, err_msg=f"cell {k}")


def test_isolated_atom_and_empty_environment(model):
    beta, sigma = model
    box = np.array([30.0, 30.0, 30.0])
    pos = np.array([[5.0, 5, 5], [6.0, 5, 5], [20.0, 20, 20], [15.0, 15.0, 9.55]])
    species = np.array([1, 0, 1, 0], np.int32)   # atom 3 has a neighbour only beyond r_c
    pos[3] = pos[2] + np.array([0.0, 0.0, -4.6])
    print("case: isolated atoms", flush=True)
    res = gpu_eval(pos, species, box, beta, sigma)
    ref = oev.evaluate(pos, species, box, beta, sigma)
    _compare(res, ref)
    assert res["e"][2] == 0.0 and res["e"][3] == 0.0
    assert np.all(res["f"][2:] == 0.0)


def test_empty_system_and_empty_cell(model):
    """No atoms at all, and an empty cell between two copies of the 80-atom cell: the
    empty parts give zero energy and raise no flag, the copies give the same bits as each
    other and the oracle's values."""
    from paper_2204_12573_amd import engine
    beta, sigma = model
    print("case: empty system", flush=True)
    m = engine.Model(beta, sigma)
    ev = engine.Evaluator(m, max_atoms=16, max_pairs=1024)
    p, s = engine.to_device(np.zeros((0, 3)), np.zeros(0, np.int32))
    ev.neighbors(p, s, [0, 0], np.array([10.0, 10.0, 10.0]), 0.2)
    ev.descriptors(p)
    out = ev.energy_forces(want_var=True)
    torch.cuda.synchronize()
    assert out["E"].cpu().numpy()[0] == 0.0
    assert ev.status() == 0
    print("case: empty cell inside a batch", flush=True)
    st = S.config_tiny()
    pos = np.concatenate([st.pos, st.pos])
    sp = np.concatenate([st.species, st.species])
    offsets = np.array([0, st.n, st.n, 2 * st.n], np.int32)
    boxes = np.stack([st.box, np.array([12.0, 12.0, 12.0]), st.box])
    res = gpu_eval(pos, sp, boxes, beta, sigma, offsets=offsets)
    assert res["status"] == 0
    assert res["E"][1] == 0.0 and res["E"][0] == res["E"][2]
    for key in ["e", "f", "var", "sigma"]:
        np.testing.assert_array_equal(res[key][:st.n], res[key][st.n:], err_msg=key)
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    _compare({k: (v[:st.n] if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == 2 * st.n else v)
              for k, v in res.items()}, ref)
    assert abs(res["E"][0] - ref.energy) <= TOL * abs(ref.energy)


def test_error_paths(model):
    from paper_2204_12573_amd import binding as Bd, engine
    beta, sigma = model
    st = S.config_tiny()
    m = engine.Model(beta, sigma)
    ev = engine.Evaluator(m, max_atoms=st.n, max_pairs=100)
    p, s = engine.to_device(st.pos, st.species)
    with pytest.raises(Bd.FlareError) as e:
        ev.descriptors(p)
    assert e.value.code == Bd.E_STALE
    with pytest.raises(Bd.FlareError) as e:
        ev.neighbors(p, s, [0, st.n], st.box, 0.2)
    assert e.value.code == Bd.E_CAPACITY
    ev2 = engine.Evaluator(m, max_atoms=st.n, max_pairs=10 * st.n * 64)
    bad = s.clone()
    bad[3] = 7
    with pytest.raises(Bd.FlareError) as e:
        ev2.neighbors(p, bad, [0, st.n], st.box, 0.2)
    assert e.value.code == Bd.E_SPECIES
    pn = p.clone()
    pn[1, 5] = float("nan")
    with pytest.raises(Bd.FlareError) as e:
        ev2.neighbors(pn, s, [0, st.n], st.box, 0.2)
    assert e.value.code == Bd.E_NONFINITE
    with pytest.raises(Bd.FlareError) as e:
        ev2.neighbors(p, s, [0, st.n], np.array([st.box[0], -1.0, st.box[2]]), 0.2)
    assert e.value.code == Bd.E_BOX
    # a later good call still works, and a large move sets the displacement flag
    ev2.neighbors(p, s, [0, st.n], st.box, 0.2)
    ev2.descriptors(p)
    assert ev2.status() == 0
    p2 = p.clone()
    p2[0, 0] += 0.15
    ev2.descriptors(p2)
    assert ev2.status() & Bd.FLAG_DISPLACED


def test_alone_and_in_batch_are_bitwise_equal(model):
    # per-row arithmetic never mixes rows and forces are gathered in list order, so a
    # cell gives the same bits alone and inside a batch of other cells
    beta, sigma = model
    b = S.config_cells(n_cells=10, seed=5)
    print("case: batch invariance, 10 cells", flush=True)
    mix = gpu_eval(b.pos, b.species, b.boxes, beta, sigma, offsets=b.offsets)
    for k in [0, 3, 9]:
        st = b.structure(k)
        lo, hi = b.offsets[k], b.offsets[k + 1]
        alone = gpu_eval(st.pos, st.species, st.box, beta, sigma)
        for key in ["e", "f", "var", "sigma"]:
            np.testing.assert_array_equal(alone[key], mix[key][lo:hi], err_msg=f"cell {k} {key}")
        assert alone["E"][0] == mix["E"][k]


def test_repeat_is_bitwise_equal(model):
    beta, sigma = model
    st = S.config_tiny()
    a = gpu_eval(st.pos, st.species, st.box, beta, sigma)
    b = gpu_eval(st.pos, st.species, st.box, beta, sigma)
    for key in ["e", "f", "sigma", "E"]:
        np.testing.assert_array_equal(a[key], b[key])


def _fcc(a, n, rng, jitter):
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.array([[i, j, k] for i in range(n) for j in range(n) for k in range(n)], float)
    pos = ((cells[:, None, :] + base[None, :, :]).reshape(-1, 3)) * a
    return pos + rng.normal(0.0, jitter, pos.shape), np.full(3, n * a)


def test_dense_cells_long_rows(model):
    # compressed fcc cells: 60-80 neighbours per atom, beyond the largest neighbour-count
    # class of the row ordering (63), in a single-species cell (144-wide rows) and a
    # random H/Pt cell (544-wide rows), batched together
    beta, sigma = model
    rng = np.random.default_rng(8)
    p1, b1 = _fcc(2.9, 3, rng, 0.05)
    p2, b2 = _fcc(3.0, 3, rng, 0.05)
    s1 = np.ones(len(p1), np.int32)
    s2 = rng.integers(0, 2, len(p2)).astype(np.int32)
    pos = np.concatenate([S._wrap(p1, b1), S._wrap(p2, b2)])
    species = np.concatenate([s1, s2])
    offsets = np.array([0, len(p1), len(p1) + len(p2)], np.int32)
    print("case: dense fcc cells, 108 + 108 atoms", flush=True)
    res = gpu_eval(pos, species, np.stack([b1, b2]), beta, sigma, offsets=offsets, max_pairs=100 * len(species))
    off, j, s = res["ev"].export_list()
    counts = np.diff(off)
    assert counts[:len(p1)].max() > 63 and counts[len(p1):].max() > 63
    for k, (pk, sk, bk) in enumerate([(p1, s1, b1), (p2, s2, b2)]):
        lo, hi = offsets[k], offsets[k + 1]
        pk = S._wrap(pk, bk)
        i0, j0, s0 = onl.brute_force(pk, bk, 4.7)
        np.testing.assert_array_equal(j[off[lo]:off[hi]], j0 + lo)
        np.testing.assert_array_equal(s[off[lo]:off[hi]], s0)
        ref = oev.evaluate(pk, sk, bk, beta, sigma)
        sub = {key: (res[key][lo:hi] if isinstance(res[key], np.ndarray) and res[key].ndim >= 1
                     and len(res[key]) == len(species) else res[key]) for key in res}
        print(_compare(sub, ref))
        assert abs(res["E"][k] - ref.energy) <= TOL * abs(ref.energy)
