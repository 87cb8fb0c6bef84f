"""Pins for the mapped quadratic forms, the forces and the NVE integrator."""
import math

import numpy as np
import pytest

from oracle import descriptors, evaluate as ev, forces, md, model, neighbors
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import structures as S


@pytest.fixture(scope="module")
def tiny():
    st = S.config_tiny()
    beta, gamma = S.random_model(DEFAULT.n_desc)
    return st, beta, gamma, ev.evaluate(st.pos, st.species, st.box, beta, gamma)


def test_quadratic_forms_closed_forms(tiny):
    st, beta, gamma, res = tiny
    n = DEFAULT.n_desc
    eye = np.stack([np.eye(n), 2 * np.eye(n)])
    e = model.energies(res.d, st.species, eye)
    # |d| = 1 for every atom with neighbours: e = 1 (H) or 2 (Pt)
    np.testing.assert_allclose(e, np.where(st.species == 0, 1.0, 2.0), rtol=1e-13)
    v = np.random.default_rng(1).standard_normal(n)
    rank1 = np.stack([np.outer(v, v)] * 2)
    np.testing.assert_allclose(model.energies(res.d, st.species, rank1), (res.d @ v) ** 2, rtol=1e-12, atol=1e-14)


def test_variance_nonnegative_and_sigma(tiny):
    st, beta, gamma, res = tiny
    assert np.all(res.v > 0)
    np.testing.assert_allclose(res.sigma ** 2, res.v, rtol=1e-14)


def test_energy_gradient_in_dtilde_fd(tiny):
    st, beta, gamma, res = tiny
    rng = np.random.default_rng(2)
    dt = res.d * res.norm[:, None]
    g = model.energy_grad_dtilde(res.d, res.norm, st.species, beta)
    for atom in [0, 70]:
        h = 1e-5 * res.norm[atom]
        for k in rng.choice(DEFAULT.n_desc, 6, replace=False):
            p = dt[atom:atom + 1].copy()
            p[0, k] += h
            ep = model.energies(descriptors.normalise(p)[0], st.species[atom:atom + 1], beta)[0]
            p[0, k] -= 2 * h
            em = model.energies(descriptors.normalise(p)[0], st.species[atom:atom + 1], beta)[0]
            np.testing.assert_allclose(g[atom, k], (ep - em) / (2 * h), rtol=1e-6,
                                       atol=1e-8 * np.abs(g[atom]).max())


def test_forces_match_richardson_fd(tiny):
    st, beta, gamma, res = tiny
    fn = lambda p: ev.total_energy(p, st.species, st.box, beta)
    atoms = [0, 17, 40, 63, 64, 65, 72, 79]
    f1 = forces.forces_fd(fn, st.pos, atoms, step=1e-4)
    f2 = forces.forces_fd(fn, st.pos, atoms, step=5e-5)
    rich = (4 * f2 - f1) / 3
    scale = np.abs(res.f).max()
    assert np.abs(f1 - res.f[atoms]).max() / scale < 1e-6
    assert np.abs(rich - res.f[atoms]).max() / scale < 1e-9


def test_force_sum_is_zero(tiny):
    st, beta, gamma, res = tiny
    assert np.abs(res.f.sum(0)).max() < 1e-15 * len(res.f) + 1e-18
    assert np.abs(res.f).max() > 1e-5


def test_rotation_covariance_of_forces():
    rng = np.random.default_rng(12)
    pos = rng.uniform(-3.0, 3.0, (20, 3))
    keep = [0]
    for k in range(1, len(pos)):
        if np.min(np.linalg.norm(pos[keep] - pos[k], axis=1)) > 1.2:
            keep.append(k)
    pos, species = pos[keep], rng.integers(0, 2, len(keep))
    beta, gamma = S.random_model(DEFAULT.n_desc)
    box = np.array([50.0, 50.0, 50.0])
    a = ev.evaluate(pos + 25, species, box, beta, gamma)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    b = ev.evaluate(pos @ q.T + 25, species, box, beta, gamma)
    np.testing.assert_allclose(b.e, a.e, rtol=1e-11)
    np.testing.assert_allclose(b.f, a.f @ q.T, atol=1e-12 * np.abs(a.f).max() + 1e-16)


def test_subset_evaluation_matches_full(tiny):
    st, beta, gamma, res = tiny
    tg = [3, 50, 66, 77]
    sub = ev.evaluate(st.pos, st.species, st.box, beta, gamma, targets=tg)
    np.testing.assert_allclose(sub.f, res.f[tg], rtol=1e-12, atol=1e-18)
    rows = sub.row_of(tg)
    np.testing.assert_allclose(sub.e[rows], res.e[tg], rtol=1e-13)
    np.testing.assert_allclose(sub.sigma[rows], res.sigma[tg], rtol=1e-13)


def test_energy_is_fsum(tiny):
    st, beta, gamma, res = tiny
    assert res.energy == math.fsum(res.e.tolist())


def _nve(st, beta, v0, n):
    def fn(p):
        r = ev.evaluate(p, st.species, st.box, beta, np.zeros_like(beta))
        return r.energy, r.f
    return md.nve(st.pos, v0, st.species, 0.5, n, fn)


def test_nve_energy_exchange_and_reversibility(tiny):
    # velocity Verlet conserves a shadow energy: the total-energy error is O(dt^2), so
    # halving dt over the same time span divides it by 4, while the potential energy
    # exchanged stays the same. A force inconsistent with the energy breaks both.
    st, beta, gamma, _ = tiny
    v0 = S.maxwell_boltzmann(st.species, 450.0, seed=9)
    ep, ek, x, v = _nve(st, beta, v0, 10)
    ep2, ek2, _, _ = _nve_dt(st, beta, v0, 0.25, 20)
    err1 = np.abs((ep + ek) - (ep[0] + ek[0])).max()
    err2 = np.abs((ep2 + ek2) - (ep2[0] + ek2[0])).max()
    swing = np.abs(ep - ep[0]).max()
    assert swing > 1e-5                                  # energy is actually exchanged
    assert err1 <= 1e-2 * swing
    assert 3.6 < err1 / err2 < 4.4
    # time reversal: run back from (x, -v)
    def fn(p):
        r = ev.evaluate(p, st.species, st.box, beta, np.zeros_like(beta))
        return r.energy, r.f
    _, _, xb, vb = md.nve(x, -v, st.species, 0.5, 10, fn)
    assert np.abs(xb - st.pos).max() < 1e-10
    assert np.abs(vb + v0).max() < 1e-10


def _nve_dt(st, beta, v0, dt, n):
    def fn(p):
        r = ev.evaluate(p, st.species, st.box, beta, np.zeros_like(beta))
        return r.energy, r.f
    return md.nve(st.pos, v0, st.species, dt, n, fn)


def test_virial_diagonal_matches_strain_fd(tiny):
    """W_aa = -dE/deps_aa: central differences of a uniaxial strain of the periodic cell
    (positions and box together), Richardson-extrapolated."""
    st, beta, gamma, _ = tiny
    res = ev.evaluate(st.pos, st.species, st.box, beta, gamma, want_virial=True)
    fn = lambda p, b: ev.total_energy(p, st.species, b, beta)
    scale = np.abs(res.virial).max()
    assert scale > 1e-4
    for axis in range(3):
        w1 = forces.virial_fd(fn, st.pos, st.box, axis, step=2e-5)
        w2 = forces.virial_fd(fn, st.pos, st.box, axis, step=1e-5)
        rich = (4 * w2 - w1) / 3
        assert abs(rich - res.virial[axis, axis]) / scale < 1e-8


def test_virial_free_cluster_is_sum_r_times_f():
    """A cluster far from its periodic images: W_ab = sum_i r_i,a F_i,b with F from
    central differences of the energy (a route that never forms h_p), and W symmetric."""
    st = S.config_tiny()
    beta, gamma = S.random_model(DEFAULT.n_desc)
    centre = st.pos[70]
    sel = np.nonzero(np.linalg.norm(st.pos - centre, axis=1) < 5.0)[0]
    box = np.array([40.0, 40.0, 40.0])
    pos = st.pos[sel] - centre + box / 2
    sp = st.species[sel]
    assert len(sel) >= 6 and len(set(sp.tolist())) == 2
    res = ev.evaluate(pos, sp, box, beta, gamma, want_virial=True)
    fn = lambda p: ev.total_energy(p, sp, box, beta)
    f = forces.forces_fd(fn, pos, step=1e-5)
    w_fd = (pos - box / 2).T @ f
    scale = np.abs(res.virial).max()
    assert scale > 1e-4
    assert np.abs(res.virial - w_fd).max() / scale < 1e-7
    assert np.abs(res.virial - res.virial.T).max() / scale < 1e-12


def test_virial_symmetric_periodic(tiny):
    st, beta, gamma, _ = tiny
    w = ev.evaluate(st.pos, st.species, st.box, beta, gamma, want_virial=True).virial
    assert np.abs(w - w.T).max() < 1e-12 * np.abs(w).max()
