"""Pins of the oracle's production-run pieces (Section VI.A): the Nose-Hoover NVT
integrator and the hydrogen coordination / reaction-event counts.

NVT: with an infinite damping time the thermostat never moves and the integrator is the
velocity-Verlet NVE integrator, bit for bit; on a harmonic system the extended energy H'
is conserved to O(dt^2) (halving dt quarters the drift); a system started hotter than the
target cools towards it (the thermostat force has the right sign). Coordination:
hand-placed atoms with known answers, including a pair across a periodic face and pairs
just inside and just outside 1 A."""
import numpy as np

from oracle import md as omd


def _harmonic(k_spring, x0):
    # E = sum k/2 |x - x0|^2 (independent oscillators), F = -k (x - x0)
    def fn(x):
        d = x - x0
        return 0.5 * k_spring * float((d * d).sum()), -k_spring * d
    return fn


def _setup(n=12, seed=0):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, 10.0, (n, 3))
    species = np.array([i % 2 for i in range(n)], np.int32)
    v0 = rng.standard_normal((n, 3)) * 0.01
    return x0, species, v0


def test_nvt_without_coupling_is_nve():
    x0, species, v0 = _setup()
    fn = _harmonic(0.5, x0)
    xs = x0 + 0.05
    ep, ek, xn, vn = omd.nve(xs, v0, species, 0.5, 25, fn)
    rec, xt, vt = omd.nvt(xs, v0, species, 0.5, 25, fn, t0=450.0, tau=np.inf)
    np.testing.assert_array_equal(xt, xn)
    np.testing.assert_array_equal(vt, vn)
    np.testing.assert_array_equal(rec[:, 0], ep)
    assert np.all(rec[:, 2] == 0.0)


def test_nvt_extended_energy_second_order():
    x0, species, v0 = _setup(seed=1)
    fn = _harmonic(2.0, x0)
    xs = x0 + 0.1
    drift = []
    for dt in (0.2, 0.1):
        n = int(round(40.0 / dt))
        rec, _, _ = omd.nvt(xs, v0, species, dt, n, fn, t0=300.0, tau=5.0)
        h = omd.extended_energy(rec, len(species), 300.0, 5.0)
        drift.append(np.abs(h - h[0]).max())
        assert np.abs(rec[:, 2]).max() > 1e-3          # the thermostat is active
    ratio = drift[0] / drift[1]
    assert 3.0 < ratio < 5.5, (drift, ratio)


def test_nvt_cools_towards_target():
    x0, species, v0 = _setup(n=30, seed=2)
    fn = _harmonic(1.0, x0)
    m = omd.masses(species)
    v_hot = v0 * 10.0
    rec, _, _ = omd.nvt(x0, v_hot, species, 0.5, 400, fn, t0=100.0, tau=10.0)
    nf = omd.n_free(len(species))
    t_inst = 2.0 * rec[:, 1] / (nf * omd.KB)
    assert t_inst[0] > 400.0
    assert rec[1, 2] > 0.0                         # zeta grows while too hot
    assert t_inst[-100:].mean() < 0.5 * t_inst[0]


def test_coordination_hand_placed():
    box = np.array([12.0, 12.0, 12.0])
    pos = np.array([
        [1.0, 1.0, 1.0], [1.74, 1.0, 1.0],          # H2 at 0.74 A: both 1
        [5.0, 5.0, 5.0],                             # isolated H: 0
        [8.0, 8.0, 8.0], [8.0, 8.0, 9.001],          # H-H at 1.001 A: 0
        [11.8, 3.0, 3.0], [0.3, 3.0, 3.0],           # across the x face, 0.5 A: 1
        [3.0, 9.0, 3.0], [3.0, 9.0, 3.9],            # H-Pt at 0.9 A: 0 (Pt reported 0)
        [6.0, 1.0, 9.0], [6.0, 1.0, 9.9995],         # H-H at 0.9995 A: 1
    ])
    species = np.array([0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0], np.int32)
    c = omd.coordination(pos, species, box)
    np.testing.assert_array_equal(c, [1, 1, 0, 0, 0, 1, 1, 0, 0, 1, 1])
    assert omd.reaction_events([1, 1, 0, 0, 1], [0, 1, 1, 0, 0]) == (2, 1)
