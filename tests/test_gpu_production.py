"""Production-run pieces on the GPU (Section VI.A) against the oracle: Nose-Hoover NVT
trajectories, per-cell thermostat independence, hydrogen coordination numbers and the
reaction events between snapshots, and the uncertainty monitor."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev, md as omd
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, engine, structures as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    return S.random_model(DEFAULT.n_desc)


def _nvt(beta, sigma, pos, species, offsets, boxes, v0, n_steps, t0, tau, dt, skin=0.4):
    """NVT on the GPU, list rebuilt every 5 steps. The default skin of 0.4 A keeps every
    atom of the seeded starts used here within half the skin of its list-build position
    (fastest atom: 0.070 A/fs at 700 K, 0.067 A/fs at 450 K, i.e. < 0.18 A in 2.5 fs), so
    no interval raises FLARE_FLAG_DISPLACED."""
    m = engine.Model(beta, sigma)
    n = len(species)
    ev = engine.Evaluator(m, max_atoms=n, max_pairs=64 * n)
    p, s = engine.to_device(pos, species)
    v = torch.from_numpy(np.ascontiguousarray(v0.T)).cuda()
    md = engine.NVT(ev, p, v, s, offsets, boxes, t_target=t0, tau=tau, dt=dt, skin=skin, rebuild=5)
    epot = [md.out["E"].cpu().numpy().copy()]
    for _ in range(n_steps):
        out = md.step()
        epot.append(out["E"].cpu().numpy().copy())
    torch.cuda.synchronize()
    return p.cpu().numpy().T, v.cpu().numpy().T, md.thermo.cpu().numpy(), np.array(epot), ev


def test_nvt_matches_oracle(model):
    beta, sigma = model
    st = S.config_tiny()
    v0 = S.maxwell_boltzmann(st.species, 700.0, seed=4)
    t0, tau, dt, n = 450.0, 10.0, 0.5, 10
    print("case: tiny NVT 10 steps", flush=True)

    def fn(x):
        r = oev.evaluate(x, st.species, st.box, beta, sigma)
        return r.energy, r.f

    rec, x_ref, v_ref = omd.nvt(st.pos, v0, st.species, dt, n, fn, t0, tau)
    x, v, thermo, epot, ev = _nvt(beta, sigma, st.pos, st.species, [0, st.n], st.box, v0, n, t0, tau, dt)
    print("max |dx|", np.abs(x - x_ref).max(), "zeta", thermo[0, 0], rec[-1, 2], "K", thermo[0, 2], rec[-1, 1])
    assert np.abs(x - x_ref).max() < 1e-7
    np.testing.assert_allclose(epot[:, 0], rec[:, 0], rtol=1e-5)
    assert abs(thermo[0, 2] - rec[-1, 1]) <= 1e-6 * rec[-1, 1]
    assert abs(thermo[0, 0] - rec[-1, 2]) <= 1e-6 * abs(rec[-1, 2])
    assert abs(thermo[0, 1] - rec[-1, 3]) <= 1e-6 * abs(rec[-1, 3])
    assert rec[-1, 2] > 0.0                      # started hot: the thermostat is braking
    assert ev.status() == 0


def test_nvt_cells_are_independent(model):
    beta, sigma = model
    b = S.config_cells(n_cells=3, seed=6)
    v0 = S.maxwell_boltzmann(b.species, 450.0, seed=2)
    print("case: NVT batch of 3 cells vs cell 1 alone", flush=True)
    xb, vb, thb, _, _ = _nvt(beta, sigma, b.pos, b.species, b.offsets, b.boxes, v0, 6, 450.0, 20.0, 0.5)
    st = b.structure(1)
    lo, hi = b.offsets[1], b.offsets[2]
    xa, va, tha, _, _ = _nvt(beta, sigma, st.pos, st.species, [0, st.n], st.box, v0[lo:hi], 6, 450.0, 20.0, 0.5)
    np.testing.assert_array_equal(xa, xb[lo:hi])
    np.testing.assert_array_equal(va, vb[lo:hi])
    np.testing.assert_array_equal(tha[0], thb[1])


def test_coordination_and_events(model):
    beta, sigma = model
    b = S.config_cells(n_cells=4, seed=3)
    pos2 = b.pos.copy()
    rng = np.random.default_rng(1)
    # stretch some H-H bonds past 1 A and move a few H atoms of different molecules together
    h = np.nonzero(b.species == 0)[0]
    for a in rng.choice(h, 12, replace=False):
        pos2[a] += rng.normal(0.0, 0.35, 3)
    print("case: coordination, 4 cells", flush=True)
    m = engine.Model(beta, sigma)
    ev = engine.Evaluator(m, max_atoms=b.n, max_pairs=300 * b.n)
    p, s = engine.to_device(b.pos, b.species)
    ev.neighbors(p, s, b.offsets, b.boxes, 4.0)     # skin 4 A: the list covers moves below 2 A
    ev.descriptors(p)
    c1, _ = ev.coordination(p)
    p2, _ = engine.to_device(pos2, b.species)
    ev.descriptors(p2)
    assert np.abs(pos2 - b.pos).max() < 2.0 / np.sqrt(3.0)
    assert ev.status() == 0            # the moves stay within half the skin
    c2, events = ev.coordination(p2, c1)
    ev.descriptors(p)                  # back: the broken bonds recombine
    c3, back = ev.coordination(p, c2)
    torch.cuda.synchronize()
    c1, c2, events = c1.cpu().numpy(), c2.cpu().numpy(), events.cpu().numpy()
    np.testing.assert_array_equal(c3.cpu().numpy(), c1)
    np.testing.assert_array_equal(back.cpu().numpy(), events[:, ::-1])
    for k in range(4):
        lo, hi = b.offsets[k], b.offsets[k + 1]
        r1 = omd.coordination(b.pos[lo:hi], b.species[lo:hi], b.boxes[k])
        r2 = omd.coordination(pos2[lo:hi], b.species[lo:hi], b.boxes[k])
        np.testing.assert_array_equal(c1[lo:hi], r1)
        np.testing.assert_array_equal(c2[lo:hi], r2)
        assert tuple(events[k]) == omd.reaction_events(r1, r2)
    assert events.sum() > 0


def test_production_monitor(model):
    beta, sigma = model
    st = S.config_tiny()
    v0 = S.maxwell_boltzmann(st.species, 450.0, seed=5)
    m = engine.Model(beta, sigma)
    ev = engine.Evaluator(m, max_atoms=st.n, max_pairs=64 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    v = torch.from_numpy(np.ascontiguousarray(v0.T)).cuda()
    nvt = engine.NVT(ev, p, v, s, [0, st.n], st.box, t_target=450.0, tau=10.0, dt=0.1)
    assert ev.status() == 0
    low = engine.Production(nvt, every=2, threshold=0.0)
    for _ in range(4):
        low.step()
    # the monitor ran at steps 2 and 4 and found the cell above a zero threshold both times
    assert low.over.cpu().tolist() == [2]
    assert low.flagged_cells() == [0]
    assert ev.status() & Bd.FLAG_UNCERTAIN
    high = engine.Production(nvt, every=2, threshold=1e9)
    seen = []
    for _ in range(4):
        high.step()
        if nvt.nstep % 2 == 0:
            seen.append(float(ev.variance()["sigma_max"][0]))
    assert high.flagged_cells() == []
    assert ev.status() == 0
    # the running maximum is the largest per-cell maximum of the monitor points, and that
    # maximum is the oracle's largest sigma at the positions of the last one
    assert float(high.sigma_max[0]) == max(seen)
    ref = oev.evaluate(p.cpu().numpy().T, st.species, st.box, beta, sigma)
    assert abs(seen[-1] - ref.sigma.max()) <= 1e-5 * ref.sigma.max()
