"""Virial W = -dE/d(strain) of each cell from the per-pair adjoint terms, against the
oracle's explicit-gradient virial (itself pinned by strain finite differences)."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, engine, structures as S

from .gpu_util import TOL

pytestmark = pytest.mark.gpu


def _gpu_virial(pos, species, boxes, offsets, beta, sigma):
    model = engine.Model(beta, sigma)
    n = len(species)
    ev = engine.Evaluator(model, max_atoms=n, max_pairs=64 * n)
    p, s = engine.to_device(pos, species)
    ev.neighbors(p, s, offsets, np.asarray(boxes, np.float64).reshape(-1, 3), 0.2)
    ev.descriptors(p)
    ev.energy_forces(want_var=False)
    w = ev.virial()
    torch.cuda.synchronize()
    return w.cpu().numpy(), ev


def test_virial_tiny():
    st = S.config_tiny()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    print("case: virial tiny", flush=True)
    w, _ = _gpu_virial(st.pos, st.species, st.box, [0, st.n], beta, sigma)
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma, want_virial=True).virial
    err = np.abs(w[0] - ref).max() / np.abs(ref).max()
    print("virial rel err", err)
    assert err <= TOL


def test_virial_batch_of_cells_and_stale():
    b = S.config_cells(n_cells=8, seed=5)
    beta, sigma = S.random_model(DEFAULT.n_desc)
    print("case: virial 8 cells", flush=True)
    w, ev = _gpu_virial(b.pos, b.species, b.boxes, b.offsets, beta, sigma)
    for k in range(8):
        st = b.structure(k)
        ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma, want_virial=True).virial
        assert np.abs(w[k] - ref).max() / np.abs(ref).max() <= TOL
    # new positions without forces: the adjoint terms are stale
    p, _ = engine.to_device(b.pos, b.species)
    ev.descriptors(p)
    with pytest.raises(Bd.FlareError):
        ev.virial()
