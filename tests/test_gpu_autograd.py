"""Differentiation form: per-cell energies through torch.autograd, backward by the
hand-written adjoint, against the FP64 oracle (its analytic gradient, and central
differences of its energy)."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev, forces as ofo
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import autograd as AG, engine, structures as S

from .gpu_util import TOL, rel_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    beta, sigma = S.random_model(DEFAULT.n_desc)
    b = S.config_cells(n_cells=256, seed=0)
    model = engine.Model(beta, sigma)
    mod = AG.FlareEnergy(model, b.species, b.offsets, b.boxes)
    return beta, sigma, b, mod


def _pos(b):
    return torch.from_numpy(np.ascontiguousarray(b.pos.T)).cuda().requires_grad_(True)


def test_energy_and_gradient_vs_oracle(setup):
    beta, sigma, b, mod = setup
    print("case: autograd, 256 cells", flush=True)
    pos = _pos(b)
    E = mod(pos)
    w = torch.linspace(0.5, 1.5, len(E), dtype=torch.float64, device="cuda")
    (g,) = torch.autograd.grad((w * E).sum(), pos)
    E = E.detach().cpu().numpy()
    g = g.cpu().numpy().T
    w = w.cpu().numpy()
    for k in [0, 1, 77, 128, 255]:
        st = b.structure(k)
        lo, hi = b.offsets[k], b.offsets[k + 1]
        ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
        assert abs(E[k] - ref.energy) <= TOL * abs(ref.energy)
        assert rel_vec(g[lo:hi], -w[k] * ref.f) <= TOL


def test_gradient_vs_oracle_finite_differences(setup):
    beta, sigma, b, mod = setup
    pos = _pos(b)
    E = mod(pos)
    (g,) = torch.autograd.grad(E[3], pos)
    g = g.cpu().numpy().T
    st = b.structure(3)
    lo = b.offsets[3]
    atoms = [0, 50, 143, 144, st.n - 1]
    fn = lambda p: oev.total_energy(p, st.species, st.box, beta)
    fd = ofo.forces_fd(fn, st.pos, atoms, step=1e-4)     # central differences, FP64
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    scale = np.linalg.norm(ref.f, axis=1).max()
    assert np.linalg.norm(g[lo + np.array(atoms)] + fd, axis=1).max() / scale <= 2e-5
    # and the gradient of one cell's energy is zero on every other cell
    other = np.r_[0:lo, b.offsets[4]:b.n]
    assert np.all(g[other] == 0.0)


def test_backward_after_another_forward_recomputes(setup):
    beta, sigma, b, mod = setup
    pos1 = _pos(b)
    E1 = mod(pos1)
    pos2 = (pos1.detach() + 0.01).requires_grad_(True)
    E2 = mod(pos2)
    (g1,) = torch.autograd.grad(E1.sum(), pos1)
    (g2,) = torch.autograd.grad(E2.sum(), pos2)
    pos3 = pos1.detach().clone().requires_grad_(True)
    (g3,) = torch.autograd.grad(mod(pos3).sum(), pos3)
    assert torch.equal(g1, g3)
    assert not torch.equal(g1, g2)


def test_double_backward_raises(setup):
    beta, sigma, b, mod = setup
    pos = _pos(b)
    E = mod(pos)
    (g,) = torch.autograd.grad(E.sum(), pos, create_graph=True)
    with pytest.raises(RuntimeError):
        torch.autograd.grad(g.sum(), pos)


def test_memory_report(setup):
    beta, sigma, b, mod = setup
    pos = _pos(b)
    mod(pos)
    npairs, counts = mod.ev.list_info()
    held = mod.ev.memory_bytes(with_model=False)
    stored = AG.stored_gradient_bytes(npairs, counts[:4].sum(), counts[4:].sum(), npairs, 0)
    print({"held": held, **stored})
    assert held < stored["dd_dr_full"] / 4
