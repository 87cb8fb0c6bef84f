"""Differentiation form: per-cell energies through torch.autograd, backward by the
hand-written adjoint, against the FP64 oracle (its analytic gradient, and central
differences of its energy)."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev, forces as ofo
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import autograd as AG, engine, structures as S

from . import oracle_pool as OP
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
    """Every one of the 256 cells: its energy and the gradient of a weighted sum of all
    cell energies against the oracle's energy and analytic forces (FP64)."""
    beta, sigma, b, mod = setup
    print("case: autograd, 256 cells vs oracle gradient", flush=True)
    pos = _pos(b)
    E = mod(pos)
    w = torch.linspace(0.5, 1.5, len(E), dtype=torch.float64, device="cuda")
    (g,) = torch.autograd.grad((w * E).sum(), pos)
    E = E.detach().cpu().numpy()
    g = g.cpu().numpy().T
    w = w.cpu().numpy()
    jobs = [(b.structure(k).pos, b.structure(k).species, b.structure(k).box, beta, sigma) for k in range(len(b.boxes))]
    refs = OP.run(OP.cell_energy_forces, jobs)
    err_e, err_g = [], []
    for k, (e_ref, f_ref) in enumerate(refs):
        lo, hi = b.offsets[k], b.offsets[k + 1]
        err_e.append(abs(E[k] - e_ref) / abs(e_ref))
        err_g.append(rel_vec(g[lo:hi], -w[k] * f_ref))
    print(f"max over 256 cells: energy {max(err_e):.2e}, gradient {max(err_g):.2e}", flush=True)
    assert max(err_e) <= TOL and max(err_g) <= TOL


def test_gradient_vs_oracle_finite_differences(setup):
    """Four seeded cells, every atom and component: the adjoint gradient of the sum of their
    energies against central differences (h = 1e-4 A) of the FP64 oracle energy."""
    beta, sigma, b, mod = setup
    rng = np.random.default_rng(4)
    cells = np.sort(rng.choice(len(b.boxes), 4, replace=False))
    print(f"case: autograd FD, cells {cells.tolist()}", flush=True)
    pos = _pos(b)
    E = mod(pos)
    sel = torch.zeros(len(E), dtype=torch.float64, device="cuda")
    sel[torch.from_numpy(cells).cuda()] = 1.0
    (g,) = torch.autograd.grad((sel * E).sum(), pos)
    g = g.cpu().numpy().T
    jobs, where = [], []
    for k in cells:
        st = b.structure(k)
        for chunk in np.array_split(np.arange(st.n), 12):
            jobs.append((st.pos, st.species, st.box, beta, 1e-4, chunk))
            where.append(b.offsets[k] + chunk)
    fd = np.concatenate(OP.run(OP.local_fd_forces, jobs))
    where = np.concatenate(where)
    scale = np.linalg.norm(fd, axis=1).max()
    err = np.linalg.norm(g[where] + fd, axis=1).max() / scale
    print(f"adjoint vs FD: {err:.2e} over {len(where)} atoms", flush=True)
    assert err <= 2e-5
    # the gradient is zero on every atom of the other cells
    other = np.ones(b.n, bool)
    other[where] = False
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
