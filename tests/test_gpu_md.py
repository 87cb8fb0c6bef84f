"""Short NVE run on the GPU (velocity Verlet, list rebuilt every 10 steps) vs the FP64
oracle integrator on the 80-atom cell."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev, md as omd
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import engine, structures as S

pytestmark = pytest.mark.gpu


def test_nve_matches_oracle():
    st = S.config_tiny()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    v0 = S.maxwell_boltzmann(st.species, 450.0, seed=9)
    print("case: tiny NVE 10 steps", flush=True)

    def fn(p):
        r = oev.evaluate(p, st.species, st.box, beta, sigma)
        return r.energy, r.f

    ep_ref, ek_ref, x_ref, v_ref = omd.nve(st.pos, v0, st.species, 0.5, 10, fn)
    model = engine.Model(beta, sigma)
    ev = engine.Evaluator(model, max_atoms=st.n, max_pairs=64 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    v = torch.from_numpy(np.ascontiguousarray(v0.T)).cuda()
    md = engine.MD(ev, p, v, s, [0, st.n], st.box, dt=0.5, skin=0.2, rebuild=5)
    epot = [md.out["E"].item()]
    for _ in range(10):
        out = md.step()
        epot.append(out["E"].item())
    torch.cuda.synchronize()
    x = p.cpu().numpy().T
    assert np.abs(x - x_ref).max() < 1e-7
    np.testing.assert_allclose(epot, ep_ref, rtol=1e-5)
    assert ev.status() == 0
