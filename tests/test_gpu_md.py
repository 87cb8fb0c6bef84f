"""Short NVE run on the GPU (velocity Verlet, list rebuilt every 10 steps) vs the FP64
oracle integrator on the 80-atom cell."""
import numpy as np
import pytest
import torch

from oracle import evaluate as oev, md as omd
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, engine, structures as S

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


def test_displaced_interval_raises_at_the_rebuild():
    """An atom moved more than half the skin between two list builds: the rebuild that ends
    the interval raises (the flag is not lost by the build), and flare_status still has it."""
    st = S.config_tiny()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    model = engine.Model(beta, sigma)
    ev = engine.Evaluator(model, max_atoms=st.n, max_pairs=64 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    v = torch.zeros_like(p)
    print("case: tiny NVE, forced displacement", flush=True)
    md = engine.MD(ev, p, v, s, [0, st.n], st.box, dt=0.5, skin=0.2, rebuild=3)
    md.step()
    p[0, 7] += 0.15              # more than skin/2 = 0.1 A
    md.step()                    # step 2: descriptors raise the flag, no rebuild yet
    with pytest.raises(engine.DisplacedError):
        md.step()                # step 3 rebuilds and reports the ended interval
    assert ev.interval_status() & Bd.FLAG_DISPLACED
    assert ev.status() & Bd.FLAG_DISPLACED
    assert ev.status() == 0      # read and cleared


def test_state_memory_fixed_across_rebuilds():
    """Every buffer of a state is allocated at flare_state_create: 20 NVE steps with a list
    rebuild every 5 change neither the state's device memory (flare_memory_bytes) nor the
    device's free memory (no allocation by the library, and none by the driver loop)."""
    b = S.config_cells(n_cells=3, seed=2)
    beta, sigma = S.random_model(DEFAULT.n_desc)
    model = engine.Model(beta, sigma)
    ev = engine.Evaluator(model, max_atoms=b.n, max_pairs=64 * b.n)
    held = ev.memory_bytes(with_model=False)
    p, s = engine.to_device(b.pos, b.species)
    v = torch.zeros_like(p)
    print("case: memory across 20 NVE steps, 3 cells", flush=True)
    md = engine.MD(ev, p, v, s, b.offsets, b.boxes, dt=0.5, skin=0.2, rebuild=5)
    for _ in range(5):
        md.step()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        md.step()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert ev.memory_bytes(with_model=False) == held
    assert ev.status() == 0


@pytest.mark.parametrize("prec", [pytest.param(Bd.FP32, id="fp32"), pytest.param(Bd.BF16X6_SPLIT, id="bf16x6")])
def test_md_step_matches_the_separate_calls(prec):
    """flare_md_step (one call per step, fused drift/displacement and output/second-half
    kernels) against the same steps through the separate calls: bit for bit, over 25 steps
    with two list rebuilds, in a batch of three cells, in the plain and the three-way BF16
    form."""
    b = S.config_cells(n_cells=3, seed=5)
    beta, sigma = S.random_model(DEFAULT.n_desc)
    v0 = S.maxwell_boltzmann(b.species, 450.0, seed=3)
    runs = []
    for fused in (True, False):
        model = engine.Model(beta, sigma, precision=prec)
        ev = engine.Evaluator(model, max_atoms=b.n, max_pairs=64 * b.n)
        p, s = engine.to_device(b.pos, b.species)
        v = torch.from_numpy(np.ascontiguousarray(v0.T)).cuda()
        # skin 1 A: at 450 K and 0.5 fs the fastest H atoms move up to about 0.4 A per
        # 10-step interval (the rebuild would rightly raise with a thinner skin)
        md = engine.MD(ev, p, v, s, b.offsets, b.boxes, dt=0.5, skin=1.0, rebuild=10)
        how = "one call" if fused else "separate calls"
        print(f"case: {b.n} atoms in 3 cells, 25 NVE steps, precision {prec}, {how}", flush=True)
        for _ in range(25):
            out = md.step() if fused else md.step_in_calls()
        torch.cuda.synchronize()
        runs.append({"x": p.cpu().numpy(), "v": v.cpu().numpy(), **{k: t.cpu().numpy() for k, t in out.items()}})
        assert ev.status() == 0
    for k in runs[0]:
        np.testing.assert_array_equal(runs[0][k], runs[1][k], err_msg=k)
