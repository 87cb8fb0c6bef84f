"""With forces, the 544-wide (mixed) rows run on the state's second stream beside the
fused kernel of the single-species rows; with the stage timers on, every stage runs in
order on the caller's stream. Both orders run the same kernels on the same inputs and
write disjoint rows and slots, so the results agree bit for bit: a dependency missing
between the two streams would show up here as a difference."""
import numpy as np
import pytest
import torch

from oracle.hyper import DEFAULT
from paper_2204_12573_amd import engine, structures as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, "bf16x6"])
def test_mixed_rows_beside_the_fused_kernel_equal_the_ordered_run(precision):
    from paper_2204_12573_amd import binding as B
    prec = 0 if precision == 0 else B.BF16X6_SPLIT
    # a 40x40x12 slab under an H2 column: ~60 k atoms, mixed rows at the surfaces
    st = S.h2_over_pt111(40, 40, 12, gas_height=150.0, jitter=0.05, seed=5)
    beta, sigma = S.random_model(DEFAULT.n_desc)
    print(f"case: {st.n} atoms, precision {precision}", flush=True)
    model = engine.Model(beta, sigma, precision=prec)
    ev = engine.Evaluator(model, max_atoms=st.n, max_pairs=64 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    ev.neighbors(p, s, [0, st.n], st.box, 0.2)
    _, counts = ev.list_info()
    assert counts[4:].sum() > 0, "the cell must have mixed rows"
    runs = []
    for timed in (False, True, False):
        ev.timers(timed)
        out = ev.compute(p, want_var=True)
        torch.cuda.synchronize()
        runs.append({k: v.clone() if torch.is_tensor(v) else v for k, v in out.items()})
    ev.timers(False)
    assert ev.status() == 0
    for other in runs[1:]:
        for k, v in runs[0].items():
            if torch.is_tensor(v):
                assert torch.equal(v, other[k]), k
            else:
                assert np.array_equal(np.asarray(v), np.asarray(other[k])), k
