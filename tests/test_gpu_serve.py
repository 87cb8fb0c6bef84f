"""Serving form on the GPU: continuous batching of uneven requests; every served result
equals the same structure evaluated alone (bitwise), and matches the FP64 oracle."""
import numpy as np
import pytest

from oracle import evaluate as oev
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import engine, serve, structures as S

from .gpu_util import TOL, gpu_eval, rel_max, rel_vec

pytestmark = pytest.mark.gpu


def test_served_equals_alone_and_oracle():
    beta, sigma = S.random_model(DEFAULT.n_desc)
    model = engine.Model(beta, sigma)
    reqs = serve.poisson_requests(40, rate=2000.0, sizes=(100, 3000), seed=4)
    print("case: serving 40 requests", flush=True)
    ex = serve.GpuExecutor(model, n_lanes=2, lane_atoms=40_000)
    done, stats = serve.Scheduler(ex).run(reqs)
    print(stats)
    assert stats["batches"] < len(reqs)                # requests were batched
    by_id = {r.rid: r for r in done}
    for rid in [0, 7, 19, 39]:
        r = by_id[rid]
        alone = gpu_eval(r.pos, r.species, r.box, beta, sigma, skin=0.0)
        np.testing.assert_array_equal(r.e, alone["e"])
        np.testing.assert_array_equal(r.f, alone["f"])
        np.testing.assert_array_equal(r.sigma, alone["sigma"])
        assert r.energy == alone["E"][0]
    for rid in [3, 11]:
        r = by_id[rid]
        ref = oev.evaluate(r.pos, r.species, r.box, beta, sigma)
        assert rel_max(r.e, ref.e) <= TOL and rel_vec(r.f, ref.f) <= TOL and rel_max(r.sigma, ref.sigma) <= TOL
