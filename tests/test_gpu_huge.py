"""The ~16 M-atom size of the precision workload (400 x 400 x 24 Pt(111) under the same H2
gas column) in every arithmetic form, checked on seeded samples.

The cell is the 100 x 100 x 24 cell of the 1 M-atom workload repeated 4 x 4 laterally:
the same generator at the same density, built in seconds instead of minutes. Every atom's
environment in the tiled cell is its original's environment translated by whole box
lengths, so the oracle evaluated on the 1 M-atom cell gives the expected values of all 16
copies (descriptors, energies and variances are invariant under the translation, forces
unchanged). The samples are taken from several copies."""
import numpy as np
import pytest

from oracle import evaluate as oev
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, structures as S

from .gpu_util import TOL, gpu_eval, rel_max, rel_vec

pytestmark = pytest.mark.gpu

TOLS = {Bd.FP32: TOL, Bd.BF16_SPLIT: 1e-4, Bd.FP8_SPLIT: 1e-2, Bd.BF16X6_SPLIT: TOL}
SIGMA_TOL = 1e-5


def test_huge_tiled_all_forms():
    small = S.config_large()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    big_st = S.tiled(small, 4, 4)
    pos, species, box, n1 = big_st.pos, big_st.species, big_st.box, small.n
    n = len(species)
    print(f"case: tiled cell, {n} atoms", flush=True)
    rng = np.random.default_rng(31)
    ztop = 23 * S.DZ
    surf = np.nonzero(np.abs(small.pos[:, 2] - ztop) < 4.0)[0]
    tg = np.unique(np.concatenate([rng.choice(n1, 60, replace=False), rng.choice(surf, 40, replace=False)]))
    ref = oev.evaluate(small.pos, small.species, small.box, beta, sigma, targets=tg)
    rows = ref.row_of(tg)
    copies = rng.integers(0, 16, len(tg))
    big = copies * n1 + tg
    for prec in (Bd.FP32, Bd.BF16_SPLIT, Bd.FP8_SPLIT, Bd.BF16X6_SPLIT):
        print(f"case: tiled cell, precision {prec}", flush=True)
        res = gpu_eval(pos, species, box, beta, sigma, max_pairs=12 * n, precision=prec)
        assert res["status"] == 0
        npairs, counts = res["ev"].list_info()
        assert counts[4] + counts[5] > 0          # mixed environments exist
        errs = {"e": rel_max(res["e"][big], ref.e[rows]), "f": rel_vec(res["f"][big], ref.f),
                "sigma": rel_max(res["sigma"][big], ref.sigma[rows])}
        print(npairs, errs, flush=True)
        assert errs["e"] <= TOLS[prec] and errs["f"] <= TOLS[prec] and errs["sigma"] <= SIGMA_TOL
        del res
