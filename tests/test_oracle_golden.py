"""Regression anchor: the oracle reproduces its committed values for the 80-atom cell."""
import os

import numpy as np

from oracle import evaluate as ev
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import structures as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_oracle.txt")


def test_oracle_matches_committed_values():
    lines = [l.split() for l in open(GOLDEN) if not l.startswith("#")]
    e_total = float(lines[0][1])
    rows = np.array([[float(x) for x in l] for l in lines[1:]])
    st = S.config_tiny()
    beta, gamma = S.random_model(DEFAULT.n_desc)
    r = ev.evaluate(st.pos, st.species, st.box, beta, gamma)
    assert abs(r.energy - e_total) <= 1e-12 * abs(e_total)
    a = rows[:, 0].astype(int)
    np.testing.assert_array_equal(st.species[a], rows[:, 1].astype(int))
    np.testing.assert_allclose(r.e[a], rows[:, 2], rtol=1e-11)
    np.testing.assert_allclose(r.sigma[a], rows[:, 3], rtol=1e-11)
    np.testing.assert_allclose(r.f[a], rows[:, 4:7], rtol=1e-9, atol=1e-13)
