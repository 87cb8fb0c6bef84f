"""Input generators: the lateral tiling used for the ~16 M-atom precision workload.

The 16 M-atom parity test and benchmark leg take their expected values from the 1 M-atom
cell, relying on every copy of a tiled cell seeing its original's environment. That is
checked here with the FP64 oracle on a small cell."""
import numpy as np

from oracle import evaluate as oev
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import structures as S


def test_tiled_layout():
    st = S.config_tiny()
    big = S.tiled(st, 3, 2)
    assert big.n == 6 * st.n
    np.testing.assert_array_equal(big.box, [3 * st.box[0], 2 * st.box[1], st.box[2]])
    np.testing.assert_array_equal(big.species, np.tile(st.species, 6))
    # copy c = a + 3 b is the original moved by (a Lx, b Ly, 0)
    for c, (a, b) in enumerate([(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (2, 1)]):
        np.testing.assert_array_equal(big.pos[c * st.n:(c + 1) * st.n],
                                      st.pos + np.array([a * st.box[0], b * st.box[1], 0.0]))


def test_tiled_copies_share_the_original_environments():
    st = S.config_tiny()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    big = S.tiled(st, 2, 2)
    tg = np.array([0, 17, 40, 63, 64, 79])          # Pt atoms (bulk, surface) and H atoms
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma, targets=tg)
    rows = ref.row_of(tg)
    for c in (1, 3):
        tc = c * st.n + tg
        got = oev.evaluate(big.pos, big.species, big.box, beta, sigma, targets=tc)
        rc = got.row_of(tc)
        np.testing.assert_allclose(got.e[rc], ref.e[rows], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(got.sigma[rc], ref.sigma[rows], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(got.f, ref.f, rtol=1e-10, atol=1e-13)   # per target, in order
