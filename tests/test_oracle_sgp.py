"""Pins for the sparse-GP mapping: mapped quadratic forms equal the unmapped sums."""
import numpy as np

from oracle import evaluate as oev, sgp
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import structures as S


def _descriptors():
    st = S.config_tiny()
    beta, gamma = S.random_model(DEFAULT.n_desc)
    return st, oev.evaluate(st.pos, st.species, st.box, beta, gamma, want_forces=False).d


def test_mean_mapping_is_exact():
    st, d = _descriptors()
    rng = np.random.default_rng(0)
    ds = d[rng.choice(len(d), 20, replace=False)]
    alpha = rng.standard_normal(20)
    beta = sgp.beta_mapped(ds, alpha, 0.7)
    mapped = np.einsum("ik,kl,il->i", d, beta, d)
    np.testing.assert_allclose(mapped, sgp.mean_unmapped(d, ds, alpha, 0.7), rtol=1e-11, atol=1e-14)


def test_variance_mapping_is_exact_and_near_cancelling():
    st, d = _descriptors()
    ds = d[::4]                                   # sparse set: every 4th environment
    sigma2, noise = 2.0, 1e-5
    gamma = sgp.gamma_mapped(ds, sigma2, noise)
    mapped = np.einsum("ik,kl,il->i", d, gamma, d)
    unmapped = sgp.variance_unmapped(d, ds, sigma2, noise)
    np.testing.assert_allclose(mapped, unmapped, rtol=1e-7, atol=1e-12)
    # one sparse point: V(d_s) = sigma^2 noise / (sigma^2 + noise) (closed form, |d_s| = 1)
    one = d[5:6]
    v1 = sgp.variance_unmapped(one, one, sigma2, noise)
    np.testing.assert_allclose(v1, sigma2 * noise / (sigma2 + noise), rtol=1e-9)
    # environments in the sparse set have V << sigma^2: the difference cancels
    assert np.all(unmapped[::4] < 1e-3 * sigma2)
    assert np.all(unmapped >= -1e-12)
    # gamma is positive definite (Cholesky exists)
    np.linalg.cholesky(gamma)
