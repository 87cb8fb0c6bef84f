"""The mapped quadratic forms on given vectors (flare_quadratic_forms, Eqs. 1-2) against
an extended-precision evaluation of d^T beta d and d^T Sigma d, for every bucket kind and
arithmetic form, including a near-cancelling variance down to V/sigma^2 = 1e-8.

Inputs (seeded, none from the HIP path): Sigma_s = gamma_s of Eq. 2 built by the oracle
(oracle/sgp.py) from a synthetic sparse set of unit vectors; beta_s random PSD. The test
vectors are FP32: d = normalise(sum_t c_t d_t + eps r), d_t sparse vectors, r random, so
that V/sigma^2 ~ eps^2 spans 1e-8 .. 1. The reference evaluates the FP64 matrices at the
FP32 vectors in numpy's long double (64-bit significand), far below the errors tested.

Bars. Energies: the form's energy bar (FP32 and three-way BF16 1e-5, two-way BF16 1e-4,
FP8 1e-2 of the largest energy). Variance: the split forms compute |L^T d|^2 with the FP64
factor on FP64 matrix cores, so every row with V/sigma^2 >= 1e-8 is held to 1e-6
pointwise relative error (the FP64 Cholesky factor's own backward error, about
sqrt(n) 2^-53 sigma^2, is 1e-7 of V there). The plain FP32 form rounds L to FP32 and sums in
FP32: its error is about 2^-24 sigma |z| / |z|^2 relative, so it is held to 1e-5 only where
V/sigma^2 >= 1e-2, and its near-cancelling errors are printed beside the FP64 ones; a split
form with FLARE_VAR_FP32 takes the same variance path and bar."""
import numpy as np
import pytest
import torch

from oracle import sgp
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, engine, structures as S

pytestmark = pytest.mark.gpu

ND, NB = DEFAULT.n_desc, 144
SIGMA2, NOISE = 1e-2, 1e-14
EPS = [1e-4, 1e-3, 1e-2, 1e-1, 1.0]
E_TOL = {Bd.FP32: 1e-5, Bd.BF16_SPLIT: 1e-4, Bd.FP8_SPLIT: 1e-2, Bd.BF16X6_SPLIT: 1e-5}
# bucket -> (species, first component, width)
BUCKETS = {0: (0, 0, NB), 3: (1, ND - NB, NB), 4: (0, 0, ND), 5: (1, 0, ND)}


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


@pytest.fixture(scope="module")
def setup():
    rng = np.random.default_rng(2022)
    # species H: a sparse set inside the H-H block; species Pt: full 544-wide vectors
    dh = np.zeros((40, ND))
    dh[:, :NB] = _unit(rng.standard_normal((40, NB)))
    dp = _unit(rng.standard_normal((40, ND)))
    gamma = np.stack([sgp.gamma_mapped(dh, SIGMA2, NOISE), sgp.gamma_mapped(dp, SIGMA2, NOISE)])
    beta, _ = S.random_model(ND)
    vecs = {}
    for b, (s, st, w) in BUCKETS.items():
        base = (dh if s == 0 else dp)[:, st:st + w]
        rows = []
        for eps in EPS:
            for _ in range(4):
                c = rng.standard_normal(len(base))
                v = c @ base + eps * _unit(rng.standard_normal(w)) * np.linalg.norm(c @ base)
                rows.append(_unit(v))
        vecs[b] = np.asarray(rows, np.float32)
    return beta, gamma, vecs


def _reference(mat, d32):
    d = d32.astype(np.longdouble)
    m = mat.astype(np.longdouble)
    return np.einsum("ik,kl,il->i", d, m, d)


@pytest.mark.parametrize("prec", [pytest.param(Bd.FP32, id="fp32"), pytest.param(Bd.BF16_SPLIT, id="bf16"),
                                  pytest.param(Bd.FP8_SPLIT, id="fp8"), pytest.param(Bd.BF16X6_SPLIT, id="bf16x6"),
                                  pytest.param(Bd.BF16X6_SPLIT | Bd.VAR_FP32, id="bf16x6-var32")])
def test_forms_of_given_vectors(setup, prec):
    beta, gamma, vecs = setup
    model = engine.Model(beta, gamma, precision=prec)
    ev = engine.Evaluator(model, max_atoms=1024, max_pairs=1024)
    for b, (s, st, w) in BUCKETS.items():
        print(f"case: quadratic forms, precision {prec}, bucket {b}", flush=True)
        d = vecs[b]
        e, v = ev.quadratic_forms(b, torch.from_numpy(d).cuda())
        torch.cuda.synchronize()
        e, v = e.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        blk = np.s_[st:st + w, st:st + w]
        e_ref = _reference(beta[s][blk], d).astype(np.float64)
        v_ref = _reference(gamma[s][blk], d).astype(np.float64)
        err_e = np.abs(e - e_ref).max() / np.abs(e_ref).max()
        rel_v = np.abs(v - v_ref) / v_ref
        ratio = v_ref / SIGMA2
        print(f"  e {err_e:.2e}; V/sigma^2 from {ratio.min():.1e}: pointwise rel. error of V by decade "
              + ", ".join(f"{lo:.0e}:{rel_v[(ratio >= lo) & (ratio < lo * 100)].max():.1e}"
                          for lo in (1e-9, 1e-7, 1e-5, 1e-3, 1e-1) if np.any((ratio >= lo) & (ratio < lo * 100))))
        assert err_e <= E_TOL[prec & ~Bd.VAR_FP32]
        if prec == Bd.FP32 or prec & Bd.VAR_FP32:
            assert rel_v[ratio >= 1e-2].max() <= 1e-5
        else:
            assert rel_v[ratio >= 1e-8].max() <= 1e-6
        if b in (0, 4, 5):
            assert ratio.min() < 1e-7            # the sample reaches the near-cancelling range


def test_forms_argument_checks(setup):
    beta, gamma, vecs = setup
    model = engine.Model(beta, gamma)
    ev = engine.Evaluator(model, max_atoms=16, max_pairs=64)
    d = torch.zeros((4, NB), dtype=torch.float32, device="cuda")
    with pytest.raises(Bd.FlareError):
        ev.quadratic_forms(6, d)
    with pytest.raises(Bd.FlareError):
        ev.quadratic_forms(0, torch.zeros((17, NB), dtype=torch.float32, device="cuda"))
    e, v = ev.quadratic_forms(0, d)
    torch.cuda.synchronize()
    assert torch.all(e == 0) and torch.all(v == 0)
