"""Precision forms: the split quadratic forms (beta = beta_hi + beta_lo and
d = d_hi + d_lo on BF16 or FP8-e4m3 matrix cores, FP32 accumulation; variance as
|L^T d|^2 with the FP64 Cholesky factor on FP64 matrix cores, FP64 sums) against the FP64
oracle, beside plain FP32.

Tolerances. BF16 has 8 significant bits: each split operand keeps ~16 bits and the
dropped lo*lo product is ~2^-16 of a term, so E and F land near 1e-5 of their scale;
1e-4 leaves room for the sum over 144^2 terms. FP8 e4m3 has 4 significant bits: with
power-of-two scales keeping every operand normal, each term 16 x b is represented to
3 * 2^-8 of |x||b| (two rounded lo' parts and the dropped lo*lo), so the worst case is
about 1.2e-2 of sum_kl |d_k||beta_kl||d_l| / |d|^2; random rounding errors average down
and the test asks for 1e-2 of the largest energy and force. The variance of these two
split forms never touches the narrow formats. The three-way BF16 form splits d and beta
into three BF16 parts (together the 24 bits of the FP32 value) and drops only part
products below 2^-23 of a term, so it is held to the FP32 bar, 1e-5, in E, F and sigma."""
import numpy as np
import pytest

from oracle import evaluate as oev, sgp
from oracle.hyper import DEFAULT
from paper_2204_12573_amd import binding as Bd, structures as S

from .gpu_util import gpu_eval, rel_max, rel_vec

pytestmark = pytest.mark.gpu

SPLIT_TOL_E = 1e-4     # energies, forces of the BF16 split form (BF16 x 3 products)
SPLIT_TOL_S = 1e-5     # sigma of the split forms (sum of squares, no cancellation)
FP8_TOL_E = 1e-2       # energies, forces of the FP8 split form (e4m3 x 3 products)
X6_TOL_E = 1e-5        # three-way BF16 form: the FP32 bar
TOL_E = {Bd.BF16_SPLIT: SPLIT_TOL_E, Bd.FP8_SPLIT: FP8_TOL_E, Bd.BF16X6_SPLIT: X6_TOL_E}
PREC = [pytest.param(Bd.BF16_SPLIT, id="bf16"), pytest.param(Bd.FP8_SPLIT, id="fp8"),
        pytest.param(Bd.BF16X6_SPLIT, id="bf16x6"), pytest.param(Bd.BF16X6_SPLIT | Bd.VAR_FP32, id="bf16x6-var32")]
TOL_E[Bd.BF16X6_SPLIT | Bd.VAR_FP32] = X6_TOL_E


def _errs(res, ref):
    return {"e": rel_max(res["e"], ref.e), "f": rel_vec(res["f"], ref.f), "sigma": rel_max(res["sigma"], ref.sigma),
            "var_pointwise": float(np.max(np.abs(res["var"] - ref.v) / np.abs(ref.v)))}


@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("case", ["tiny", "cells"])
def test_split_form_random_models(case, prec):
    beta, sigma = S.random_model(DEFAULT.n_desc)
    if case == "tiny":
        st = S.config_tiny()
        cells = [(st, 0, st.n)]
        pos, species, boxes, offsets = st.pos, st.species, st.box, None
    else:
        b = S.config_cells(n_cells=6, seed=3)
        cells = [(b.structure(k), b.offsets[k], b.offsets[k + 1]) for k in range(6)]
        pos, species, boxes, offsets = b.pos, b.species, b.boxes, b.offsets
    print(f"case: split form {case} precision {prec}", flush=True)
    res = gpu_eval(pos, species, boxes, beta, sigma, offsets=offsets, precision=prec)
    for st, lo, hi in cells:
        ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
        sub = {k: res[k][lo:hi] for k in ["e", "f", "sigma", "var"]}
        errs = _errs(sub, ref)
        print(errs)
        assert errs["e"] <= TOL_E[prec] and errs["f"] <= TOL_E[prec] and errs["sigma"] <= SPLIT_TOL_S


def test_near_cancelling_variance():
    """Sigma_s = gamma_s of a sparse GP whose sparse set contains half the environments:
    V = sigma^2 - (a term of nearly the same size). Every form evaluates |L^T d~|^2 / |d~|^2;
    the split forms with the FP64 factor on FP64 matrix cores, the FP32 form with the factor
    rounded to FP32. Bounds per atom, from the arithmetic (gamma <= sigma^2 I, |d| = 1):
      descriptor rounding   2 sigma sqrt(V) |dd| + sigma^2 |dd|^2, |dd| the largest
                            descriptor error (exported descriptors against the oracle's);
      split forms           + 1e-6 V (FP64 form; pinned on given vectors in test_gpu_forms);
      FP32 form (and a split form with FLARE_VAR_FP32)
                            + 2 sqrt(V) 2^-22 |L|_F (L rounded to FP32 and 144-term FP32
                            sums: four roundings at the scale of a column of L).
    Each is asserted with a factor of 2. A direct FP32 d^T gamma d, formed with torch on
    the exported descriptors, is printed for comparison."""
    import torch
    st = S.config_tiny()
    beta, _ = S.random_model(DEFAULT.n_desc)
    d = oev.evaluate(st.pos, st.species, st.box, beta, beta, want_forces=False).d
    sigma2, noise = 1e-3, 1e-7
    gamma = np.stack([sgp.gamma_mapped(d[(st.species == s)][::2], sigma2, noise) for s in (0, 1)])
    ref = oev.evaluate(st.pos, st.species, st.box, beta, gamma)
    lf = max(np.linalg.norm(np.linalg.cholesky(g)) for g in gamma)      # |L|_F (FP64 oracle)
    sig = np.sqrt(sigma2)
    out = {}
    for name, prec in [("fp32", Bd.FP32), ("split", Bd.BF16_SPLIT), ("fp8", Bd.FP8_SPLIT),
                       ("bf16x6", Bd.BF16X6_SPLIT), ("bf16x6_var32", Bd.BF16X6_SPLIT | Bd.VAR_FP32)]:
        res = gpu_eval(st.pos, st.species, st.box, beta, gamma, precision=prec, want_d=True)
        dd = float(np.linalg.norm(res["d"] - ref.d, axis=1).max())
        err = np.abs(res["var"] - ref.v)
        bound = 2.0 * sig * np.sqrt(ref.v) * dd + sigma2 * dd * dd
        fp32_factor = prec == Bd.FP32 or bool(prec & Bd.VAR_FP32)
        bound += 2.0 * np.sqrt(ref.v) * 2.0 ** -22 * lf if fp32_factor else 1e-6 * ref.v
        out[name] = {"rel": float(np.max(err / ref.v)), "descriptor_err": dd,
                     "err_over_bound": float(np.max(err / bound))}
        if name == "fp32":
            torch.backends.cuda.matmul.allow_tf32 = False
            dv = torch.from_numpy(res["d"]).cuda()
            g = torch.from_numpy(gamma.astype(np.float32)).cuda()
            sp = torch.from_numpy(st.species.astype(np.int64)).cuda()
            v_direct = ((dv @ g[0]) * dv).sum(1) * (sp == 0) + ((dv @ g[1]) * dv).sum(1) * (sp == 1)
            out["direct_fp32"] = {"rel": float(np.max(np.abs(v_direct.cpu().numpy() - ref.v) / ref.v))}
    print("variance errors:", out, "V/sigma^2 range:", ref.v.min() / sigma2, ref.v.max() / sigma2)
    assert ref.v.min() < 1e-3 * sigma2              # genuinely near-cancelling
    for name in ("fp32", "split", "fp8", "bf16x6", "bf16x6_var32"):
        assert out[name]["err_over_bound"] <= 2.0
        assert out[name]["rel"] < out["direct_fp32"]["rel"] / 5


def test_fp32_full_sigma_when_not_positive_definite():
    """A rank-deficient Sigma has no Cholesky factor: the FP32 form then evaluates d^T Sigma d
    with the full matrix (the split forms refuse such a model)."""
    st = S.config_tiny()
    beta, _ = S.random_model(DEFAULT.n_desc)
    rng = np.random.default_rng(9)
    a = rng.standard_normal((2, DEFAULT.n_desc, 40))
    sigma = 1e-3 * np.einsum("sik,sjk->sij", a, a) / 40      # PSD, rank 40
    print("case: rank-deficient Sigma, FP32", flush=True)
    res = gpu_eval(st.pos, st.species, st.box, beta, sigma, precision=Bd.FP32)
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    errs = _errs(res, ref)
    print(errs)
    assert errs["e"] <= 1e-5 and errs["f"] <= 1e-5 and errs["sigma"] <= 1e-5
    with pytest.raises(Bd.FlareError):
        gpu_eval(st.pos, st.species, st.box, beta, sigma, precision=Bd.BF16_SPLIT)


@pytest.mark.parametrize("prec", PREC)
def test_split_form_large_sample(prec):
    st = S.config_large()
    beta, sigma = S.random_model(DEFAULT.n_desc)
    print(f"case: split form, large cell, precision {prec}", flush=True)
    res = gpu_eval(st.pos, st.species, st.box, beta, sigma, max_pairs=12 * st.n, precision=prec)
    rng = np.random.default_rng(21)
    tg = np.unique(rng.choice(st.n, 200, replace=False))
    ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma, targets=tg)
    rows = ref.row_of(tg)
    errs = {"e": rel_max(res["e"][tg], ref.e[rows]), "f": rel_vec(res["f"][tg], ref.f),
            "sigma": rel_max(res["sigma"][tg], ref.sigma[rows])}
    print(errs)
    assert errs["e"] <= TOL_E[prec] and errs["f"] <= TOL_E[prec] and errs["sigma"] <= SPLIT_TOL_S
