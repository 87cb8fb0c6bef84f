"""Host logic of the benchmark script: the one-GPU contract and the per-form bound of the
fused kernel (arithmetic only, no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2204_12573_amd import binding as B  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


@pytest.mark.parametrize("prec,products,e_peak,v_peak", [
    (B.BF16_SPLIT, 3, 2.5e15, 78.6e12),
    (B.FP8_SPLIT, 3, 5.0e15, 78.6e12),
    (B.BF16X6_SPLIT, 6, 2.5e15, 78.6e12),
    (B.BF16X6_SPLIT | B.VAR_FP32, 6, 2.5e15, 157.3e12),
])
def test_form_bound_sums_each_part_at_its_peak(prec, products, e_peak, v_peak):
    # one row and no vector work: the bound is the energy pass's part products plus the
    # triangular variance, each at its own peak
    work = {"n144": 1000, "valu_flops": 0.0, "vchol": True}
    r = bench.form_roofline(prec, work, 1e-3)
    t_e = 1000 * products * 2 * 144 * 144 / e_peak
    t_v = 1000 * 144 * 145 / v_peak
    assert r["parts_us"]["energy_pass_us"] == pytest.approx(t_e * 1e6, abs=0.06)
    assert r["parts_us"]["variance_pass_us"] == pytest.approx(t_v * 1e6, abs=0.06)
    assert r["t_min_us"] == pytest.approx((t_e + t_v) * 1e6, abs=0.1)
    assert r["frac"] == pytest.approx((t_e + t_v) / 1e-3, abs=1e-3)
    # vector work adds at the FP32 vector peak; the full Sigma replaces the factor's 144*145
    work2 = {"n144": 1000, "valu_flops": 78.6e6, "vchol": False}
    r2 = bench.form_roofline(prec, work2, 1e-3)
    assert r2["parts_us"]["vector_us"] == pytest.approx(1.0, abs=1e-6)
    assert r2["parts_us"]["variance_pass_us"] == pytest.approx(1000 * 2 * 144 * 144 / v_peak * 1e6, abs=0.06)
