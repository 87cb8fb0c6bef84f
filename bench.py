#!/usr/bin/env python3
"""Throughput of the FLARE B2 force-field MD step on one MI355X.

Workload: periodic Pt(111) slab 100x100x24 (240,000 Pt) under an H2 gas at 1 molecule
per 200 A^3 in a 1142.2 A column (~1.0 M atoms), 0.05 A Gaussian jitter, random PSD
beta/Sigma (scale 1e-3), 2 species, 8 radial functions, l <= 3, r_cut 4.5 A (544 B2
components). One step = velocity-Verlet NVE step with energies, forces and per-atom
uncertainty (E+F+sigma), list rebuilt every 10 steps (skin 0.2 A), dt = 0.5 fs. All
inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line. `value` is M atom-steps/s of the plain FP32 path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M atom-steps/s/GPU (E+F+σ) plain FP32 vs mixed @ force err; p50/p99 serve latency"
PEAK_FP32_MFMA = 157.3e12      # dense FP32 matrix FLOP/s, MI355X
PEAK_HBM = 8.0e12              # B/s
PEAK_FP32_VALU = 78.6e12       # FP32 vector FMA without packed instructions
# algorithmic vector work beside the quadratic forms (flop). Per pair inside the cutoff:
# densities = radial basis (24) + 16 harmonics (35) + 8x16 multiply-adds (256) = 320 with
# rounding; adjoint term = radial basis and derivative (75) + harmonics (35) + A_lm, B_lm
# (512) + the radial sum (64) + the harmonic gradient contraction (135) + assembly (9) =
# 830. Per 144-wide row: B2 contraction 36 x 16 multiply-adds (1152), |d~|^2 (288), the
# epilogue e = Y.d, g = s(Y - e d), V = |z|^2 (1000), the adjoint transform u = G^ c
# (8 x 8 x 16 multiply-adds = 2048).
VALU_FLOP_DENS, VALU_FLOP_ADJ = 320, 830
VALU_FLOP_B2, VALU_FLOP_NORM, VALU_FLOP_EPI, VALU_FLOP_U = 1152, 288, 1000, 2048
# dense matrix peaks of the split forms' instruction types (FLOP/s, MI355X)
PEAK_BF16_MFMA, PEAK_FP8_MFMA, PEAK_FP64_MFMA = 2.5e15, 5.0e15, 78.6e12


PROFILE = os.path.join(ROOT, "profiles", "k_fused144_w_h2_pt111_1M_fp32.txt")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ["fused.hip", "adjoint.h", "half.h", "pair.h", "basis.h", "common.h", "state.h"]:
        with open(os.path.join(ROOT, "paper_2204_12573_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel="k_fused144_w<0, false>"):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    try:
        with open(PROFILE) as fh:
            txt = fh.read()
        data = json.loads(txt.split("# json\n", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if data.get("sha256") != kernel_sources_sha():
        return None
    k = data["kernels"].get(kernel)
    if not k:
        return None
    return (k["fetch_MB"] + k["write_MB"]) * 1e6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_crop_part(job):
    """One worker's share of the oracle crop: E+F+sigma of the given target atoms."""
    from oracle import evaluate as oev
    pos, species, box, beta, sigma, tg = job
    t0 = time.perf_counter()
    oev.evaluate(pos, species, box, beta, sigma, targets=tg)
    return time.perf_counter() - t0


def _n_workers():
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cpus = os.cpu_count() or 1
    return max(1, min(16, cpus))


def cpu_baseline(st, beta, sigma, n_crop=100_000, seed=2204):
    """The FP64 oracle on a bounded sample of the workload: a seeded crop of n_crop atoms of
    the 1 M-atom cell (every atom of a lateral square column through slab and gas, centred at
    a seeded point), one E+F+sigma evaluation of those atoms, their targets split into
    contiguous spatial blocks over one worker process per core (each worker one BLAS thread).
    The oracle's cost is linear in the atoms it evaluates (neighbour lists from a k-d tree,
    per-atom descriptors and forms), so a full evaluation of the cell takes N / rate."""
    import multiprocessing as mp

    import numpy as np
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(0.0, 1.0, 2) * st.box[:2]
    dx = np.abs((st.pos[:, 0] - cx + 0.5 * st.box[0]) % st.box[0] - 0.5 * st.box[0])
    dy = np.abs((st.pos[:, 1] - cy + 0.5 * st.box[1]) % st.box[1] - 0.5 * st.box[1])
    r = np.maximum(dx, dy)
    tg = np.argsort(r, kind="stable")[:n_crop]            # the n_crop atoms nearest the column axis
    order = tg[np.lexsort((st.pos[tg, 1], st.pos[tg, 0], st.pos[tg, 2]))]
    nw = _n_workers()
    parts = np.array_split(order, nw)
    jobs = [(st.pos, st.species, st.box, beta, sigma, np.sort(p)) for p in parts]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(nw, initializer=_one_blas_thread) as pool:
        busy = pool.map(_oracle_crop_part, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    rate = len(tg) / wall
    return {"value": rate / 1e6, "unit": "M atom-steps/s", "cores": int(nw), "kind": "oracle",
            "sample": f"seeded {len(tg)}-atom crop of the {st.n}-atom cell (a lateral square column through slab "
                      f"and gas), one E+F+sigma evaluation of those atoms in {wall:.1f} s wall over {nw} worker "
                      f"processes ({sum(busy):.1f} s of worker time); numpy FP64, one BLAS thread per worker",
            "full_cell_extrapolation_s": round(st.n / rate, 1)}


def _one_blas_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:  # pragma: no cover
        pass


def oracle_tiny_run(beta, sigma, n_steps=10, dt=0.5):
    """The small workload in full on the host: one E+F+sigma evaluation of the 80-atom cell and
    a 10-step NVE run (dt 0.5 fs) with the FP64 oracle, single process."""
    import numpy as np

    from oracle import evaluate as oev, md as omd
    from paper_2204_12573_amd import structures as S
    st = S.config_tiny()
    t0 = time.perf_counter()
    oev.evaluate(st.pos, st.species, st.box, beta, sigma)
    t_eval = time.perf_counter() - t0

    def fn(x):
        r = oev.evaluate(x, st.species, st.box, beta, sigma)
        return r.energy, r.f

    t0 = time.perf_counter()
    omd.nve(st.pos, np.zeros_like(st.pos), st.species, dt, n_steps, fn)
    t_md = time.perf_counter() - t0
    return {"atoms": st.n, "eval_s": round(t_eval, 3), "nve_steps": n_steps, "nve_s": round(t_md, 3),
            "M_atom_steps_per_s": st.n * (n_steps + 1) / (t_eval + t_md) / 1e6,
            "note": "80-atom H2/Pt(111) cell: one evaluation plus a 10-step NVE run (11 evaluations), FP64 oracle"}


def md_throughput(engine, torch, st, beta, sigma, steps, warmup, precision, settle=0):
    n = st.n
    model = engine.Model(beta, sigma, precision=precision)
    ev = engine.Evaluator(model, max_atoms=n, max_pairs=12 * n)
    p, s = engine.to_device(st.pos, st.species)
    v = torch.zeros_like(p)
    md = engine.MD(ev, p, v, s, [0, n], st.box, dt=0.5, skin=0.2, rebuild=10, want_var=True)
    # a fresh GPU speeds up during its first few tens of ms under load (the fused kernel's
    # launches fall from about 880 to 780 us over the first 40 steps, the list build's by
    # 4 %, then stay flat), so untimed settle steps come before the warm-up: the timed
    # steps are then those of a long run whatever the warm-up count
    for _ in range(settle):
        md.step()
    for _ in range(warmup):
        md.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        md.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the stage breakdown from further steps with the stage timers on (their events add
    # queue packets between the kernels, so the timed steps above run without them)
    ev.timers(True)
    ev.read_timers(reset=True)
    for _ in range(min(steps, 20)):
        md.step()
    tm = ev.read_timers(reset=True)
    ev.timers(False)
    return ev, model, el, tm


def production_nvt(engine, torch, st, beta, sigma, steps, warmup, every=10):
    """The production-run form (Section VI.A): Nose-Hoover NVT at 450 K, dt 0.1 fs, tau
    10 fs, starting from Maxwell-Boltzmann velocities at 450 K, with hydrogen coordination,
    reaction events and the uncertainty monitor (threshold 0.005) every `every` steps."""
    import numpy as np

    from paper_2204_12573_amd import structures as S
    n = st.n
    model = engine.Model(beta, sigma)
    ev = engine.Evaluator(model, max_atoms=n, max_pairs=12 * n)
    p, s = engine.to_device(st.pos, st.species)
    v = torch.from_numpy(np.ascontiguousarray(S.maxwell_boltzmann(st.species, 450.0, seed=1).T)).cuda()
    # skin 0.25 A: the fastest atom of this 450 K start moves 0.107 A per 10-step interval,
    # more than half of a 0.2 A skin (the engine raises when an interval exceeds it)
    nvt = engine.NVT(ev, p, v, s, [0, n], st.box, t_target=450.0, tau=10.0, dt=0.1, skin=0.25, rebuild=10)
    prod = engine.Production(nvt, every=every, threshold=0.005)
    # its own warm-up: at least two monitor intervals and one list rebuild, so that the
    # first coordination, monitor and rebuild calls are outside the timed region whatever
    # the caller's --warmup
    for _ in range(max(warmup, 2 * every, 10)):
        prod.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prod.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    th = nvt.thermo.cpu().numpy()[0]
    nf = 3 * n - 3
    return {"value": round(n * steps / el / 1e6, 3), "ms_per_step": round(el / steps * 1e3, 4),
            "steps": steps, "monitor_every": every, "t_kinetic_K": float(2 * th[2] / (nf * 8.617333262e-5)),
            "zeta_per_fs": float(th[0]), "reaction_events": prod.events.cpu().numpy()[0].tolist(),
            "max_sigma": float(prod.sigma_max.max()), "cells_over_threshold": len(prod.flagged_cells()),
            "note": "Nose-Hoover NVT 450 K, dt 0.1 fs, tau 10 fs, list every 10 steps (skin 0.25 A); coordination, "
                    "reaction events and max-sigma monitor every 10 steps (synthetic random-weight model: "
                    "sigma values are not physical)"}


def form_roofline(prec, fused_work, t_launch):
    """Bound of the fused kernel of the 144-wide rows in a split form: its matrix work at the
    peak of each instruction type plus its vector work at the FP32 vector peak (the matrix
    and vector instructions share the SIMD datapath). Per row: the energy pass takes
    `products` part products of 2*144^2 flop (BF16 x3: 3, FP8 x3: 3, BF16 x6: 6) on the
    form's matrix type; the variance |L^T d|^2 takes 144*145 flop on FP64 matrix cores, or on
    FP32 ones with FLARE_VAR_FP32."""
    from paper_2204_12573_amd import binding as B
    base = prec & ~B.VAR_FP32
    products, peak, kind = {B.BF16_SPLIT: (3, PEAK_BF16_MFMA, "bf16"), B.FP8_SPLIT: (3, PEAK_FP8_MFMA, "fp8"),
                            B.BF16X6_SPLIT: (6, PEAK_BF16_MFMA, "bf16")}[base]
    var_peak = PEAK_FP32_MFMA if prec & B.VAR_FP32 else PEAK_FP64_MFMA
    n144 = fused_work["n144"]
    e_flops = n144 * products * 2 * 144 * 144
    v_flops = n144 * (144 * 145 if fused_work["vchol"] else 2 * 144 * 144)
    parts = {"energy_pass_us": e_flops / peak * 1e6, "variance_pass_us": v_flops / var_peak * 1e6,
             "vector_us": fused_work["valu_flops"] / PEAK_FP32_VALU * 1e6}
    t_min = sum(parts.values()) * 1e-6
    return {"bound": "alu", "t_min_us": round(t_min * 1e6, 1), "avg_launch_us": round(t_launch * 1e6, 1),
            "frac": round(t_min / t_launch, 3), "parts_us": {k: round(v, 1) for k, v in parts.items()},
            "peak_derivation": f"energy pass {products} products on {kind} matrix cores "
                               f"({peak / 1e12:.0f} TFLOP/s), variance on "
                               f"{'FP32' if prec & B.VAR_FP32 else 'FP64'} matrix cores "
                               f"({var_peak / 1e12:.1f} TFLOP/s), vector work at 78.6 TFLOP/s, summed "
                               f"(one datapath)"}


def measured_ceilings(torch):
    """Ceilings reached on this device by plain library work, beside the published peaks the
    roofline uses: a 1 GiB device-to-device copy (read + write bytes) and a 8192^3 FP32
    matrix product through torch (the ROCm BLAS library, no reduced-precision modes),
    each the best of five after a warm-up."""
    x = torch.empty(2**28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    a = torch.randn(8192, 8192, dtype=torch.float32, device="cuda")
    b = torch.randn(8192, 8192, dtype=torch.float32, device="cuda")
    torch.backends.cuda.matmul.allow_tf32 = False

    def best(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts)

    t_copy = best(lambda: y.copy_(x))
    t_mm = best(lambda: torch.matmul(a, b))
    out = {"hbm_copy_TBps": round(2 * x.numel() * 4 / t_copy / 1e12, 2),
           "sgemm_fp32_TFLOPs": round(2 * 8192**3 / t_mm / 1e12, 1),
           "note": "best of 5: 1 GiB device copy (read + write), torch FP32 8192^3 matmul; the roofline "
                   "fractions use the published peaks (HBM 8 TB/s, FP32 matrix 157.3 TFLOP/s)"}
    del x, y, a, b
    torch.cuda.empty_cache()
    return out


def valu_work(engine, st):
    """Pairs inside the cutoff whose centre has a single-species environment (the rows of
    the fused kernel), from the library's own list of the initial positions."""
    import numpy as np
    model = engine.Model(np.zeros((2, 544, 544)), np.zeros((2, 544, 544)))
    ev = engine.Evaluator(model, max_atoms=st.n, max_pairs=12 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    ev.neighbors(p, s, [0, st.n], st.box, 0.2)
    off, j, sh = ev.export_list()
    del ev, model
    cnt = np.diff(off)
    i = np.repeat(np.arange(st.n), cnt)
    d = st.pos[j] + sh * st.box - st.pos[i]
    inside = (d * d).sum(1) < 4.5 ** 2
    # environment class over the listed pairs, as the library classifies rows
    spj = st.species[j]
    n_h = np.bincount(i, weights=(spj == 0), minlength=st.n)
    n_pt = np.bincount(i, weights=(spj == 1), minlength=st.n)
    single = (n_h > 0) ^ (n_pt > 0)
    mixed = (n_h > 0) & (n_pt > 0)
    return {"pairs144": int(np.count_nonzero(inside & single[i])),
            "pairs544": int(np.count_nonzero(inside & mixed[i]))}


def sample_errors(engine, torch, st, beta, sigma, precision, tg, ref):
    """E, F, sigma of one evaluation at the initial positions vs the FP64 oracle sample."""
    import numpy as np
    model = engine.Model(beta, sigma, precision=precision)
    ev = engine.Evaluator(model, max_atoms=st.n, max_pairs=12 * st.n)
    p, s = engine.to_device(st.pos, st.species)
    ev.neighbors(p, s, [0, st.n], st.box, 0.2)
    out = ev.compute(p, want_var=True)
    torch.cuda.synchronize()
    rows = ref.row_of(tg)
    e = out["e"].cpu().numpy()[tg]
    f = out["f"].cpu().numpy().T[tg]
    sg = out["sigma"].cpu().numpy()[tg]
    return {"e": float(np.abs(e - ref.e[rows]).max() / np.abs(ref.e[rows]).max()),
            "f": float(np.linalg.norm(f - ref.f, axis=1).max() / np.linalg.norm(ref.f, axis=1).max()),
            "sigma": float(np.abs(sg - ref.sigma[rows]).max() / np.abs(ref.sigma[rows]).max())}


def precision_16m(engine, torch, small, beta, sigma, half_width=13.1, evals=5):
    """The ~16 M-atom precision workload: the 1 M-atom cell tiled 4 x 4 laterally
    (400 x 400 x 24 Pt(111) under the same gas column), one list build and `evals` timed
    E + F + sigma evaluations per arithmetic form (inputs resident), errors against the FP64
    oracle on a seeded subsample of ~10,000 atoms: every atom of a 2*half_width A square
    column through slab, surface and gas at a seeded position (neighbouring sampled atoms
    share the oracle's work), each taken from a random copy. The oracle evaluates them in the
    1 M-atom cell, whose environments all copies share."""
    import numpy as np

    from oracle import evaluate as oev
    from paper_2204_12573_amd import binding, structures as S
    big = S.tiled(small, 4, 4)
    n, n1 = big.n, small.n
    rng = np.random.default_rng(2204)
    cx, cy = rng.uniform(0.0, 1.0, 2) * small.box[:2]
    dx = np.abs((small.pos[:, 0] - cx + 0.5 * small.box[0]) % small.box[0] - 0.5 * small.box[0])
    dy = np.abs((small.pos[:, 1] - cy + 0.5 * small.box[1]) % small.box[1] - 0.5 * small.box[1])
    tg = np.nonzero((dx < half_width) & (dy < half_width))[0]
    n_sample = len(tg)
    log(f"  oracle on {n_sample} sampled atoms ...")
    t0 = time.perf_counter()
    ref = oev.evaluate(small.pos, small.species, small.box, beta, sigma, targets=tg)
    t_oracle = time.perf_counter() - t0
    rows = ref.row_of(tg)
    atoms = rng.integers(0, 16, len(tg)) * n1 + tg
    # environment class of each sampled atom from the oracle's descriptor blocks: (H,H)
    # components only, (Pt,Pt) only, or some in the cross block (mixed)
    dref = ref.d[rows]
    hh, cross, ptpt = (np.abs(dref[:, :144]).max(1) > 0, np.abs(dref[:, 144:400]).max(1) > 0,
                       np.abs(dref[:, 400:]).max(1) > 0)
    classes = {"h_only": hh & ~cross & ~ptpt, "pt_only": ptpt & ~cross & ~hh, "mixed": cross}
    p, s = engine.to_device(big.pos, big.species)
    forms = {}
    for name, prec in (("plain_fp32", 0), ("mixed_bf16_split", binding.BF16_SPLIT),
                       ("mixed_fp8_split", binding.FP8_SPLIT), ("mixed_bf16x6_split", binding.BF16X6_SPLIT),
                       ("mixed_bf16x6_split_var32", binding.BF16X6_SPLIT | binding.VAR_FP32)):
        log(f"  {name} on {n} atoms ...")
        model = engine.Model(beta, sigma, precision=prec)
        ev = engine.Evaluator(model, max_atoms=n, max_pairs=12 * n)
        ev.neighbors(p, s, [0, n], big.box, 0.2)
        out = ev.compute(p, want_var=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(evals):
            out = ev.compute(p, want_var=True, out=out)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / evals
        status = ev.status()
        e = out["e"].cpu().numpy()[atoms]
        f = out["f"].cpu().numpy().T[atoms]
        sg = out["sigma"].cpu().numpy()[atoms]
        def errs(m):
            return {"atoms": int(m.sum()),
                    "e": float(np.abs(e[m] - ref.e[rows][m]).max() / np.abs(ref.e[rows][m]).max()),
                    "f": float(np.linalg.norm(f[m] - ref.f[m], axis=1).max()
                               / np.linalg.norm(ref.f[m], axis=1).max()),
                    "sigma": float(np.abs(sg[m] - ref.sigma[rows][m]).max() / np.abs(ref.sigma[rows][m]).max())}
        forms[name] = {
            "M_atom_evals_per_s": round(n / el / 1e6, 1), "ms_per_eval": round(el * 1e3, 3),
            "status_flags": status,
            "err_vs_fp64_oracle": {k: v for k, v in errs(np.ones(len(tg), bool)).items() if k != "atoms"},
            "err_by_class": {c: errs(m) for c, m in classes.items() if m.any()}}
        del out, ev, model
        torch.cuda.synchronize()
    return {"atoms": n, "cell": "1 M-atom cell tiled 4 x 4 (400 x 400 x 24 Pt(111) + H2 gas)",
            "evals_timed": evals,
            "sample": f"{n_sample} atoms of a {2*half_width:.1f} A square column at a seeded position, each "
                      f"from a random copy; FP64 oracle {t_oracle:.1f} s",
            "forms": forms}


def serving(engine, torch, beta, sigma, n_req, rate, warmup=1000, pool=2000):
    """Open-loop Poisson stream of warmup + n_req requests (structures drawn from a pool of
    distinct slabs of log-uniform size); statistics over the n_req after the warm-up."""
    import sys as _sys

    from paper_2204_12573_amd import binding, serve
    _sys.setswitchinterval(1e-4)       # quick hand-offs between the scheduler and lane threads
    out = {}
    reqs_proto = serve.poisson_requests(warmup + n_req, rate=rate, seed=7, pool=pool)
    for name, prec, lanes, mb, chunk in [("batched_split", binding.BF16_SPLIT, 2, 10**9, None),
                                         ("one_at_a_time_fp32", binding.FP32, 1, 1, None)]:
        reqs = [serve.Request(r.rid, r.arrival, r.pos, r.species, r.box) for r in reqs_proto]
        model = engine.Model(beta, sigma, precision=prec)
        ex = serve.GpuExecutor(model, n_lanes=lanes, lane_atoms=400_000)
        # first use of each lane outside the stream
        serve.Scheduler(ex, max_batch=mb).run([serve.Request(-1 - k, 0.0, r.pos, r.species, r.box)
                                               for k, r in enumerate(reqs[:4])])
        torch.cuda.synchronize()
        _, stats = serve.Scheduler(ex, max_batch=mb, chunk_atoms=chunk).run(reqs, warmup=warmup)
        stats = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()}
        stats["chunk_atoms"] = chunk
        stats["lanes"] = lanes
        stats["lane_state_bytes"] = int(ex.lane_bytes)
        out[name] = stats
        ex.close()
        del ex, model
    out["offered"] = {"rate_req_s": rate, "requests": n_req, "warmup_requests": warmup,
                      "distinct_structures": pool,
                      "mean_atoms": float(sum(r.n for r in reqs_proto[warmup:]) / n_req)}
    return out


def autograd_cells(engine, torch, beta, sigma):
    import numpy as np

    from paper_2204_12573_amd import autograd as AG, structures as S
    b = S.config_cells(n_cells=256, seed=0)
    model = engine.Model(beta, sigma)
    mod = AG.FlareEnergy(model, b.species, b.offsets, b.boxes)
    pos = torch.from_numpy(np.ascontiguousarray(b.pos.T)).cuda().requires_grad_(True)
    for _ in range(2):
        E = mod(pos)
        (g,) = torch.autograd.grad(E.sum(), pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        E = mod(pos)
        (g,) = torch.autograd.grad(E.sum(), pos)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    npairs, counts = mod.ev.list_info()
    held = mod.ev.memory_bytes(with_model=False)
    stored = AG.stored_gradient_bytes(npairs, counts[:4].sum(), counts[4:].sum(), npairs, 0)
    return {"cells": 256, "atoms": int(b.n), "pairs": int(npairs), "ms_forward_backward": round(dt * 1e3, 3),
            "M_atom_grad_per_s": round(b.n / dt / 1e6, 3), "state_bytes": int(held),
            "stored_dd_dr_bytes": int(stored["dd_dr_full"]), "stored_dc_dr_bytes": int(stored["dc_dr"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--settle", type=int, default=60,
                    help="untimed MD steps before the warm-up (the GPU's speed settles under load)")
    ap.add_argument("--no-forms", action="store_true", help="skip the split-precision, serving and autograd legs")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--no-huge", action="store_true", help="skip the ~16 M-atom precision leg")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8", "bf16x6", "bf16x6-var32"],
                    help="arithmetic form of the main MD leg (default fp32; the others for profiling)")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured ceilings (library copy and GEMM), e.g. under a profiler")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy, a kernel of known traffic for counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design "
                                   "note, not part of this build", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_12573_amd import engine, structures as S

    if args.copy_calibration:
        a = torch.empty(64 * 2**20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
    log("generating workload ...")
    st = S.config_large()
    beta, sigma = S.random_model(544)
    n = st.n
    from paper_2204_12573_amd import binding as B
    main_prec = {"fp32": 0, "bf16": B.BF16_SPLIT, "fp8": B.FP8_SPLIT, "bf16x6": B.BF16X6_SPLIT,
                 "bf16x6-var32": B.BF16X6_SPLIT | B.VAR_FP32}[args.precision]
    ev, model, el, tm = md_throughput(engine, torch, st, beta, sigma, args.steps, args.warmup, main_prec,
                                      settle=args.settle)
    npairs, counts = ev.list_info()
    status = ev.status()
    log(f"atoms {n}, pairs {npairs}, buckets {counts.tolist()}")
    value = n * args.steps / el / 1e6
    log(f"{args.steps} steps in {el*1e3:.1f} ms -> {value:.2f} M atom-steps/s, status {status}")
    for k, (ms, c) in tm.items():
        if c:
            log(f"  {k:9s} {ms/c*1e3:9.1f} us/launch x {c}")
    vchol = model.variance_cholesky
    del ev, model
    work = valu_work(engine, st)

    # dominant kernel: quadratic forms on the 144-wide rows (beta and Sigma, E+V). Algorithmic
    # flops per row: Y = beta d (2*144^2) and V = |L^T d|^2 through the triangular factor
    # (144*145, one multiply-add per nonzero of L), or d^T Sigma d (2*144^2) without it.
    n144 = int(counts[:4].sum())
    n544 = int(counts[4:].sum())
    q_ms, q_cnt = tm["qform144"]
    flops_per_row = 2 * 144 * 144 + (144 * 145 if vchol else 2 * 144 * 144)
    flops_per_launch = n144 * flops_per_row
    t_launch = q_ms / q_cnt * 1e-3
    # FP32 matrix instructions and FP32 vector instructions share one datapath on gfx950
    # (measured: a wave issuing MFMAs and a wave issuing FMAs on the same SIMD take the sum
    # of their separate times), so the kernel is bound by that datapath: its time is at
    # least the MFMA work at the matrix peak plus the vector work at the non-packed vector
    # peak. The bound's peak is the blend of the two for this kernel's mix of work.
    valu_flops = work["pairs144"] * (VALU_FLOP_DENS + VALU_FLOP_ADJ) + n144 * (
        VALU_FLOP_B2 + VALU_FLOP_NORM + VALU_FLOP_EPI + VALU_FLOP_U)
    t_min = flops_per_launch / PEAK_FP32_MFMA + valu_flops / PEAK_FP32_VALU
    fused_work = {"n144": n144, "valu_flops": valu_flops, "vchol": vchol}
    total = flops_per_launch + valu_flops
    roofline = {"bound": "alu", "achieved": total / t_launch / 1e12, "peak": total / t_min / 1e12,
                "unit": "TFLOP/s", "frac": t_min / t_launch, "traffic": profiled_traffic(),
                "kernel": "k_fused144_w (144-wide rows: descriptors, D[L] and D[beta] on FP32 MFMA, adjoint "
                          "terms; FP32 matrix and vector instructions share the SIMD datapath)",
                "peak_derivation": "blend of the FP32 MFMA peak (157.3 TFLOP/s) and the non-packed FP32 vector "
                                   "peak (78.6 TFLOP/s = 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz) "
                                   "weighted by this kernel's matrix and vector flops",
                "mfma_flop_per_launch": flops_per_launch, "mfma_flop_per_row": flops_per_row,
                "valu_flop_per_launch": int(valu_flops), "pairs_in_cutoff_144": int(work["pairs144"]),
                "t_min_us": t_min * 1e6, "avg_launch_us": t_launch * 1e6,
                "variance_form": "cholesky" if vchol else "full",
                "mfma_only": {"achieved": flops_per_launch / t_launch / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                              "frac": flops_per_launch / t_launch / PEAK_FP32_MFMA}}
    # whole step against its ideal time: every stage at the bound of its algorithmic work
    # (the per-unit figures of the method; stage-internal layouts such as the per-slot pair
    # geometry are implementation, not algorithmic work):
    #   144-wide rows  the fused kernel's t_min above (matrix + vector flops);
    #   544-wide rows  Y = D beta (2 544^2) and Z = D L (544 * 545) per row on the FP32 matrix
    #                  cores, vector work per pair (densities 320, adjoint 830) and per row
    #                  (B2 4352, |d~|^2 1088, epilogue e, g, V 3808, u 8192) at the vector peak;
    #   list build     100 B per Pt atom, 50 B per H atom of HBM traffic, every `rebuild` steps;
    #   integrator, reductions and outputs  100 B per atom of HBM traffic.
    n_pt = int((st.species == 1).sum())
    mx_mfma = n544 * (2 * 544 * 544 + (544 * 545 if vchol else 2 * 544 * 544))
    mx_valu = work["pairs544"] * (VALU_FLOP_DENS + VALU_FLOP_ADJ) + n544 * (4352 + 1088 + 3808 + 8192)
    t_parts = {"rows144_fused": t_min,
               "rows544": mx_mfma / PEAK_FP32_MFMA + mx_valu / PEAK_FP32_VALU,
               "list_build": (n_pt * 100 + (n - n_pt) * 50) / PEAK_HBM / 10,
               "integrator_outputs": n * 100 / PEAK_HBM}
    t_ideal = sum(t_parts.values())
    t_step = el / args.steps
    step_roofline = {"t_ideal_us": t_ideal * 1e6, "t_measured_us": t_step * 1e6, "frac": t_ideal / t_step,
                     "parts_us": {k: round(v * 1e6, 2) for k, v in t_parts.items()},
                     "note": "T_ideal / T_measured of one whole MD step (list rebuilds amortised), each stage "
                             "at the bound of its algorithmic work (FP32 matrix 157.3, FP32 vector 78.6 "
                             "TFLOP/s, HBM 8 TB/s)"}
    stage_us = {k: round(ms / max(c, 1) * 1e3, 1) for k, (ms, c) in tm.items() if c}
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "M atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_steps": args.settle,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "H2 gas over Pt(111) 100x100x24, ~1.0 M atoms, NVE dt 0.5 fs, rebuild every 10",
                   "atoms": n, "pairs": int(npairs), "rows144": n144, "rows544": n544,
                   "n_desc": 544, "r_cut": 4.5, "skin": 0.2, "precision": args.precision},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "measured_ceilings": None if args.no_ceilings else measured_ceilings(torch),
        "stage_us_per_launch": stage_us,
        "status_flags": status,
    }
    if not args.no_forms:
        from paper_2204_12573_amd import binding
        from oracle import evaluate as oev
        log("split-precision MD ...")
        ev2, m2, el2, tm2 = md_throughput(engine, torch, st, beta, sigma, args.steps, args.warmup,
                                          binding.BF16_SPLIT)
        del ev2, m2
        ev3, m3, el3, tm3 = md_throughput(engine, torch, st, beta, sigma, args.steps, args.warmup,
                                          binding.FP8_SPLIT)
        del ev3, m3
        ev6, m6, el6, tm6 = md_throughput(engine, torch, st, beta, sigma, args.steps, args.warmup,
                                          binding.BF16X6_SPLIT)
        del ev6, m6
        ev7, m7, el7, tm7 = md_throughput(engine, torch, st, beta, sigma, args.steps, args.warmup,
                                          binding.BF16X6_SPLIT | binding.VAR_FP32)
        del ev7, m7
        log("errors vs the FP64 oracle on a 300-atom sample ...")
        rng = np.random.default_rng(12)
        ztop = 23 * S.DZ
        surf = np.nonzero(np.abs(st.pos[:, 2] - ztop) < 4.0)[0]
        tg = np.unique(np.concatenate([rng.choice(n, 200, replace=False), rng.choice(surf, 100, replace=False)]))
        ref = oev.evaluate(st.pos, st.species, st.box, beta, sigma, targets=tg)
        out["plain_fp32"] = {"value": round(value, 3),
                             "err_vs_fp64_oracle": sample_errors(engine, torch, st, beta, sigma, 0, tg, ref)}
        out["mixed_bf16_split"] = {
            "value": round(n * args.steps / el2 / 1e6, 3), "ms_per_step": round(el2 / args.steps * 1e3, 4),
            "err_vs_fp64_oracle": sample_errors(engine, torch, st, beta, sigma, binding.BF16_SPLIT, tg, ref),
            "stage_us_per_launch": {k: round(ms / max(c, 1) * 1e3, 1) for k, (ms, c) in tm2.items() if c},
            "roofline": form_roofline(binding.BF16_SPLIT, fused_work, tm2["qform144"][0] / tm2["qform144"][1] * 1e-3),
            "note": "energy pass BF16 x3 (d and beta split hi/lo), variance |L^T d|^2 with the FP64 factor "
                    "on FP64 matrix cores, FP64 sums; mixed-environment rows: FP32 energy, FP64 variance"}
        out["mixed_fp8_split"] = {
            "value": round(n * args.steps / el3 / 1e6, 3), "ms_per_step": round(el3 / args.steps * 1e3, 4),
            "err_vs_fp64_oracle": sample_errors(engine, torch, st, beta, sigma, binding.FP8_SPLIT, tg, ref),
            "stage_us_per_launch": {k: round(ms / max(c, 1) * 1e3, 1) for k, (ms, c) in tm3.items() if c},
            "roofline": form_roofline(binding.FP8_SPLIT, fused_work, tm3["qform144"][0] / tm3["qform144"][1] * 1e-3),
            "note": "energy pass OCP e4m3 x3 with power-of-two row and block scales (d and beta split "
                    "hi/lo'), variance as in the BF16 form (FP64); mixed-environment rows: FP32 energy"}
        out["mixed_bf16x6_split"] = {
            "value": round(n * args.steps / el6 / 1e6, 3), "ms_per_step": round(el6 / args.steps * 1e3, 4),
            "err_vs_fp64_oracle": sample_errors(engine, torch, st, beta, sigma, binding.BF16X6_SPLIT, tg, ref),
            "stage_us_per_launch": {k: round(ms / max(c, 1) * 1e3, 1) for k, (ms, c) in tm6.items() if c},
            "roofline": form_roofline(binding.BF16X6_SPLIT, fused_work, tm6["qform144"][0] / tm6["qform144"][1] * 1e-3),
            "note": "energy pass on BF16 matrix cores with d and beta split into three BF16 parts "
                    "(x0 + x1 + x2 = the FP32 value), six of the nine part products, FP32 accumulation "
                    "(FP32-level error); variance |L^T d|^2 with the FP64 factor on FP64 matrix cores; FP64 "
                    "norms and sums; mixed-environment rows: FP32 energy, FP64 variance"}
        out["mixed_bf16x6_split_var32"] = {
            "value": round(n * args.steps / el7 / 1e6, 3), "ms_per_step": round(el7 / args.steps * 1e3, 4),
            "err_vs_fp64_oracle": sample_errors(engine, torch, st, beta, sigma,
                                                binding.BF16X6_SPLIT | binding.VAR_FP32, tg, ref),
            "stage_us_per_launch": {k: round(ms / max(c, 1) * 1e3, 1) for k, (ms, c) in tm7.items() if c},
            "roofline": form_roofline(binding.BF16X6_SPLIT | binding.VAR_FP32, fused_work, tm7["qform144"][0] / tm7["qform144"][1] * 1e-3),
            "note": "the three-way BF16 energy pass with the variance through the FP32 factor on FP32 "
                    "matrix cores (FLARE_VAR_FP32: the plain form's variance error, not FP64)"}
        if not args.no_huge:
            log("precision forms at ~16 M atoms ...")
            out["precision_16m"] = precision_16m(engine, torch, st, beta, sigma)
        log("production NVT ...")
        out["production_nvt"] = production_nvt(engine, torch, st, beta, sigma, args.steps, args.warmup)
        log("serving ...")
        out["serving"] = serving(engine, torch, beta, sigma, args.serve_requests, 2000.0)
        log("autograd (256 cells) ...")
        out["autograd"] = autograd_cells(engine, torch, beta, sigma)
    if not args.no_cpu_baseline:
        log("oracle CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline(st, beta, sigma)
        out["cpu_oracle_tiny"] = oracle_tiny_run(beta, sigma)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
