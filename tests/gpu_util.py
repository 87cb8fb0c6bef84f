"""Helpers for the GPU tests: run the HIP path through the C ABI and compare with the
FP64 oracle using the relative error measures of the parity bar:
  energy, sigma: max_i |x_i - ref_i| / max_i |ref_i|
  forces:        max_i |F_i - F_ref_i|_2 / max_i |F_ref_i|_2
"""
import numpy as np
import torch

from paper_2204_12573_amd import engine

TOL = 1e-5     # relative bound on energies, forces and sigma (FP32 path vs FP64 oracle)


def rel_max(x, ref):
    x, ref = np.asarray(x, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def rel_vec(f, ref):
    f, ref = np.asarray(f, np.float64), np.asarray(ref, np.float64)
    return float(np.linalg.norm(f - ref, axis=1).max() / max(np.linalg.norm(ref, axis=1).max(), 1e-300))


def gpu_eval(pos, species, box_or_boxes, beta, sigma, offsets=None, skin=0.2, want_d=False,
             max_pairs=None, precision=0):
    """Full evaluation on the GPU; returns numpy arrays in the caller's atom order."""
    n = len(species)
    boxes = np.asarray(box_or_boxes, np.float64).reshape(-1, 3)
    if offsets is None:
        offsets = np.array([0, n], np.int32)
    model = engine.Model(beta, sigma, precision=precision)
    ev = engine.Evaluator(model, max_atoms=max(n, 1), max_pairs=max_pairs or max(64 * n, 1024))
    p, s = engine.to_device(pos, species)
    ev.neighbors(p, s, offsets, boxes, skin)
    d, nrm = ev.descriptors(p, want_d=want_d, want_norm=True)
    out = ev.energy_forces(want_var=True)
    var = ev.variance()
    torch.cuda.synchronize()
    res = {
        "e": out["e"].cpu().numpy(),
        "f": out["f"].cpu().numpy().T.copy(),
        "E": out["E"].cpu().numpy(),
        "var": out["var"].cpu().numpy(),
        "sigma": out["sigma"].cpu().numpy(),
        "var2": var["var"].cpu().numpy(),
        "sigma_max": var["sigma_max"].cpu().numpy(),
        "norm": nrm.cpu().numpy(),
        "d": d.cpu().numpy() if d is not None else None,
        "ev": ev,
        "model": model,
        "status": ev.status(),
    }
    return res
