"""Differentiation form: per-cell energies as a torch.autograd.Function.

forward(pos) evaluates E_k = sum_{i in cell k} e_i (Eq. 1) for every cell; backward(gE)
returns dL/dr = -gE_k F_i through the hand-written adjoint (the reordered sum of the
paper's Section V.B). Nothing per pair is kept between the two passes except the pair
geometry and the per-atom energy gradients g_i = de_i/dd~_i: the densities and every
pair term of the adjoint are recomputed in backward, instead of storing the descriptor
gradients dd/dr that a generic autodiff of the descriptor would keep (the memory the
paper bounds by batching atoms, Section V.C).

First order only: a second backward raises.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.autograd.function import once_differentiable

from . import engine


class _EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, module):
        module._stage(pos)
        out = module.ev.energies()
        ctx.module = module
        ctx.gen = module._gen
        ctx.save_for_backward(pos)
        return out["E"].clone()

    @staticmethod
    @once_differentiable
    def backward(ctx, gE):
        (pos,) = ctx.saved_tensors
        m = ctx.module
        if m._gen != ctx.gen:          # another forward ran since: recompute for these positions
            m._stage(pos.detach())
            m.ev.energies()
        scale = (-gE).to(torch.float64).contiguous()
        f = m.ev.forces(cell_scale=scale)
        return f.to(pos.dtype), None


class FlareEnergy(torch.nn.Module):
    """E per cell for positions pos [3, N] (FP64, device) of a fixed batch of cells.

    model: engine.Model; species: int32 [N] (numpy or device); offsets: host int32
    [n_cells+1]; boxes: host [n_cells, 3]. The neighbour list (radius r_cut + skin) is
    rebuilt every `rebuild_every` forward calls (1 = always).
    """

    def __init__(self, model, species, offsets, boxes, skin=0.2, max_pairs=None, rebuild_every=1):
        super().__init__()
        n = int(offsets[-1])
        self.ev = engine.Evaluator(model, max_atoms=max(n, 1), max_pairs=max_pairs or max(64 * n, 1024))
        self.species = species if isinstance(species, torch.Tensor) else \
            torch.from_numpy(np.asarray(species, np.int32)).to(self.ev.device)
        self.offsets = np.asarray(offsets, np.int32)
        self.boxes = np.asarray(boxes, np.float64).reshape(-1, 3)
        self.skin = skin
        self.rebuild_every = rebuild_every
        self._calls = 0
        self._gen = 0

    def _stage(self, pos):
        p = pos.detach()
        if p.dtype != torch.float64 or not p.is_contiguous():
            p = p.to(torch.float64).contiguous()
        if self._calls % self.rebuild_every == 0:
            self.ev.neighbors(p, self.species, self.offsets, self.boxes, self.skin)
        self._calls += 1
        self._gen += 1
        self.ev.descriptors(p)

    def forward(self, pos):
        return _EnergyFn.apply(pos, self)


def stored_gradient_bytes(n_pairs_in_cutoff, n_rows_single, n_rows_mixed, pairs_single, pairs_mixed):
    """Bytes a store-everything backward would keep (FP32), for comparison:
    dd~/dr per pair over the full 544 components, over the blocks actually non-zero
    (144 for single-species rows), and dc/dr per pair (16 x 8 channels of one species)."""
    return {
        "dd_dr_full": int(n_pairs_in_cutoff) * 544 * 3 * 4,
        "dd_dr_blocks": (int(pairs_single) * 144 + int(pairs_mixed) * 544) * 3 * 4,
        "dc_dr": int(n_pairs_in_cutoff) * 8 * 16 * 3 * 4,
    }
