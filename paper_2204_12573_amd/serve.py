"""Continuous-batching service for energy / force / uncertainty requests.

Requests are periodic cells of uneven size (active-learning candidate screening). The
scheduler keeps several *lanes*: one HIP stream, one device-resident evaluation state
(neighbour list, descriptors, gradients) and pinned host staging buffers each. Whenever
a lane is free it takes the oldest waiting requests (FIFO) up to the lane's HBM
footprint budget, uploads them, and enqueues one launch sequence for the whole batch
(list build, descriptors, energies + forces + variances, download). Requests arriving
while batches run wait in the queue and are admitted as soon as a lane frees up; with
two or more lanes the batches of different lanes overlap on the device. Latency is
measured from a request's arrival to its results being on the host.

Per-cell results do not depend on the batch composition (the library computes each row
independently and gathers forces in a fixed order), so a structure gives the same bits
alone and in any mix.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds, on the server clock
    pos: np.ndarray           # [n, 3] FP64
    species: np.ndarray       # [n] int32
    box: np.ndarray           # [3]
    t_start: float = -1.0
    t_done: float = -1.0
    e: np.ndarray | None = None
    f: np.ndarray | None = None
    sigma: np.ndarray | None = None
    energy: float | None = None

    @property
    def n(self) -> int:
        return len(self.species)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Footprint:
    """Device bytes a batch needs: per-atom arrays, per-pair list, sliced slots
    (with padding headroom) and descriptor/gradient rows."""

    def __init__(self, pairs_per_atom=22.0, slot_overhead=1.6):
        self.ppa = pairs_per_atom
        self.slot = slot_overhead

    def atoms_pairs(self, n_atoms):
        return n_atoms, int(self.ppa * n_atoms) + 64

    def bytes(self, n_atoms):
        n, p = self.atoms_pairs(n_atoms)
        per_atom = 4 * 16 + 8 * 12 + 4 * 6 + 8 * 32   # int arrays, FP64 SoA, FP32 outputs, pair cache
        per_pair = 4 * 4                                # j, shift, reverse, slot of pair
        per_slot = 4 * 3 + 16 * 3                       # slot ints, fixed pair vector, geometry, reverse term
        rows = 2 * 144 * 4 + 16 + 5 * 4                 # descriptor + gradient, own force, row copies
        return n * (per_atom + rows) + p * (per_pair + self.slot * per_slot)


class GpuExecutor:
    """Lanes on the GPU: each has its own torch stream and flare state."""

    def __init__(self, model, n_lanes=2, lane_atoms=400_000, footprint=None, want_var=True):
        import torch

        from . import engine

        self.torch = torch
        self.engine = engine
        self.model = model
        self.fp = footprint or Footprint()
        self.want_var = want_var
        self.lanes = []
        for _ in range(n_lanes):
            st = torch.cuda.Stream()
            n, p = self.fp.atoms_pairs(lane_atoms)
            ev = engine.Evaluator(model, max_atoms=n, max_pairs=p, stream=st)
            self.lanes.append({"stream": st, "ev": ev, "busy": None,
                               "pin_pos": torch.empty((3, n), dtype=torch.float64).pin_memory(),
                               "pin_sp": torch.empty(n, dtype=torch.int32).pin_memory(),
                               "dev_pos": torch.empty((3, n), dtype=torch.float64, device="cuda"),
                               "dev_sp": torch.empty(n, dtype=torch.int32, device="cuda"),
                               "host": {"e": torch.empty(n, dtype=torch.float32).pin_memory(),
                                        "f": torch.empty((3, n), dtype=torch.float32).pin_memory(),
                                        "sigma": torch.empty(n, dtype=torch.float32).pin_memory(),
                                        "E": torch.empty(n, dtype=torch.float64).pin_memory()}})
        self.lane_atoms = lane_atoms
        self.budget = self.fp.bytes(lane_atoms)

    def launch(self, k, batch):
        """Upload and enqueue one batch on lane k (returns after the list build)."""
        torch = self.torch
        lane = self.lanes[k]
        n = sum(r.n for r in batch)
        offs = np.zeros(len(batch) + 1, np.int32)
        offs[1:] = np.cumsum([r.n for r in batch])
        boxes = np.stack([r.box for r in batch])
        pp = lane["pin_pos"][:, :n].numpy()
        ps = lane["pin_sp"][:n].numpy()
        for r, a in zip(batch, offs[:-1]):
            pp[:, a:a + r.n] = r.pos.T
            ps[a:a + r.n] = r.species
        st = lane["stream"]
        with torch.cuda.stream(st):
            pos = lane["dev_pos"][:, :n]
            sp = lane["dev_sp"][:n]
            pos.copy_(lane["pin_pos"][:, :n], non_blocking=True)
            sp.copy_(lane["pin_sp"][:n], non_blocking=True)
            ev = lane["ev"]
            ev.neighbors(pos, sp, offs, boxes, 0.0)
            ev.descriptors(pos)
            out = ev.energy_forces(want_var=self.want_var)
            hb = lane["host"]
            host = {"e": hb["e"][:n], "f": hb["f"][:, :n], "E": hb["E"][:len(batch)]}
            host["e"].copy_(out["e"], non_blocking=True)
            host["f"].copy_(out["f"], non_blocking=True)
            host["E"].copy_(out["E"], non_blocking=True)
            if self.want_var:
                host["sigma"] = hb["sigma"][:n]
                host["sigma"].copy_(out["sigma"], non_blocking=True)
            done = torch.cuda.Event()
            done.record(st)
        lane["busy"] = (batch, offs, host, done)

    def poll(self, k):
        lane = self.lanes[k]
        if lane["busy"] is None:
            return None
        batch, offs, host, done = lane["busy"]
        if not done.query():
            return None
        lane["busy"] = None
        e = host["e"].numpy()
        f = host["f"].numpy()
        E = host["E"].numpy()
        sg = host["sigma"].numpy() if "sigma" in host else None
        for idx, (r, a) in enumerate(zip(batch, offs[:-1])):
            r.e = e[a:a + r.n].copy()
            r.f = f[:, a:a + r.n].T.copy()
            r.energy = float(E[idx])
            if sg is not None:
                r.sigma = sg[a:a + r.n].copy()
        return batch

    def idle(self, k):
        return self.lanes[k]["busy"] is None

    @property
    def n_lanes(self):
        return len(self.lanes)


class Scheduler:
    """FIFO continuous batching over an executor's lanes.

    max_batch: cap on requests per batch (1 = one at a time).
    """

    def __init__(self, executor, clock=time.perf_counter, max_batch=10**9, spin=None):
        self.ex = executor
        self.clock = clock
        self.max_batch = max_batch
        self.spin = spin            # called when nothing is ready (tests advance a fake clock)

    def _form_batch(self, queue):
        fp = self.ex.fp
        batch, used, atoms = [], 0, 0
        while queue and len(batch) < self.max_batch:
            r = queue[0]
            b = fp.bytes(atoms + r.n) - used if batch else fp.bytes(r.n)
            if batch and (used + b > self.ex.budget or atoms + r.n > self.ex.lane_atoms):
                break
            if not batch and r.n > self.ex.lane_atoms:
                raise ValueError(f"request {r.rid} with {r.n} atoms exceeds a lane ({self.ex.lane_atoms})")
            batch.append(queue.popleft())
            used = fp.bytes(atoms + r.n)
            atoms += r.n
        return batch

    def run(self, requests):
        """Serve `requests` (sorted by arrival, arrival times relative to the start)."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        done = []
        t0 = self.clock()
        stats = {"batches": 0, "batch_atoms": []}
        total = len(pending)
        while len(done) < total:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for k in range(self.ex.n_lanes):
                fin = self.ex.poll(k)
                if fin:
                    t = self.clock() - t0
                    for r in fin:
                        r.t_done = t
                    done.extend(fin)
                    progressed = True
            for k in range(self.ex.n_lanes):
                if queue and self.ex.idle(k):
                    batch = self._form_batch(queue)
                    t = self.clock() - t0
                    for r in batch:
                        r.t_start = t
                    self.ex.launch(k, batch)
                    stats["batches"] += 1
                    stats["batch_atoms"].append(sum(r.n for r in batch))
                    progressed = True
            if not progressed and self.spin is not None:
                self.spin()
        span = max(r.t_done for r in done) - min(r.arrival for r in done)
        lat = np.array([r.latency for r in done])
        atoms = sum(r.n for r in done)
        stats.update({
            "requests": total,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "throughput_req_s": total / span,
            "throughput_Matom_s": atoms / span / 1e6,
            "mean_batch_atoms": float(np.mean(stats["batch_atoms"])),
        })
        del stats["batch_atoms"]
        return done, stats


def poisson_requests(n, rate, sizes=(100, 50_000), seed=0):
    """Open-loop arrivals: Poisson process of `rate` per second, slabs of log-uniform size."""
    from . import structures as S
    out = []
    for k, (t, st) in enumerate(S.serving_requests(n, rate=rate, lo=sizes[0], hi=sizes[1], seed=seed)):
        out.append(Request(k, t, st.pos, st.species.astype(np.int32), st.box))
    return out
