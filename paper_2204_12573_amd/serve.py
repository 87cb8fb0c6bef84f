"""Continuous-batching service for energy / force / uncertainty requests.

Requests are periodic cells of uneven size (active-learning candidate screening). The
scheduler keeps several *lanes*: one HIP stream, one device-resident evaluation state
(neighbour list, descriptors, gradients; every buffer sized when the lane is made, its
bytes read back with flare_memory_bytes) and pinned host staging buffers each, served by a
host thread of its own. Whenever a lane is free it takes the oldest waiting requests (FIFO)
as long as the batch fits the lane's state (atoms, estimated pairs, cells), and its thread
uploads them and runs one launch sequence for the whole batch (list build, descriptors,
energies + forces + variances, download), so a lane waiting for its list build never holds
up the scheduler or the other lanes. Requests arriving while batches run wait in the queue
and are admitted as soon as a lane frees up; the batches of different lanes overlap on the
device. Latency is measured from a request's arrival to its results being on the host.

Per-cell results do not depend on the batch composition (the library computes each row
independently and gathers forces in a fixed order), so a structure gives the same bits
alone and in any mix.

Requests larger than a lane, and optionally all above `chunk_atoms`, are split by atom
ranges: along the longer
lateral axis into equal slabs, each evaluated with a halo of 2 r_c (plus a margin) on both
sides in a box widened so that no periodic image reaches across the cut. An atom's energy
and uncertainty depend on its neighbours within r_c, and its force on the energies of
those neighbours, i.e. on atoms within 2 r_c; so every atom of a slab's own range gets the
values of the whole structure (up to the order of FP32 sums), and the request's results
are those atoms' values put back in its order, its energy their FP64 sum. The slabs of one
request are batched like any other requests, on any lane.
"""
from __future__ import annotations

import dataclasses
import threading
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
    # a slab of a chunked request: the request, the slab atoms' indices in it, and which
    # slab atoms are the slab's own (their results are kept)
    parent: "Request | None" = None
    index: np.ndarray | None = None
    own: np.ndarray | None = None

    @property
    def n(self) -> int:
        return len(self.species)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def split_request(r: Request, chunk_atoms: int, r_cut: float, margin: float = 0.5, max_atoms: int | None = None):
    """Slabs of request r along its longer lateral axis, about chunk_atoms own atoms each,
    with a halo of 2 r_cut + margin on both sides; each slab's box along that axis is its
    width plus r_cut + margin, so that no pair crosses the cut through a periodic image.
    With max_atoms, more slabs are taken until each (with its halo) holds at most that many
    atoms. The request itself comes back when the slabs would be thinner than the halo."""
    m = max(int(np.ceil(r.n / chunk_atoms)), 1)
    while True:
        slabs = _slabs(r, m, r_cut, margin)
        if max_atoms is None or len(slabs) == 1 or max(c.n for c in slabs) <= max_atoms:
            return slabs
        m += 1


def _slabs(r: Request, m: int, r_cut: float, margin: float):
    axis = 0 if r.box[0] >= r.box[1] else 1
    L = float(r.box[axis])
    halo = 2.0 * r_cut + margin
    width = L / m
    if m < 2 or width < halo:
        return [r]
    x = np.mod(r.pos[:, axis], L)
    owner = np.minimum((x / width).astype(np.int64), m - 1)     # each atom's own slab
    slabs = []
    for k in range(m):
        # coordinate measured from the slab's lower halo edge, wrapped into [0, L)
        u = np.mod(x - (k * width - halo), L)
        keep = np.nonzero((u < width + 2.0 * halo) | (owner == k))[0]
        pos = r.pos[keep].copy()
        pos[:, axis] = u[keep]
        box = r.box.astype(np.float64).copy()
        box[axis] = width + 2.0 * halo + r_cut + margin
        slabs.append(Request(r.rid, r.arrival, pos, r.species[keep], box, parent=r, index=keep,
                             own=owner[keep] == k))
    return slabs


def join_slabs(r: Request, slabs) -> None:
    """The request's results from its slabs' own atoms (each atom owned by exactly one)."""
    r.e = np.zeros(r.n, np.float32)
    r.f = np.zeros((r.n, 3), np.float32)
    r.sigma = np.zeros(r.n, np.float32) if slabs[0].sigma is not None else None
    for c in slabs:
        idx = c.index[c.own]
        r.e[idx] = c.e[c.own]
        r.f[idx] = c.f[c.own]
        if r.sigma is not None:
            r.sigma[idx] = c.sigma[c.own]
    r.energy = float(np.sum(r.e.astype(np.float64)))
    r.t_start = min(c.t_start for c in slabs)
    r.t_done = max(c.t_done for c in slabs)


class Footprint:
    """What a batch needs of a lane's state: its atoms and an estimate of its listed pairs
    (pairs_per_atom; bulk Pt(111) has 18 at the list radius, a surface or H atom fewer)."""

    def __init__(self, pairs_per_atom=22.0):
        self.ppa = pairs_per_atom

    def atoms_pairs(self, n_atoms):
        return n_atoms, int(self.ppa * n_atoms) + 64

    def fits(self, n_atoms, n_cells, lane_atoms):
        """A batch of n_atoms in n_cells fits a lane made for lane_atoms atoms."""
        return n_atoms <= lane_atoms and n_cells <= lane_atoms + 1


class GpuExecutor:
    """Lanes on the GPU: each has its own torch stream, flare state, pinned staging and a
    host thread that runs its batches (launch() hands a batch over and returns at once)."""

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
            lane = {"stream": st, "ev": ev, "busy": None, "result": None, "error": None,
                    "work": threading.Event(), "ready": threading.Event(),
                    "pin_pos": torch.empty((3, n), dtype=torch.float64).pin_memory(),
                    "pin_sp": torch.empty(n, dtype=torch.int32).pin_memory(),
                    "dev_pos": torch.empty((3, n), dtype=torch.float64, device="cuda"),
                    "dev_sp": torch.empty(n, dtype=torch.int32, device="cuda"),
                    "host": {"e": torch.empty(n, dtype=torch.float32).pin_memory(),
                             "f": torch.empty((3, n), dtype=torch.float32).pin_memory(),
                             "sigma": torch.empty(n, dtype=torch.float32).pin_memory(),
                             "E": torch.empty(n, dtype=torch.float64).pin_memory()}}
            lane["thread"] = threading.Thread(target=self._worker, args=(lane,), daemon=True)
            lane["thread"].start()
            self.lanes.append(lane)
        self.lane_atoms = lane_atoms
        # the device memory a lane holds: its state, fixed when the lane is made
        self.lane_bytes = self.lanes[0]["ev"].memory_bytes(with_model=False)

    def _worker(self, lane):
        torch = self.torch
        torch.cuda.set_device(0)
        while True:
            lane["work"].wait()
            lane["work"].clear()
            batch = lane["busy"]
            if batch is None:
                return
            try:
                lane["result"] = self._run(lane, batch)
            except Exception as exc:      # reported to the scheduler by poll()
                lane["error"] = exc
            lane["ready"].set()

    def _run(self, lane, batch):
        """Upload one batch, build its list, evaluate E, F, sigma, download (waits)."""
        torch = self.torch
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
        st.synchronize()
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

    def launch(self, k, batch):
        """Hand one batch to lane k's thread (returns at once)."""
        lane = self.lanes[k]
        lane["busy"] = batch
        lane["ready"].clear()
        lane["work"].set()

    def poll(self, k):
        lane = self.lanes[k]
        if lane["busy"] is None or not lane["ready"].is_set():
            return None
        lane["busy"] = None
        if lane["error"] is not None:
            exc, lane["error"] = lane["error"], None
            raise exc
        return lane["result"]

    def idle(self, k):
        return self.lanes[k]["busy"] is None

    def close(self):
        for lane in self.lanes:
            lane["busy"] = None
            lane["work"].set()
            lane["thread"].join()

    @property
    def n_lanes(self):
        return len(self.lanes)


class Scheduler:
    """FIFO continuous batching over an executor's lanes.

    max_batch: cap on requests per batch (1 = one at a time).
    """

    def __init__(self, executor, clock=time.perf_counter, max_batch=10**9, spin=None, chunk_atoms=None,
                 r_cut=4.5):
        self.ex = executor
        self.clock = clock
        self.max_batch = max_batch
        # requests above chunk_atoms are split by atom ranges; a request larger than a lane
        # always is (into slabs of at most a lane each, about half a lane of own atoms)
        self.chunk_atoms = chunk_atoms
        self.r_cut = r_cut
        # called when nothing is ready: tests advance a fake clock; by default a short sleep
        # that lets the lane threads run
        self.spin = spin if spin is not None else (lambda: time.sleep(2e-5))

    def _form_batch(self, queue):
        fp = self.ex.fp
        batch, atoms = [], 0
        while queue and len(batch) < self.max_batch:
            r = queue[0]
            if not fp.fits(atoms + r.n, len(batch) + 1, self.ex.lane_atoms):
                if not batch:
                    raise ValueError(f"request {r.rid} with {r.n} atoms exceeds a lane ({self.ex.lane_atoms})")
                break
            batch.append(queue.popleft())
            atoms += r.n
        return batch

    def run(self, requests, warmup=0):
        """Serve `requests` (sorted by arrival, arrival times relative to the start); the
        first `warmup` requests by arrival are served but left out of the statistics."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue = deque()
        done = []
        t0 = self.clock()
        stats = {"batches": 0, "batch_atoms": []}
        total = len(pending)
        open_slabs = {}          # chunked request -> [its slabs, slabs still out]
        while len(done) < total:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                lane = self.ex.lane_atoms
                if r.n > lane or (self.chunk_atoms is not None and r.n > self.chunk_atoms):
                    target = min(self.chunk_atoms or lane // 2, lane // 2)
                    slabs = split_request(r, target, self.r_cut, max_atoms=lane)
                    if len(slabs) > 1:
                        open_slabs[id(r)] = [slabs, len(slabs)]
                    queue.extend(slabs)
                else:
                    queue.append(r)
            progressed = False
            for k in range(self.ex.n_lanes):
                fin = self.ex.poll(k)
                if fin:
                    t = self.clock() - t0
                    for r in fin:
                        r.t_done = t
                        if r.parent is None:
                            done.append(r)
                            continue
                        entry = open_slabs[id(r.parent)]
                        entry[1] -= 1
                        if entry[1] == 0:
                            join_slabs(r.parent, entry[0])
                            del open_slabs[id(r.parent)]
                            done.append(r.parent)
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
            if not progressed:
                self.spin()
        ordered = sorted(done, key=lambda r: r.arrival)
        timed = ordered[warmup:] if warmup < len(ordered) else ordered
        span = max(r.t_done for r in timed) - min(r.arrival for r in timed)
        lat = np.array([r.latency for r in timed])
        wait = np.array([r.t_start - r.arrival for r in timed])
        atoms = sum(r.n for r in timed)
        sizes = np.array([r.n for r in timed])
        edges = np.percentile(sizes, np.linspace(0, 100, 11))
        deciles = []
        for q in range(10):
            m = (sizes >= edges[q]) & ((sizes < edges[q + 1]) if q < 9 else (sizes <= edges[q + 1]))
            if m.any():
                deciles.append({"atoms": [int(sizes[m].min()), int(sizes[m].max())],
                                "p50_ms": round(float(np.percentile(lat[m], 50) * 1e3), 3),
                                "p99_ms": round(float(np.percentile(lat[m], 99) * 1e3), 3)})
        stats.update({
            "requests": len(timed),
            "warmup_requests": len(ordered) - len(timed),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "queue_wait_p50_ms": float(np.percentile(wait, 50) * 1e3),
            "queue_wait_p99_ms": float(np.percentile(wait, 99) * 1e3),
            "throughput_req_s": len(timed) / span,
            "throughput_Matom_s": atoms / span / 1e6,
            "mean_batch_atoms": float(np.mean(stats["batch_atoms"])),
            "by_size_decile": deciles,
        })
        del stats["batch_atoms"]
        return done, stats


def poisson_requests(n, rate, sizes=(100, 50_000), seed=0, pool=None):
    """Open-loop arrivals: Poisson process of `rate` per second, slabs of log-uniform size.
    With `pool`, the structures are drawn (seeded, with repetition) from `pool` distinct
    slabs of the same distribution, which bounds the host memory of long streams."""
    from . import structures as S
    if pool is None or pool >= n:
        return [Request(k, t, st.pos, st.species.astype(np.int32), st.box)
                for k, (t, st) in enumerate(S.serving_requests(n, rate=rate, lo=sizes[0], hi=sizes[1], seed=seed))]
    base = S.serving_requests(pool, rate=rate, lo=sizes[0], hi=sizes[1], seed=seed)
    rng = np.random.default_rng(seed + 1)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    pick = rng.integers(0, pool, n)
    return [Request(k, float(t[k]), base[p][1].pos, base[p][1].species.astype(np.int32), base[p][1].box)
            for k, p in enumerate(pick)]
