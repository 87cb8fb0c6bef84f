"""Device-resident evaluator and MD driver over the C ABI.

Every step of the force-field evaluation runs in the HIP library; this module only
owns torch tensors (device memory), orders the calls and converts arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B

MASSES = np.array([1.008, 195.084])   # amu, H and Pt


class Model:
    """Mapped per-species (beta_s, Sigma_s), FP64 host arrays [S, n_d, n_d] (Eqs. 1-2)."""

    def __init__(self, beta, sigma, r_cut=4.5, n_rad=8, l_max=3, precision=B.FP32, _handle=None):
        lib = B.load()
        if _handle is None:
            beta = np.ascontiguousarray(beta, dtype=np.float64)
            sigma = np.ascontiguousarray(sigma, dtype=np.float64)
            h = ctypes.c_void_p()
            B.check(lib.flare_model_create(ctypes.byref(h), beta.shape[0], n_rad, l_max, float(r_cut),
                                           B.ptr(beta), B.ptr(sigma), precision))
        else:
            h = _handle
        self.handle = h
        self.r_cut = r_cut
        d = ctypes.c_int()
        B.check(lib.flare_descriptor_dim(h, ctypes.byref(d)))
        self.n_desc = d.value
        p, c = ctypes.c_int(), ctypes.c_int()
        B.check(lib.flare_model_info(h, ctypes.byref(p), ctypes.byref(c)))
        self.precision = p.value
        self.variance_cholesky = bool(c.value)   # V = |L^T d|^2 (else the full Sigma)

    @classmethod
    def from_sparse_set(cls, d_sparse, alpha, n_sparse, signal_var, noise, r_cut=4.5, n_rad=8, l_max=3,
                        precision=B.FP32, want_matrices=False):
        """The mapped model of a sparse set (flare_model_from_sparse_set, built on the device
        in FP64): d_sparse [n_S, n_d] normalised descriptors grouped by central species
        (n_sparse[s] rows of species s, species 0 first), alpha [n_S] the mean weights,
        signal_var sigma^2, noise on the sparse-set kernel diagonal. With want_matrices the
        device FP64 beta and gamma [S, n_d, n_d] are returned as well."""
        lib = B.load()
        d = torch.as_tensor(np.ascontiguousarray(d_sparse, np.float64)).cuda()
        a = torch.as_tensor(np.ascontiguousarray(alpha, np.float64)).cuda()
        ns = np.ascontiguousarray(n_sparse, np.int32)
        nd = d.shape[1]
        bm = torch.empty((len(ns), nd, nd), dtype=torch.float64, device="cuda") if want_matrices else None
        gm = torch.empty_like(bm) if want_matrices else None
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        B.check(lib.flare_model_from_sparse_set(ctypes.byref(h), len(ns), n_rad, l_max, float(r_cut), B.ptr(ns),
                                                B.ptr(d), B.ptr(a), float(signal_var), float(noise), precision,
                                                B.ptr(bm), B.ptr(gm)))
        m = cls(None, None, r_cut, n_rad, l_max, precision, _handle=h)
        return (m, bm, gm) if want_matrices else m

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                B.load().flare_model_destroy(self.handle)
            except (AttributeError, TypeError):   # interpreter shutdown: module already gone
                pass
            self.handle = None


class Evaluator:
    """One flare_state: neighbour list, resident descriptors, outputs in caller order."""

    def __init__(self, model: Model, max_atoms: int, max_pairs: int, stream=None,
                 device="cuda"):
        self.lib = B.load()
        self.model = model
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        B.check(self.lib.flare_state_create(ctypes.byref(h), model.handle, int(max_atoms),
                                            int(max_pairs), ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h
        self.max_atoms = max_atoms
        self.max_pairs = max_pairs
        self.n = 0
        self.n_struct = 0

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.flare_state_destroy(self.handle)
            self.handle = None

    # ---- list ----
    def neighbors(self, pos, species, offsets, boxes, skin=0.2):
        """pos: device FP64 [3, N]; species: device int32 [N]; offsets/boxes: host arrays."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[1]
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_neighbors(self.handle, n, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]),
                                             B.ptr(species), len(boxes), B.ptr(offsets), B.ptr(boxes),
                                             float(skin)))
        self.n = n
        self.n_struct = len(boxes)
        self.species = species

    def list_info(self):
        npairs = ctypes.c_longlong()
        counts = np.zeros(6, np.int32)
        B.check(self.lib.flare_list_info(self.handle, ctypes.byref(npairs), B.ptr(counts)))
        return npairs.value, counts

    def export_list(self):
        npairs, _ = self.list_info()
        off = np.zeros(self.n + 1, np.int64)
        j = np.zeros(max(npairs, 1), np.int32)
        s = np.zeros((max(npairs, 1), 3), np.int32)
        B.check(self.lib.flare_neighbors_export(self.handle, B.ptr(off), B.ptr(j), B.ptr(s)))
        return off, j[:npairs], s[:npairs]

    # ---- per step ----
    def descriptors(self, pos, want_d=False, want_norm=False):
        d = torch.empty((self.n, self.model.n_desc), dtype=torch.float32, device=self.device) if want_d else None
        nrm = torch.empty(self.n, dtype=torch.float32, device=self.device) if want_norm else None
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_descriptors(self.handle, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]),
                                               B.ptr(d), B.ptr(nrm)))
        return d, nrm

    def energy_forces(self, out=None, want_var=False):
        out = self._outputs(out, want_var)
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_energy_forces(self.handle, B.ptr(out["e"]), B.ptr(out["f"][0]),
                                                 B.ptr(out["f"][1]), B.ptr(out["f"][2]), B.ptr(out["E"]),
                                                 B.ptr(out.get("var")), B.ptr(out.get("sigma"))))
        return out

    def energies(self, out=None, want_var=False):
        """Energies (and variances) without forces; the gradients stay resident."""
        out = {} if out is None else out
        dev = self.device
        out.setdefault("e", torch.empty(self.n, dtype=torch.float32, device=dev))
        out.setdefault("E", torch.empty(self.n_struct, dtype=torch.float64, device=dev))
        if want_var:
            out.setdefault("var", torch.empty(self.n, dtype=torch.float32, device=dev))
            out.setdefault("sigma", torch.empty(self.n, dtype=torch.float32, device=dev))
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_energy_forces(self.handle, B.ptr(out["e"]), None, None, None, B.ptr(out["E"]),
                                                 B.ptr(out.get("var")), B.ptr(out.get("sigma"))))
        return out

    def forces(self, cell_scale=None, f=None):
        """Forces of the last energies() / energy_forces() positions, optionally scaled per cell."""
        f = torch.empty((3, self.n), dtype=torch.float32, device=self.device) if f is None else f
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_forces(self.handle, B.ptr(cell_scale), B.ptr(f[0]), B.ptr(f[1]), B.ptr(f[2])))
        return f

    def virial(self, out=None):
        """Per-cell virial W = -dE/d(strain), [n_struct, 3, 3] FP64, from the last forces."""
        out = torch.empty((self.n_struct, 3, 3), dtype=torch.float64, device=self.device) if out is None else out
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_virial(self.handle, B.ptr(out)))
        return out

    def virial_noalloc(self, out):
        """As virial(), through the allocation-free entry point; `out` is a device FP64
        [n_struct, 3, 3] tensor (the call allocates nothing)."""
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_virial_noalloc(self.handle, B.ptr(out)))
        return out

    def memory_bytes(self, with_model=True):
        b = ctypes.c_longlong()
        B.check(self.lib.flare_memory_bytes(self.model.handle if with_model else None, self.handle,
                                            ctypes.byref(b)))
        return b.value

    def variance(self, out=None):
        out = out or {}
        dev = self.device
        out.setdefault("var", torch.empty(self.n, dtype=torch.float32, device=dev))
        out.setdefault("sigma", torch.empty(self.n, dtype=torch.float32, device=dev))
        out.setdefault("sigma_max", torch.empty(self.n_struct, dtype=torch.float32, device=dev))
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_variance(self.handle, B.ptr(out["var"]), B.ptr(out["sigma"]),
                                            B.ptr(out["sigma_max"])))
        return out

    def compute(self, pos, want_var=True, out=None):
        self.descriptors(pos)
        return self.energy_forces(out, want_var)

    def timers(self, on=True):
        B.check(self.lib.flare_timers_enable(self.handle, 1 if on else 0))

    def read_timers(self, reset=True):
        ms = np.zeros(len(B.TIMER_NAMES), np.float64)
        cnt = np.zeros(len(B.TIMER_NAMES), np.int64)
        B.check(self.lib.flare_timers_read(self.handle, B.ptr(ms), B.ptr(cnt), 1 if reset else 0))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(B.TIMER_NAMES)}

    def status(self):
        """Status bits raised since the last call (synchronising; sticky across list builds)."""
        f = np.zeros(1, np.int32)
        B.check(self.lib.flare_status(self.handle, B.ptr(f)))
        return int(f[0])

    def interval_status(self):
        """Status bits of the interval the last list build ended (no wait)."""
        f = np.zeros(1, np.int32)
        B.check(self.lib.flare_interval_status(self.handle, B.ptr(f)))
        return int(f[0])

    def uncertainty_monitor(self, threshold, sigma_max_run, over_count):
        """Per-cell running max of sigma and count of evaluations above `threshold`
        (device FP32 / int32 [n_struct], updated in place) for the staged positions."""
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_uncertainty_monitor(self.handle, float(threshold), B.ptr(sigma_max_run),
                                                       B.ptr(over_count)))

    def _outputs(self, out, want_var):
        out = {} if out is None else out
        dev = self.device
        out.setdefault("e", torch.empty(self.n, dtype=torch.float32, device=dev))
        out.setdefault("f", torch.empty((3, self.n), dtype=torch.float32, device=dev))
        out.setdefault("E", torch.empty(self.n_struct, dtype=torch.float64, device=dev))
        if want_var:
            out.setdefault("var", torch.empty(self.n, dtype=torch.float32, device=dev))
            out.setdefault("sigma", torch.empty(self.n, dtype=torch.float32, device=dev))
        return out

    # ---- integrator ----
    def md_first_half(self, pos, vel, f, dt):
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_md_first_half(self.handle, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]),
                                                 B.ptr(vel[0]), B.ptr(vel[1]), B.ptr(vel[2]), B.ptr(f[0]),
                                                 B.ptr(f[1]), B.ptr(f[2]), B.ptr(self.species),
                                                 B.ptr(MASSES), float(dt)))

    def md_second_half(self, vel, f, dt):
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_md_second_half(self.handle, B.ptr(vel[0]), B.ptr(vel[1]), B.ptr(vel[2]),
                                                  B.ptr(f[0]), B.ptr(f[1]), B.ptr(f[2]), B.ptr(self.species),
                                                  B.ptr(MASSES), float(dt)))

    def md_step(self, pos, vel, out, dt, rebuild, want_var=True):
        """One NVE step in one call (flare_md_step): out["f"] holds the forces at the current
        positions on entry and at the new ones on return; e, E (and var, sigma) are refreshed."""
        f = out["f"]
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_md_step(
                self.handle, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]), B.ptr(vel[0]), B.ptr(vel[1]),
                B.ptr(vel[2]), B.ptr(f[0]), B.ptr(f[1]), B.ptr(f[2]), B.ptr(self.species), B.ptr(MASSES),
                float(dt), 1 if rebuild else 0, B.ptr(out["e"]), B.ptr(out["E"]),
                B.ptr(out["var"]) if want_var else None, B.ptr(out["sigma"]) if want_var else None))

    # ---- Nose-Hoover NVT and coordination (production runs) ----
    def new_thermostat(self, vel):
        """Per-cell thermostat state (zeta, eta, K) on the device, zeta = eta = 0 and K of vel."""
        thermo = torch.zeros((self.n_struct, 3), dtype=torch.float64, device=self.device)
        self.kinetic(vel, thermo)
        return thermo

    def kinetic(self, vel, thermo):
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_kinetic(self.handle, B.ptr(vel[0]), B.ptr(vel[1]), B.ptr(vel[2]),
                                           B.ptr(self.species), B.ptr(MASSES), B.ptr(thermo)))

    def nvt_first_half(self, pos, vel, f, dt, t_target, tau, thermo):
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_nvt_first_half(self.handle, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]),
                                                  B.ptr(vel[0]), B.ptr(vel[1]), B.ptr(vel[2]), B.ptr(f[0]),
                                                  B.ptr(f[1]), B.ptr(f[2]), B.ptr(self.species), B.ptr(MASSES),
                                                  float(dt), float(t_target), float(tau), B.ptr(thermo)))

    def nvt_second_half(self, vel, f, dt, t_target, tau, thermo):
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_nvt_second_half(self.handle, B.ptr(vel[0]), B.ptr(vel[1]), B.ptr(vel[2]),
                                                   B.ptr(f[0]), B.ptr(f[1]), B.ptr(f[2]), B.ptr(self.species),
                                                   B.ptr(MASSES), float(dt), float(t_target), float(tau),
                                                   B.ptr(thermo)))

    def quadratic_forms(self, bucket, d_rows):
        """e = d^T beta d and V = d^T Sigma d of given FP32 vectors (device [n, 144 or 544])
        with the model of environment bucket `bucket` (flare_quadratic_forms); discards the
        resident descriptors."""
        n = d_rows.shape[0]
        e = torch.empty(n, dtype=torch.float32, device=self.device)
        v = torch.empty(n, dtype=torch.float32, device=self.device)
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_quadratic_forms(self.handle, int(bucket), n, B.ptr(d_rows), B.ptr(e), B.ptr(v)))
        return e, v

    def coordination(self, pos, prev=None):
        """H coordination numbers (device int32 [N], caller order) of `pos`, the positions last
        passed to `descriptors`, and, given an earlier snapshot, the (dissociation,
        recombination) counts per cell."""
        coord = torch.empty(self.n, dtype=torch.int32, device=self.device)
        events = torch.zeros((self.n_struct, 2), dtype=torch.int64, device=self.device) if prev is not None else None
        with torch.cuda.stream(self.stream):
            B.check(self.lib.flare_coordination(self.handle, B.ptr(pos[0]), B.ptr(pos[1]), B.ptr(pos[2]),
                                                B.ptr(coord), B.ptr(prev), B.ptr(events)))
        return coord, events


def to_device(pos, species, device="cuda"):
    """numpy [N,3] FP64 + [N] int -> device SoA [3,N] FP64 and int32 [N]."""
    p = torch.from_numpy(np.ascontiguousarray(np.asarray(pos, np.float64).T)).to(device)
    s = torch.from_numpy(np.asarray(species, np.int32)).to(device)
    return p, s


class DisplacedError(RuntimeError):
    """An interval between two list builds raised FLARE_FLAG_DISPLACED or NONFINITE: some
    atom moved more than half the skin (the list may have missed pairs) or a position
    became non-finite."""


def check_interval(ev):
    flags = ev.interval_status()
    bad = flags & (B.FLAG_DISPLACED | B.FLAG_NONFINITE)
    if bad:
        raise DisplacedError(f"list interval ended with status flags {flags:#x} (displaced > skin/2 or non-finite)")
    return flags


class MD:
    """Velocity-Verlet NVE with a neighbour-list rebuild every `rebuild` steps.

    One step: half kick + drift, list rebuild when due, descriptors, energies, forces
    (and variances), half kick. State (x, v) stays FP64 on the device. Every rebuild checks
    the status bits of the interval it ends (no extra wait: the build reads them at its
    own synchronisation point) and raises DisplacedError if an atom moved more than half
    the skin or a position became non-finite.
    """

    def __init__(self, ev: Evaluator, pos, vel, species, offsets, boxes, dt=0.5, skin=0.2,
                 rebuild=10, want_var=True):
        self.ev, self.pos, self.vel = ev, pos, vel
        self.species, self.offsets, self.boxes = species, offsets, boxes
        self.dt, self.skin, self.rebuild, self.want_var = dt, skin, rebuild, want_var
        self.nstep = 0
        ev.neighbors(pos, species, offsets, boxes, skin)
        self.out = ev.compute(pos, want_var)

    def step(self):
        ev = self.ev
        self.nstep += 1
        rebuild = self.nstep % self.rebuild == 0
        ev.md_step(self.pos, self.vel, self.out, self.dt, rebuild, self.want_var)
        if rebuild:
            check_interval(ev)
        return self.out

    def step_in_calls(self):
        """The same step through the separate calls (first half, list, descriptors, energies and
        forces, second half); bit for bit the result of step()."""
        ev = self.ev
        ev.md_first_half(self.pos, self.vel, self.out["f"], self.dt)
        self.nstep += 1
        if self.nstep % self.rebuild == 0:
            ev.neighbors(self.pos, self.species, self.offsets, self.boxes, self.skin)
            check_interval(ev)
        ev.descriptors(self.pos)
        ev.energy_forces(self.out, self.want_var)
        ev.md_second_half(self.vel, self.out["f"], self.dt)
        return self.out


class NVT(MD):
    """Nose-Hoover NVT (one thermostat per cell, flare_nvt_*_half) with the same list cadence.
    `thermo` holds (zeta, eta, K) per cell on the device."""

    def __init__(self, ev: Evaluator, pos, vel, species, offsets, boxes, t_target, tau, dt=0.1, skin=0.2,
                 rebuild=10, want_var=True):
        super().__init__(ev, pos, vel, species, offsets, boxes, dt, skin, rebuild, want_var)
        self.t_target, self.tau = t_target, tau
        self.thermo = ev.new_thermostat(vel)

    def step(self):
        ev = self.ev
        ev.nvt_first_half(self.pos, self.vel, self.out["f"], self.dt, self.t_target, self.tau, self.thermo)
        self.nstep += 1
        if self.nstep % self.rebuild == 0:
            ev.neighbors(self.pos, self.species, self.offsets, self.boxes, self.skin)
            check_interval(ev)
        ev.descriptors(self.pos)
        ev.energy_forces(self.out, self.want_var)
        ev.nvt_second_half(self.vel, self.out["f"], self.dt, self.t_target, self.tau, self.thermo)
        return self.out


class Production:
    """The in-situ work of the paper's production runs (Section VI.A) around an NVT run:
    every `every` steps, hydrogen coordination numbers, the reaction events since the last
    snapshot (dissociations 1 -> 0, recombinations 0 -> 1) and the largest uncertainty per
    cell against the active-learning threshold, all on the device (flare_coordination,
    flare_uncertainty_monitor): `sigma_max` is the running maximum per cell, `over` counts
    the monitor points at which a cell exceeded the threshold, and the status bit
    FLARE_FLAG_UNCERTAIN, read at list builds, says whether any did."""

    def __init__(self, nvt: NVT, every=1000, threshold=0.005):
        self.nvt, self.every, self.threshold = nvt, every, threshold
        self.coord, _ = nvt.ev.coordination(nvt.pos)
        self.events = torch.zeros((nvt.ev.n_struct, 2), dtype=torch.int64, device=nvt.ev.device)
        self.sigma_max = torch.zeros(nvt.ev.n_struct, dtype=torch.float32, device=nvt.ev.device)
        self.over = torch.zeros(nvt.ev.n_struct, dtype=torch.int32, device=nvt.ev.device)

    def step(self):
        out = self.nvt.step()
        if self.nvt.nstep % self.every == 0:
            ev = self.nvt.ev
            coord, ev_counts = ev.coordination(self.nvt.pos, self.coord)
            with torch.cuda.stream(ev.stream):
                self.events += ev_counts
            self.coord = coord
            ev.uncertainty_monitor(self.threshold, self.sigma_max, self.over)
        return out

    def flagged_cells(self):
        """Cells whose largest sigma exceeded the threshold at some monitor point (waits)."""
        return torch.nonzero(self.over).flatten().cpu().tolist()
