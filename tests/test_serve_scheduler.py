"""Scheduler logic of the serving loop on the CPU with a fake executor and a fake clock:
FIFO admission, lane capacity, lane overlap, latency bookkeeping, warm-up exclusion and
the per-size-decile latencies."""
import numpy as np
import pytest

from paper_2204_12573_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-4):
        self.t += dt


class FakeExecutor:
    """Charges `per_atom` seconds per atom plus `per_batch` per launch; results are a
    function of each request alone (its atom count), like the real kernels."""

    def __init__(self, clock, n_lanes=2, lane_atoms=10_000, per_atom=1e-7, per_batch=5e-4):
        self.clock, self.per_atom, self.per_batch = clock, per_atom, per_batch
        self.fp = serve.Footprint()
        self.lane_atoms = lane_atoms
        self.busy = [None] * n_lanes
        self.launched = []

    @property
    def n_lanes(self):
        return len(self.busy)

    def idle(self, k):
        return self.busy[k] is None

    def launch(self, k, batch):
        n = sum(r.n for r in batch)
        assert self.fp.fits(n, len(batch), self.lane_atoms)
        self.busy[k] = (batch, self.clock() + self.per_batch + self.per_atom * n)
        self.launched.append([r.rid for r in batch])

    def poll(self, k):
        if self.busy[k] is None or self.clock() < self.busy[k][1]:
            return None
        batch = self.busy[k][0]
        self.busy[k] = None
        for r in batch:
            r.e = np.full(r.n, float(r.n))
        return batch


def _reqs(sizes, arrivals):
    return [serve.Request(k, t, np.zeros((n, 3)), np.zeros(n, np.int32), np.ones(3) * 10)
            for k, (n, t) in enumerate(zip(sizes, arrivals))]


def test_fifo_and_capacity():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sched = serve.Scheduler(ex, clock=clock, spin=clock.advance)
    rng = np.random.default_rng(0)
    sizes = rng.integers(100, 4000, 60)
    arrivals = np.cumsum(rng.exponential(2e-4, 60))
    done, stats = sched.run(_reqs(sizes, arrivals))
    assert len(done) == 60
    order = [rid for b in ex.launched for rid in b]
    assert order == sorted(order)                   # FIFO admission
    for b in ex.launched:
        assert sum(sizes[i] for i in b) <= ex.lane_atoms or len(b) == 1
    for r in done:
        assert r.t_start >= r.arrival and r.t_done > r.t_start
        assert np.all(r.e == r.n)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    assert stats["queue_wait_p99_ms"] <= stats["p99_ms"]
    dec = stats["by_size_decile"]
    assert len(dec) == 10 and sum(1 for _ in dec) == 10
    assert dec[0]["atoms"][0] == sizes.min() and dec[-1]["atoms"][1] == sizes.max()


def test_warmup_left_out_of_the_statistics():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sizes = [200] * 30
    arrivals = np.arange(30) * 1e-3
    done, stats = serve.Scheduler(ex, clock=clock, spin=clock.advance).run(_reqs(sizes, arrivals), warmup=10)
    assert len(done) == 30 and stats["requests"] == 20 and stats["warmup_requests"] == 10


def test_continuous_batching_beats_one_at_a_time():
    rng = np.random.default_rng(1)
    sizes = rng.integers(100, 3000, 200)
    arrivals = np.cumsum(rng.exponential(1e-4, 200))
    res = {}
    for name, mb, lanes in [("one", 1, 1), ("batched", 10**9, 2)]:
        clock = FakeClock()
        ex = FakeExecutor(clock, n_lanes=lanes)
        sched = serve.Scheduler(ex, clock=clock, max_batch=mb, spin=clock.advance)
        _, res[name] = sched.run(_reqs(sizes, arrivals))
    assert res["batched"]["p99_ms"] < res["one"]["p99_ms"]
    assert res["batched"]["throughput_Matom_s"] > res["one"]["throughput_Matom_s"]


def test_oversized_request_rejected():
    clock = FakeClock()
    ex = FakeExecutor(clock, lane_atoms=1000)
    sched = serve.Scheduler(ex, clock=clock, spin=clock.advance)
    with pytest.raises(ValueError):
        sched.run(_reqs([500, 5000], [0.0, 0.0]))
