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


def _slab_request(n_target=6000, seed=4):
    from paper_2204_12573_amd import structures as S
    for t, st in S.serving_requests(40, lo=n_target, hi=n_target + 1, seed=seed):
        return serve.Request(0, t, st.pos, st.species.astype(np.int32), st.box)


def test_split_owns_every_atom_once_and_keeps_two_cutoffs_of_neighbours():
    """Each atom is owned by exactly one slab, and in its slab every atom within 2 r_c of it
    (as in the whole periodic structure: same atoms, same pair vectors) is present."""
    from oracle.neighbors import neighbor_list
    r = _slab_request()
    slabs = serve.split_request(r, 1500, 4.5)
    assert len(slabs) == int(np.ceil(r.n / 1500))
    owned = np.concatenate([c.index[c.own] for c in slabs])
    np.testing.assert_array_equal(np.sort(owned), np.arange(r.n))
    reach = 2 * 4.5
    i0, j0, s0 = neighbor_list(r.pos, r.box, reach)
    d0 = r.pos[j0] + s0 * r.box - r.pos[i0]
    for c in slabs:
        i1, j1, s1 = neighbor_list(c.pos, c.box, reach)
        d1 = c.pos[j1] + s1 * c.box - c.pos[i1]
        for a in np.nonzero(c.own)[0][::7]:
            want = sorted((int(j), tuple(np.round(d, 6))) for j, d in zip(j0[i0 == c.index[a]], d0[i0 == c.index[a]]))
            got = sorted((int(c.index[j]), tuple(np.round(d, 6))) for j, d in zip(j1[i1 == a], d1[i1 == a]))
            assert got == want, f"atom {c.index[a]}"


class SlabExecutor(FakeExecutor):
    """Results that name each atom of the request: e = f = sigma = its index in the request."""

    def poll(self, k):
        batch = super().poll(k)
        if batch:
            for r in batch:
                idx = (r.index if r.parent is not None else np.arange(r.n)).astype(np.float32)
                r.e, r.sigma = idx.copy(), idx.copy()
                r.f = np.repeat(idx[:, None], 3, axis=1)
        return batch


def test_chunked_requests_are_joined_in_order():
    clock = FakeClock()
    ex = SlabExecutor(clock, lane_atoms=4000)
    big = _slab_request()
    reqs = _reqs([500, 700], [0.0, 0.0005])
    reqs.append(serve.Request(2, 0.0002, big.pos, big.species, big.box))
    done, stats = serve.Scheduler(ex, clock=clock, spin=clock.advance, chunk_atoms=2000).run(reqs)
    assert sorted(r.rid for r in done) == [0, 1, 2] and stats["requests"] == 3
    joined = next(r for r in done if r.rid == 2)
    np.testing.assert_array_equal(joined.e, np.arange(big.n, dtype=np.float32))
    np.testing.assert_array_equal(joined.f[:, 1], np.arange(big.n, dtype=np.float32))
    assert joined.energy == float(np.sum(np.arange(big.n, dtype=np.float64)))
    assert joined.t_done >= joined.t_start >= joined.arrival
    # the slabs went through the lanes as requests of their own
    assert sum(len(b) for b in ex.launched) == 2 + int(np.ceil(big.n / 2000))


def test_request_larger_than_a_lane_is_split_to_fit():
    clock = FakeClock()
    ex = SlabExecutor(clock, lane_atoms=2500)
    big = _slab_request()
    done, stats = serve.Scheduler(ex, clock=clock, spin=clock.advance).run(
        [serve.Request(0, 0.0, big.pos, big.species, big.box)])
    assert len(done) == 1 and stats["requests"] == 1
    np.testing.assert_array_equal(done[0].e, np.arange(big.n, dtype=np.float32))
    assert len(ex.launched) >= int(np.ceil(big.n / 1250))     # slabs of about half a lane each
