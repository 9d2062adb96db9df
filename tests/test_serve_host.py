"""Host logic of the serving loop (setup cache, lanes, routing) on the CPU.

A fake backend stands in for the library: its "solver" of key (field, mass)
returns x = b / (f + m) after a number of steps that depends on b, so a result
routed to the wrong key, column or slot shows up as a wrong value.
"""

import contextlib
import threading
import time

import numpy as np
import pytest

from paper_0710_3612_amd import serve


class FakeSolver:
    def __init__(self, be, field, mass, derived_from=None):
        self.be, self.field, self.mass = be, field, mass
        self.derived_from = derived_from
        self.closed = False

    def memory_bytes(self):
        return self.be.bytes_per_solver

    def derive(self, mass, stream=None):
        return FakeSolver(self.be, self.field, mass, derived_from=self)

    def close(self):
        assert not self.closed
        self.closed = True
        self.be.closed += 1


class FakeBatch:
    def __init__(self, be, solver, capacity):
        self.be, self.solver, self.cap = be, solver, capacity
        self.slots = [None] * capacity  # [rhs, steps left, done]
        self.closed = False

    def memory_bytes(self):
        return self.be.bytes_per_batch

    def admit(self, rhs, stream=None):
        assert not self.solver.closed
        assert not self.closed, "batch used after close"
        for j in range(self.cap):
            if self.slots[j] is None:
                steps = 1 + int(abs(rhs[0].real) * 3) % 4
                self.slots[j] = [np.array(rhs), steps, False]
                return j
        return None

    def step(self, iters=1, stream=None):
        assert not self.closed, "batch used after close"
        with self.be.lock:
            self.be.stepping += 1
            self.be.max_stepping = max(self.be.max_stepping, self.be.stepping)
        time.sleep(0.0005)
        for s in self.slots:
            if s is not None and not s[2]:
                s[1] -= iters
                if s[1] <= 0:
                    s[2] = True
        with self.be.lock:
            self.be.stepping -= 1

    def poll(self):
        return [(j, {"status": 0, "iterations": 3, "true_relres": 1e-11})
                for j, s in enumerate(self.slots) if s is not None and s[2]]

    def harvest(self, slot, out, stream=None):
        rhs = self.slots[slot][0]
        out[:] = rhs / (self.solver.field + self.solver.mass)
        self.slots[slot] = None

    def close(self):
        time.sleep(self.be.batch_close_delay)
        self.closed = True


class FakeBackend:
    def __init__(self, est=100, bytes_per_solver=80, bytes_per_batch=20, fail_fields=(), setup_delay=0.0):
        self.est = est
        self.bytes_per_solver = bytes_per_solver
        self.bytes_per_batch = bytes_per_batch
        self.fail_fields = set(fail_fields)
        self.setup_delay = setup_delay
        self.setups = []
        self.derives = []
        self.closed = 0
        self.lock = threading.Lock()
        self.stepping = 0
        self.max_stepping = 0
        self.cache_ref = None
        self.max_used = 0
        self.batch_close_delay = 0.0

    def _watch(self):
        if self.cache_ref is not None:
            self.max_used = max(self.max_used, self.cache_ref.used)

    def estimate(self, field, capacity):
        return self.est if capacity else self.est - self.bytes_per_batch

    def batch_estimate(self, field, capacity):
        return self.bytes_per_batch

    def setup(self, field, mass, stream):
        time.sleep(self.setup_delay)
        if field in self.fail_fields:
            raise RuntimeError("setup failed")
        self.setups.append((field, mass))
        self._watch()
        return FakeSolver(self, field, mass)

    def derive(self, solver, mass, stream):
        self.derives.append((solver.field, mass))
        self._watch()
        return solver.derive(mass)

    def new_stream(self):
        return object()

    def stream_context(self, stream):
        return contextlib.nullcontext()

    def new_batch(self, solver, capacity, tol, maxiter, precision, stream):
        return FakeBatch(self, solver, capacity)

    def new_output(self, rhs):
        return np.zeros_like(rhs)


def make_requests(spec, n=6, seed=0):
    """spec: list of (field, mass, k, arrival)."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (f, m, k, t) in enumerate(spec):
        rhs = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
        out.append(serve.Request(i, f, m, rhs, k, t))
    return out


def check_results(reqs, results):
    for req, res in zip(reqs, results):
        assert res.ok, res.error
        np.testing.assert_array_equal(res.x, req.rhs / (req.field + req.mass))
        assert res.admitted >= res.arrival - 1e-9
        assert res.finished >= res.admitted
        assert len(res.status) == req.k


def test_all_requests_complete_and_route_correctly():
    be = FakeBackend()
    spec = [(f, m, k, 0.002 * i) for i, (f, m, k) in enumerate(
        [(1, 0.1, 3), (2, 0.1, 1), (1, 0.2, 5), (1, 0.1, 2), (3, 0.05, 16), (2, 0.3, 4)] * 3)]
    reqs = make_requests(spec)
    with serve.Server(be, budget_bytes=10_000, capacity=4, max_lanes=3) as srv:
        results = srv.run_trace(reqs, timeout=30)
        # first mass of a field is a full setup, the others derive from it
        assert sorted(set(f for f, _ in be.setups)) == [1, 2, 3]
        assert len(be.setups) == 3
        assert len(be.derives) == 2
    check_results(reqs, results)
    assert be.max_stepping <= 3


def test_request_wider_than_the_batch_streams_through_slots():
    be = FakeBackend()
    reqs = make_requests([(1, 0.0, 11, 0.0)])
    with serve.Server(be, budget_bytes=10_000, capacity=2, max_lanes=1) as srv:
        results = srv.run_trace(reqs, timeout=30)
    check_results(reqs, results)


def test_budget_evicts_least_recently_used_idle_setups():
    be = FakeBackend(est=100, bytes_per_solver=80, bytes_per_batch=20)
    spec = [(f, 0.0, 2, 0.0) for f in (1, 2, 3, 1, 4, 2)]
    reqs = make_requests(spec)
    with serve.Server(be, budget_bytes=250, capacity=4, max_lanes=1, linger=0.0) as srv:
        be.cache_ref = srv.cache
        results = srv.run_trace(reqs, timeout=30)
        assert srv.cache.used <= 250
        assert srv.cache.evictions >= 2
        assert be.max_used <= 250
    check_results(reqs, results)
    assert be.closed >= 2


def test_pinned_setups_are_not_evicted_and_waiters_proceed():
    # room for one hierarchy: the second key waits for the first lane to retire
    be = FakeBackend(est=100)
    reqs = make_requests([(1, 0.0, 3, 0.0), (2, 0.0, 3, 0.0), (1, 0.5, 2, 0.0)])
    with serve.Server(be, budget_bytes=150, capacity=2, max_lanes=3, linger=0.0) as srv:
        results = srv.run_trace(reqs, timeout=30)
    check_results(reqs, results)


def test_over_budget_and_failed_setups_fail_only_their_requests():
    be = FakeBackend(est=100, fail_fields={7})
    reqs = make_requests([(7, 0.0, 2, 0.0), (1, 0.0, 2, 0.0)])
    with serve.Server(be, budget_bytes=1000, capacity=2, max_lanes=2) as srv:
        results = srv.run_trace(reqs, timeout=30)
    assert results[0].error and "setup failed" in results[0].error
    check_results(reqs[1:], results[1:])

    be2 = FakeBackend(est=5000)
    reqs2 = make_requests([(1, 0.0, 1, 0.0)])
    with serve.Server(be2, budget_bytes=1000, capacity=2) as srv:
        res = srv.run_trace(reqs2, timeout=30)
    assert res[0].error and "exceed the budget" in res[0].error


def test_concurrent_requests_for_a_key_share_one_setup():
    be = FakeBackend(setup_delay=0.05)
    reqs = make_requests([(1, 0.0, 1, 0.0)] * 6)
    with serve.Server(be, budget_bytes=10_000, capacity=8, max_lanes=4) as srv:
        results = srv.run_trace(reqs, timeout=30)
    assert len(be.setups) == 1 and not be.derives
    check_results(reqs, results)


def test_poisson_trace_and_summary():
    fields = ["a", "b"]
    masses = {"a": [0.1, 0.2], "b": [0.3]}
    tr = serve.poisson_trace(4000, rate=200.0, fields=fields, masses=masses, k_range=(1, 16), seed=3)
    t = np.array([x[0] for x in tr])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(np.mean(np.diff(t)) - 1 / 200.0) < 0.1 / 200.0
    ks = np.array([x[3] for x in tr])
    assert ks.min() == 1 and ks.max() == 16
    for _, f, m, _, _ in tr:
        assert m in masses[f]
    assert tr == serve.poisson_trace(4000, 200.0, fields, masses, (1, 16), seed=3)
    res = [serve.Result(i, "a", 0.1, 2, arrival=0.0, admitted=0.0, finished=0.01 * (i + 1), status=[0, 0])
           for i in range(100)]
    s = serve.latency_summary(res)
    assert s["ok"] == 100 and s["solves"] == 200
    assert abs(s["p50_ms"] - 505.0) < 1e-9 and abs(s["p99_ms"] - 990.1) < 1e-9  # linear interpolation at rank 98.01


def test_levels_for_and_estimate():
    assert serve.levels_for(64) == 3  # 64 -> 16 -> 4
    assert serve.levels_for(128) == 3  # 128 -> 32 -> 8
    assert serve.levels_for(256) == 4  # 256 -> 64 -> 16 -> 4
    assert serve.levels_for(512) == 4  # 512 -> 128 -> 32 -> 8
    import paper_0710_3612_amd as smg

    p = smg.make_params(256, 256, 0.1, levels=3, blocks=[(4, 4)] * 2, nv=[12, 12])
    a = serve.estimate_bytes(p, capacity=16)
    b = serve.estimate_bytes(p, capacity=1)
    c = serve.estimate_bytes(p, capacity=1, mixed=False)
    assert a > b > c > 0
    setup, _, batch = smg.query_bytes(p, 16, smg.MIXED)
    assert a == setup + batch


def test_worker_threads_get_large_stacks():
    """Warm-up workers and lanes start with THREAD_STACK_BYTES of stack, and the
    process default is restored afterwards."""
    import threading

    seen = []
    before = threading.stack_size()
    with serve._thread_stack():
        t = threading.Thread(target=lambda: seen.append(threading.stack_size()))
        t.start()
        t.join()
    assert seen == [serve.THREAD_STACK_BYTES]
    assert threading.stack_size() == before


def test_warm_builds_every_key_once():
    be = FakeBackend()
    keys = [(f, m) for f in (1, 2, 3) for m in (0.1, 0.2)]
    with serve.Server(be, budget_bytes=10_000, capacity=4) as srv:
        srv.warm(keys, workers=2)
        assert len(be.setups) == 3 and len(be.derives) == 3
        # hierarchies stay resident; batches live with the lanes only
        assert all(srv.cache.entry(f, m) is not None and srv.cache.entry(f, m).batch is None for f, m in keys)
        reqs = make_requests([(f, m, 2, 0.0) for f, m in keys])
        results = srv.run_trace(reqs, timeout=30)
        assert len(be.setups) == 3 and len(be.derives) == 3  # served from the warm cache
    check_results(reqs, results)


def test_eviction_keeps_full_setups_longer():
    """Derived hierarchies (another mass of a resident field) are evicted before full
    setups, least recently used first within each kind, and a new mass derives from
    the field's full setup when it is resident."""
    be = FakeBackend(est=100)
    cache = serve.SetupCache(be, budget_bytes=300)
    for f, m in ((1, 0.1), (1, 0.2), (2, 0.1)):  # setup 1, derive (1, 0.2), setup 2
        assert cache.acquire(f, m, 4) is not None
        cache.release(f, m)
    assert be.setups == [(1, 0.1), (2, 0.1)] and be.derives == [(1, 0.2)]
    assert cache.entry(1, 0.1).base and not cache.entry(1, 0.2).base
    # a fourth key needs room: the derived (1, 0.2) goes, although (1, 0.1) is older
    assert cache.acquire(3, 0.1, 4) is not None
    cache.release(3, 0.1)
    assert cache.entry(1, 0.2) is None and cache.entry(1, 0.1) is not None
    # the next mass of field 1 derives from its full setup, which is kept while room is
    # made (the least recently used other full setup, field 2's, goes instead)
    assert cache.acquire(1, 0.3, 4) is not None
    assert be.derives[-1] == (1, 0.3) and len(be.setups) == 3
    assert cache.entry(2, 0.1) is None and cache.entry(1, 0.1) is not None


def test_batches_live_with_lanes_and_are_accounted():
    """A lane opens its key's batch when it starts (its bytes count against the
    budget) and closes it when it retires; the hierarchy stays resident and only
    its own bytes remain counted."""
    be = FakeBackend(est=100, bytes_per_solver=80, bytes_per_batch=20)
    with serve.Server(be, budget_bytes=10_000, capacity=4, linger=0.0) as srv:
        reqs = make_requests([(1, 0.1, 2, 0.0), (2, 0.1, 3, 0.0)])
        results = srv.run_trace(reqs, timeout=30)
        deadline = time.time() + 10
        while srv.lanes and time.time() < deadline:
            time.sleep(0.01)
        assert not srv.lanes
        assert srv.cache.used == 2 * 80
        assert all(e.batch is None for e in srv.cache.entries.values())
    check_results(reqs, results)


def test_fitted_batch_capacity():
    """With fit_capacity a lane's batch has the smallest power of two >= the minimum
    that holds the right-hand sides queued for its key, at most `capacity`; a request
    wider than that streams through the slots and every result is still right."""
    be = FakeBackend()
    caps = []
    make = be.new_batch

    def recording(solver, capacity, *a):
        caps.append((solver.field, capacity))
        return make(solver, capacity, *a)

    be.new_batch = recording
    srv = serve.Server(be, budget_bytes=10_000, capacity=16, fit_capacity=True, min_capacity=4)
    assert [srv.batch_capacity(w) for w in (0, 1, 4, 5, 8, 9, 16, 40)] == [4, 4, 4, 8, 8, 16, 16, 16]
    assert serve.Server(be, 10_000, capacity=16).batch_capacity(1) == 16  # fixed by default
    assert serve.Server(be, 10_000, capacity=2, fit_capacity=True).batch_capacity(1) == 2
    with srv:
        reqs = make_requests([(1, 0.1, 1, 0.0), (2, 0.1, 6, 0.0), (3, 0.1, 13, 0.0), (4, 0.1, 30, 0.0)])
        results = srv.run_trace(reqs, timeout=30)
    check_results(reqs, results)
    assert sorted(caps) == [(1, 4), (2, 8), (3, 16), (4, 16)]
    times = srv.phase_times()
    assert times["lanes"] == 4 and times["serve_s"] > 0 and times["batch_create_s"] >= 0


def test_retiring_lane_keeps_its_key_until_its_batch_is_closed():
    """A request for a key whose lane is retiring (between its decision to retire and
    the close of its batch) waits for that lane to finish and then gets a lane and a
    batch of its own: it never reaches the batch that is being closed."""
    be = FakeBackend()
    made = []
    make = be.new_batch

    def recording(solver, capacity, *a):
        b = make(solver, capacity, *a)
        made.append(b)
        return b

    be.new_batch = recording
    with serve.Server(be, budget_bytes=10_000, capacity=4, linger=0.0) as srv:
        close = srv.cache.close_batch

        def slow_close(field, mass):  # the retiring lane is slow to reach the close
            time.sleep(0.3)
            close(field, mass)

        srv.cache.close_batch = slow_close
        first = make_requests([(1, 0.1, 2, 0.0)], seed=1)
        check_results(first, srv.run_trace(first, timeout=30))
        time.sleep(0.1)  # the idle lane (linger 0) has decided to retire and is not done
        second = make_requests([(1, 0.1, 3, 0.0)], seed=2)
        second[0].rid = 99
        check_results(second, srv.run_trace(second, timeout=30))
    assert len(made) == 2 and made[1] is not made[0]
    assert all(b.closed for b in made)
