"""Serving: a continuous-batching request loop over the adaptive-MG library.

The paper separates the adaptive setup from the solves and reuses one setup for
many right-hand sides and for other masses (Results section).  A server that
answers solve requests for many gauge fields therefore keeps each field's setup
resident on the device and sends every right-hand side through a batch of column
slots of that setup:

* ``SetupCache`` holds hierarchies keyed by (field, mass) under an HBM budget,
  evicting the least recently used idle one when a new one does not fit.  The
  first mass of a field runs the full adaptive setup; another mass of a field
  with a resident hierarchy is derived from it (same near-null vectors, new
  Galerkin operators), as the paper does when it changes the mass.
* A ``Lane`` serves one (field, mass) key on its own stream and host thread.  It
  owns a ``Batch`` (``smg_batch_*``): right-hand sides are admitted into free
  slots whenever they arrive, all running slots advance together, and finished
  slots are harvested and refilled.  Lanes of different keys run at the same
  time, so their kernels overlap on the device.
* ``Server`` routes requests (each 1..k right-hand sides) to lanes, limits the
  number of live lanes, and records arrival, admission and completion times.

All numerical work is in the library; this module only schedules it.  The cache,
lanes and server accept any backend object with the methods used here, which
lets the host logic be tested without a GPU.
"""

from __future__ import annotations

import collections
import contextlib
import dataclasses
import math
import threading
import time
from typing import Callable, Dict, Hashable, List, Optional, Sequence, Tuple

__all__ = [
    "Request",
    "Result",
    "SetupCache",
    "Server",
    "estimate_bytes",
    "poisson_trace",
    "latency_summary",
    "levels_for",
]

Z64, Z32 = 16, 8


def levels_for(l: int, block: int = 4, max_coarse: int = 8) -> int:
    """Number of levels for an l x l lattice with block x block aggregates: coarsen
    while the coarse extent stays >= 4 and the coarse lattice exceeds max_coarse."""
    levels, c = 1, l
    while c % block == 0 and c // block >= 4 and c > max_coarse:
        c //= block
        levels += 1
    return levels


def estimate_bytes(params, capacity: int = 1, mixed: bool = True) -> int:
    """Device bytes of one hierarchy plus a batch of `capacity` slots (none for 0),
    from the library's own allocation plan (smg_query_bytes: no device call)."""
    from . import FP64, MIXED, query_bytes

    setup, _solve, batch = query_bytes(params, max(capacity, 1), MIXED if mixed else FP64)
    return setup + (batch if capacity > 0 else 0)


# Stack of every thread that calls into the library here (warm-up workers, lanes).
# A launch from a fresh thread can run deep in the HIP runtime and, under a
# profiler's tracing callbacks, beyond the 8 MiB that threads get by default.
THREAD_STACK_BYTES = 64 << 20


@contextlib.contextmanager
def _thread_stack(nbytes: int = THREAD_STACK_BYTES):
    """Threads started inside the block get `nbytes` of stack."""
    old = threading.stack_size(nbytes)
    try:
        yield
    finally:
        threading.stack_size(old)


@dataclasses.dataclass
class Request:
    """A solve request: A(field, mass) x_i = b_i for its k right-hand sides.

    `rhs` is a [k, n] complex128 device tensor or a callable returning one (called
    on the serving lane's stream when the request is first admitted)."""

    rid: int
    field: Hashable
    mass: float
    rhs: object
    k: int
    arrival: float = 0.0


@dataclasses.dataclass
class Result:
    rid: int
    field: Hashable
    mass: float
    k: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    x: object = None
    status: List[int] = dataclasses.field(default_factory=list)
    iterations: List[int] = dataclasses.field(default_factory=list)
    true_relres: List[float] = dataclasses.field(default_factory=list)
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def ok(self) -> bool:
        return self.error is None and all(s == 0 for s in self.status)


class BudgetExceeded(RuntimeError):
    pass


@dataclasses.dataclass
class _Entry:
    solver: object
    bytes: int
    pins: int = 0
    batch: object = None  # the key's slot batch, kept with the hierarchy
    base: bool = False    # built by the full adaptive setup (it holds the mass coefficients)
    ready: threading.Event = dataclasses.field(default_factory=threading.Event)
    failed: Optional[BaseException] = None


class SetupCache:
    """Resident hierarchies keyed by (field, mass), least recently used first out.

    backend.setup(field, mass, stream) -> solver   full adaptive setup
    backend.derive(solver, mass, stream) -> solver  another mass, same vectors
    backend.estimate(field, capacity) -> bytes      before allocating
    solver.memory_bytes(), solver.close()

    Setups run outside the cache lock (other keys stay available meanwhile); a
    second request for a key being built waits for it.
    """

    def __init__(self, backend, budget_bytes: int):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.entries: "collections.OrderedDict[Tuple, _Entry]" = collections.OrderedDict()
        self.used = 0
        self.lock = threading.RLock()
        self.setups = 0
        self.derives = 0
        self.evictions = 0
        # seconds spent in setups, derives, evictions (closing hierarchies and batches)
        # and trims, summed over the threads that ran them
        self.times = collections.Counter()

    def _time(self, name: str, t0: float):
        dt = time.perf_counter() - t0
        with self.lock:
            self.times[name] += dt

    def _evict_for(self, need: int) -> bool:
        # least recently used first; hierarchies derived from another mass (cheap to
        # derive again) before full setups (a field's adaptive setup costs far more)
        t0 = time.perf_counter()
        try:
            return self._evict_lru(need)
        finally:
            self.times["evict_s"] += time.perf_counter() - t0  # called under the lock

    def _evict_lru(self, need: int) -> bool:
        for bases in (False, True):
            for key in list(self.entries.keys()):
                if self.used + need <= self.budget:
                    break
                e = self.entries[key]
                if e.pins == 0 and e.ready.is_set() and e.base == bases:
                    if e.batch is not None:
                        e.batch.close()
                    if e.solver is not None:
                        e.solver.close()
                    self.used -= e.bytes
                    del self.entries[key]
                    self.evictions += 1
        return self.used + need <= self.budget

    def entry(self, field, mass: float) -> Optional[_Entry]:
        with self.lock:
            return self.entries.get((field, float(mass)))

    def acquire(self, field, mass: float, capacity: int, stream=None):
        """Pinned solver for (field, mass); None while the budget cannot make room
        (every resident hierarchy is in use).  Raises BudgetExceeded when it could
        never fit, and what the setup raised when it failed."""
        key = (field, float(mass))
        with self.lock:
            e = self.entries.get(key)
            if e is not None:
                self.entries.move_to_end(key)
                e.pins += 1
                build = evicted = False
            else:
                need = self.backend.estimate(field, 0)  # the hierarchy; a lane's batch is added by open_batch
                if need + self.backend.estimate(field, capacity) - need > self.budget:
                    raise BudgetExceeded(f"{key}: {need} bytes exceed the budget of {self.budget}")
                # derive from a resident hierarchy of the field, its full setup first; it is
                # pinned before room is made, so that the eviction cannot take it
                same = [(k, v) for k, v in reversed(self.entries.items())
                        if k[0] == field and v.ready.is_set() and v.solver is not None]
                same.sort(key=lambda kv: not kv[1].base)
                src = same[0][0] if same else None
                if src is not None:
                    self.entries[src].pins += 1
                ev0 = self.evictions
                if not self._evict_for(need):
                    if src is not None:
                        self.entries[src].pins -= 1
                    return None
                evicted = self.evictions != ev0
                e = _Entry(None, need, pins=1)
                self.entries[key] = e
                self.used += need
                build = True
        if build and evicted and hasattr(self.backend, "trim"):
            t0 = time.perf_counter()
            self.backend.trim()  # memory the evicted hierarchies held goes back to the device
            self._time("trim_s", t0)
        if not build:
            e.ready.wait()
            if e.failed is not None:
                self.release(field, mass)
                raise e.failed
            return e.solver
        t0 = time.perf_counter()
        try:
            if src is not None:
                solver = self.backend.derive(self.entries[src].solver, float(mass), stream)
            else:
                solver = self.backend.setup(field, float(mass), stream)
            self._time("derive_s" if src is not None else "setup_s", t0)
        except BaseException as exc:
            with self.lock:
                e.failed = exc
                self.used -= e.bytes
                e.bytes = 0
                if self.entries.get(key) is e:
                    del self.entries[key]
                if src is not None:
                    self.entries[src].pins -= 1
            e.ready.set()
            raise
        with self.lock:
            e.solver = solver
            if src is not None:
                self.entries[src].pins -= 1
                self.derives += 1
            else:
                e.base = True
                self.setups += 1
        e.ready.set()
        return solver

    def open_batch(self, field, mass: float, capacity: int, make: Callable[[], object]):
        """A new batch for a pinned key, made by make(), its bytes counted against the
        budget; None while the budget cannot make room for it, or while the key's
        previous batch (another caller's) is not closed yet."""
        key = (field, float(mass))
        with self.lock:
            e = self.entries[key]
            if e.batch is not None:
                return None
            need = self.backend.batch_estimate(field, capacity)
            ev0 = self.evictions
            if not self._evict_for(need):
                return None
            evicted = self.evictions != ev0
            e.bytes += need
            self.used += need
        if evicted and hasattr(self.backend, "trim"):
            t0 = time.perf_counter()
            self.backend.trim()
            self._time("trim_s", t0)
        t0 = time.perf_counter()
        try:
            batch = make()
        except BaseException:
            with self.lock:
                e.bytes -= need
                self.used -= need
            raise
        self._time("batch_create_s", t0)
        with self.lock:
            e.batch = batch
            actual = e.solver.memory_bytes() + batch.memory_bytes()
            self.used += actual - e.bytes
            e.bytes = actual
        return batch

    def close_batch(self, field, mass: float):
        """Close a key's batch (its slots are all harvested); the hierarchy stays."""
        key = (field, float(mass))
        with self.lock:
            e = self.entries.get(key)
            if e is None or e.batch is None:
                return
            batch, e.batch = e.batch, None
            actual = e.solver.memory_bytes()
            self.used += actual - e.bytes
            e.bytes = actual
        t0 = time.perf_counter()
        batch.close()
        self._time("batch_close_s", t0)

    def settle(self, field, mass: float, actual: int):
        """Replace the estimate of a resident entry by its measured bytes."""
        with self.lock:
            e = self.entries.get((field, float(mass)))
            if e is not None:
                self.used += int(actual) - e.bytes
                e.bytes = int(actual)

    def release(self, field, mass: float):
        with self.lock:
            e = self.entries.get((field, float(mass)))
            if e is not None and e.pins > 0:
                e.pins -= 1

    def close(self):
        with self.lock:
            for e in self.entries.values():
                if e.batch is not None:
                    e.batch.close()
                if e.solver is not None:
                    e.solver.close()
            self.entries.clear()
            self.used = 0


class _Lane:
    """One (field, mass) key: a batch of slots on its own stream and thread."""

    def __init__(self, server: "Server", field, mass: float):
        self.server = server
        self.field = field
        self.mass = float(mass)
        self.pending: "collections.deque[Tuple[Result, Request, int]]" = collections.deque()
        self.slots: Dict[int, Tuple[Result, int]] = {}
        self.remaining: Dict[int, int] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.last_busy = time.perf_counter()
        with _thread_stack():
            self.thread = threading.Thread(target=self._run, daemon=True, name=f"lane-{field}-{mass}")
        self.solver = None
        self.batch = None
        self.cap = server.capacity  # slots of this lane's batch (Server.batch_capacity)
        self.stream = server._take_stream()

    def push(self, res: Result, req: Request):
        with self.cv:
            for j in range(req.k):
                self.pending.append((res, req, j))
            self.remaining[res.rid] = req.k
            self.last_busy = time.perf_counter()
            self.cv.notify()

    def idle(self) -> bool:
        with self.cv:
            return not self.pending and not self.slots

    def _fail(self, msg: str):
        srv = self.server
        with self.cv:
            items = list(self.pending)
            self.pending.clear()
            held = list(self.slots.values())
            self.slots.clear()
        done = set()
        for res, _req, _j in items:
            if res.rid not in done:
                res.error = msg
                done.add(res.rid)
                srv._complete(res)
        for res, _j in held:
            if res.rid not in done:
                res.error = msg
                done.add(res.rid)
                srv._complete(res)

    def _run(self):
        srv = self.server
        be = srv.backend
        ctx = be.stream_context(self.stream)
        t_start = time.perf_counter()
        with ctx:
            try:
                while True:
                    self.solver = srv.cache.acquire(self.field, self.mass, srv.capacity, self.stream)
                    if self.solver is not None:
                        break
                    if self.stop:
                        return
                    time.sleep(srv.poll_sleep)
                t_acq = time.perf_counter()
                srv._lane_time("acquire_s", t_acq - t_start)
                # the key's batch lives while the lane does: idle keys keep only their hierarchy
                with self.cv:
                    want = len(self.pending)
                self.cap = srv.batch_capacity(want)
                make = lambda: be.new_batch(self.solver, self.cap, srv.tol, srv.maxiter,  # noqa: E731
                                            srv.precision, self.stream)
                while True:
                    self.batch = srv.cache.open_batch(self.field, self.mass, self.cap, make)
                    if self.batch is not None:
                        break
                    if self.stop:
                        srv.cache.release(self.field, self.mass)
                        self.solver = None
                        return
                    time.sleep(srv.poll_sleep)
                srv._lane_time("open_batch_s", time.perf_counter() - t_acq)
            except Exception as exc:  # setup failed: fail what is queued here
                self._fail(f"setup: {exc}")
                if self.solver is not None:
                    srv.cache.release(self.field, self.mass)
                    self.solver = None
                srv._lane_done(self)
                return
            t_serve = time.perf_counter()
            try:
                self._serve()
            except Exception as exc:
                self._fail(f"solve: {exc}")
            finally:
                t_end = time.perf_counter()
                srv._lane_time("serve_s", t_end - t_serve)
                try:
                    srv.cache.close_batch(self.field, self.mass)
                except Exception:
                    pass
                self.batch = None
                srv.cache.release(self.field, self.mass)
                self.solver = None
                srv._lane_done(self)
                srv._lane_time("close_s", time.perf_counter() - t_end)
                srv._lane_time("lanes", 1)

    def _serve(self):
        srv = self.server
        be = srv.backend
        while True:
            idle = 0.0
            with self.cv:
                if not self.pending and not self.slots and not self.stop:
                    t_idle = time.perf_counter()
                    self.cv.wait(timeout=srv.poll_sleep * 10)
                    idle = time.perf_counter() - t_idle
                has_work = bool(self.pending or self.slots)
                stop = self.stop
                todo = []
                free = self.cap - len(self.slots)
                while self.pending and len(todo) < free:
                    todo.append(self.pending.popleft())
            if idle:
                srv._lane_time("idle_s", idle)  # takes the server lock: never under self.cv
            if not has_work:
                if stop or srv._want_retire(self):  # takes the server lock: never under self.cv
                    return
                continue
            for i, (res, req, j) in enumerate(todo):
                if res.x is None:
                    rhs = req.rhs() if callable(req.rhs) else req.rhs
                    req.rhs = rhs
                    res.x = be.new_output(rhs)
                    res.status = [1] * req.k
                    res.iterations = [0] * req.k
                    res.true_relres = [math.nan] * req.k
                if math.isnan(res.admitted):
                    res.admitted = srv.now()
                slot = self.batch.admit(req.rhs[j], self.stream)
                if slot is None:  # cannot happen while slots are counted; keep the columns
                    with self.cv:
                        self.pending.extendleft(reversed(todo[i:]))
                    break
                self.slots[slot] = (res, j)
            if self.slots:
                t_step = time.perf_counter()
                self.batch.step(srv.iters_per_step, self.stream)
                polled = self.batch.poll()
                srv._lane_time("step_poll_s", time.perf_counter() - t_step)
                for slot, st in polled:
                    res, j = self.slots.pop(slot)
                    self.batch.harvest(slot, res.x[j], self.stream)
                    res.status[j] = st["status"]
                    res.iterations[j] = st["iterations"]
                    res.true_relres[j] = st["true_relres"]
                    self.remaining[res.rid] -= 1
                    if self.remaining[res.rid] == 0:
                        del self.remaining[res.rid]
                        res.finished = srv.now()
                        srv._complete(res)
                self.last_busy = time.perf_counter()


class Server:
    """Routes requests to per-(field, mass) lanes; at most `max_lanes` are live.

    backend: new_stream(), stream_context(stream), new_batch(solver, capacity, tol,
    maxiter, precision, stream), new_output(rhs), plus the SetupCache methods.
    """

    def __init__(self, backend, budget_bytes: int, capacity: int = 16, tol: float = 1e-10, maxiter: int = 5000,
                 precision: int = 1, max_lanes: int = 8, iters_per_step: int = 1, poll_sleep: float = 0.0005,
                 linger: float = 0.5, keep_solutions: bool = True, fit_capacity: bool = False,
                 min_capacity: int = 4):
        self.backend = backend
        self.cache = SetupCache(backend, budget_bytes)
        self.capacity = int(capacity)
        # fit_capacity: a lane's batch gets the smallest power of two >= min_capacity
        # that holds the right-hand sides queued for its key when it opens (at most
        # `capacity`), so that small requests do not hold a full batch of memory
        self.fit_capacity = bool(fit_capacity)
        self.min_capacity = max(1, int(min_capacity))
        self.tol = float(tol)
        self.maxiter = int(maxiter)
        self.precision = int(precision)
        self.max_lanes = int(max_lanes)
        self.iters_per_step = int(iters_per_step)
        self.poll_sleep = float(poll_sleep)
        self.linger = float(linger)
        self.lanes: Dict[Tuple, _Lane] = {}
        self.waiting: "collections.deque[Tuple[Result, Request]]" = collections.deque()
        self.lock = threading.RLock()
        self.done_cv = threading.Condition(self.lock)
        self.results: Dict[int, Result] = {}
        self.open = 0
        self.t0 = time.perf_counter()
        self.lanes_started = 0
        # lane seconds by phase (acquire, open_batch, serve with its idle_s part, close)
        # and the number of lanes that ended, summed over the lanes
        self.lane_times = collections.Counter()
        self.streams: list = []
        # False: a finished request drops its right-hand sides and solutions (its
        # statistics stay), so that a long trace does not hold them all on the device
        self.keep_solutions = bool(keep_solutions)
        self.requests: Dict[int, Request] = {}

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def batch_capacity(self, want: int) -> int:
        """Slots of a lane's batch when `want` right-hand sides wait for its key."""
        if not self.fit_capacity:
            return self.capacity
        c = min(self.min_capacity, self.capacity)
        while c < want and c < self.capacity:
            c *= 2
        return min(c, self.capacity)

    def _lane_time(self, name: str, value: float):
        with self.lock:
            self.lane_times[name] += value

    def phase_times(self) -> dict:
        """Lane phases and cache work so far (seconds summed over threads; `lanes`
        counts the lanes that ended)."""
        with self.lock:
            out = dict(self.lane_times)
        with self.cache.lock:
            out.update(self.cache.times)
        return out

    # -- routing ---------------------------------------------------------------
    def submit(self, req: Request, arrival: Optional[float] = None) -> Result:
        res = Result(req.rid, req.field, float(req.mass), req.k, self.now() if arrival is None else arrival)
        with self.lock:
            self.results[req.rid] = res
            self.requests[req.rid] = req
            self.open += 1
            self._route(res, req)
        return res

    def _route(self, res: Result, req: Request):
        key = (req.field, float(req.mass))
        lane = self.lanes.get(key)
        if lane is None:
            if len(self.lanes) >= self.max_lanes:
                self.waiting.append((res, req))
                return
            lane = _Lane(self, req.field, req.mass)
            self.lanes[key] = lane
            self.lanes_started += 1
            lane.push(res, req)
            lane.thread.start()
            return
        lane.push(res, req)

    def _want_retire(self, lane: _Lane) -> bool:
        """An idle lane leaves when others wait for a lane or it lingered long.  It
        stays the key's lane until its batch is closed (_lane_done): a request for the
        key that arrives meanwhile is queued on it and goes back to the waiting queue
        then, so that no second lane of the key can reach the batch being closed."""
        with self.lock:
            if lane.pending or lane.slots:
                return False
            return bool(self.waiting) or time.perf_counter() - lane.last_busy > self.linger

    def _take_stream(self):
        with self.lock:
            return self.streams.pop() if self.streams else self.backend.new_stream()

    def _lane_done(self, lane: _Lane):
        with self.lock:
            self.streams.append(lane.stream)
            key = (lane.field, lane.mass)
            if self.lanes.get(key) is lane:
                del self.lanes[key]
            # requests routed to the lane after it decided to retire
            with lane.cv:
                left = list(lane.pending)
                lane.pending.clear()
            seen = set()
            for res, req, _j in left:
                if res.rid not in seen:
                    seen.add(res.rid)
                    self.waiting.appendleft((res, req))
            self._drain_waiting()

    def _drain_waiting(self):
        keep = collections.deque()
        while self.waiting:
            res, req = self.waiting.popleft()
            key = (req.field, float(req.mass))
            if key in self.lanes or len(self.lanes) < self.max_lanes:
                self._route(res, req)
            else:
                keep.append((res, req))
        self.waiting = keep

    def _complete(self, res: Result):
        with self.lock:
            if math.isnan(res.finished):
                res.finished = self.now()
            req = self.requests.pop(res.rid, None)
            if not self.keep_solutions:
                res.x = None
                if req is not None:
                    req.rhs = None
            self.open -= 1
            self.done_cv.notify_all()

    # -- warm-up -----------------------------------------------------------------
    def warm(self, keys: Sequence[Tuple], workers: int = 4, serial: int = 1):
        """Build the hierarchy of each (field, mass) key before serving (the masses of
        one field in order, so that the first one runs the adaptive setup and the
        others derive from it).  The first `serial` fields are built on this thread
        alone, so that the kernels they use have all been launched once before several
        threads launch them at the same time; the other fields in parallel."""
        by_field: Dict = collections.OrderedDict()
        for f, m in keys:
            by_field.setdefault(f, []).append(float(m))
        items = list(by_field.items())
        errors: list = []

        def work(i):
            stream = self._take_stream()
            try:
                with self.backend.stream_context(stream):
                    for f, ms in items[i::workers]:
                        build(f, ms, stream)
            except BaseException as exc:
                errors.append(exc)
            finally:
                with self.lock:
                    self.streams.append(stream)

        def build(f, ms, stream):
            for m in ms:
                solver = self.cache.acquire(f, m, self.capacity, stream)
                if solver is None:
                    raise BudgetExceeded(f"no room to warm {(f, m)}")
                # a batch made once readies the operators its precision needs; the lanes make their own
                b = self.cache.open_batch(f, m, self.capacity, lambda s_=solver: self.backend.new_batch(
                    s_, self.capacity, self.tol, self.maxiter, self.precision, stream))
                if b is not None:
                    self.cache.close_batch(f, m)
                self.cache.release(f, m)

        if serial > 0 and items:
            stream = self._take_stream()
            try:
                with self.backend.stream_context(stream):
                    for f, ms in items[:serial]:
                        build(f, ms, stream)
            finally:
                with self.lock:
                    self.streams.append(stream)
            items = items[serial:]
        with _thread_stack():
            threads = [threading.Thread(target=work, args=(i,)) for i in range(min(workers, len(items)))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]

    # -- driving ---------------------------------------------------------------
    def run_trace(self, requests: Sequence[Request], timeout: float = 600.0,
                  progress: Optional[Callable[[int, int], None]] = None) -> List[Result]:
        """Submit each request at its arrival time (seconds from now) and wait for
        all of them; returns the results in request order.  progress(open, total), if
        given, is called about every 10 s while waiting."""
        self.t0 = time.perf_counter()
        order = sorted(requests, key=lambda r: r.arrival)
        for req in order:
            dt = req.arrival - self.now()
            if dt > 0:
                time.sleep(dt)
            self.submit(req, arrival=req.arrival)
            with self.lock:
                self._drain_waiting()
        self.wait(timeout, progress=(None if progress is None else (lambda o: progress(o, len(order)))))
        return [self.results[r.rid] for r in requests]

    def wait(self, timeout: float = 600.0, progress: Optional[Callable[[int], None]] = None):
        end = time.perf_counter() + timeout
        tick = time.perf_counter() + 10.0
        with self.lock:
            while self.open > 0:
                self._drain_waiting()
                now = time.perf_counter()
                left = end - now
                if left <= 0:
                    raise TimeoutError(f"{self.open} requests still open")
                if progress is not None and now >= tick:
                    progress(self.open)
                    tick = now + 10.0
                self.done_cv.wait(timeout=min(left, 0.01))

    def close(self):
        with self.lock:
            lanes = list(self.lanes.values())
        for lane in lanes:
            with lane.cv:
                lane.stop = True
                lane.cv.notify()
        for lane in lanes:
            lane.thread.join(timeout=60)
        self.cache.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# -- workloads -------------------------------------------------------------------
def poisson_trace(n_requests: int, rate: float, fields: Sequence, masses: Dict, k_range=(1, 16),
                  seed: int = 0) -> List[Tuple[float, object, float, int, int]]:
    """(arrival, field, mass, k, rhs_seed) for a Poisson stream of `rate`
    requests/s; field uniform over `fields`, mass uniform over masses[field], k
    uniform over k_range (inclusive)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        f = fields[int(rng.integers(len(fields)))]
        ms = masses[f]
        m = float(ms[int(rng.integers(len(ms)))])
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        out.append((float(t[i]), f, m, k, int(rng.integers(1 << 31))))
    return out


def latency_summary(results: Sequence[Result]) -> dict:
    import numpy as np

    lat = np.array([r.latency for r in results if r.ok], dtype=np.float64)
    solves = sum(r.k for r in results if r.ok)
    span = max(r.finished for r in results) - min(r.arrival for r in results) if results else 0.0
    if lat.size == 0:
        return {"requests": len(results), "ok": 0}
    wait = np.array([r.admitted - r.arrival for r in results if r.ok], dtype=np.float64)
    service = np.array([r.finished - r.admitted for r in results if r.ok], dtype=np.float64)
    return {
        "requests": len(results),
        "ok": int(sum(r.ok for r in results)),
        "solves": int(solves),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "wait_p50_ms": float(np.percentile(wait, 50) * 1e3),
        "wait_p99_ms": float(np.percentile(wait, 99) * 1e3),
        "service_p50_ms": float(np.percentile(service, 50) * 1e3),
        "service_p99_ms": float(np.percentile(service, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "span_s": float(span),
        "solves_per_s": float(solves / span) if span > 0 else math.nan,
    }


class DeviceBackend:
    """The library on the GPU: one torch stream per lane.

    fields: {key: (gauge tensor [2, lt, lx] on the device, Params template)}."""

    def __init__(self, fields: Dict, mixed: bool = True):
        import torch

        from . import Batch, Solver

        self.torch = torch
        self.Solver = Solver
        self.Batch = Batch
        self.fields = fields
        self.mixed = mixed

    def estimate(self, field, capacity: int) -> int:
        """Hierarchy bytes, plus a batch of `capacity` slots when capacity > 0."""
        _g, p = self.fields[field]
        return estimate_bytes(p, capacity, mixed=self.mixed)

    def batch_estimate(self, field, capacity: int) -> int:
        _g, p = self.fields[field]
        return estimate_bytes(p, capacity, mixed=self.mixed) - estimate_bytes(p, 0, mixed=self.mixed)

    def setup(self, field, mass: float, stream):
        g, p = self.fields[field]
        q = type(p)()
        ctypes_copy(q, p)
        q.mass = mass
        return self.Solver(g, q, stream=stream)

    def derive(self, solver, mass: float, stream):
        return solver.derive(mass, stream=stream)

    def new_stream(self):
        return self.torch.cuda.Stream()

    def trim(self, slack: int = 8 << 30):
        """Return torch's cached free blocks (where the library's evicted arrays went)
        to the device once they exceed `slack` bytes, so that allocations outside
        torch's cache (rocBLAS workspaces) still find memory."""
        t = self.torch
        if t.cuda.memory_reserved() - t.cuda.memory_allocated() > slack:
            t.cuda.empty_cache()

    def stream_context(self, stream):
        return self.torch.cuda.stream(stream)

    def new_batch(self, solver, capacity, tol, maxiter, precision, stream):
        return self.Batch(solver, capacity, tol=tol, maxiter=maxiter, precision=precision, stream=stream)

    def new_output(self, rhs):
        return self.torch.empty_like(rhs)


def ctypes_copy(dst, src):
    import ctypes

    ctypes.memmove(ctypes.addressof(dst), ctypes.addressof(src), ctypes.sizeof(src))
