"""Request loop over the sparse LU library: factor, refactor and solve requests for
many matrix patterns, served concurrently on one GPU.

Every pattern keeps one resident handle (symbolic analysis + factors on the device).
Worker threads are the slots: a free slot takes the oldest queued request whose pattern
is idle and whose handle fits the HBM budget (evicting idle least-recently-used handles
when it does not), so requests that arrive while others run are admitted as slots and
memory free up.  Library calls release the GIL and every handle runs on its own HIP
stream, so admitted requests overlap on the device.  Requests of one pattern run one at
a time in arrival order, which makes every result identical to running that pattern's
requests alone, in the same order.  An evicted pattern is rebuilt from host copies of
its values (a factorization with the values that chose its pivots, then a
refactorization with its latest values), so eviction does not change results either.
A pattern larger than the whole budget runs once nothing else is running.

The numeric work is the library's: this module only schedules calls.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import Handle, default_options, BaskerError

FACTOR, REFACTOR, SOLVE = "factor", "refactor", "solve"


@dataclass
class Pattern:
    """A sparsity pattern the server knows: CSC structure plus the options to analyse it."""
    key: str
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    values: np.ndarray          # values used by the matching at analysis time
    options: dict = field(default_factory=dict)


@dataclass
class Request:
    kind: str                    # factor | refactor | solve
    pattern: str
    values: Optional[np.ndarray] = None   # factor / refactor
    rhs: Optional[np.ndarray] = None      # solve: n x nrhs, column-major
    arrival: float = 0.0         # perf_counter time the request entered the queue
    start: float = 0.0
    done: float = 0.0
    status: int = 0
    result: Optional[np.ndarray] = None   # solve: the solution
    error: Optional[str] = None
    event: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Csc:
    """The minimal CSC view Handle.symbolic needs."""

    def __init__(self, p: Pattern):
        self.n = p.n
        self.colptr = p.colptr
        self.rowind = p.rowind
        self.values = p.values
        self.nnz = int(p.colptr[-1])


class _Resident:
    def __init__(self, estimate: int):
        self.handle: Optional[Handle] = None
        self.bytes = estimate     # device bytes; the estimate until a request has run
        self.busy = False
        self.factored = False
        self.last_use = 0.0


class _State:
    """Host copy of what a pattern's factors are made of, to rebuild them bit for bit
    after an eviction: the values of the last full factorization (pivots chosen there)
    and the values of the last factor or refactor."""

    def __init__(self):
        self.base: Optional[np.ndarray] = None
        self.cur: Optional[np.ndarray] = None


def library_estimate(p: Pattern) -> int:
    """Device bytes a handle of pattern p will hold after its first factorization and a
    solve with up to 8 right-hand sides, as the library computes them from its own
    plan (a host-only symbolic analysis: no device memory is touched)."""
    h = Handle.symbolic(_Csc(p), default_options(**dict(p.options, device=-1)))
    try:
        return int(h.info()["device_bytes_plan"])
    finally:
        h.free()


class Server:
    """slots: concurrent requests; hbm_budget: bytes of device memory the resident
    handles may hold.  A pattern not yet resident is admitted on its estimate (by
    default the library's own, from a host-only analysis, computed once per pattern);
    once it has run, its handle's actual device bytes count instead."""

    def __init__(self, patterns: list, slots: int = 8, hbm_budget: int = 200 << 30,
                 estimate: Optional[Callable[[Pattern], int]] = None):
        self.patterns = {p.key: p for p in patterns}
        self.slots = slots
        self.budget = hbm_budget
        self._est_fn = estimate or library_estimate
        self._est_cache: dict = {}
        self.peak_bytes = 0
        self.resident: dict = {}
        self.state = {p.key: _State() for p in patterns}
        self.restores = 0
        self.queue: collections.deque = collections.deque()
        self.cv = threading.Condition()
        self.stop = False
        self.evictions = 0
        self.completed = 0
        self.workers = [threading.Thread(target=self._work, daemon=True) for _ in range(slots)]
        for w in self.workers:
            w.start()

    # ---- client side -------------------------------------------------------------
    def submit(self, req: Request) -> Request:
        if req.pattern not in self.patterns:
            raise KeyError("unknown pattern %s" % req.pattern)
        req.arrival = req.arrival or time.perf_counter()
        with self.cv:
            self.queue.append(req)
            self.cv.notify()
        return req

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()
        for r in self.resident.values():
            if r.handle is not None:
                r.handle.free()
        self.resident.clear()

    def estimate(self, p: Pattern) -> int:
        if p.key not in self._est_cache:
            self._est_cache[p.key] = int(self._est_fn(p))
        return self._est_cache[p.key]

    def resident_bytes(self) -> int:
        return sum(r.bytes for r in self.resident.values())

    # ---- scheduling --------------------------------------------------------------
    def _admissible(self, req: Request) -> bool:
        """Called with the lock held: can req start now (pattern idle, memory fits)?"""
        r = self.resident.get(req.pattern)
        if r is not None:
            return not r.busy
        need = self.estimate(self.patterns[req.pattern])
        used = self.resident_bytes()
        if used + need <= self.budget:
            return True
        busy = [x for x in self.resident.values() if x.busy]
        if sum(x.bytes for x in busy) + need <= self.budget:
            return True
        # larger than the budget even alone: runs once nothing else does
        return not busy

    def _make_room(self, need: int):
        """Called with the lock held: evict idle handles, least recently used first."""
        used = self.resident_bytes()
        for key, r in sorted(self.resident.items(), key=lambda kv: kv[1].last_use):
            if used + need <= self.budget:
                break
            if r.busy:
                continue
            used -= r.bytes
            if r.handle is not None:
                r.handle.free()
            del self.resident[key]
            self.evictions += 1

    def _next(self) -> Optional[Request]:
        """Called with the lock held: the oldest admissible request, removed from the
        queue; a pattern's requests never overtake each other."""
        blocked = set()
        for i, req in enumerate(self.queue):
            if req.pattern in blocked:
                continue
            if self._admissible(req):
                del self.queue[i]
                return req
            blocked.add(req.pattern)
        return None

    def _work(self):
        while True:
            with self.cv:
                req = None
                while not self.stop:
                    req = self._next()
                    if req is not None:
                        break
                    self.cv.wait()
                if req is None:
                    return
                r = self.resident.get(req.pattern)
                if r is None:
                    est = self.estimate(self.patterns[req.pattern])
                    self._make_room(est)
                    r = _Resident(est)
                    self.resident[req.pattern] = r
                r.busy = True
            try:
                req.start = time.perf_counter()
                self._run(req, r)
            except BaseException as e:  # reported on the request, the server keeps going
                req.error = str(e)
                req.status = getattr(e, "status", -6)
            finally:
                req.done = time.perf_counter()
                if r.handle is not None:
                    r.bytes = int(r.handle.info()["device_bytes"])
                with self.cv:
                    r.busy = False
                    r.last_use = req.done
                    self.completed += 1
                    self.peak_bytes = max(self.peak_bytes, self.resident_bytes())
                    self.cv.notify_all()
                req.event.set()

    def _run(self, req: Request, r: _Resident):
        p = self.patterns[req.pattern]
        st = self.state[req.pattern]
        if r.handle is None:
            r.handle = Handle.symbolic(_Csc(p), default_options(**p.options))
            if st.base is not None:
                # rebuilt after an eviction: same pivots, same values as before
                r.handle.factor(st.base)
                if st.cur is not st.base:
                    r.handle.refactor(st.cur)
                r.factored = True
                self.restores += 1
        h = r.handle
        if req.kind == FACTOR or (req.kind == REFACTOR and not r.factored):
            h.factor(req.values)
            r.factored = True
            st.base = st.cur = np.array(req.values, dtype=np.float64, copy=True)
        elif req.kind == REFACTOR:
            req.status = h.refactor(req.values)
            st.cur = np.array(req.values, dtype=np.float64, copy=True)
            if req.status != 0:     # fell back to a full factorization: new pivots
                st.base = st.cur
        elif req.kind == SOLVE:
            if not r.factored:
                raise BaskerError(-5, "solve before any factor of pattern %s" % req.pattern)
            req.result = h.solve(req.rhs)
        else:
            raise ValueError("unknown request kind %s" % req.kind)


def run_sequential(patterns: list, requests: list) -> list:
    """The plain path: one request at a time, in arrival order, one handle per pattern
    (no eviction), on the calling thread."""
    pats = {p.key: p for p in patterns}
    handles, factored = {}, set()
    for req in requests:
        p = pats[req.pattern]
        req.start = time.perf_counter()
        if req.arrival == 0.0:
            req.arrival = req.start
        h = handles.get(req.pattern)
        if h is None:
            h = handles[req.pattern] = Handle.symbolic(_Csc(p), default_options(**p.options))
        if req.kind == FACTOR or (req.kind == REFACTOR and req.pattern not in factored):
            h.factor(req.values)
            factored.add(req.pattern)
        elif req.kind == REFACTOR:
            req.status = h.refactor(req.values)
        else:
            req.result = h.solve(req.rhs)
        req.done = time.perf_counter()
        req.event.set()
    for h in handles.values():
        h.free()
    return requests
