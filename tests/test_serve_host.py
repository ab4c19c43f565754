"""Scheduling logic of the serving loop, on the CPU: the library handle is replaced by a
stand-in whose solve result depends on the whole factor/refactor history of its
pattern, so any reordering of a pattern's requests, or an eviction that does not
rebuild the same state, changes a result.  Random delays interleave the slots."""
import threading
import time

import numpy as np
import pytest


class FakeHandle:
    live = 0
    lock = threading.Lock()

    def __init__(self, n):
        self.n = n
        self.base = None
        self.cur = None
        self.busy = False
        with FakeHandle.lock:
            FakeHandle.live += 1

    @staticmethod
    def symbolic(a, options=None):
        return FakeHandle(a.n)

    def _enter(self):
        assert not self.busy, "a handle was used by two requests at once"
        self.busy = True
        time.sleep(np.random.default_rng().uniform(0, 2e-3))

    def factor(self, v):
        self._enter()
        self.base = self.cur = float(np.asarray(v).sum())
        self.busy = False

    def refactor(self, v):
        self._enter()
        self.cur = float(np.asarray(v).sum())
        self.busy = False
        return 0

    def solve(self, b):
        self._enter()
        assert self.base is not None
        self.busy = False
        return np.asarray(b) * (1.0 + self.base) + self.cur

    def info(self):
        return {"device_bytes": 1000 * self.n}

    def free(self):
        with FakeHandle.lock:
            FakeHandle.live -= 1


@pytest.fixture
def serve(monkeypatch):
    from paper_1601_05725_amd import serve as s
    monkeypatch.setattr(s, "Handle", FakeHandle)
    monkeypatch.setattr(s, "default_options", lambda **kw: None)
    return s


def stream(s, npat=5, nreq=120, seed=3):
    rng = np.random.default_rng(seed)
    pats = [s.Pattern("p%d" % i, 100 + 50 * i, np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0))
            for i in range(npat)]
    reqs, touched = [], set()
    for t in range(nreq):
        p = pats[int(rng.integers(npat))]
        u = rng.random()
        if p.key not in touched or u < 0.15:
            touched.add(p.key)
            reqs.append(s.Request(s.FACTOR, p.key, values=rng.uniform(size=4)))
        elif u < 0.45:
            reqs.append(s.Request(s.REFACTOR, p.key, values=rng.uniform(size=4)))
        else:
            reqs.append(s.Request(s.SOLVE, p.key, rhs=rng.uniform(size=3)))
    return pats, reqs


def clone(s, reqs):
    return [s.Request(r.kind, r.pattern, values=r.values, rhs=r.rhs) for r in reqs]


@pytest.mark.parametrize("budget", [10 ** 9, 250_000])
def test_served_equals_sequential(serve, budget):
    pats, reqs = stream(serve)
    seq = serve.run_sequential(pats, clone(serve, reqs))
    srv = serve.Server(pats, slots=4, hbm_budget=budget, estimate=lambda p: 1000 * p.n)
    mine = [srv.submit(r) for r in clone(serve, reqs)]
    for r in mine:
        assert r.event.wait(30)
    ev, rs = srv.evictions, srv.restores
    srv.close()
    assert FakeHandle.live == 0
    for a, b in zip(seq, mine):
        assert b.error is None, b.error
        if a.kind == serve.SOLVE:
            np.testing.assert_array_equal(a.result, b.result)
    if budget < 10 ** 6:
        assert ev > 0 and rs > 0
    else:
        assert ev == 0


def test_budget_bounds_resident(serve):
    pats, reqs = stream(serve, npat=6, nreq=80, seed=5)
    budget = 2 * 1000 * max(p.n for p in pats)
    srv = serve.Server(pats, slots=3, hbm_budget=budget, estimate=lambda p: 1000 * p.n)
    peak = [0]

    def watch():
        while not stop.is_set():
            with srv.cv:
                peak[0] = max(peak[0], srv.resident_bytes())
            time.sleep(1e-4)

    stop = threading.Event()
    th = threading.Thread(target=watch)
    th.start()
    mine = [srv.submit(r) for r in reqs]
    for r in mine:
        assert r.event.wait(30)
    stop.set()
    th.join()
    srv.close()
    assert peak[0] <= budget


def test_unknown_pattern_rejected(serve):
    pats, _ = stream(serve, npat=1, nreq=1)
    srv = serve.Server(pats, slots=1)
    with pytest.raises(KeyError):
        srv.submit(serve.Request(serve.SOLVE, "nope", rhs=np.zeros(1)))
    srv.close()
