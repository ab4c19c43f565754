"""Serving loop on the GPU: a mixed stream of factor, refactor and solve requests over
several patterns, served with concurrent slots, must give every request the same result
as the plain one-at-a-time path (bitwise: each pattern's requests run in order on one
handle, and every kernel is deterministic), also under an HBM budget so small that
handles are evicted and rebuilt."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_05725_amd as bk
    bk.load()
    return bk


def make_stream(serve, seed=11, nreq=48):
    sizes = [600, 900, 1500, 2500, 4000, 6500]
    pats, seqs = [], {}
    for i, n in enumerate(sizes):
        a = synth.gen_mna(n, seed=seed + i)
        key = "p%d" % i
        pats.append(serve.Pattern(key, a.n, a.colptr, a.rowind, a.values))
        seqs[key] = (a, iter(synth.value_sequence(a, nreq, seed=seed + 100 + i)))
    rng = np.random.default_rng(seed)
    reqs, touched = [], set()
    for t in range(nreq):
        key = pats[int(rng.integers(len(pats)))].key
        a, vs = seqs[key]
        if key not in touched:
            reqs.append(serve.Request(serve.FACTOR, key, values=a.values.copy()))
            touched.add(key)
            continue
        u = rng.random()
        if u < 0.1:
            reqs.append(serve.Request(serve.FACTOR, key, values=next(vs)))
        elif u < 0.4:
            reqs.append(serve.Request(serve.REFACTOR, key, values=next(vs)))
        else:
            nrhs = int(rng.integers(1, 5))
            reqs.append(serve.Request(serve.SOLVE, key, rhs=synth.rhs(a.n, nrhs, ident=1000 + t)))
    return pats, reqs


def clone(serve, reqs):
    return [serve.Request(r.kind, r.pattern, values=r.values, rhs=r.rhs) for r in reqs]


@pytest.mark.parametrize("budget_mb", [200_000, 6])
def test_served_results_equal_sequential(bk, budget_mb):
    from paper_1601_05725_amd import serve
    pats, reqs = make_stream(serve)
    say("sequential %d requests" % len(reqs))
    seq = serve.run_sequential(pats, clone(serve, reqs))
    say("served, budget %d MB" % budget_mb)
    srv = serve.Server(pats, slots=4, hbm_budget=budget_mb << 20, estimate=lambda p: 1 << 20)
    mine = [srv.submit(r) for r in clone(serve, reqs)]
    for r in mine:
        assert r.event.wait(120), "request did not finish"
    evictions, restores = srv.evictions, srv.restores
    srv.close()
    say("evictions %d restores %d" % (evictions, restores))
    for a, b in zip(seq, mine):
        assert b.error is None, b.error
        assert a.status == b.status, (a.kind, a.pattern)
        if a.kind == serve.SOLVE:
            np.testing.assert_array_equal(a.result, b.result)
    if budget_mb < 100:
        assert evictions > 0 and restores > 0


def test_admission_budget_binds_with_library_estimate(bk):
    """Default admission (the library's own device-byte estimate): with a budget that
    holds only about two of the patterns, the resident handles' actual device bytes
    never exceed it, handles are evicted, and every result still equals the
    one-at-a-time path."""
    from paper_1601_05725_amd import serve
    pats, reqs = make_stream(serve, seed=23, nreq=40)
    est = {p.key: serve.library_estimate(p) for p in pats}
    say("estimates MB %s" % {k: round(v / 2**20, 1) for k, v in est.items()})
    budget = 2 * max(est.values()) + 1
    seq = serve.run_sequential(pats, clone(serve, reqs))
    srv = serve.Server(pats, slots=4, hbm_budget=budget)
    mine = [srv.submit(r) for r in clone(serve, reqs)]
    for r in mine:
        assert r.event.wait(120), "request did not finish"
    peak, evictions = srv.peak_bytes, srv.evictions
    srv.close()
    say("budget %d peak %d evictions %d" % (budget, peak, evictions))
    assert peak <= budget
    assert evictions > 0
    for a, b in zip(seq, mine):
        assert b.error is None, b.error
        if a.kind == serve.SOLVE:
            np.testing.assert_array_equal(a.result, b.result)
