"""GPU parity: the HIP factorization, refactorization and solve (called through the
C ABI) against the oracle on the same inputs and orderings.

The kernel updates every column in ascending pivot order with separately rounded
multiply-subtract and IEEE division, so against the oracle run in that order
(update_order = ascending) pivots, patterns and values must agree bit for bit.
Against the oracle's default DFS order the pivots agree at every column whose
decision margin is not ambiguous (>= 1e-10) and the patterns are identical.  The solve
subtracts every update in the order of the oracle's block back-substitution, so on
identical factors the solutions are identical bit for bit.  Backward error <= 1e-13
and solve residual <= 1e-12 are checked too.
"""
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

VAL_TOL = 1e-12
BERR_TOL = 1e-13
RES_TOL = 1e-12


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


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def compare_exact(ext, f):
    np.testing.assert_array_equal(ext.piv, f.piv)
    np.testing.assert_array_equal(ext.Lp, f.Lp)
    np.testing.assert_array_equal(ext.Li, f.Li)
    np.testing.assert_array_equal(ext.Up, f.Up)
    np.testing.assert_array_equal(ext.Ui, f.Ui)
    np.testing.assert_array_equal(ext.Lx, f.Lx)
    np.testing.assert_array_equal(ext.Ux, f.Ux)


def col_rel_err(p, x, y):
    worst = 0.0
    for k in range(len(p) - 1):
        a, b = x[p[k]:p[k + 1]], y[p[k]:p[k + 1]]
        if a.size:
            den = max(np.abs(b).max(), 1e-300)
            worst = max(worst, np.abs(a - b).max() / den)
    return worst


def compare_tol(ext, f, n):
    """GPU (ascending update order) vs the oracle's DFS update order: the same
    elimination with the terms of every sum added in another order.  Pivots must
    agree except at columns whose decision margin is ambiguous (< 1e-10), and the L
    and U patterns must then be identical.  Values are not compared entry by entry
    here: two summation orders differ by forward error, which cancellation can make
    large in relative terms for tiny entries even when both factorizations are
    backward stable (seen: 79% in one entry of a 300-row natural-order MNA case with
    backward error 1e-16 for both).  Values are held to bitwise equality against the
    oracle in the kernel's own order, and to the backward-error gate."""
    amb = f.margin < 1e-10
    same = np.array_equal(ext.piv, f.piv)
    if not same:
        diff = np.nonzero(ext.piv != f.piv)[0]
        assert amb[diff[0]], "pivot differs at a non-ambiguous column %d" % diff[0]
        return False
    np.testing.assert_array_equal(ext.Lp, f.Lp)
    np.testing.assert_array_equal(ext.Li, f.Li)
    np.testing.assert_array_equal(ext.Up, f.Up)
    np.testing.assert_array_equal(ext.Ui, f.Ui)
    return True


def as_factors(orc, ext, n):
    return orc.Factors(n, 0, -1, ext.Lp, ext.Li, ext.Lx, ext.Up, ext.Ui, ext.Ux, ext.piv, np.zeros(n), 0.0)


def run_case(bk, orc, a, order=None, tau=1e-3, diag_pref=1, label="", nrhs=2, **opt):
    say("case %s n=%d nnz=%d tau=%g" % (label, a.n, a.nnz, tau))
    o = bk.default_options(pivot_tol=tau, diag_pref=diag_pref, **opt)
    if order is None:
        h = bk.Handle.symbolic(a, o)
        prow, qcol, bp, gp = h.ordering()
        order = orc.Ordering(prow, qcol, bp, gp)
    else:
        h = bk.Handle.symbolic_ordered(a, order.prow, order.qcol, order.blkptr, order.grpptr, o)
    h.factor(a.values)
    ext = h.extract()
    f_asc = orc.factor(a, order, tau=tau, diag_pref=bool(diag_pref), update_order=orc.ORDER_ASCENDING)
    assert f_asc.status == 0
    compare_exact(ext, f_asc)
    f_dfs = orc.factor(a, order, tau=tau, diag_pref=bool(diag_pref), update_order=orc.ORDER_DFS)
    compare_tol(ext, f_dfs, a.n)
    berr = orc.backward_error(a, order, as_factors(orc, ext, a.n))
    assert berr <= BERR_TOL, berr
    b = synth.rhs(a.n, nrhs)
    x = h.solve(b)
    assert orc.residual(a, x, b) <= RES_TOL
    # the solve subtracts every update in the order of the oracle's column sweep:
    # identical factors give an identical solution, bit for bit
    xo = orc.solve(a, order, f_asc, b)
    np.testing.assert_array_equal(x, xo)
    return h, order, ext


# ---------------------------------------------------------------------------

def test_tiny_identity_ordering(bk, orc):
    a = synth.csc_from_dense(np.array([[1.0, 0, 4], [4, 2, 0], [0, 3, 1]]))
    run_case(bk, orc, a, orc.Ordering.natural(3), tau=0.1, label="golden3x3")
    run_case(bk, orc, a, orc.Ordering.natural(3), tau=1.0, diag_pref=0, label="golden3x3-pp")


def test_one_by_one_and_diagonal(bk, orc):
    run_case(bk, orc, synth.csc_from_dense(np.array([[2.5]])), orc.Ordering.natural(1), label="1x1")
    d = synth.csc_from_dense(np.diag([3.0, -2.0, 0.5, 7.0]))
    run_case(bk, orc, d, orc.Ordering.natural(4), label="diag")


@pytest.mark.parametrize("tau,dp", [(1.0, 0), (0.1, 1), (1e-3, 1)])
def test_mna_natural_order_forces_pivoting(bk, orc, tau, dp):
    a = synth.gen_mna(300, seed=21)
    run_case(bk, orc, a, orc.Ordering.natural(a.n), tau=tau, diag_pref=dp, label="mna300-natural")


@pytest.mark.parametrize("n", [64, 300])
def test_dense(bk, orc, n):
    """Dense columns: 300 rows exceed the LDS workspace and use the global fallback."""
    A = synth.random_dense(n, 31 + n)
    a = synth.csc_from_dense(A)
    run_case(bk, orc, a, orc.Ordering.natural(n), tau=1.0, diag_pref=0, label="dense%d" % n)


@pytest.mark.parametrize("seed", [41, 42])
def test_blocks_and_groups_user_ordering(bk, orc, seed):
    n = 240
    a0 = synth.random_sparse(n, 0.03, seed)
    s = synth.Stream(synth.substream_key(seed, 77))
    blkptr = np.unique(np.concatenate([[0, n], s.integers(1, n, 12)])).astype(np.int32)
    grpptr = np.unique(np.concatenate([blkptr, s.integers(1, n, 30)])).astype(np.int32)
    blk = np.repeat(np.arange(len(blkptr) - 1), np.diff(blkptr))
    D = a0.to_dense()
    D = np.where(blk[:, None] > blk[None, :], 0.0, D)
    pr, pc = s.permutation(n), s.permutation(n)
    A = np.zeros((n, n))
    A[np.ix_(pr, pc)] = D
    a = synth.csc_from_dense(A)
    order = orc.Ordering(pr.astype(np.int32), pc.astype(np.int32), blkptr, grpptr)
    run_case(bk, orc, a, order, tau=0.1, label="groups-%d" % seed, nrhs=3)


def test_c0_full_pipeline(bk, orc):
    a = synth.gen_mna(2000)
    h, order, ext = run_case(bk, orc, a, label="C0", nrhs=1)
    inf = h.info()
    say("C0 info %s" % {k: inf[k] for k in ("nblocks", "lnz", "unz", "max_depth", "factor_kernel_ms", "offdiag_pivots")})


def nd_separator_groups(h):
    """Groups that are ND separators (some group names them as parent)."""
    gpar = h.group_tree()
    return set(int(g) for g in gpar[gpar >= 0])


def test_nd_block(bk, orc):
    a = synth.gen_mna(12000, seed=6)
    h, order, ext = run_case(bk, orc, a, label="mna12k-nd", nd_min_block=3000, nd_leaves=8)
    inf = h.info()
    assert inf["nd_blocks"] >= 1
    # both separator paths ran: the dense kernel counts the separators it completed
    seps = nd_separator_groups(h)
    say("separators %d: dense %d sparse %d" % (len(seps), inf["dense_seps"], inf["sparse_seps"]))
    assert inf["dense_seps"] > 0 and inf["sparse_seps"] > 0
    assert inf["dense_seps"] + inf["sparse_seps"] == len(seps)


@pytest.mark.parametrize("leaves", [16, 32, 64])
def test_nd_block_leaf_counts(bk, orc, leaves):
    # deeper ND trees (more leaves than the configurations' 16): smaller leaves, one more
    # level of small sparse separators per doubling, each separator a work item of its own
    a = synth.gen_mna(30000, seed=8)
    h, order, ext = run_case(bk, orc, a, label="mna30k-nd%d" % leaves, nd_min_block=3000, nd_leaves=leaves)
    inf = h.info()
    assert inf["nd_blocks"] >= 1
    assert inf["nlevels"] == leaves.bit_length()   # log2(leaves) separator levels + the first level
    assert inf["sparse_seps"] > 0


def test_first_step_tables_agree(bk, orc):
    # the separator first step on the 2,048-slot table (two waves a CU, chosen when the
    # symbolic workspace bound fits 3/4 of it) and on the 4,096-slot table (sched_flags
    # bit 3): the same factors, bit for bit, and the oracle's
    a = synth.gen_mna(30000, seed=8)
    h0, order, ext0 = run_case(bk, orc, a, label="mna30k-nd32-step1-2048", nd_min_block=3000, nd_leaves=32)
    h1, _, ext1 = run_case(bk, orc, a, order=order, label="mna30k-nd32-step1-4096", nd_min_block=3000,
                           nd_leaves=32, sched_flags=8)
    assert h0.info()["sym_ws_rows"] <= 1536
    for key in ("piv", "Lp", "Li", "Lx", "Up", "Ui", "Ux"):
        np.testing.assert_array_equal(getattr(ext0, key), getattr(ext1, key), err_msg=key)


def test_solve_abort_path_ends_and_reports(bk, orc):
    # sched_flags bit 4 starts the one-launch solve with its abort bit set: every wait
    # that has to wait (per-entry waits on coupled solution entries, ND task flags) gives
    # up at its first failed poll, the launch still ends, and the solve reports the stall;
    # a handle without the flag then solves bit for bit as the oracle does
    inp = synth.gen_batched_btf(nblocks=300, big=4000, seed=7)
    a = inp.a
    b = synth.rhs(a.n, 1)
    h_bad = bk.Handle.symbolic(a, bk.default_options(nd_min_block=2000, nd_leaves=4, sched_flags=16))
    h_bad.factor(a.values)
    say("abort-path solve, n=%d" % a.n)
    with pytest.raises(bk.BaskerError) as ei:
        h_bad.solve(b)
    assert "did not end" in str(ei.value)
    h_bad.free()
    h, order, ext = run_case(bk, orc, a, label="after-abort", nd_min_block=2000, nd_leaves=4, nrhs=1)
    assert h.info()["nd_blocks"] >= 1


def test_large_block_without_nd(bk, orc):
    # one 11k-row block: its solve work vectors exceed LDS and live in global memory
    a = synth.gen_mna(12000, seed=6)
    h, order, ext = run_case(bk, orc, a, label="mna12k-no-nd", nd_min_block=10**9, nrhs=3)
    assert np.diff(order.blkptr).max() > 10000


def test_batched_btf_small(bk, orc):
    inp = synth.gen_batched_btf(nblocks=400, big=4000, seed=5)
    h, order, ext = run_case(bk, orc, inp.a, label="btf400", nd_min_block=2000, nd_leaves=4)
    assert h.info()["nblocks"] >= 400


def test_refactor_bitwise_and_sequence(bk, orc):
    a = synth.gen_mna(1500, seed=9)
    h = bk.Handle.symbolic(a)
    prow, qcol, bp, gp = h.ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    h.factor(a.values)
    e0 = h.extract()
    say("refactor same values")
    assert h.refactor(a.values) == bk.OK
    compare_exact(h.extract(), orc.factor(a, order, update_order=orc.ORDER_ASCENDING))
    compare_exact(h.extract(), e0)
    for t, vals in enumerate(synth.value_sequence(a, 4)):
        say("refactor step %d" % t)
        at = a.with_values(vals)
        st = h.refactor(vals)
        ref = orc.refactor(at, order, e0.piv, update_order=orc.ORDER_ASCENDING)
        if ref.status == 0:
            assert st == bk.OK
            compare_exact(h.extract(), ref)
        else:
            assert st == bk.REFACTOR_FELL_BACK
            compare_exact(h.extract(), orc.factor(at, order, update_order=orc.ORDER_ASCENDING))
            e0 = h.extract()
        b = synth.rhs(a.n, 1, ident=t)
        assert orc.residual(at, h.solve(b), b) <= RES_TOL


def test_refactor_graph_replays_match_eager(bk, orc):
    """Refactorizations replayed from the captured HIP graph against eager launches on a
    second handle: every replay bitwise equal, with eager work and host synchronisation
    between replays, device- and host-resident values, and a forced fallback (which
    drops the graph) in the middle of the sequence."""
    import torch
    a = synth.gen_mna(12000, seed=6)
    og = bk.default_options(nd_min_block=3000, nd_leaves=8)
    oe = bk.default_options(nd_min_block=3000, nd_leaves=8)
    oe.refactor_graph = 0
    hg = bk.Handle.symbolic(a, og)
    he = bk.Handle.symbolic(a, oe)
    hg.factor(a.values)
    he.factor(a.values)
    seq = list(synth.value_sequence(a, 6))
    replays = 0
    for t, vals in enumerate(seq):
        if t == 3:
            # a tiny pivot in the first column of the ND block forces the threshold
            # check to fail on both handles
            vals = vals.copy()
            prow, qcol, bp, gp = hg.ordering()
            k = int(bp[np.argmax(np.diff(bp))])
            acol, arow = int(qcol[k]), int(prow[hg.extract().piv[k]])
            q = a.colptr[acol] + int(np.nonzero(a.rowind[a.colptr[acol]:a.colptr[acol + 1]] == arow)[0][0])
            vals[q] *= 1e-14
        say("graph/eager refactor step %d" % t)
        v = torch.from_numpy(vals).cuda() if t % 2 == 0 else vals
        sg = hg.refactor(v)
        se = he.refactor(vals)
        assert sg == se
        if t == 3:
            assert sg == bk.REFACTOR_FELL_BACK
        else:
            replays += int(sg == bk.OK)
        compare_exact(hg.extract(), he.extract())
        b = synth.rhs(a.n, 1, ident=100 + t)
        np.testing.assert_array_equal(hg.solve(b), he.solve(b))
        torch.cuda.synchronize()
    assert hg.info()["refactor_calls"] == he.info()["refactor_calls"] == 6
    assert replays >= 3


def test_refactor_fallback_forced(bk, orc):
    a = synth.gen_mna(400, seed=10)
    order = orc.Ordering.natural(a.n)
    h = bk.Handle.symbolic_ordered(a, order.prow, order.qcol, order.blkptr, order.grpptr)
    h.factor(a.values)
    e0 = h.extract()
    vals = a.values.copy()
    p = e0.piv[0]
    sel = a.rowind[a.colptr[0]:a.colptr[1]] == p
    vals[a.colptr[0]:a.colptr[1]][sel] *= 1e-12
    say("refactor forced failure")
    assert h.refactor(vals) == bk.REFACTOR_FELL_BACK
    at = a.with_values(vals)
    compare_exact(h.extract(), orc.factor(at, order, update_order=orc.ORDER_ASCENDING))
    assert h.info()["refactor_fallbacks"] == 1


def test_singular_reported(bk, orc):
    n = 6
    s = synth.Stream(61)
    L0 = np.tril(s.integers(-1, 2, n * n).reshape(n, n), -1) + np.eye(n)
    U0 = np.triu(s.integers(-1, 2, n * n).reshape(n, n), 1) + np.diag(np.where(s.uniform(n) < 0.5, 1.0, -1.0))
    A = L0 @ U0
    A[:, 4] = A[:, 2]
    a = synth.csc_from_dense(A)
    o = bk.default_options(pivot_tol=1e-300)
    h = bk.Handle.symbolic_ordered(a, np.arange(n), np.arange(n), [0, n], [0, n], o)
    with pytest.raises(bk.BaskerError) as e:
        h.factor(a.values)
    assert e.value.status == bk.ERR_NUM_SINGULAR
    assert h.info()["fail_col"] == 4


def test_deterministic_repeat(bk, orc):
    inp = synth.gen_batched_btf(nblocks=300, big=0, seed=7)
    h = bk.Handle.symbolic(inp.a)
    h.factor(inp.a.values)
    e1 = h.extract()
    h.factor(inp.a.values)
    e2 = h.extract()
    compare_exact(e1, orc.Factors(inp.a.n, 0, -1, e2.Lp, e2.Li, e2.Lx, e2.Up, e2.Ui, e2.Ux, e2.piv, None, 0.0))


def test_device_pointers(bk, orc):
    import torch
    a = synth.gen_mna(500, seed=11)
    h = bk.Handle.symbolic(a)
    vals = torch.from_numpy(a.values.copy()).cuda()
    h.factor(vals)
    b = synth.rhs(a.n, 2)
    Bt = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()   # (nrhs, n) rows = columns of B
    h.solve(Bt)
    torch.cuda.synchronize()
    x = Bt.cpu().numpy().T
    assert orc.residual(a, x, b) <= RES_TOL



# ---------------------------------------------------------------------------
# exact ties, full-size parity, determinism, refactor on ND blocks
# ---------------------------------------------------------------------------

def integer_matrix(n, density, seed):
    """{-1, 0, 1} entries with a +-1 diagonal: magnitudes tie exactly, so the pivot
    choices exercise the smallest-index tie-break and the threshold equality."""
    s = synth.Stream(synth.substream_key(seed, 5))
    D = s.integers(-1, 2, n * n).astype(float).reshape(n, n)
    D[s.uniform(n * n).reshape(n, n) >= density] = 0.0
    D[np.arange(n), np.arange(n)] = np.where(s.uniform(n) < 0.5, 1.0, -1.0)
    return D


@pytest.mark.parametrize("tau,dp", [(1.0, 0), (1.0, 1), (0.5, 1)])
@pytest.mark.parametrize("n,density,seed", [(12, 1.0, 20), (12, 1.0, 24), (160, 0.03, 22), (400, 0.012, 23)])
def test_exact_ties_integer(bk, orc, tau, dp, n, density, seed):
    a = synth.csc_from_dense(integer_matrix(n, density, seed))
    order = orc.Ordering.natural(n)
    f = orc.factor(a, order, tau=tau, diag_pref=bool(dp), update_order=orc.ORDER_ASCENDING)
    if f.status != 0:
        pytest.skip("singular draw")
    assert np.count_nonzero(f.margin == 0.0) > 0     # the case really holds exact ties
    run_case(bk, orc, a, order, tau=tau, diag_pref=dp, label="ties-%d-%d" % (n, seed), nrhs=1)


@pytest.mark.parametrize("waves,bin_edge", [(0, 0), (7, 128)])
def test_full_c2_bitwise(bk, orc, waves, bin_edge):
    """The batched-BTF workload at full size (50,000 blocks + the 100k ND block, 16
    leaves, n = 346,411), as the benchmark factors it (the default schedule, and the
    autotuner's usual pick: 7 waves, bin edge 128): pivots, patterns and values bit for
    bit against the oracle, dense separators included; solve residual."""
    inp = synth.gen_batched_btf()
    a = inp.a
    say("C2 full n=%d nnz=%d waves %d bin edge %d" % (a.n, a.nnz, waves, bin_edge))
    h = bk.Handle.symbolic(a, bk.default_options(nd_leaves=16, coop_waves=waves, bin_edge=bin_edge))
    prow, qcol, bp, gp = h.ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    h.factor(a.values)
    ext = h.extract()
    f = orc.factor(a, order, update_order=orc.ORDER_ASCENDING)
    assert f.status == 0
    compare_exact(ext, f)
    inf = h.info()
    say("C2 dense separators %d sparse %d offdiag pivots %d" % (inf["dense_seps"], inf["sparse_seps"],
                                                                inf["offdiag_pivots"]))
    assert inf["dense_seps"] > 0
    b = synth.rhs(a.n, 1)
    x = h.solve(b)
    assert orc.residual(a, x, b) <= RES_TOL
    np.testing.assert_array_equal(x, orc.solve(a, order, f, b))


@pytest.mark.parametrize("max_grid,flags", [(1, 0), (37, 1), (0, 1)])
def test_deterministic_under_schedule(bk, orc, max_grid, flags):
    """Schedule determinism: other grid sizes and the reverse order of work items change
    which workgroup factors what and when; the factors must not change by a bit."""
    inp = synth.gen_batched_btf(nblocks=300, big=4000, seed=7)
    a = inp.a
    h0 = bk.Handle.symbolic(a, bk.default_options(nd_min_block=2000, nd_leaves=4))
    h0.factor(a.values)
    e0 = h0.extract()
    h1 = bk.Handle.symbolic(a, bk.default_options(nd_min_block=2000, nd_leaves=4, max_grid=max_grid,
                                                  sched_flags=flags))
    h1.factor(a.values)
    e1 = h1.extract()
    for x, y in ((e0.piv, e1.piv), (e0.Lp, e1.Lp), (e0.Li, e1.Li), (e0.Lx, e1.Lx), (e0.Up, e1.Up),
                 (e0.Ui, e1.Ui), (e0.Ux, e1.Ux)):
        np.testing.assert_array_equal(x, y)
    b = synth.rhs(a.n, 2)
    np.testing.assert_array_equal(h0.solve(b), h1.solve(b))


def test_refactor_nd_block_vs_oracle(bk, orc):
    """Refactorization on an ND block with dense and sparse separators (the known-pattern
    separator first step, known-pattern columns at separator levels and the dense
    kernel in refactor mode) against the oracle's refactorization, step by step; steps
    whose threshold check fails fall back and match the oracle's full factorization."""
    a = synth.gen_mna(12000, seed=6)
    h = bk.Handle.symbolic(a, bk.default_options(nd_min_block=3000, nd_leaves=8))
    prow, qcol, bp, gp = h.ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    h.factor(a.values)
    assert h.info()["dense_seps"] > 0
    base = h.extract()
    assert h.refactor(a.values) == bk.OK
    compare_exact(h.extract(), orc.refactor(a, order, base.piv, update_order=orc.ORDER_ASCENDING))
    passed = fell = 0
    for t, vals in enumerate(synth.value_sequence(a, 6, sigma=0.002)):
        say("nd refactor step %d" % t)
        at = a.with_values(vals)
        st = h.refactor(vals)
        ref = orc.refactor(at, order, base.piv, update_order=orc.ORDER_ASCENDING)
        if ref.status == 0:
            assert st == bk.OK
            compare_exact(h.extract(), ref)
            passed += 1
        else:
            assert st == bk.REFACTOR_FELL_BACK
            compare_exact(h.extract(), orc.factor(at, order, update_order=orc.ORDER_ASCENDING))
            base = h.extract()
            fell += 1
    say("nd refactor passed %d fell back %d" % (passed, fell))
    assert passed >= 1


def test_hbm_budget_and_estimate(bk, orc):
    """The handle's device memory after a factorization and an 8-RHS solve matches the
    analysis estimate; a budget below it refuses the analysis with BASKER_ERR_OOM, one
    above it holds."""
    a = synth.gen_mna(5000, seed=13)
    est = bk.Handle.symbolic(a, bk.default_options(device=-1)).info()["device_bytes_plan"]
    h = bk.Handle.symbolic(a, bk.default_options(hbm_budget=est + (1 << 20)))
    h.factor(a.values)
    b = synth.rhs(a.n, 8)
    x = h.solve(b)
    inf = h.info()
    say("estimate %d held %d regrows %d" % (est, inf["device_bytes"], inf["pool_regrows"]))
    assert inf["pool_regrows"] == 0
    assert 0.9 * est <= inf["device_bytes"] <= est
    assert orc.residual(a, x, b) <= RES_TOL
    h.free()
    with pytest.raises(bk.BaskerError) as e:
        bk.Handle.symbolic(a, bk.default_options(hbm_budget=est // 2))
    assert e.value.status == bk.ERR_OOM


# ---------------------------------------------------------------------------
# first-level cooperative schedule: speculation, redo, learned dependencies
# ---------------------------------------------------------------------------

def test_speculation_redo_and_learning(bk, orc):
    """Natural ordering of an MNA circuit (zero diagonals of the voltage-source rows):
    the dependencies predicted without row exchanges are wrong, so the speculative
    first level must detect it, redo the item with elimination-tree dependencies and
    still give the oracle's factors bit for bit; the observed dependencies are then
    learned and the next factorization of the same values needs no redo."""
    a = synth.gen_mna(3000, seed=31)
    order = orc.Ordering.natural(a.n)
    h = bk.Handle.symbolic_ordered(a, order.prow, order.qcol, order.blkptr, order.grpptr)
    assert h.info()["coop_items"] >= 1
    f = orc.factor(a, order, update_order=orc.ORDER_ASCENDING)
    assert f.status == 0 and np.count_nonzero(f.piv != np.arange(a.n)) > 0
    h.factor(a.values)
    inf = h.info()
    say("first factor: redo %d learn %d" % (inf["redo_items"], inf["learn_events"]))
    assert inf["redo_items"] >= 1 and inf["learn_events"] == 1
    compare_exact(h.extract(), f)
    h.factor(a.values)
    inf = h.info()
    assert inf["redo_items"] == 0 and inf["learn_events"] == 1
    compare_exact(h.extract(), f)
    b = synth.rhs(a.n, 1)
    assert orc.residual(a, h.solve(b), b) <= RES_TOL


@pytest.mark.parametrize("waves,flags,item_cols", [(4, 0, 64), (7, 0, 256), (8, 0, 1024), (6, 2, 256), (6, 3, 128)])
def test_first_level_schedules_agree(bk, orc, waves, flags, item_cols):
    """Wavefronts per workgroup, item size, reverse item order and the safe-only
    schedule (flag 2) change who factors which column when; the factors stay the
    oracle's bit for bit."""
    inp = synth.gen_batched_btf(nblocks=600, big=6000, seed=19)
    a = inp.a
    o = bk.default_options(nd_min_block=3000, nd_leaves=8, coop_waves=waves, sched_flags=flags, item_cols=item_cols)
    h = bk.Handle.symbolic(a, o)
    prow, qcol, bp, gp = h.ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    h.factor(a.values)
    inf = h.info()
    say("waves %d flags %d items %d redo %d" % (waves, flags, inf["coop_items"], inf["redo_items"]))
    assert inf["coop_items"] > 1 and inf["coop_waves"] == waves
    compare_exact(h.extract(), orc.factor(a, order, update_order=orc.ORDER_ASCENDING))


@pytest.mark.gpu
@pytest.mark.parametrize("bin_edge", [-1, 4, 64, 4096])
def test_first_level_bins_agree(bk, orc, bin_edge):
    """Size bins of the first level (thread per 1 x 1 block, wavefront per segment of at
    most bin_edge columns, shared workgroups above it) change who factors which column;
    factorization and refactorization stay the oracle's bit for bit."""
    inp = synth.gen_batched_btf(nblocks=600, big=6000, seed=23)
    a = inp.a
    o = bk.default_options(nd_min_block=3000, nd_leaves=8, bin_edge=bin_edge)
    h = bk.Handle.symbolic(a, o)
    prow, qcol, bp, gp = h.ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    say("bin_edge %d: items %d" % (bin_edge, h.info()["coop_items"]))
    h.factor(a.values)
    e0 = h.extract()
    compare_exact(e0, orc.factor(a, order, update_order=orc.ORDER_ASCENDING))
    vals = next(iter(synth.value_sequence(a, 1, sigma=0.002)))
    st = h.refactor(vals)
    ref = orc.refactor(a.with_values(vals), order, e0.piv, update_order=orc.ORDER_ASCENDING)
    if ref.status == 0:
        assert st == bk.OK
        compare_exact(h.extract(), ref)


@pytest.mark.gpu
def test_one_by_one_block_singular(bk, orc):
    """A 1 x 1 diagonal block holding an explicit zero is numerically singular: the
    thread-per-block bin reports it at that column, like the oracle."""
    # diagonal with an explicit zero at (2, 2), and one coupling entry (0, 5)
    r = np.array([0, 1, 2, 3, 4, 5, 0])
    c = np.array([0, 1, 2, 3, 4, 5, 5])
    v = np.array([2.0, 3.0, 0.0, 4.0, 5.0, 1.5, 1.0])
    a = synth.csc_from_coo(6, r, c, v)
    assert a.nnz == 7
    h = bk.Handle.symbolic(a, bk.default_options(matching=0))
    prow, qcol, bp, gp = h.ordering()
    f = orc.factor(a, orc.Ordering(prow, qcol, bp, gp))
    assert f.status != 0
    with pytest.raises(bk.BaskerError) as e:
        h.factor(a.values)
    assert e.value.status == bk.ERR_NUM_SINGULAR
    assert h.info()["fail_col"] == f.fail_col


@pytest.mark.gpu
def test_autotune_keeps_the_factors(bk, orc):
    """With autotune on, the first factorizations time the schedule candidates (bin
    edges, wavefronts per workgroup) and the fastest is kept; every factorization on the
    way, and the ones after, equal the oracle's bit for bit."""
    inp = synth.gen_batched_btf(nblocks=500, big=5000, seed=29)
    a = inp.a
    h = bk.Handle.symbolic(a, bk.default_options(nd_min_block=2500, nd_leaves=8, autotune=1))
    prow, qcol, bp, gp = h.ordering()
    ref = orc.factor(a, orc.Ordering(prow, qcol, bp, gp), update_order=orc.ORDER_ASCENDING)
    trials = []
    for call in range(10):
        h.factor(a.values)
        inf = h.info()
        trials.append(inf["autotune_trials"])
        compare_exact(h.extract(), ref)
    say("trials %s -> bin edge %d, waves %d" % (trials, inf["sched_bin_edge"], inf["coop_waves"]))
    assert trials[0] == 0 and trials[-1] == max(trials) >= 6
    assert inf["coop_waves"] in (4, 6, 7, 8) and inf["sched_bin_edge"] in (0, 8, 32, 128)


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["nd12k", "btf400"])
def test_one_launch_solve_equals_level_launches(bk, orc, case):
    """The solve runs every task in one launch (workgroups wait on their predecessors'
    done flags) unless sched_flags bit 2 asks for one launch per level; both give the
    oracle's solution bit for bit, also over repeated solves on one handle (the flags
    and the task counter are cleared before every launch)."""
    if case == "nd12k":
        a = synth.gen_mna(12000, seed=6)
        opt = dict(nd_min_block=3000, nd_leaves=8)
    else:
        a = synth.gen_batched_btf(nblocks=400, big=4000, seed=5).a
        opt = dict(nd_min_block=2000, nd_leaves=4)
    hs = []
    for flags in (0, 4):
        say("case %s sched_flags %d" % (case, flags))
        h = bk.Handle.symbolic(a, bk.default_options(sched_flags=flags, **opt))
        h.factor(a.values)
        hs.append(h)
    prow, qcol, bp, gp = hs[0].ordering()
    order = orc.Ordering(prow, qcol, bp, gp)
    f_asc = orc.factor(a, order, update_order=orc.ORDER_ASCENDING)
    for rep, nrhs in enumerate((1, 3, 8, 2)):
        b = synth.rhs(a.n, nrhs, ident=500 + rep)
        xo = orc.solve(a, order, f_asc, b)
        for h in hs:
            np.testing.assert_array_equal(h.solve(b), xo)
