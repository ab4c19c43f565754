"""Pins of the oracle against things other than itself (CPU only).

* P1 textbook: tau = 1, no diagonal preference, natural order -> identical pivots
  to LAPACK getrf partial pivoting (scipy.linalg.lu), factors within 1e-13.
* P2 brute force: an independent dense right-looking threshold LU written below,
  with the same pivot rule and candidate groups; integer {-1,0,1} matrices make
  exact ties, pinning the smallest-index tie-break.
* P3 reach: the pattern of every column equals a boolean fixed-point closure.
* P4 invariants: unit lower L, |l_ij| <= 1/tau, backward error, ND fill only on
  ancestor paths.
* P5 special cases: diagonal, upper triangular, permutation, tridiagonal (Thomas),
  block diagonal (each block alone == batched).
* P6 refactor: bitwise equal to the factorization it replays.
* P8 solve: residual and agreement with scipy's splu.
* A hand-derived example in tests/golden/diag_pref_3x3.txt.
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent dense reference (right-looking elimination, original row space)
# ---------------------------------------------------------------------------

def dense_threshold_lu(R, blkptr, grpptr, tau, diag_pref, stats=None):
    """Dense right-looking LU of the block-diagonal part of R with the pivot rule of
    the sparse path.  Returns (status, fail_col, piv, L, U) with L, U in pivot order.

    With a dict ``stats`` it also records, by their definitions and from this
    elimination alone:
      * ``margin[k]``: the decision margin of column k's pivot choice, clipped at 1.
        With C the non-pivotal rows of k's group and m = max |x_C|: if the diagonal
        test applies (diag_pref, k in C) it passes iff |x_k| >= tau * m_o, m_o the
        largest magnitude over C minus row k, so its margin is | |x_k| - tau m_o | / m;
        when the pivot is not the preferred diagonal, the argmax also matters, with
        margin (m - m2) / m, m2 the runner-up.  No competitor gives margin 1.
      * ``flops``: multiply-subtract pairs (2 flops each) applied to structurally
        nonzero entries plus one division per entry of L, counted as the
        right-looking elimination performs them.
    Structure is tracked symbolically (an entry is structural if it is in the input
    or receives an update), so an entry whose value cancels to zero stays in L or U,
    as the sparse factorization keeps it.
    """
    n = R.shape[0]
    A = np.zeros_like(R)
    for b in range(len(blkptr) - 1):
        s, e = blkptr[b], blkptr[b + 1]
        A[s:e, s:e] = R[s:e, s:e]
    S = A != 0.0
    grp = np.repeat(np.arange(len(grpptr) - 1), np.diff(grpptr))
    blk = np.repeat(np.arange(len(blkptr) - 1), np.diff(blkptr))
    pivoted = np.zeros(n, bool)
    piv = np.zeros(n, np.int64)
    Lrow = np.zeros((n, n))
    Urows = np.zeros((n, n))
    margin = np.ones(n)
    flops = 0
    for k in range(n):
        cand = np.nonzero((~pivoted) & (grp == grp[k]))[0]
        x = A[:, k]
        m = np.abs(x[cand]).max() if cand.size else 0.0
        if not m > 0:
            return -3, k, None, None, None
        dtest = diag_pref and not pivoted[k]
        amax = int(cand[np.nonzero(np.abs(x[cand]) == m)[0][0]])
        if dtest and abs(x[k]) >= tau * m:
            p = k
        else:
            p = amax
        mu = 1.0
        if dtest:
            others = cand[cand != k]
            if others.size:
                mu = min(mu, abs(abs(x[k]) - tau * np.abs(x[others]).max()) / m)
        if p != k or not dtest:
            others = cand[cand != amax]
            if others.size:
                mu = min(mu, (m - np.abs(x[others]).max()) / m)
        margin[k] = mu
        piv[k] = p
        pivoted[p] = True
        Urows[k, k:] = A[p, k:]
        rows = np.nonzero((~pivoted) & (blk == blk[k]))[0]
        ucnt = int(np.count_nonzero(S[p, k + 1:] & (blk[k + 1:] == blk[k])))
        for i in rows:
            if S[i, k]:
                l = A[i, k] / A[p, k]
                Lrow[i, k] = l
                flops += 1 + 2 * ucnt
                A[i, k + 1:] = A[i, k + 1:] - l * A[p, k + 1:]
                S[i, k + 1:] |= S[p, k + 1:]
                A[i, k] = 0.0
    if stats is not None:
        stats["margin"] = margin
        stats["flops"] = flops
    pos = np.empty(n, np.int64)
    pos[piv] = np.arange(n)
    L = np.eye(n)
    for i in range(n):
        for k in range(n):
            if Lrow[i, k] != 0.0:
                L[pos[i], k] = Lrow[i, k]
    return 0, -1, piv, L, Urows


def permuted_dense(a, order):
    return a.to_dense()[np.ix_(order.prow, order.qcol)]


def rel_col_err(Fa, Fb_dense, n):
    return np.abs(Fa - Fb_dense).max() / max(1.0, np.abs(Fb_dense).max())


# ---------------------------------------------------------------------------
# P1: LAPACK partial pivoting
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (5, 3), (16, 4), (40, 5), (64, 6)])
def test_p1_dense_matches_lapack(oracle_lib, n, seed):
    A = synth.random_dense(n, seed)
    a = synth.csc_from_dense(A)
    for upd in (oracle_lib.ORDER_DFS, oracle_lib.ORDER_ASCENDING):
        f = oracle_lib.factor(a, tau=1.0, diag_pref=False, update_order=upd)
        assert f.status == 0
        p, l, u = scipy.linalg.lu(A, p_indices=True)
        np.testing.assert_array_equal(f.piv, np.argsort(p))
        assert np.abs(f.L_dense() - l).max() <= 1e-13 * max(1, np.abs(l).max())
        assert np.abs(f.U_dense() - u).max() <= 1e-13 * max(1, np.abs(u).max())


@pytest.mark.parametrize("n,density,seed", [(30, 0.1, 7), (64, 0.05, 8), (64, 0.2, 9)])
def test_p1_sparse_matches_lapack(oracle_lib, n, density, seed):
    a = synth.random_sparse(n, density, seed)
    A = a.to_dense()
    f = oracle_lib.factor(a, tau=1.0, diag_pref=False)
    assert f.status == 0
    p, l, u = scipy.linalg.lu(A, p_indices=True)
    np.testing.assert_array_equal(f.piv, np.argsort(p))
    assert np.abs(f.L_dense() - l).max() <= 1e-13 * max(1, np.abs(l).max())
    assert np.abs(f.U_dense() - u).max() <= 1e-13 * max(1, np.abs(u).max())


# ---------------------------------------------------------------------------
# P2: dense threshold LU with candidate groups and diagonal preference
# ---------------------------------------------------------------------------

def _groups_case(n, seed):
    """Blocks and nested groups over [0, n) (block-upper-triangular A with zero
    lower off-diagonal blocks, random groups inside each block)."""
    s = synth.Stream(synth.substream_key(seed, 77))
    cuts = np.unique(np.concatenate([[0, n], s.integers(1, n, max(1, n // 12))]))
    blkptr = cuts.astype(np.int32)
    gcuts = np.unique(np.concatenate([blkptr, s.integers(1, n, max(1, n // 6))]))
    return blkptr, gcuts.astype(np.int32)


def _block_upper(a_dense, blkptr):
    n = a_dense.shape[0]
    blk = np.repeat(np.arange(len(blkptr) - 1), np.diff(blkptr))
    return np.where(blk[:, None] > blk[None, :], 0.0, a_dense)


@pytest.mark.parametrize("tau", [1.0, 0.1, 0.001])
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_p2_threshold_groups_random(oracle_lib, tau, seed):
    n = 48
    a0 = synth.random_sparse(n, 0.12, seed)
    blkptr, grpptr = _groups_case(n, seed)
    D = _block_upper(a0.to_dense(), blkptr)
    a = synth.csc_from_dense(D)
    order = oracle_lib.Ordering(np.arange(n), np.arange(n), blkptr, grpptr)
    st, fc, piv, L, U = dense_threshold_lu(D, blkptr, grpptr, tau, True)
    for upd in (oracle_lib.ORDER_DFS, oracle_lib.ORDER_ASCENDING):
        f = oracle_lib.factor(a, order, tau=tau, diag_pref=True, update_order=upd)
        assert f.status == st and f.fail_col == fc
        if st == 0:
            np.testing.assert_array_equal(f.piv, piv)
            # every factor entry stays inside its column's diagonal block
            blk = np.repeat(np.arange(len(blkptr) - 1), np.diff(blkptr))
            colL = np.repeat(np.arange(n), np.diff(f.Lp))
            colU = np.repeat(np.arange(n), np.diff(f.Up))
            assert np.all(blk[f.Li] == blk[colL]) and np.all(blk[f.Ui] == blk[colU])
            assert np.abs(f.L_dense() - L).max() <= 1e-12 * max(1, np.abs(L).max())
            assert np.abs(f.U_dense() - U).max() <= 1e-12 * max(1, np.abs(U).max())


@pytest.mark.parametrize("seed", list(range(20, 32)))
@pytest.mark.parametrize("diag_pref,tau", [(False, 1.0), (True, 1.0), (True, 0.5)])
def test_p2_exact_ties_integer(oracle_lib, seed, diag_pref, tau):
    """Entries in {-1, 0, 1}: every quantity stays a small integer or an exact ratio,
    so ties are exact and the smallest-index tie-break is pinned."""
    n = 12
    s = synth.Stream(synth.substream_key(seed, 5))
    D = s.integers(-1, 2, n * n).astype(float).reshape(n, n)
    D[np.arange(n), np.arange(n)] = np.where(s.uniform(n) < 0.5, 1.0, -1.0)
    a = synth.csc_from_dense(D)
    st, fc, piv, L, U = dense_threshold_lu(D, np.array([0, n]), np.array([0, n]), tau, diag_pref)
    f = oracle_lib.factor(a, tau=tau, diag_pref=diag_pref)
    assert f.status == st and f.fail_col == fc
    if st == 0:
        np.testing.assert_array_equal(f.piv, piv)
        assert np.abs(f.L_dense() - L).max() <= 1e-12 * max(1, np.abs(L).max())
        assert np.abs(f.U_dense() - U).max() <= 1e-12 * max(1, np.abs(U).max())


def test_golden_hand_example(oracle_lib):
    lines = [l for l in open(os.path.join(GOLDEN, "diag_pref_3x3.txt")) if not l.startswith("#")]
    A = np.array([float(v) for v in lines[0].split()[1:]]).reshape(3, 3)
    a = synth.csc_from_dense(A)
    for line in lines[1:]:
        head, piv, L, U = line.split("|")
        tau, dp = float(head.split()[1]), bool(int(head.split()[2]))
        f = oracle_lib.factor(a, tau=tau, diag_pref=dp)
        assert f.status == 0
        np.testing.assert_array_equal(f.piv, [int(v) for v in piv.split()])
        np.testing.assert_allclose(f.L_dense(), np.array([float(v) for v in L.split()]).reshape(3, 3), rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(f.U_dense(), np.array([float(v) for v in U.split()]).reshape(3, 3), rtol=1e-15, atol=1e-15)


# ---------------------------------------------------------------------------
# P3: reach = boolean closure
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [41, 42])
def test_p3_reach_is_closure(oracle_lib, seed):
    a = synth.gen_mna(300, seed=seed)
    f = oracle_lib.factor(a)
    assert f.status == 0
    n = a.n
    pos = np.empty(n, np.int64)
    pos[f.piv] = np.arange(n)
    Lrows = [set(f.piv[f.Li[f.Lp[j]:f.Lp[j + 1]]].tolist()) for j in range(n)]
    for k in range(n):
        S = set(a.rowind[a.colptr[k]:a.colptr[k + 1]].tolist())
        while True:
            grow = set()
            for i in S:
                if pos[i] < k:
                    grow |= Lrows[pos[i]]
            if grow <= S:
                break
            S |= grow
        got = set(f.piv[f.Ui[f.Up[k]:f.Up[k + 1]]].tolist()) | Lrows[k]
        assert S == got, k


# ---------------------------------------------------------------------------
# P4: invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [1.0, 0.1, 0.001])
def test_p4_invariants_mna(oracle_lib, tau):
    a = synth.gen_mna(400, seed=3)
    order = oracle_lib.Ordering.natural(a.n)
    f = oracle_lib.factor(a, order, tau=tau)
    assert f.status == 0
    n = a.n
    for k in range(n):
        li = f.Li[f.Lp[k]:f.Lp[k + 1]]
        assert np.all(li > k)                      # strictly lower, unit diagonal implicit
        ui = f.Ui[f.Up[k]:f.Up[k + 1]]
        assert np.all(ui <= k) and ui[-1] == k     # upper with diagonal last
    assert np.abs(f.Lx).max() <= 1.0 / tau * (1 + 1e-15)
    assert oracle_lib.backward_error(a, order, f) <= 1e-13


def test_p4_nd_fill_on_ancestor_paths(oracle_lib):
    """Geometric ND of a grid (two leaves, one separator): leaf columns never put fill
    into the sibling leaf, and pivots stay inside each column's group."""
    m = 9
    g0 = synth.gen_power_grid(m, relabel=False, long_frac=0.0, unsym_frac=0.0)
    # unsymmetric values on the mesh pattern (keeps the separator property)
    g = g0.with_values(g0.values * (1.0 + 0.3 * (synth.Stream(4).uniform(g0.nnz) - 0.5)))
    mid = m // 2
    idx = np.arange(m * m).reshape(m, m)
    left, sep, right = idx[:, :mid].ravel(), idx[:, mid].ravel(), idx[:, mid + 1:].ravel()
    perm = np.concatenate([left, right, sep]).astype(np.int32)
    n = m * m
    grpptr = np.array([0, left.size, left.size + right.size, n], np.int32)
    order = oracle_lib.Ordering(perm, perm.copy(), np.array([0, n], np.int32), grpptr)
    f = oracle_lib.factor(g, order, tau=0.1)
    assert f.status == 0
    grp = np.repeat(np.arange(3), np.diff(grpptr))
    assert np.all(grp[f.piv] == grp[np.arange(n)])     # pivots inside their group
    for k in range(n):
        li = f.Li[f.Lp[k]:f.Lp[k + 1]]
        rows_grp = grp[li]
        if grp[k] == 0:
            assert not np.any(rows_grp == 1)
        if grp[k] == 1:
            assert not np.any(rows_grp == 0)
    assert oracle_lib.backward_error(g, order, f) <= 1e-13


# ---------------------------------------------------------------------------
# P5: special cases
# ---------------------------------------------------------------------------

def test_p5_diagonal(oracle_lib):
    d = np.array([3.0, -2.0, 0.5, 7.0])
    a = synth.csc_from_dense(np.diag(d))
    f = oracle_lib.factor(a, tau=1.0, diag_pref=False)
    np.testing.assert_array_equal(f.piv, np.arange(4))
    assert f.lnz == 0
    np.testing.assert_array_equal(f.Ux, d)


def test_p5_upper_triangular(oracle_lib):
    A = np.triu(synth.random_dense(10, 51)) + 3 * np.eye(10)
    a = synth.csc_from_dense(A)
    f = oracle_lib.factor(a, tau=1.0, diag_pref=False)
    np.testing.assert_array_equal(f.piv, np.arange(10))
    assert f.lnz == 0
    np.testing.assert_array_equal(f.U_dense(), A)


def test_p5_permutation(oracle_lib):
    perm = synth.Stream(9).permutation(12)
    P = np.zeros((12, 12)); P[perm, np.arange(12)] = 1.0
    f = oracle_lib.factor(synth.csc_from_dense(P), tau=1.0, diag_pref=False)
    np.testing.assert_array_equal(f.piv, perm)
    assert f.lnz == 0
    np.testing.assert_array_equal(f.U_dense(), np.eye(12))


def test_p5_tridiagonal_thomas(oracle_lib):
    n = 50
    s = synth.Stream(3)
    lo, up = s.uniform(n - 1) - 0.5, s.uniform(n - 1) - 0.5
    di = 2.0 + s.uniform(n)
    A = np.diag(di) + np.diag(lo, -1) + np.diag(up, 1)
    f = oracle_lib.factor(synth.csc_from_dense(A), tau=1.0, diag_pref=True)
    np.testing.assert_array_equal(f.piv, np.arange(n))
    # Thomas algorithm: c'_0 = d_0, l_i = a_i / c'_{i-1}, c'_i = d_i - l_i u_{i-1}
    cp = np.zeros(n); l = np.zeros(n - 1)
    cp[0] = di[0]
    for i in range(1, n):
        l[i - 1] = lo[i - 1] / cp[i - 1]
        cp[i] = di[i] - l[i - 1] * up[i - 1]
    np.testing.assert_array_equal(f.Lx, l)
    np.testing.assert_array_equal(np.diag(f.U_dense()), cp)


def test_p5_block_diagonal_alone_equals_batched(oracle_lib):
    blocks = [synth.gen_mna(s, seed=100 + s) for s in (1, 3, 17, 40, 90)]
    n = sum(b.n for b in blocks)
    D = scipy.linalg.block_diag(*[b.to_dense() for b in blocks])
    big = synth.csc_from_dense(D)
    blkptr = np.concatenate([[0], np.cumsum([b.n for b in blocks])]).astype(np.int32)
    order = oracle_lib.Ordering(np.arange(n), np.arange(n), blkptr, blkptr)
    fb = oracle_lib.factor(big, order, tau=0.001)
    assert fb.status == 0
    for bi, b in enumerate(blocks):
        s0 = blkptr[bi]
        f1 = oracle_lib.factor(b, tau=0.001)
        np.testing.assert_array_equal(fb.piv[s0:s0 + b.n] - s0, f1.piv)
        Lb = fb.L_dense()[s0:s0 + b.n, s0:s0 + b.n]
        Ub = fb.U_dense()[s0:s0 + b.n, s0:s0 + b.n]
        np.testing.assert_array_equal(Lb, f1.L_dense())
        np.testing.assert_array_equal(Ub, f1.U_dense())


def test_singular_detection(oracle_lib):
    """A = L0 U0 with integer factors and unit-magnitude pivots, then column 4 := column 2.
    With the diagonal preferred, every operation is exact, so the Schur complement
    column at step 4 is exactly zero: numerically singular at column 4."""
    n = 6
    s = synth.Stream(61)
    L0 = np.tril(s.integers(-1, 2, n * n).reshape(n, n), -1) + np.eye(n)
    U0 = np.triu(s.integers(-1, 2, n * n).reshape(n, n), 1) + np.diag(np.where(s.uniform(n) < 0.5, 1.0, -1.0))
    A = L0 @ U0
    A[:, 4] = A[:, 2]
    f = oracle_lib.factor(synth.csc_from_dense(A), tau=1e-300, diag_pref=True)
    assert f.status == oracle_lib.ERR_NUM_SINGULAR and f.fail_col == 4
    # a column whose rows are all pivotal already (structurally singular)
    B = np.eye(n); B[0, 3] = 2.0; B[3, 3] = 0.0
    f = oracle_lib.factor(synth.csc_from_dense(B), tau=1.0, diag_pref=False)
    assert f.status == oracle_lib.ERR_NUM_SINGULAR and f.fail_col == 3


# ---------------------------------------------------------------------------
# P6: refactor
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("upd", [0, 1])
def test_p6_refactor_bitwise(oracle_lib, upd):
    a = synth.gen_mna(500, seed=8)
    f = oracle_lib.factor(a, update_order=upd)
    r = oracle_lib.refactor(a, oracle_lib.Ordering.natural(a.n), f.piv, update_order=upd)
    assert r.status == 0
    for x, y in ((f.Lp, r.Lp), (f.Li, r.Li), (f.Lx, r.Lx), (f.Up, r.Up), (f.Ui, r.Ui), (f.Ux, r.Ux)):
        np.testing.assert_array_equal(x, y)


def test_p6_refactor_sequence_and_fallback(oracle_lib):
    a = synth.gen_mna(300, seed=9)
    order = oracle_lib.Ordering.natural(a.n)
    f0 = oracle_lib.factor(a, order)
    same = 0
    for vals in synth.value_sequence(a, 5):
        at = a.with_values(vals)
        ft = oracle_lib.factor(at, order)
        rt = oracle_lib.refactor(at, order, f0.piv)
        if np.array_equal(ft.piv, f0.piv):
            same += 1
            assert rt.status == 0
            np.testing.assert_array_equal(rt.Ux, ft.Ux)
            np.testing.assert_array_equal(rt.Lx, ft.Lx)
    # forcing a tiny pivot makes the threshold check fail
    vals = a.values.copy()
    k = 0
    p = f0.piv[k]
    col = a.qcol if hasattr(a, "qcol") else None
    sel = (a.rowind[a.colptr[0]:a.colptr[1]] == p)
    vals[a.colptr[0]:a.colptr[1]][sel] *= 1e-12
    rt = oracle_lib.refactor(a.with_values(vals), order, f0.piv)
    assert rt.status == oracle_lib.REFACTOR_FAIL and rt.fail_col == 0


# ---------------------------------------------------------------------------
# P8: solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nrhs", [1, 3])
def test_p8_solve_vs_splu(oracle_lib, nrhs):
    a = synth.gen_mna(600, seed=10)
    order = oracle_lib.Ordering.natural(a.n)
    f = oracle_lib.factor(a, order)
    b = synth.rhs(a.n, nrhs)
    x = oracle_lib.solve(a, order, f, b)
    assert oracle_lib.residual(a, x, b) <= 1e-12
    ref = spla.splu(a.to_scipy()).solve(b)
    cond = np.linalg.cond(a.to_dense(), 1)
    assert np.abs(x - ref).max() / np.abs(ref).max() <= 1e-15 * cond * 10


def test_p8_solve_block_triangular(oracle_lib):
    """Upper block-triangular coupling exercises the off-diagonal back-substitution."""
    n = 60
    a0 = synth.random_sparse(n, 0.15, 71)
    blkptr, grpptr = _groups_case(n, 71)
    D = _block_upper(a0.to_dense(), blkptr)
    s = synth.Stream(5)
    perm_r = s.permutation(n); perm_c = s.permutation(n)
    # hide the ordering: A(perm_r, perm_c) = D  =>  prow = perm_r, qcol = perm_c
    A = np.zeros((n, n)); A[np.ix_(perm_r, perm_c)] = D
    a = synth.csc_from_dense(A)
    order = oracle_lib.Ordering(perm_r, perm_c, blkptr, grpptr)
    f = oracle_lib.factor(a, order, tau=0.1)
    assert f.status == 0
    b = synth.rhs(n, 2)
    x = oracle_lib.solve(a, order, f, b)
    assert oracle_lib.residual(a, x, b) <= 1e-12
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------
# update order: DFS reverse postorder vs ascending pivot index
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tau", [1.0, 0.1, 0.001])
def test_update_orders_agree(oracle_lib, tau):
    """Two topological update orders of the same elimination: no column of these MNA
    cases has an ambiguous decision, so pivots and patterns agree exactly and values
    to rounding."""
    a = synth.gen_mna(800, seed=12)
    f0 = oracle_lib.factor(a, tau=tau, update_order=0)
    f1 = oracle_lib.factor(a, tau=tau, update_order=1)
    assert not np.any(f0.margin < 1e-10) and not np.any(f1.margin < 1e-10)
    np.testing.assert_array_equal(f0.piv, f1.piv)
    for x, y in ((f0.Lp, f1.Lp), (f0.Li, f1.Li), (f0.Up, f1.Up), (f0.Ui, f1.Ui)):
        np.testing.assert_array_equal(x, y)
    assert np.abs(f0.Lx - f1.Lx).max() <= 1e-12 * max(1, np.abs(f0.Lx).max())
    assert np.abs(f0.Ux - f1.Ux).max() <= 1e-12 * max(1, np.abs(f0.Ux).max())


# ---------------------------------------------------------------------------
# decision margins and the flop count, against the dense elimination
# ---------------------------------------------------------------------------

def test_margin_golden(oracle_lib):
    """Hand-derived margins (tests/golden/margins.txt) on tiny integer matrices with
    exact ties, an exact threshold equality and clear decisions."""
    for line in open(os.path.join(GOLDEN, "margins.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, mat, want = line.split("|")
        name, n, tau, dp = head.split()
        n = int(n)
        A = np.array([float(v) for v in mat.split()]).reshape(n, n)
        f = oracle_lib.factor(synth.csc_from_dense(A), tau=float(tau), diag_pref=bool(int(dp)))
        assert f.status == 0, name
        np.testing.assert_allclose(f.margin, [float(v) for v in want.split()], rtol=1e-15, atol=0, err_msg=name)


def _margin_case(oracle_lib, D, blkptr, grpptr, tau, dp):
    n = D.shape[0]
    a = synth.csc_from_dense(D)
    order = oracle_lib.Ordering(np.arange(n), np.arange(n), blkptr, grpptr)
    st = {}
    ds, _, dpiv, _, _ = dense_threshold_lu(D, blkptr, grpptr, tau, dp, stats=st)
    f = oracle_lib.factor(a, order, tau=tau, diag_pref=dp)
    assert f.status == ds == 0
    np.testing.assert_array_equal(f.piv, dpiv)
    return f, st


@pytest.mark.parametrize("seed", list(range(20, 28)))
@pytest.mark.parametrize("diag_pref,tau", [(False, 1.0), (True, 1.0), (True, 0.5), (True, 0.1)])
def test_margin_vs_dense_integer(oracle_lib, seed, diag_pref, tau):
    """{-1, 0, 1} matrices with a nonzero diagonal (so a non-pivotal diagonal row is
    always structurally present): exact ties and threshold equalities occur, and
    every margin equals the one the dense elimination derives by definition."""
    n = 12
    s = synth.Stream(synth.substream_key(seed, 5))
    D = s.integers(-1, 2, n * n).astype(float).reshape(n, n)
    D[np.arange(n), np.arange(n)] = np.where(s.uniform(n) < 0.5, 1.0, -1.0)
    f, st = _margin_case(oracle_lib, D, np.array([0, n]), np.array([0, n]), tau, diag_pref)
    np.testing.assert_allclose(np.minimum(f.margin, 1.0), st["margin"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12, 13])
@pytest.mark.parametrize("tau", [1.0, 0.1])
def test_margin_and_flops_vs_dense_groups(oracle_lib, seed, tau):
    """Random sparse matrices (continuous values, no exact cancellation) with blocks and
    candidate groups: margins agree with the dense definition to rounding, and the flop
    count F equals the dense elimination's count of structural multiply-subtracts and
    divisions exactly."""
    n = 48
    a0 = synth.random_sparse(n, 0.12, seed)
    blkptr, grpptr = _groups_case(n, seed)
    D = _block_upper(a0.to_dense(), blkptr)
    f, st = _margin_case(oracle_lib, D, blkptr, grpptr, tau, True)
    np.testing.assert_allclose(np.minimum(f.margin, 1.0), st["margin"], rtol=0, atol=1e-12)
    assert f.flops == st["flops"]
    f0 = oracle_lib.factor(synth.csc_from_dense(D), oracle_lib.Ordering(np.arange(n), np.arange(n), blkptr, grpptr),
                           tau=tau, update_order=oracle_lib.ORDER_DFS)
    assert f0.flops == st["flops"]


def test_flops_closed_form_dense(oracle_lib):
    """Fully dense n x n with partial pivoting: sum_k (n-k-1) (1 + 2 (n-k-1)) flops."""
    n = 20
    A = synth.random_dense(n, 3)
    f = oracle_lib.factor(synth.csc_from_dense(A), tau=1.0, diag_pref=False)
    want = sum((n - k - 1) * (1 + 2 * (n - k - 1)) for k in range(n))
    assert f.flops == want


def test_margin_rarely_ambiguous_on_mna(oracle_lib):
    """Continuous circuit values: ambiguous decisions (margin < 1e-10) are absent."""
    for n, seed in ((300, 21), (2000, 160105725)):
        a = synth.gen_mna(n, seed=seed)
        for tau in (1.0, 0.1, 0.001):
            f = oracle_lib.factor(a, tau=tau)
            assert np.count_nonzero(f.margin < 1e-10) == 0, (n, tau)
