"""Host-side checks of the C-ABI library (no GPU): it loads, exports every symbol the
header declares, and its symbolic analysis (run with device = -1) produces valid
orderings -- checked against scipy and brute force, not against itself."""
import itertools
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bk():
    import paper_1601_05725_amd as bk
    if not os.path.exists(bk.LIB_PATH):
        from paper_1601_05725_amd import build
        build.build()
    bk.load()
    return bk


def header_symbols():
    text = open(os.path.join(ROOT, "include", "basker.h")).read()
    return sorted(set(re.findall(r"^\s*(?:basker_status|void|const char\*)\s+(basker_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(bk):
    lib = bk.load()
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(bk.EXPORTED)


def test_status_strings(bk):
    lib = bk.load()
    for code in range(-7, 2):
        assert lib.basker_status_string(code)


def analyse(bk, a, **kw):
    return bk.Handle.symbolic(a, bk.default_options(device=-1, **kw))


def check_ordering(a, prow, qcol, blkptr, grpptr):
    n = a.n
    assert sorted(prow.tolist()) == list(range(n))
    assert sorted(qcol.tolist()) == list(range(n))
    assert blkptr[0] == 0 and blkptr[-1] == n and np.all(np.diff(blkptr) > 0)
    assert grpptr[0] == 0 and grpptr[-1] == n and np.all(np.diff(grpptr) > 0)
    assert set(blkptr.tolist()) <= set(grpptr.tolist())   # groups nested in blocks
    R = a.to_scipy()[prow][:, qcol].tocoo()
    blk = np.repeat(np.arange(len(blkptr) - 1), np.diff(blkptr))
    assert not np.any(blk[R.row] > blk[R.col])               # block upper triangular
    d = a.to_scipy()[prow][:, qcol].diagonal()
    assert np.all(d != 0)                                    # matched diagonal is structurally nonzero
    return R


@pytest.mark.parametrize("n,seed", [(200, 1), (2000, 2)])
def test_btf_blocks_are_the_strong_components(bk, n, seed):
    a = synth.gen_mna(n, seed=seed)
    h = analyse(bk, a)
    prow, qcol, bp, gp = h.ordering()
    check_ordering(a, prow, qcol, bp, gp)
    # strong components of the matched matrix (rows moved onto the diagonal) = blocks
    B = a.to_scipy()[prow][:, qcol]
    nc, lab = csgraph.connected_components(B, directed=True, connection="strong")
    assert nc == len(bp) - 1
    blk = np.repeat(np.arange(len(bp) - 1), np.diff(bp))
    # same partition: each block holds exactly one label and labels are distinct
    for b in range(len(bp) - 1):
        assert len(set(lab[bp[b]:bp[b + 1]].tolist())) == 1
    assert len(set(lab[bp[:-1]].tolist())) == nc
    del blk


def _bottleneck_by_threshold(a):
    """Independent bottleneck value: largest t such that entries |a| >= t admit a
    perfect matching (scipy's Hopcroft-Karp), by bisection over the magnitudes."""
    m = a.to_scipy().tocsr()
    mags = np.unique(np.abs(m.data))
    lo, hi = 0, len(mags) - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        keep = np.abs(m.data) >= mags[mid]
        t = sp.csr_matrix((np.ones(keep.sum()), m.indices[keep], np.repeat(np.arange(m.shape[0]), np.diff(m.indptr))[keep]), shape=m.shape) if False else None
        mm = m.copy()
        mm.data = np.where(keep, 1.0, 0.0)
        mm.eliminate_zeros()
        match = csgraph.maximum_bipartite_matching(mm, perm_type="column")
        if np.all(match >= 0):
            lo = mid
        else:
            hi = mid - 1
    return mags[lo]


@pytest.mark.parametrize("n,seed", [(150, 3), (600, 4)])
def test_bottleneck_matching_value(bk, n, seed):
    a = synth.gen_mna(n, seed=seed)
    h = analyse(bk, a)
    prow, qcol, bp, gp = h.ordering()
    d = np.abs(a.to_scipy()[prow][:, qcol].diagonal())
    assert d.min() == pytest.approx(_bottleneck_by_threshold(a), rel=0, abs=0)
    assert h.info()["bottleneck"] == d.min()


def test_bottleneck_matching_brute_force(bk):
    for seed in range(5):
        n = 6
        a = synth.random_sparse(n, 0.5, seed=200 + seed, diag=False)
        M = a.to_dense()
        best = -1.0
        for perm in itertools.permutations(range(n)):
            vals = np.abs(M[list(perm), range(n)])
            if np.all(vals > 0):
                best = max(best, vals.min())
        if best < 0:
            with pytest.raises(bk.BaskerError):
                analyse(bk, a)
            continue
        h = analyse(bk, a)
        prow, qcol, bp, gp = h.ordering()
        d = np.abs(a.to_scipy()[prow][:, qcol].diagonal())
        assert d.min() == best


def test_structurally_singular_rejected(bk):
    A = np.eye(5)
    A[:, 2] = 0.0
    A[2, 3] = 1.0
    with pytest.raises(bk.BaskerError) as e:
        analyse(bk, synth.csc_from_dense(A))
    assert e.value.status == bk.ERR_STRUCT_SINGULAR


def test_invalid_csc_rejected(bk):
    a = synth.gen_mna(50, seed=5)
    bad = synth.Csc(a.n, a.colptr.copy(), a.rowind.copy(), a.values.copy())
    bad.rowind[bad.colptr[3]], bad.rowind[bad.colptr[3] + 1] = bad.rowind[bad.colptr[3] + 1], bad.rowind[bad.colptr[3]]
    with pytest.raises(bk.BaskerError) as e:
        analyse(bk, bad)
    assert e.value.status == bk.ERR_INVALID


def test_nd_separator_property(bk):
    """Large block ordered by ND: no entry of A + A^T joins two different subtrees of
    a separator (checked on the group tree recovered from the group ranges)."""
    a = synth.gen_mna(12000, seed=6)
    h = analyse(bk, a, nd_min_block=3000, nd_leaves=8)
    prow, qcol, bp, gp = h.ordering()
    R = check_ordering(a, prow, qcol, bp, gp)
    assert h.info()["nd_blocks"] >= 1
    sizes = np.diff(bp)
    b = int(np.argmax(sizes))
    b0, b1 = bp[b], bp[b + 1]
    groups = gp[(gp >= b0) & (gp <= b1)]
    grp = np.full(a.n, -1)
    for g in range(len(groups) - 1):
        grp[groups[g]:groups[g + 1]] = g
    gpar = h.group_tree()
    def ancestors(g):
        out = set()
        while g >= 0:
            out.add(g)
            g = gpar[g]
        return out
    S = (R + R.T).tocoo()
    inb = (S.row >= b0) & (S.row < b1) & (S.col >= b0) & (S.col < b1)
    pairs = set(zip(grp[S.row[inb]].tolist(), grp[S.col[inb]].tolist()))
    ngrp_blk = len(groups) - 1
    assert ngrp_blk >= 3
    # every coupled pair of groups lies on one root path of the ND tree
    for gi, gj in pairs:
        gi_abs = int(np.searchsorted(gp, groups[gi], side="right") - 1)
        gj_abs = int(np.searchsorted(gp, groups[gj], side="right") - 1)
        assert gi_abs in ancestors(gj_abs) or gj_abs in ancestors(gi_abs), (gi, gj)
    # a leaf count matching the request (some separators may be empty)
    roots = [g for g in range(len(gp) - 1) if gp[g] >= b0 and gp[g] < b1 and gpar[g] < 0]
    assert len(roots) == 1


def test_ordered_symbolic_validation(bk):
    a = synth.gen_mna(100, seed=7)
    n = a.n
    r = np.arange(n, dtype=np.int32)
    h = bk.Handle.symbolic_ordered(a, r, r, [0, n], [0, n], bk.default_options(device=-1))
    assert h.info()["nblocks"] == 1
    with pytest.raises(bk.BaskerError):
        bk.Handle.symbolic_ordered(a, r, r, [0, 10, n], [0, n], bk.default_options(device=-1))  # group crosses block
    bad = r.copy()
    bad[0] = 1
    with pytest.raises(bk.BaskerError):
        bk.Handle.symbolic_ordered(a, bad, r, [0, n], [0, n], bk.default_options(device=-1))


@pytest.mark.parametrize("field,value", [("pivot_tol", 0.0), ("pivot_tol", -1e-3), ("pivot_tol", 1.5),
                                         ("pivot_tol", float("nan")), ("nd_leaves", 3), ("nd_leaves", 0),
                                         ("hbm_budget", -1), ("max_grid", -2)])
def test_options_rejected(bk, field, value):
    """Options outside their documented ranges are refused before any analysis."""
    a = synth.gen_mna(200, seed=3)
    with pytest.raises(bk.BaskerError) as e:
        analyse(bk, a, **{field: value})
    assert e.value.status == bk.ERR_INVALID


def _c_layout(struct, fields):
    """sizeof and offsetof of the header's struct, from the C compiler."""
    import subprocess
    import tempfile
    body = "\n".join('printf("%%s %%zu\\n", "%s", offsetof(%s, %s));' % (f, struct, f) for f in fields)
    src = ('#include <stddef.h>\n#include <stdio.h>\n#include "basker.h"\nint main(void) {\n'
           'printf("sizeof %%zu\\n", sizeof(%s));\n%s\nreturn 0;\n}\n' % (struct, body))
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return {out[i]: int(out[i + 1]) for i in range(0, len(out), 2)}


@pytest.mark.parametrize("name", ["basker_options", "basker_info_t"])
def test_struct_layouts_match_the_header(bk, name):
    """Every field of the binding's ctypes structs sits where the C compiler puts the
    header's field, and the sizes agree."""
    cls = getattr(bk, name)
    fields = [f for f, _ in cls._fields_]
    lay = _c_layout(name, fields)
    import ctypes
    assert lay["sizeof"] == ctypes.sizeof(cls)
    for f in fields:
        assert lay[f] == getattr(cls, f).offset, f


def test_device_bytes_plan_estimate(bk):
    """The host-only analysis reports the device memory a handle will hold: at least the
    L/U pools (capacity_factor * nnz(diagonal blocks) entries of 4 + 8 bytes, twice),
    the value arrays and the solve vectors for 8 right-hand sides."""
    a = synth.gen_mna(3000, seed=5)
    for cf in (2.0, 6.0):
        inf = analyse(bk, a, capacity_factor=cf).info()
        pools = 2 * 12 * int(cf * inf["nnz_diag"])
        assert inf["device_bytes_plan"] >= pools + 8 * a.nnz + 3 * 8 * 8 * a.n
    small = analyse(bk, a, capacity_factor=2.0).info()["device_bytes_plan"]
    big = analyse(bk, a, capacity_factor=6.0).info()["device_bytes_plan"]
    assert big - small >= 2 * 12 * int(4.0 * analyse(bk, a).info()["nnz_diag"]) - 64


def _diag_dominant(n, density, seed):
    a = synth.random_sparse(n, density, seed=seed)
    d = a.to_dense()
    np.fill_diagonal(d, np.abs(d).sum(axis=1) + 1.0)
    return synth.csc_from_dense(d)


@pytest.mark.parametrize("n,seed,kw", [(300, 11, {}), (900, 12, {"nd_min_block": 400, "nd_leaves": 4})])
def test_fill_bound_is_the_fill_without_row_exchanges(bk, n, seed, kw):
    """The analysis's fill counts are the factorization's when no row leaves the
    diagonal: on a diagonally dominant matrix the oracle (same ordering) pivots on the
    diagonal, and its nnz(L), nnz(U) equal the reported bound."""
    import oracle
    a = _diag_dominant(n, 0.01, seed)
    h = analyse(bk, a, **kw)
    inf = h.info()
    assert inf["fill_bound"] == 1
    prow, qcol, bp, gp = h.ordering()
    f = oracle.factor(a, oracle.Ordering(prow, qcol, bp, gp), update_order=oracle.ORDER_ASCENDING)
    assert f.status == oracle.OK
    assert np.array_equal(f.piv, np.arange(n))   # no row exchange
    assert inf["sym_lnz"] == f.lnz and inf["sym_unz"] == f.unz
    # a column's workspace holds its L and U rows: at least the longest column of L + U
    longest = max(int(f.Lp[k + 1] - f.Lp[k] + f.Up[k + 1] - f.Up[k]) for k in range(n))
    assert inf["sym_ws_rows"] >= longest


def test_factor_refuses_a_column_beyond_the_workspace(bk):
    """An arrow matrix whose dense column reaches 9,000 rows exceeds the 8,192-row
    per-wave workspace: basker_factor refuses it before any device work."""
    n = 9000
    r = np.concatenate([np.arange(n), np.arange(n - 1), np.full(n - 1, n - 1)])
    c = np.concatenate([np.arange(n), np.full(n - 1, n - 1), np.arange(n - 1)])
    v = np.concatenate([np.full(n, 4.0), np.ones(2 * (n - 1))])
    a = synth.csc_from_coo(n, r, c, v)
    h = analyse(bk, a, nd_min_block=1 << 30)
    inf = h.info()
    assert inf["fill_bound"] == 1 and inf["sym_ws_rows"] > 8192
    with pytest.raises(bk.BaskerError) as e:
        h.factor(a.values)
    assert e.value.status == bk.ERR_WORKSPACE
