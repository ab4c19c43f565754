"""Seeded synthetic inputs for the sparse LU path and for the oracle that checks it.

This module only builds matrices, right-hand sides and value sequences.  It holds
none of the factorization's arithmetic, so both the oracle and the GPU library can
be fed from it.

Random numbers come from SplitMix64 used as a counter-based generator: draw i of a
stream with key s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), where mix is the
published SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).  A sub-stream
for an object id (a block, a step, a request) has key mix(seed ^ id).  Every draw is
therefore vectorisable and reproducible on any machine.

Workloads (the paper evaluates circuit and power-grid matrices, Sec. V, Table I;
those matrices are not available, so these generators stand in for them with the
same shapes: a few nonzeros per row, fill ratios below about 4, many small BTF
blocks):

* ``gen_mna(n)``        modified-nodal-analysis circuit matrix (resistor graph,
                         controlled sources, voltage sources with zero diagonal).
* ``gen_power_grid(m)`` m x m resistor mesh with long-range branches.
* ``gen_batched_btf()`` many power-law-sized MNA blocks plus one large coupled
                         block, joined by upper block-triangular coupling.
* ``value_sequence()``  multiplicative perturbation of values (transient steps).

All matrices are returned as ``Csc`` (int32 colptr/rowind, float64 values, rows
sorted and unique within each column).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
BASE_SEED = 160105725


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def substream_key(seed: int, ident: int) -> int:
    return int(_mix(np.uint64((seed ^ ident) & 0xFFFFFFFFFFFFFFFF)))


class Stream:
    """Counter-based SplitMix64 stream: successive calls continue the counter."""

    def __init__(self, key: int):
        self.key = np.uint64(key & 0xFFFFFFFFFFFFFFFF)
        self.ctr = 0

    def raw(self, count: int) -> np.ndarray:
        idx = np.arange(self.ctr + 1, self.ctr + 1 + count, dtype=np.uint64)
        self.ctr += count
        with np.errstate(over="ignore"):
            return _mix(self.key + idx * GOLDEN)

    def uniform(self, count: int) -> np.ndarray:
        """U[0,1): top 53 bits of each draw."""
        return (self.raw(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def uniform_pos(self, count: int) -> np.ndarray:
        """U(0,1]: never zero, safe under log."""
        return 1.0 - self.uniform(count)

    def integers(self, lo: int, hi: int, count: int) -> np.ndarray:
        """Uniform integers in [lo, hi) (multiply-shift on the 53-bit uniform)."""
        u = self.uniform(count)
        return lo + np.minimum((u * (hi - lo)).astype(np.int64), hi - lo - 1)

    def normal(self, count: int) -> np.ndarray:
        """Box-Muller, one normal per pair of uniforms (the cosine branch)."""
        u1 = self.uniform_pos(count)
        u2 = self.uniform(count)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)

    def log_uniform(self, lo: float, hi: float, count: int) -> np.ndarray:
        u = self.uniform(count)
        return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))

    def geometric(self, p: float, count: int) -> np.ndarray:
        """Failures before the first success, P(k) = (1-p)^k p (inverse CDF)."""
        u = self.uniform_pos(count)
        return np.floor(np.log(u) / np.log1p(-p)).astype(np.int64)

    def permutation(self, n: int) -> np.ndarray:
        """Uniform random permutation: argsort of n 64-bit draws (ties broken by index)."""
        return np.argsort(self.raw(n), kind="stable").astype(np.int64)


@dataclasses.dataclass
class Csc:
    n: int
    colptr: np.ndarray  # int32[n+1]
    rowind: np.ndarray  # int32[nnz]
    values: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_scipy(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.values, self.rowind, self.colptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def with_values(self, values: np.ndarray) -> "Csc":
        assert values.shape == self.values.shape
        return Csc(self.n, self.colptr, self.rowind, np.ascontiguousarray(values, dtype=np.float64))


def csc_from_coo(n: int, rows, cols, vals) -> Csc:
    """Assemble; duplicate (row, col) entries are summed; rows sorted per column."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsc()
    m.sum_duplicates()
    m.sort_indices()
    return Csc(n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def csc_from_dense(a: np.ndarray, keep_zeros: bool = False) -> Csc:
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if keep_zeros:
        r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        return csc_from_coo(n, r.ravel(), c.ravel(), a.ravel())
    r, c = np.nonzero(a)
    return csc_from_coo(n, r, c, a[r, c])


def symmetric_relabel(a: Csc, perm: np.ndarray) -> Csc:
    """B(perm[i], perm[j]) = A(i, j): the same permutation on rows and columns."""
    coo = a.to_scipy().tocoo()
    return csc_from_coo(a.n, perm[coo.row], perm[coo.col], coo.data)


# ---------------------------------------------------------------------------
# MNA circuit generator
# ---------------------------------------------------------------------------

def mna_parts(n: int) -> tuple[int, int, int]:
    """n = graph nodes + auxiliary (controlled-source) nodes + voltage-source rows,
    in fractions 0.90 / 0.075 / 0.025 (the stated 1,800 + 150 + 50 = 2,000)."""
    n_g = int(round(0.90 * n))
    n_vs = int(round(0.025 * n))
    n_aux = n - n_g - n_vs
    if n_aux < 0:
        n_aux = 0
        n_vs = n - n_g
    return n_g, n_aux, n_vs


def mna_triplets(n: int, key: int, p_long: float = 1e-3, edges_per_node: int = 3,
                 g_lo: float = 1e-3, g_hi: float = 1e3):
    """Triplets (rows, cols, vals) of one MNA matrix of order n, before relabelling.

    Graph nodes 0..n_g-1: every node v >= 1 starts ``edges_per_node`` resistors.  The
    first goes to an earlier node (connectivity); each partner sits at offset
    1 + Geom(0.25), or with probability p_long at a uniform node.  Conductances are
    log-uniform in [g_lo, g_hi] and stamped symmetrically.  Node 0 and 1% of nodes are
    grounded.  Auxiliary nodes hang off a random graph node and are grounded.  There
    are n_aux controlled-source entries U(-1,1) at random off-diagonal node positions
    (uniform for n <= 2,000; above that at a local offset, uniform only with
    probability p_long, so large circuits keep circuit-like fill), and n_vs voltage sources, each tying a distinct graph node to ground through a
    +1/+1 pair with no diagonal entry.
    """
    n_g, n_aux, n_vs = mna_parts(n)
    s = Stream(key)
    R, C, V = [], [], []

    def stamp(u, v, g):
        R.extend([u, v, u, v]); C.extend([u, v, v, u]); V.extend([g, g, -g, -g])

    if n_g >= 2:
        v = np.arange(1, n_g, dtype=np.int64)
        m = v.size
        # edge 0: to an earlier node
        off0 = 1 + s.geometric(0.25, m)
        u0 = np.maximum(v - off0, 0)
        lng = s.uniform(m) < p_long
        u0 = np.where(lng, s.integers(0, n_g, m) % np.maximum(v, 1), u0)
        us = [u0]
        for _ in range(edges_per_node - 1):
            off = 1 + s.geometric(0.25, m)
            sign = np.where(s.uniform(m) < 0.5, -1, 1)
            u = v + sign * off
            u = np.where(u < 0, -u, u)
            u = np.where(u >= n_g, 2 * (n_g - 1) - u, u)
            u = np.clip(u, 0, n_g - 1)
            lng = s.uniform(m) < p_long
            u = np.where(lng, s.integers(0, n_g, m), u)
            us.append(u)
        for u in us:
            keep = u != v
            g = s.log_uniform(g_lo, g_hi, m)
            uu, vv, gg = u[keep], v[keep], g[keep]
            R.append(np.concatenate([uu, vv, uu, vv])); C.append(np.concatenate([uu, vv, vv, uu]))
            V.append(np.concatenate([gg, gg, -gg, -gg]))
    # grounding: node 0 plus 1% of graph nodes
    n_gnd = max(0, int(round(0.01 * n_g)))
    gnd = np.unique(np.concatenate([[0], s.integers(0, max(n_g, 1), n_gnd)])) if n_g > 0 else np.zeros(0, np.int64)
    R.append(gnd); C.append(gnd); V.append(s.log_uniform(g_lo, g_hi, gnd.size))
    # auxiliary nodes
    if n_aux > 0:
        a = np.arange(n_g, n_g + n_aux, dtype=np.int64)
        tgt = s.integers(0, n_g, n_aux)
        g = s.log_uniform(g_lo, g_hi, n_aux)
        R.append(np.concatenate([a, tgt, a, tgt])); C.append(np.concatenate([a, tgt, tgt, a]))
        V.append(np.concatenate([g, g, -g, -g]))
        R.append(a); C.append(a); V.append(s.log_uniform(g_lo, g_hi, n_aux))
        # controlled sources: off-diagonal node positions -- uniform up to n = 2,000;
        # above that local like the resistor partners (uniform with probability p_long)
        nn = n_g + n_aux
        i = s.integers(0, nn, n_aux)
        j = (i + 1 + s.integers(0, nn - 1, n_aux)) % nn
        if n > 2000:
            off = 1 + s.geometric(0.25, n_aux)
            sign = np.where(s.uniform(n_aux) < 0.5, -1, 1)
            jl = np.clip(i + sign * off, 0, nn - 1)
            jl = np.where(jl == i, np.where(i > 0, i - 1, i + 1), jl)
            j = np.where(s.uniform(n_aux) < p_long, j, jl)
        R.append(i); C.append(j); V.append(2.0 * s.uniform(n_aux) - 1.0)
    # voltage sources
    if n_vs > 0:
        nodes = s.permutation(n_g)[:n_vs]
        mrow = np.arange(n - n_vs, n, dtype=np.int64)
        R.append(np.concatenate([nodes, mrow])); C.append(np.concatenate([mrow, nodes]))
        V.append(np.ones(2 * n_vs))
    rows = np.concatenate([np.asarray(x, dtype=np.int64).ravel() for x in R]) if R else np.zeros(0, np.int64)
    cols = np.concatenate([np.asarray(x, dtype=np.int64).ravel() for x in C]) if C else np.zeros(0, np.int64)
    vals = np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in V]) if V else np.zeros(0)
    return rows, cols, vals


def mna_p_long(n: int) -> float:
    """Probability of a uniform long-range partner: 1e-3 up to n = 2,000, then
    1e-3 * sqrt(2000 / n), so the number of long branches grows like sqrt(n) (a
    Rent-exponent-1/2 circuit) instead of linearly, which would make large circuits
    expanders with fill far above the circuit range (|L+U|/|A| < 4)."""
    return 1e-3 if n <= 2000 else 1e-3 * np.sqrt(2000.0 / n)


def gen_mna(n: int, seed: int = BASE_SEED, relabel: bool = True, p_long: float | None = None) -> Csc:
    """One nonsingular MNA circuit matrix of order n (about 6 nnz/row)."""
    key = substream_key(seed, 0x4D4E41)
    r, c, v = mna_triplets(n, key, p_long=mna_p_long(n) if p_long is None else p_long)
    a = csc_from_coo(n, r, c, v)
    if relabel:
        a = symmetric_relabel(a, Stream(substream_key(seed, 0x5045524D)).permutation(n))
    return a


# ---------------------------------------------------------------------------
# Power-grid mesh
# ---------------------------------------------------------------------------

def gen_power_grid(m: int, seed: int = BASE_SEED + 1, relabel: bool = True,
                   long_frac: float = 0.02, unsym_frac: float = 0.01) -> Csc:
    """m x m resistor mesh (4-neighbour conductances log-uniform in [1e-2, 1e2]),
    round(long_frac n) long-range branches between uniform node pairs,
    round(unsym_frac n) unsymmetric entries U(-1,1), node 0 and 1% of nodes grounded."""
    n = m * m
    s = Stream(substream_key(seed, 0x47524944))
    idx = np.arange(n, dtype=np.int64).reshape(m, m)
    eu = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    ev = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    n_long = int(round(long_frac * n))
    lu = s.integers(0, n, n_long)
    lv = (lu + 1 + s.integers(0, n - 1, n_long)) % n
    eu = np.concatenate([eu, lu]); ev = np.concatenate([ev, lv])
    g = s.log_uniform(1e-2, 1e2, eu.size)
    R = [eu, ev, eu, ev]; C = [eu, ev, ev, eu]; V = [g, g, -g, -g]
    n_gnd = int(round(0.01 * n))
    gnd = np.unique(np.concatenate([[0], s.integers(0, n, n_gnd)]))
    R.append(gnd); C.append(gnd); V.append(s.log_uniform(1e-2, 1e2, gnd.size))
    n_un = int(round(unsym_frac * n))
    i = s.integers(0, n, n_un)
    j = (i + 1 + s.integers(0, n - 1, n_un)) % n
    R.append(i); C.append(j); V.append(2.0 * s.uniform(n_un) - 1.0)
    a = csc_from_coo(n, np.concatenate(R), np.concatenate(C), np.concatenate(V))
    if relabel:
        a = symmetric_relabel(a, Stream(substream_key(seed, 0x5045524D)).permutation(n))
    return a


# ---------------------------------------------------------------------------
# Batched BTF
# ---------------------------------------------------------------------------

def power_law_sizes(count: int, key: int, s_max: int = 2000, alpha: float = 2.0) -> np.ndarray:
    """Block sizes from p(s) proportional to s^-alpha on {1..s_max} (inverse CDF)."""
    w = np.arange(1, s_max + 1, dtype=np.float64) ** (-alpha)
    cdf = np.cumsum(w) / w.sum()
    u = Stream(key).uniform(count)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.int64).clip(1, s_max)


@dataclasses.dataclass
class BtfInput:
    a: Csc
    block_sizes: np.ndarray  # sizes in generation order (before relabel)
    big_block: int           # index of the large coupled block in generation order (-1 if none)


def gen_batched_btf(nblocks: int = 50000, big: int = 100000, seed: int = BASE_SEED + 2,
                    s_max: int = 2000, coupling_per_row: int = 3, relabel: bool = True,
                    fill_to: int | None = None) -> BtfInput:
    """Many independent power-law-sized MNA blocks plus one large MNA block, placed
    in a random order along the diagonal and joined by ``coupling_per_row`` random
    U(-1,1) entries per row in columns of later blocks (upper block triangular).
    ``fill_to`` keeps drawing small blocks until the order reaches that n."""
    sizes = power_law_sizes(nblocks, substream_key(seed, 0x53495A45), s_max)
    if fill_to is not None:
        extra_key = 1
        while sizes.sum() + big < fill_to:
            more = power_law_sizes(nblocks, substream_key(seed, 0x53495A45 + extra_key), s_max)
            sizes = np.concatenate([sizes, more])
            extra_key += 1
        cs = np.cumsum(sizes) + big
        sizes = sizes[: int(np.searchsorted(cs, fill_to)) + 1]
    all_sizes = list(sizes)
    big_at = -1
    if big > 0:
        pos = int(Stream(substream_key(seed, 0x424947)).integers(0, len(all_sizes) + 1, 1)[0])
        all_sizes.insert(pos, big)
        big_at = pos
    all_sizes = np.asarray(all_sizes, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(all_sizes)])
    n = int(off[-1])
    R, C, V = [], [], []
    for b, s_b in enumerate(all_sizes):
        r, c, v = mna_triplets(int(s_b), substream_key(seed, 0x10000000 + b), p_long=mna_p_long(int(s_b)))
        R.append(r + off[b]); C.append(c + off[b]); V.append(v)
    # upper block-triangular coupling: row i in block b -> columns in blocks > b
    s = Stream(substream_key(seed, 0x434F5550))
    blk_of_row = np.repeat(np.arange(all_sizes.size), all_sizes)
    start_after = off[blk_of_row + 1]
    has = start_after < n
    rows = np.repeat(np.arange(n)[has], coupling_per_row)
    lo = np.repeat(start_after[has], coupling_per_row)
    span = n - lo
    cols = lo + np.minimum((s.uniform(rows.size) * span).astype(np.int64), span - 1)
    R.append(rows); C.append(cols); V.append(2.0 * s.uniform(rows.size) - 1.0)
    a = csc_from_coo(n, np.concatenate(R), np.concatenate(C), np.concatenate(V))
    if relabel:
        a = symmetric_relabel(a, Stream(substream_key(seed, 0x5045524D)).permutation(n))
    return BtfInput(a, all_sizes, big_at)


# ---------------------------------------------------------------------------
# Value sequences, right-hand sides, small test matrices
# ---------------------------------------------------------------------------

def value_sequence(a: Csc, steps: int, seed: int = BASE_SEED + 3, sigma: float = 0.05):
    """values_t = values_{t-1} * (1 + sigma N(0,1)), cumulative, t = 1..steps."""
    vals = a.values.copy()
    for t in range(1, steps + 1):
        z = Stream(substream_key(seed, 0x53544550 + t)).normal(vals.size)
        vals = vals * (1.0 + sigma * z)
        yield vals.copy()


def rhs(n: int, nrhs: int = 1, seed: int = BASE_SEED, ident: int = 0x524853) -> np.ndarray:
    """Column-major n x nrhs right-hand sides, U(-1,1)."""
    u = Stream(substream_key(seed, ident)).uniform(n * nrhs)
    return np.asfortranarray((2.0 * u - 1.0).reshape(nrhs, n).T)


def random_sparse(n: int, density: float, seed: int, diag: bool = True,
                  integer: bool = False, value_range: int = 4) -> Csc:
    """Random square test matrix; optional full diagonal; optional small integers."""
    s = Stream(substream_key(seed, 0x52414E44))
    mask = s.uniform(n * n).reshape(n, n) < density
    if diag:
        mask[np.arange(n), np.arange(n)] = True
    r, c = np.nonzero(mask)
    if integer:
        v = s.integers(-value_range, value_range + 1, r.size).astype(np.float64)
        v[v == 0] = 1.0
    else:
        v = 2.0 * s.uniform(r.size) - 1.0
    return csc_from_coo(n, r, c, v)


def random_dense(n: int, seed: int) -> np.ndarray:
    s = Stream(substream_key(seed, 0x44454E53))
    return (2.0 * s.uniform(n * n) - 1.0).reshape(n, n)
