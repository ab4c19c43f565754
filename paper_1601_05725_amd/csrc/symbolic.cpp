// Host-side symbolic analysis (see symbolic.hpp).
#include "symbolic.hpp"

#include <algorithm>
#include <iterator>
#include <cmath>
#include <numeric>

namespace basker {

namespace {

bool validate_csc(int n, const int32_t* Ap, const int32_t* Ai, std::string& err) {
  if (n < 0) { err = "negative order"; return false; }
  if (Ap[0] != 0) { err = "colptr[0] != 0"; return false; }
  for (int j = 0; j < n; j++) {
    if (Ap[j + 1] < Ap[j]) { err = "colptr not monotone"; return false; }
    for (int32_t p = Ap[j]; p < Ap[j + 1]; p++) {
      if (Ai[p] < 0 || Ai[p] >= n) { err = "row index out of range"; return false; }
      if (p > Ap[j] && Ai[p] <= Ai[p - 1]) { err = "rows not sorted/unique"; return false; }
    }
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// Maximum matching: a greedy start (diagonal first, then any free row), then a
// shortest augmenting path (breadth first) from every column left unmatched.
// Entries with |a| < thresh are not usable.
// ---------------------------------------------------------------------------
int max_matching(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax, double thresh,
                 std::vector<int32_t>& m) {
  auto usable = [&](int32_t p) { return !Ax || std::fabs(Ax[p]) >= thresh; };
  std::vector<int32_t> col_of_row(n, -1), visited(n, -1), cstack(n);
  if ((int)m.size() != n) m.assign(n, -1);
  int matched = 0;
  for (int j = 0; j < n; j++) {
    int32_t i = m[j];
    bool ok = false;
    if (i >= 0) {
      for (int32_t p = Ap[j]; p < Ap[j + 1]; p++)
        if (Ai[p] == i) { ok = usable(p) && col_of_row[i] < 0; break; }
    }
    if (ok) { col_of_row[i] = j; matched++; } else m[j] = -1;
  }
  // greedy start: the diagonal entry where it is usable, then any free usable row,
  // so that the augmenting searches below only handle the few remaining columns
  for (int j = 0; j < n; j++) {
    if (m[j] >= 0 || col_of_row[j] >= 0) continue;
    for (int32_t p = Ap[j]; p < Ap[j + 1]; p++)
      if (Ai[p] == j) {
        if (usable(p)) { m[j] = j; col_of_row[j] = j; matched++; }
        break;
      }
  }
  for (int j = 0; j < n; j++) {
    if (m[j] >= 0) continue;
    for (int32_t p = Ap[j]; p < Ap[j + 1]; p++)
      if (usable(p) && col_of_row[Ai[p]] < 0) { m[j] = Ai[p]; col_of_row[Ai[p]] = j; matched++; break; }
  }
  // shortest augmenting path from every unmatched column (breadth-first over
  // alternating paths: column -> row -> the row's matched column)
  std::vector<int32_t> prev_col(n, -1), via_row(n, -1);
  for (int j0 = 0; j0 < n; j0++) {
    if (m[j0] >= 0) continue;
    int head = 0, tail = 0;
    cstack[tail++] = j0;
    visited[j0] = j0;
    prev_col[j0] = -1;
    int32_t found = -1, found_col = -1;
    while (head < tail && found < 0) {
      int32_t j = cstack[head++];
      for (int32_t p = Ap[j]; p < Ap[j + 1]; p++) {
        if (!usable(p)) continue;
        int32_t i = Ai[p];
        int32_t jj = col_of_row[i];
        if (jj < 0) { found = i; found_col = j; break; }
        if (visited[jj] != j0) {
          visited[jj] = j0;
          prev_col[jj] = j;
          via_row[jj] = i;
          cstack[tail++] = jj;
        }
      }
    }
    if (found >= 0) {
      // flip the path: found_col takes `found`, each column hands its row to the next
      int32_t c = found_col, r = found;
      while (c >= 0) {
        int32_t old = m[c];
        m[c] = r;
        col_of_row[r] = c;
        r = old;
        c = prev_col[c];
      }
      matched++;
    }
  }
  return matched;
}

// Bottleneck matching: a perfect matching maximising min |a(m[j], j)| (the MC64
// bottleneck objective), by bisection over the distinct magnitudes with a warm start.
int bottleneck_matching(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax,
                        std::vector<int32_t>& m, double* bottleneck) {
  m.assign(n, -1);
  int r = max_matching(n, Ap, Ai, nullptr, 0.0, m);
  if (r < n) { if (bottleneck) *bottleneck = 0.0; return r; }
  if (!Ax || n == 0) { if (bottleneck) *bottleneck = 0.0; return n; }
  // upper bound: every column and every row must keep one usable entry
  double ub = INFINITY;
  std::vector<double> rowmax(n, 0.0);
  for (int j = 0; j < n; j++) {
    double cm = 0.0;
    for (int32_t p = Ap[j]; p < Ap[j + 1]; p++) {
      double v = std::fabs(Ax[p]);
      cm = std::max(cm, v);
      rowmax[Ai[p]] = std::max(rowmax[Ai[p]], v);
    }
    ub = std::min(ub, cm);
  }
  for (int i = 0; i < n; i++) ub = std::min(ub, rowmax[i]);
  std::vector<double> mags;
  mags.reserve(Ap[n]);
  for (int32_t p = 0; p < Ap[n]; p++) {
    double v = std::fabs(Ax[p]);
    if (v <= ub) mags.push_back(v);
  }
  std::sort(mags.begin(), mags.end());
  mags.erase(std::unique(mags.begin(), mags.end()), mags.end());
  // current matching is feasible at the smallest magnitude
  double best = INFINITY;
  for (int j = 0; j < n; j++)
    for (int32_t p = Ap[j]; p < Ap[j + 1]; p++)
      if (Ai[p] == m[j]) best = std::min(best, std::fabs(Ax[p]));
  int lo = (int)(std::lower_bound(mags.begin(), mags.end(), best) - mags.begin());
  if (lo >= (int)mags.size()) lo = (int)mags.size() - 1;
  int hi = (int)mags.size() - 1;
  std::vector<int32_t> trial;
  while (lo < hi) {
    int mid = lo + (hi - lo + 1) / 2;
    trial = m;
    if (max_matching(n, Ap, Ai, Ax, mags[mid], trial) == n) { lo = mid; m.swap(trial); }
    else hi = mid - 1;
  }
  if (bottleneck) {
    double b = INFINITY;
    for (int j = 0; j < n; j++)
      for (int32_t p = Ap[j]; p < Ap[j + 1]; p++)
        if (Ai[p] == m[j]) b = std::min(b, std::fabs(Ax[p]));
    *bottleneck = b;
  }
  return n;
}

// ---------------------------------------------------------------------------
// Strongly connected components (Tarjan, iterative) of the directed graph with an
// edge j -> r for every off-diagonal entry B(r, j), B = A with column j's matched row
// moved to position j.  Components are emitted sinks first, which makes the
// permuted matrix block upper triangular.  perm: new index -> old column index.
// ---------------------------------------------------------------------------
int scc_order(int n, const int32_t* Ap, const int32_t* Ai, const int32_t* row_of_col,
              std::vector<int32_t>& perm, std::vector<int32_t>& blkptr) {
  std::vector<int32_t> col_of_row(n);
  for (int j = 0; j < n; j++) col_of_row[row_of_col[j]] = j;
  std::vector<int32_t> index(n, -1), low(n, 0), stack, cstack, pos(n), comp(n, -1);
  std::vector<char> onstack(n, 0);
  stack.reserve(n);
  cstack.reserve(n);
  int counter = 0, ncomp = 0;
  std::vector<int32_t> order;
  order.reserve(n);
  blkptr.assign(1, 0);
  for (int s = 0; s < n; s++) {
    if (index[s] >= 0) continue;
    cstack.push_back(s);
    index[s] = low[s] = counter++;
    pos[s] = Ap[s];
    stack.push_back(s);
    onstack[s] = 1;
    while (!cstack.empty()) {
      int v = cstack.back();
      bool descended = false;
      while (pos[v] < Ap[v + 1]) {
        int w = col_of_row[Ai[pos[v]]];
        pos[v]++;
        if (w == v) continue;
        if (index[w] < 0) {
          index[w] = low[w] = counter++;
          pos[w] = Ap[w];
          stack.push_back(w);
          onstack[w] = 1;
          cstack.push_back(w);
          descended = true;
          break;
        } else if (onstack[w]) {
          low[v] = std::min(low[v], index[w]);
        }
      }
      if (descended) continue;
      cstack.pop_back();
      if (!cstack.empty()) low[cstack.back()] = std::min(low[cstack.back()], low[v]);
      if (low[v] == index[v]) {
        // pop the component; list its nodes in ascending index for determinism
        size_t start = order.size();
        while (true) {
          int w = stack.back();
          stack.pop_back();
          onstack[w] = 0;
          comp[w] = ncomp;
          order.push_back(w);
          if (w == v) break;
        }
        std::sort(order.begin() + (long)start, order.end());
        ncomp++;
        blkptr.push_back((int32_t)order.size());
      }
    }
  }
  perm = order;
  return ncomp;
}

// ---------------------------------------------------------------------------
// Minimum-degree ordering on a symmetric graph using a quotient graph of
// variables and elements with approximate external degrees (the scheme of
// Amestoy, Davis and Duff's approximate minimum degree; no supervariables).
// Returns perm: new -> old.
// ---------------------------------------------------------------------------
std::vector<int32_t> min_degree_order(int n, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj) {
  std::vector<int32_t> perm;
  perm.reserve(n);
  if (n == 0) return perm;
  std::vector<std::vector<int32_t>> vadj(n), eadj(n), elem(n);
  std::vector<int32_t> deg(n), esize(n, 0);
  std::vector<char> state(n, 0);  // 0 variable, 1 element (alive), 2 dead element
  for (int i = 0; i < n; i++) {
    vadj[i].assign(adj.begin() + xadj[i], adj.begin() + xadj[i + 1]);
    deg[i] = (int32_t)vadj[i].size();
  }
  // degree buckets (doubly linked)
  std::vector<int32_t> head(n + 1, -1), next(n, -1), prev(n, -1);
  auto insert = [&](int i) {
    int d = deg[i];
    next[i] = head[d];
    prev[i] = -1;
    if (head[d] >= 0) prev[head[d]] = i;
    head[d] = i;
  };
  auto remove = [&](int i) {
    int d = deg[i];
    if (prev[i] >= 0) next[prev[i]] = next[i]; else head[d] = next[i];
    if (next[i] >= 0) prev[next[i]] = prev[i];
  };
  for (int i = n - 1; i >= 0; i--) insert(i);
  std::vector<int32_t> mark(n, -1), w(n, -1);
  std::vector<int32_t> Lp;
  int mindeg = 0;
  for (int k = 0; k < n; k++) {
    while (mindeg <= n && head[mindeg] < 0) mindeg++;
    int p = head[mindeg];
    remove(p);
    perm.push_back(p);
    // Lp = adjacent variables plus the variables of adjacent elements
    Lp.clear();
    mark[p] = p;
    for (int v : vadj[p])
      if (state[v] == 0 && mark[v] != p) { mark[v] = p; Lp.push_back(v); }
    for (int e : eadj[p]) {
      if (state[e] != 1) continue;
      for (int v : elem[e])
        if (state[v] == 0 && mark[v] != p) { mark[v] = p; Lp.push_back(v); }
      state[e] = 2;
      std::vector<int32_t>().swap(elem[e]);
    }
    state[p] = 1;
    elem[p] = Lp;
    esize[p] = (int32_t)Lp.size();
    std::vector<int32_t>().swap(vadj[p]);
    std::vector<int32_t>().swap(eadj[p]);
    const int lsz = (int)Lp.size();
    // |Le \ Lp| for elements adjacent to Lp
    std::vector<int32_t> touched;
    for (int i : Lp) {
      for (int e : eadj[i]) {
        if (state[e] != 1 || e == p) continue;
        if (w[e] < 0) { w[e] = esize[e]; touched.push_back(e); }
        w[e]--;
      }
    }
    const int remaining = n - k - 1;
    for (int i : Lp) {
      remove(i);
      // prune element list, drop elements absorbed by p (Le subset of Lp), add p
      auto& E = eadj[i];
      size_t o = 0;
      int64_t esum = 0;
      for (int e : E) {
        if (state[e] != 1 || e == p) continue;
        if (w[e] == 0) { state[e] = 2; continue; }   // aggressive absorption
        E[o++] = e;
        esum += w[e];
      }
      E.resize(o);
      E.push_back(p);
      // prune variable list: drop variables covered by p's element
      auto& V = vadj[i];
      o = 0;
      for (int v : V)
        if (state[v] == 0 && mark[v] != p && v != i) V[o++] = v;
      V.resize(o);
      int64_t d = (int64_t)V.size() + (lsz - 1) + esum;
      d = std::min<int64_t>(d, (int64_t)deg[i] + lsz - 1);
      d = std::min<int64_t>(d, remaining > 0 ? remaining - 1 : 0);
      if (d < 0) d = 0;
      deg[i] = (int32_t)d;
      insert(i);
      if (d < mindeg) mindeg = (int)d;
    }
    for (int e : touched) w[e] = -1;
  }
  return perm;
}

namespace {

// Column elimination tree of B^T B for columns [b0, b1) of the diagonal block part of R
// (Liu's algorithm with path compression; CSparse's cs_etree, ata variant).
void block_col_etree(int b0, int b1, const std::vector<int32_t>& Rp, const std::vector<int32_t>& Ri,
                     std::vector<int32_t>& parent, std::vector<int32_t>& prev, std::vector<int32_t>& anc,
                     int r0 = -1, int r1 = -1) {
  if (r0 < 0) { r0 = b0; r1 = b1; }
  for (int k = r0; k < r1; k++) prev[k] = -1;
  for (int k = b0; k < b1; k++) {
    parent[k] = -1;
    anc[k] = -1;
    for (int32_t p = Rp[k]; p < Rp[k + 1]; p++) {
      int32_t i = Ri[p];
      if (i < r0 || i >= r1) continue;
      int32_t j = prev[i];
      while (j != -1 && j < k) {
        int32_t jn = anc[j];
        anc[j] = k;
        if (jn == -1) { parent[j] = k; break; }
        j = jn;
      }
      prev[i] = k;
    }
  }
}

// Symmetric adjacency of B+B^T restricted to the index set `nodes` (given in the
// global column numbering via pos_of: global -> local, -1 outside).
void local_graph(const std::vector<int32_t>& nodes, const std::vector<int32_t>& pos_of,
                 const int32_t* Ap, const int32_t* Ai, const std::vector<int32_t>& row_to_node,
                 std::vector<int64_t>& xadj, std::vector<int32_t>& adj) {
  const int m = (int)nodes.size();
  std::vector<std::vector<int32_t>> nb(m);
  for (int a = 0; a < m; a++) {
    int c = nodes[a];
    for (int32_t p = Ap[c]; p < Ap[c + 1]; p++) {
      int r = row_to_node[Ai[p]];
      int b = pos_of[r];
      if (b < 0 || b == a) continue;
      nb[a].push_back(b);
      nb[b].push_back(a);
    }
  }
  xadj.assign(m + 1, 0);
  adj.clear();
  for (int a = 0; a < m; a++) {
    auto& v = nb[a];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    adj.insert(adj.end(), v.begin(), v.end());
    xadj[a + 1] = (int64_t)adj.size();
  }
}

// ---------------------------------------------------------------------------
// Nested dissection of one block (Sec. III-C) by recursive vertex bisection.
// Each bisection: breadth-first level structure from a pseudo-peripheral vertex
// (George and Liu), the smallest level near the middle as the separator, then a
// pass that moves separator vertices touching only one side into that side.
// Disconnected parts are split by whole components with an empty separator.
// ---------------------------------------------------------------------------
struct NdBuild {
  const std::vector<int64_t>& xadj;
  const std::vector<int32_t>& adj;
  std::vector<int32_t> part;    // current subset id per local vertex
  std::vector<int32_t> level;
  std::vector<int32_t> queue;
  int next_id = 1;
};

// BFS inside subset `id` from `src`; returns the last vertex reached and fills level
static int bfs_levels(NdBuild& B, int id, int src, const std::vector<int32_t>& verts, int* nlev) {
  for (int v : verts) B.level[v] = -1;
  B.queue.clear();
  B.queue.push_back(src);
  B.level[src] = 0;
  size_t h = 0;
  int last = src;
  while (h < B.queue.size()) {
    int v = B.queue[h++];
    last = v;
    for (int64_t p = B.xadj[v]; p < B.xadj[v + 1]; p++) {
      int w = B.adj[p];
      if (B.part[w] == id && B.level[w] < 0) { B.level[w] = B.level[v] + 1; B.queue.push_back(w); }
    }
  }
  *nlev = B.level[last] + 1;
  return last;
}

// ---------------------------------------------------------------------------
// Multilevel bisection (the scheme of Karypis and Kumar's METIS, restated):
// coarsen by heavy-edge matching, split the coarsest graph by greedy growing,
// refine with Fiduccia-Mattheyses moves on every level while projecting back, and
// turn the final edge cut into a vertex separator by a minimum vertex cover of the
// cut edges (Koenig's theorem on the bipartite cut graph).
// ---------------------------------------------------------------------------
struct WGraph {
  int n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj, ewgt;
  std::vector<int32_t> vwgt;
};

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// heavy-edge matching; returns the coarse graph and the fine->coarse map
static bool coarsen(const WGraph& g, WGraph& c, std::vector<int32_t>& cmap, uint64_t seed) {
  const int n = g.n;
  std::vector<int32_t> order(n), match(n, -1);
  for (int i = 0; i < n; i++) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    uint64_t ha = mix64(seed ^ (uint64_t)a), hb = mix64(seed ^ (uint64_t)b);
    return ha < hb;
  });
  for (int v : order) {
    if (match[v] >= 0) continue;
    int best = -1, bw = -1;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
      int u = g.adj[p];
      if (match[u] < 0 && u != v && g.ewgt[p] > bw) { bw = g.ewgt[p]; best = u; }
    }
    if (best >= 0) { match[v] = best; match[best] = v; }
    else match[v] = v;
  }
  cmap.assign(n, -1);
  int nc = 0;
  for (int v = 0; v < n; v++) {
    if (cmap[v] >= 0) continue;
    cmap[v] = nc;
    if (match[v] != v) cmap[match[v]] = nc;
    nc++;
  }
  if (nc > (int)(0.95 * n)) return false;
  c.n = nc;
  c.vwgt.assign(nc, 0);
  for (int v = 0; v < n; v++) c.vwgt[cmap[v]] += g.vwgt[v];
  // coarse adjacency with summed edge weights
  std::vector<int32_t> mark(nc, -1), pos(nc, 0);
  std::vector<std::vector<int32_t>> members(nc);
  for (int v = 0; v < n; v++) members[cmap[v]].push_back(v);
  c.xadj.assign(nc + 1, 0);
  c.adj.clear();
  c.ewgt.clear();
  for (int cv = 0; cv < nc; cv++) {
    size_t start = c.adj.size();
    for (int v : members[cv])
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
        int cu = cmap[g.adj[p]];
        if (cu == cv) continue;
        if (mark[cu] != cv) {
          mark[cu] = cv;
          pos[cu] = (int32_t)c.adj.size();
          c.adj.push_back(cu);
          c.ewgt.push_back(g.ewgt[p]);
        } else {
          c.ewgt[pos[cu]] += g.ewgt[p];
        }
      }
    (void)start;
    c.xadj[cv + 1] = (int64_t)c.adj.size();
  }
  return true;
}

// Fiduccia-Mattheyses refinement of a 2-way partition (side 0/1) with balance
// max side weight <= maxw.  Moves are tried greedily by gain; each pass keeps the
// best prefix of moves.
static void fm_refine(const WGraph& g, std::vector<char>& side, int64_t maxw, int passes) {
  const int n = g.n;
  int64_t w[2] = {0, 0};
  for (int v = 0; v < n; v++) w[(int)side[v]] += g.vwgt[v];
  std::vector<int64_t> gain(n);
  std::vector<char> locked(n);
  for (int pass = 0; pass < passes; pass++) {
    for (int v = 0; v < n; v++) {
      int64_t ext = 0, in = 0;
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) (side[g.adj[p]] == side[v] ? in : ext) += g.ewgt[p];
      gain[v] = ext - in;
    }
    std::fill(locked.begin(), locked.end(), 0);
    // boundary-driven priority queue (max gain; ties by vertex id)
    std::vector<std::pair<int64_t, int32_t>> heap;
    auto push = [&](int v) { heap.push_back({gain[v], -v}); std::push_heap(heap.begin(), heap.end()); };
    for (int v = 0; v < n; v++) {
      bool bnd = false;
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1] && !bnd; p++) bnd = side[g.adj[p]] != side[v];
      if (bnd) push(v);
    }
    std::vector<int32_t> moved;
    int64_t cur = 0, best = 0;
    size_t best_len = 0;
    int stall = 0;
    while (!heap.empty() && stall < 200) {
      std::pop_heap(heap.begin(), heap.end());
      auto top = heap.back();
      heap.pop_back();
      int v = -top.second;
      if (locked[v] || top.first != gain[v]) continue;
      int from = side[v], to = 1 - from;
      if (w[to] + g.vwgt[v] > maxw) continue;
      locked[v] = 1;
      side[v] = (char)to;
      w[from] -= g.vwgt[v];
      w[to] += g.vwgt[v];
      cur += gain[v];
      moved.push_back(v);
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
        int u = g.adj[p];
        if (locked[u]) continue;
        gain[u] += (side[u] == to) ? -2 * g.ewgt[p] : 2 * g.ewgt[p];
        push(u);
      }
      if (cur > best) { best = cur; best_len = moved.size(); stall = 0; }
      else stall++;
    }
    // undo the moves after the best prefix
    for (size_t i = moved.size(); i > best_len; i--) {
      int v = moved[i - 1];
      int from = side[v], to = 1 - from;
      side[v] = (char)to;
      w[from] -= g.vwgt[v];
      w[to] += g.vwgt[v];
    }
    if (best <= 0) break;
  }
}

// Greedy growing from a seed: add the frontier vertex with the largest gain until
// half of the weight is on side 0.
static void grow_partition(const WGraph& g, int seed, std::vector<char>& side) {
  const int n = g.n;
  int64_t total = 0;
  for (int v = 0; v < n; v++) total += g.vwgt[v];
  side.assign(n, 1);
  std::vector<int64_t> conn(n, 0);
  std::vector<std::pair<int64_t, int32_t>> heap;
  int64_t w0 = 0;
  auto add = [&](int v) {
    side[v] = 0;
    w0 += g.vwgt[v];
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++) {
      int u = g.adj[p];
      if (side[u] == 1) { conn[u] += g.ewgt[p]; heap.push_back({conn[u], -u}); std::push_heap(heap.begin(), heap.end()); }
    }
  };
  add(seed);
  while (w0 * 2 < total) {
    int v = -1;
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end());
      auto t = heap.back();
      heap.pop_back();
      if (side[-t.second] == 1 && t.first == conn[-t.second]) { v = -t.second; break; }
    }
    if (v < 0) {  // disconnected remainder: take any vertex
      for (int u = 0; u < n; u++) if (side[u] == 1) { v = u; break; }
      if (v < 0) break;
    }
    add(v);
  }
}

static int64_t cut_weight(const WGraph& g, const std::vector<char>& side) {
  int64_t c = 0;
  for (int v = 0; v < g.n; v++)
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; p++)
      if (side[g.adj[p]] != side[v]) c += g.ewgt[p];
  return c / 2;
}

// 2-way edge partition of g by the multilevel scheme
static void multilevel_bisect(const WGraph& g0, std::vector<char>& side, uint64_t seed) {
  std::vector<WGraph> levels;
  std::vector<std::vector<int32_t>> maps;
  levels.push_back(g0);
  while (levels.back().n > 120) {
    WGraph c;
    std::vector<int32_t> cmap;
    if (!coarsen(levels.back(), c, cmap, seed + levels.size())) break;
    maps.push_back(std::move(cmap));
    levels.push_back(std::move(c));
  }
  const WGraph& gc = levels.back();
  int64_t total = 0;
  for (int v = 0; v < gc.n; v++) total += gc.vwgt[v];
  const double imb = 1.05;
  int64_t maxw = (int64_t)(imb * (double)total / 2.0) + 1;
  // best of a few growing seeds at the coarsest level
  std::vector<char> best_side;
  int64_t best_cut = INT64_MAX;
  const int tries = std::min(gc.n, 8);
  for (int t = 0; t < tries; t++) {
    int s0 = (int)(mix64(seed * 31 + t) % (uint64_t)gc.n);
    std::vector<char> sd;
    grow_partition(gc, s0, sd);
    fm_refine(gc, sd, maxw, 4);
    int64_t c = cut_weight(gc, sd);
    if (c < best_cut) { best_cut = c; best_side = sd; }
  }
  side = best_side;
  for (int l = (int)levels.size() - 2; l >= 0; l--) {
    const WGraph& g = levels[l];
    std::vector<char> fine(g.n);
    for (int v = 0; v < g.n; v++) fine[v] = side[maps[l][v]];
    side.swap(fine);
    int64_t tw = 0;
    for (int v = 0; v < g.n; v++) tw += g.vwgt[v];
    fm_refine(g, side, (int64_t)(imb * (double)tw / 2.0) + 1, 3);
  }
}

// minimum vertex cover of the bipartite graph of cut edges (left = side 0)
static void cut_vertex_cover(const WGraph& g, const std::vector<char>& side, std::vector<char>& in_sep) {
  const int n = g.n;
  in_sep.assign(n, 0);
  std::vector<int32_t> mate(n, -1);
  // augmenting paths from every left boundary vertex (Kuhn's algorithm)
  std::vector<int32_t> seen(n, -1), stack, from_edge;
  std::vector<int64_t> it(n);
  for (int v = 0; v < n; v++) {
    if (side[v] != 0) continue;
    bool bnd = false;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1] && !bnd; p++) bnd = side[g.adj[p]] == 1;
    if (!bnd) continue;
    // DFS over alternating paths: left u -> right w (cut edge) -> left mate[w]
    stack.assign(1, v);
    it[v] = g.xadj[v];
    seen[v] = v;
    std::vector<int32_t> via;  // right vertex used to reach each stacked left vertex
    via.assign(1, -1);
    bool found = false;
    while (!stack.empty() && !found) {
      int u = stack.back();
      bool pushed = false;
      while (it[u] < g.xadj[u + 1]) {
        int w = g.adj[it[u]++];
        if (side[w] != 1) continue;
        if (mate[w] < 0) {
          // augment along the stack
          int r = w;
          for (int h = (int)stack.size() - 1; h >= 0; h--) {
            int l = stack[h];
            int prev = mate[l];
            mate[l] = r;
            mate[r] = l;
            r = prev;
          }
          found = true;
          break;
        }
        int l2 = mate[w];
        if (seen[l2] != v) {
          seen[l2] = v;
          it[l2] = g.xadj[l2];
          stack.push_back(l2);
          via.push_back(w);
          pushed = true;
          break;
        }
      }
      if (!found && !pushed) { stack.pop_back(); via.pop_back(); }
    }
  }
  // Koenig: Z = vertices reachable from unmatched left boundary vertices by alternating paths
  std::vector<char> inZ(n, 0);
  std::vector<int32_t> q;
  for (int v = 0; v < n; v++) {
    if (side[v] != 0 || mate[v] >= 0) continue;
    bool bnd = false;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1] && !bnd; p++) bnd = side[g.adj[p]] == 1;
    if (bnd) { inZ[v] = 1; q.push_back(v); }
  }
  for (size_t h = 0; h < q.size(); h++) {
    int u = q[h];
    for (int64_t p = g.xadj[u]; p < g.xadj[u + 1]; p++) {
      int w = g.adj[p];
      if (side[w] != 1 || inZ[w]) continue;
      inZ[w] = 1;
      int l = mate[w];
      if (l >= 0 && !inZ[l]) { inZ[l] = 1; q.push_back(l); }
    }
  }
  for (int v = 0; v < n; v++) {
    bool bnd = false;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1] && !bnd; p++) bnd = side[g.adj[p]] != side[v];
    if (!bnd) continue;
    if (side[v] == 0 && !inZ[v]) in_sep[v] = 1;
    if (side[v] == 1 && inZ[v]) in_sep[v] = 1;
  }
}

// split `verts` (subset id) into (left, right, sep)
static void bisect(NdBuild& B, int id, const std::vector<int32_t>& verts, std::vector<int32_t>& left,
                   std::vector<int32_t>& right, std::vector<int32_t>& sep) {
  left.clear(); right.clear(); sep.clear();
  const int m = (int)verts.size();
  if (m == 0) return;
  // induced subgraph with unit weights
  WGraph g;
  g.n = m;
  g.vwgt.assign(m, 1);
  g.xadj.assign(m + 1, 0);
  std::vector<int32_t> loc(0);
  for (int a = 0; a < m; a++) B.level[verts[a]] = a;   // reuse level[] as local index
  for (int a = 0; a < m; a++) {
    int v = verts[a];
    for (int64_t p = B.xadj[v]; p < B.xadj[v + 1]; p++) {
      int u = B.adj[p];
      if (B.part[u] == id) { g.adj.push_back(B.level[u]); g.ewgt.push_back(1); }
    }
    g.xadj[a + 1] = (int64_t)g.adj.size();
  }
  std::vector<char> side;
  multilevel_bisect(g, side, 0x5EED0000ull + (uint64_t)m);
  std::vector<char> in_sep;
  cut_vertex_cover(g, side, in_sep);
  for (int a = 0; a < m; a++) {
    int v = verts[a];
    if (in_sep[a]) sep.push_back(v);
    else (side[a] == 0 ? left : right).push_back(v);
  }
}

// Recursive ND: appends the tree nodes in postorder (left, right, separator) and the
// vertex order.  Returns the node index of this subtree's root.
static int nd_recurse(NdBuild& B, std::vector<int32_t>& verts, int depth, int max_depth,
                      std::vector<std::vector<int32_t>>& node_verts, std::vector<int32_t>& node_parent,
                      std::vector<int32_t>& node_level, std::vector<char>& node_leaf) {
  if (depth == max_depth || verts.size() < 4) {
    int idx = (int)node_verts.size();
    node_verts.push_back(verts);
    node_parent.push_back(-1);
    node_level.push_back(0);
    node_leaf.push_back(1);
    return idx;
  }
  const int id = B.part[verts[0]];
  std::vector<int32_t> left, right, sep;
  bisect(B, id, verts, left, right, sep);
  const int idL = B.next_id++, idR = B.next_id++;
  for (int v : left) B.part[v] = idL;
  for (int v : right) B.part[v] = idR;
  for (int v : sep) B.part[v] = -1;
  int cl = nd_recurse(B, left, depth + 1, max_depth, node_verts, node_parent, node_level, node_leaf);
  int cr = nd_recurse(B, right, depth + 1, max_depth, node_verts, node_parent, node_level, node_leaf);
  int idx = (int)node_verts.size();
  node_verts.push_back(sep);
  node_parent.push_back(-1);
  node_level.push_back(std::max(node_level[cl], node_level[cr]) + 1);
  node_leaf.push_back(0);
  node_parent[cl] = idx;
  node_parent[cr] = idx;
  return idx;
}

// R's diagonal-block and off-diagonal-block parts from the final permutations.
int assemble_R(int n, const int32_t* Ap, const int32_t* Ai, Plan& P) {
  std::vector<int32_t> blk(n);
  for (size_t b = 0; b + 1 < P.blkptr.size(); b++)
    for (int k = P.blkptr[b]; k < P.blkptr[b + 1]; k++) blk[k] = (int32_t)b;
  P.Rp.assign(n + 1, 0);
  P.Op.assign(n + 1, 0);
  P.Ri.clear(); P.Rmap.clear(); P.Oi.clear(); P.Omap.clear();
  std::vector<std::pair<int32_t, int32_t>> tmp;
  for (int k = 0; k < n; k++) {
    int c = P.qcol[k];
    tmp.clear();
    for (int32_t p = Ap[c]; p < Ap[c + 1]; p++) tmp.push_back({P.pinvrow[Ai[p]], p});
    std::sort(tmp.begin(), tmp.end());
    for (auto& t : tmp) {
      int i = t.first;
      if (blk[i] == blk[k]) { P.Ri.push_back(i); P.Rmap.push_back(t.second); }
      else if (blk[i] < blk[k]) { P.Oi.push_back(i); P.Omap.push_back(t.second); }
      else { P.error = "entry below the diagonal blocks (not block upper triangular)"; return -1; }
    }
    P.Rp[k + 1] = (int32_t)P.Ri.size();
    P.Op[k + 1] = (int32_t)P.Oi.size();
  }
  return 0;
}

// Dependency forest, depths and the initial ready list (deepest first).
void finish_schedule(Plan& P) {
  const int n = P.n;
  P.nchild.assign(n, 0);
  P.depth.assign(n, 0);
  for (int k = 0; k < n; k++)
    if (P.parent[k] >= 0) P.nchild[P.parent[k]]++;
  int md = 0;
  for (int k = n - 1; k >= 0; k--) {
    P.depth[k] = P.parent[k] < 0 ? 0 : P.depth[P.parent[k]] + 1;
    md = std::max(md, P.depth[k]);
  }
  P.max_depth = md;
  P.ready.clear();
  for (int k = 0; k < n; k++)
    if (P.nchild[k] == 0) P.ready.push_back(k);
  std::stable_sort(P.ready.begin(), P.ready.end(),
                   [&](int a, int b) { return P.depth[a] > P.depth[b]; });
  P.col_grp.assign(n, 0);
  for (size_t g = 0; g + 1 < P.grpptr.size(); g++)
    for (int k = P.grpptr[g]; k < P.grpptr[g + 1]; k++) P.col_grp[k] = (int32_t)g;
}

// Level lists of the factor segments (largest first inside a level) and of the
// solve's block back-substitution: block b reads the solution of the later blocks its
// off-diagonal entries touch, so level(b) = 1 + max level of those blocks.
// Tasks of the block back-substitution.  R is block upper triangular, so block b can
// start once every later block it couples to is solved.  A block without an ND tree
// is one task (residual, L sweep, U sweep).  A block with an ND tree is split per
// node: forward tasks from the leaves up (a node's L columns reach only its own rows
// and its ancestors' rows; the latter go to a per-node buffer that the ancestors
// add in a fixed order), then backward tasks from the root down (a node pulls the
// products of its rows of the ancestors' U columns with the ancestors' solution).
// A task's level is one more than the highest level of the tasks it waits for.
void build_solve_tasks(Plan& P) {
  const int n = P.n;
  const int nb = (int)P.blkptr.size() - 1;
  const int ng = (int)P.grpptr.size() - 1;
  std::vector<int32_t> blk(n);
  for (int b = 0; b < nb; b++)
    for (int k = P.blkptr[b]; k < P.blkptr[b + 1]; k++) blk[k] = b;
  std::vector<int32_t> gfirst(nb + 1, 0);   // first group of every block
  {
    int g = 0;
    for (int b = 0; b <= nb; b++) {
      while (g < ng && P.grpptr[g] < (b < nb ? P.blkptr[b] : n)) g++;
      gfirst[b] = g;
    }
  }
  std::vector<char> is_nd(nb, 0);
  if (!P.grp_parent.empty())
    for (int b = 0; b < nb; b++)
      for (int g = gfirst[b]; g < gfirst[b + 1]; g++)
        if (P.grp_parent[g] >= 0) { is_nd[b] = 1; break; }
  // group tree data: first descendant, ancestors (root first), ancestor row offsets
  P.sg_fd.assign(ng, 0);
  P.sg_choff.assign(ng, 0);
  P.sg_tbase.assign(ng, 0);
  P.sg_anc_ptr.assign(1, 0);
  P.sg_anc.clear();
  P.s_rowpos.assign(n, -1);
  int64_t tb = 0;
  for (int g = 0; g < ng; g++) P.sg_fd[g] = g;
  for (int b = 0; b < nb; b++) {
    for (int g = gfirst[b]; g < gfirst[b + 1]; g++) {
      if (is_nd[b] && P.grp_parent[g] >= 0) {
        const int p = P.grp_parent[g];
        P.sg_fd[p] = std::min(P.sg_fd[p], P.sg_fd[g]);
      }
    }
  }
  for (int g = 0; g < ng; g++) {
    std::vector<int32_t> chain;
    int b = blk[P.grpptr[g]];
    if (is_nd[b])
      for (int a = P.grp_parent[g]; a >= 0; a = P.grp_parent[a]) chain.push_back(a);
    int64_t off = 0;
    for (int t = (int)chain.size() - 1; t >= 0; t--) {
      P.sg_anc.push_back(chain[t]);
      off += P.grpptr[chain[t] + 1] - P.grpptr[chain[t]];
    }
    P.sg_anc_ptr.push_back((int32_t)P.sg_anc.size());
    P.sg_choff[g] = (int32_t)off;
    if (is_nd[b]) {
      P.sg_tbase[g] = tb;
      tb += (P.grpptr[g + 1] - P.grpptr[g]) + off;
      // a row's position in the ancestor-row buffer of any descendant of its group
      for (int r = P.grpptr[g]; r < P.grpptr[g + 1]; r++) P.s_rowpos[r] = (int32_t)off + (r - P.grpptr[g]);
    }
  }
  P.s_gbuf_total = tb;
  // levels
  std::vector<int32_t> base(nb, 0), done(nb, 0);
  std::vector<int32_t> kind, id, lev;
  std::vector<int32_t> fwd(ng, 0), bwd(ng, 0);
  for (int c = nb - 1; c >= 0; c--) {
    if (!is_nd[c]) {
      kind.push_back(0); id.push_back(c); lev.push_back(base[c]);
      done[c] = base[c];
    } else {
      int mx = base[c];
      for (int g = gfirst[c]; g < gfirst[c + 1]; g++) fwd[g] = base[c];
      for (int g = gfirst[c]; g < gfirst[c + 1]; g++) {   // postorder: children first
        kind.push_back(1); id.push_back(g); lev.push_back(fwd[g]);
        const int p = P.grp_parent[g];
        if (p >= 0) fwd[p] = std::max(fwd[p], fwd[g] + 1);
      }
      for (int g = gfirst[c + 1] - 1; g >= gfirst[c]; g--) {  // parents first
        const int p = P.grp_parent[g];
        bwd[g] = (p >= 0 ? bwd[p] : fwd[g]) + 1;
        kind.push_back(2); id.push_back(g); lev.push_back(bwd[g]);
        mx = std::max(mx, bwd[g]);
      }
      done[c] = mx;
    }
    for (int k = P.blkptr[c]; k < P.blkptr[c + 1]; k++)
      for (int32_t q = P.Op[k]; q < P.Op[k + 1]; q++) {
        const int b = blk[P.Oi[q]];
        base[b] = std::max(base[b], done[c] + 1);
      }
  }
  int nlev = 0;
  for (int32_t l : lev) nlev = std::max(nlev, l + 1);
  const int nt = (int)kind.size();
  P.st_lvl_ptr.assign(nlev + 1, 0);
  for (int t = 0; t < nt; t++) P.st_lvl_ptr[lev[t] + 1]++;
  for (int l = 0; l < nlev; l++) P.st_lvl_ptr[l + 1] += P.st_lvl_ptr[l];
  std::vector<int32_t> order(nt);
  {
    std::vector<int32_t> fp(P.st_lvl_ptr.begin(), P.st_lvl_ptr.end() - 1);
    for (int t = 0; t < nt; t++) order[fp[lev[t]]++] = t;
  }
  auto tsize = [&](int t) {
    return kind[t] == 0 ? P.blkptr[id[t] + 1] - P.blkptr[id[t]] : P.grpptr[id[t] + 1] - P.grpptr[id[t]];
  };
  for (int l = 0; l < nlev; l++)
    std::stable_sort(order.begin() + P.st_lvl_ptr[l], order.begin() + P.st_lvl_ptr[l + 1],
                     [&](int x, int y) { return tsize(x) > tsize(y); });
  P.st_kind.resize(nt); P.st_id.resize(nt); P.st_need.resize(nt);
  std::vector<int32_t> pos0(nb, -1), pos1(ng, -1), pos2(ng, -1);
  for (int q = 0; q < nt; q++) {
    const int t = order[q];
    P.st_kind[q] = kind[t];
    P.st_id[q] = id[t];
    const int m = tsize(t);
    // doubles of work storage: the task's rows
    P.st_need[q] = m;
    (kind[t] == 0 ? pos0[id[t]] : kind[t] == 1 ? pos1[id[t]] : pos2[id[t]]) = q;
  }
  // Flagged predecessors of every task (queue positions, all earlier in the queue): an
  // ND node's forward tasks of its children, and for a backward task its own forward
  // task and its parent's backward task.  The solution entries a residual reads through
  // the off-diagonal blocks are waited for one by one on the device, not through their
  // tasks' flags; their tasks (a whole block's, or the backward task of the ND node
  // holding the column) are still earlier in the queue, since the levels above count
  // those couplings.
  std::vector<std::vector<int32_t>> pred(nt);
  for (int g = 0; g < ng; g++) {
    if (pos1[g] < 0) continue;
    const int p = P.grp_parent[g];
    if (p >= 0) pred[pos1[p]].push_back(pos1[g]);
    pred[pos2[g]].push_back(pos1[g]);
    if (p >= 0) pred[pos2[g]].push_back(pos2[p]);
  }
  P.st_dep_ptr.assign(nt + 1, 0);
  P.st_dep.clear();
  P.st_succ.assign(nt, 0);
  for (int q = 0; q < nt; q++) {
    std::vector<int32_t>& v = pred[q];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    for (int32_t d : v) P.st_succ[d] = 1;
    P.st_dep.insert(P.st_dep.end(), v.begin(), v.end());
    P.st_dep_ptr[q + 1] = (int32_t)P.st_dep.size();
  }
  // Issue order of the one-launch solve: longest remaining path first.  A task's bottom
  // level is its weight (rows plus a fixed start cost) plus the largest bottom level of
  // the tasks that wait for it, through a flag or through a coupled solution entry (the
  // producer of the entry: a block's task, or the ND node's backward task).  Every
  // predecessor has a strictly larger bottom level, so the descending sort is a
  // topological order.
  std::vector<int32_t> cgrp(n, -1);
  for (int g = 0; g < ng; g++)
    for (int k = P.grpptr[g]; k < P.grpptr[g + 1]; k++) cgrp[k] = g;
  auto producer = [&](int k) { return is_nd[blk[k]] ? pos2[cgrp[k]] : pos0[blk[k]]; };
  auto owner = [&](int i) { return is_nd[blk[i]] ? pos1[cgrp[i]] : pos0[blk[i]]; };
  std::vector<std::vector<int32_t>> succ(nt);
  for (int q = 0; q < nt; q++)
    for (int e = P.st_dep_ptr[q]; e < P.st_dep_ptr[q + 1]; e++) succ[P.st_dep[e]].push_back(q);
  for (int k = 0; k < n; k++)
    for (int32_t e = P.Op[k]; e < P.Op[k + 1]; e++) succ[producer(k)].push_back(owner(P.Oi[e]));
  std::vector<int64_t> bl(nt, 0);
  for (int q = nt - 1; q >= 0; q--) {
    int64_t mx = 0;
    for (int32_t s2 : succ[q]) mx = std::max(mx, bl[s2]);
    bl[q] = mx + P.st_need[q] + 16;
  }
  P.st_issue.resize(nt);
  for (int q = 0; q < nt; q++) P.st_issue[q] = q;
  std::stable_sort(P.st_issue.begin(), P.st_issue.end(), [&](int32_t x, int32_t y) { return bl[x] > bl[y]; });
}

void build_levels(Plan& P) {
  const int ns = (int)P.seg_c0.size();
  const int kDenseSepMin = 16;
  int nl = 0;
  for (int s = 0; s < ns; s++) nl = std::max(nl, P.seg_level[s] + 1);
  // dense separators: level >= 1 segments of at least kDenseSepMin columns
  std::vector<char> dense(ns, 0);
  for (int s = 0; s < ns; s++) {
    if (P.seg_level[s] < 1 || P.seg_c1[s] - P.seg_c0[s] < kDenseSepMin || P.seg_grp.empty() || P.seg_grp[s] < 0)
      continue;
    int64_t H = 0;
    for (int g = P.seg_grp[s]; g >= 0; g = P.grp_parent[g]) H += P.grpptr[g + 1] - P.grpptr[g];
    if (H <= 11264) dense[s] = 1;   // panel rows fit the dense kernel's row bitmaps (176 words)
  }
  P.lvl_ptr.assign(nl + 1, 0);
  for (int s = 0; s < ns; s++) P.lvl_ptr[P.seg_level[s] + 1]++;
  for (int l = 0; l < nl; l++) P.lvl_ptr[l + 1] += P.lvl_ptr[l];
  P.lvl_seg.assign(ns, 0);
  {
    std::vector<int32_t> fp(P.lvl_ptr.begin(), P.lvl_ptr.end() - 1);
    for (int s = 0; s < ns; s++) P.lvl_seg[fp[P.seg_level[s]]++] = s;
  }
  P.crit_cols = 0;
  for (int l = 0; l < nl; l++) {
    auto b = P.lvl_seg.begin() + P.lvl_ptr[l], e = P.lvl_seg.begin() + P.lvl_ptr[l + 1];
    // dense separators first, then largest first
    std::stable_sort(b, e, [&](int x, int y) {
      if (dense[x] != dense[y]) return dense[x] > dense[y];
      return P.seg_c1[x] - P.seg_c0[x] > P.seg_c1[y] - P.seg_c0[y];
    });
    int mx = 0;
    for (auto it = b; it != e; ++it) mx = std::max(mx, P.seg_c1[*it] - P.seg_c0[*it]);
    P.crit_cols += mx;
  }
  // work items over the non-dense segments of every level: item i covers
  // lvl_seg[item_lo[i] .. item_hi[i]).  First-level segments are gathered up to
  // kItemCols columns an item; a separator (level >= 1) is an item of its own, since its
  // columns each take a long reach and the separators of a level are independent.
  const int kItemCols = 64;
  P.item_lo.clear();
  P.item_hi.clear();
  P.lvl_item_ptr.assign(1, 0);
  for (int l = 0; l < nl; l++) {
    int q0 = P.lvl_ptr[l];
    while (q0 < P.lvl_ptr[l + 1] && dense[P.lvl_seg[q0]]) q0++;
    int start = q0, acc = 0;
    const int cap = l == 0 ? kItemCols : 1;
    for (int q = q0; q < P.lvl_ptr[l + 1]; q++) {
      const int sz = P.seg_c1[P.lvl_seg[q]] - P.seg_c0[P.lvl_seg[q]];
      if (acc > 0 && (acc >= cap || sz >= cap)) {
        P.item_lo.push_back(start); P.item_hi.push_back(q);
        start = q;
        acc = 0;
      }
      acc += sz;
    }
    if (P.lvl_ptr[l + 1] > start) { P.item_lo.push_back(start); P.item_hi.push_back(P.lvl_ptr[l + 1]); }
    P.lvl_item_ptr.push_back((int32_t)P.item_lo.size());
  }
  // columns per level, dense separators' columns first
  P.lvl_col.clear();
  P.lvl_col_ptr.assign(1, 0);
  P.lvl_dcol_cnt.assign(nl, 0);
  for (int l = 0; l < nl; l++) {
    for (int q = P.lvl_ptr[l]; q < P.lvl_ptr[l + 1]; q++) {
      const int sg = P.lvl_seg[q];
      if (dense[sg]) P.lvl_dcol_cnt[l] += P.seg_c1[sg] - P.seg_c0[sg];
      for (int k = P.seg_c0[sg]; k < P.seg_c1[sg]; k++) P.lvl_col.push_back(k);
    }
    P.lvl_col_ptr.push_back((int32_t)P.lvl_col.size());
  }
  // dense separator panels: own rows, then each ancestor separator's rows
  P.dsep_seg.clear(); P.dsep_H.clear(); P.dsep_rng_g0.clear(); P.dsep_rng_len.clear(); P.dsep_rng_loc.clear();
  P.dsep_rng_ptr.assign(1, 0);
  P.dsep_poff.clear(); P.dsep_soff.clear();
  P.lvl_dsep_ptr.assign(1, 0);
  P.dsep_panel_total = 0;
  P.dsep_bits_total = 0;
  for (int l = 0; l < nl; l++) {
    for (int q = P.lvl_ptr[l]; q < P.lvl_ptr[l + 1]; q++) {
      const int sg = P.lvl_seg[q];
      if (!dense[sg]) continue;
      const int m = P.seg_c1[sg] - P.seg_c0[sg];
      int H = 0;
      for (int g = P.seg_grp.empty() ? -1 : P.seg_grp[sg]; g >= 0; g = P.grp_parent.empty() ? -1 : P.grp_parent[g]) {
        P.dsep_rng_g0.push_back(P.grpptr[g]);
        P.dsep_rng_len.push_back(P.grpptr[g + 1] - P.grpptr[g]);
        P.dsep_rng_loc.push_back(H);
        H += P.grpptr[g + 1] - P.grpptr[g];
      }
      P.dsep_rng_ptr.push_back((int32_t)P.dsep_rng_g0.size());
      P.dsep_seg.push_back(sg);
      P.dsep_H.push_back(H);
      P.dsep_poff.push_back(P.dsep_panel_total);
      P.dsep_soff.push_back(P.dsep_bits_total);
      P.dsep_panel_total += (int64_t)H * m;
      P.dsep_bits_total += (int64_t)((H + 63) / 64) * m;
    }
    P.lvl_dsep_ptr.push_back((int32_t)P.dsep_seg.size());
  }
  build_solve_tasks(P);
}

}  // namespace

int build_plan(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax,
               const SymbolicOptions& opt, Plan& P) {
  P = Plan();
  P.n = n;
  if (!validate_csc(n, Ap, Ai, P.error)) return -1;
  P.nnz = Ap[n];
  // 1. matching: row_of_col[j] = row of A placed on the diagonal at column j
  std::vector<int32_t> row_of_col;
  if (opt.matching) {
    P.struct_rank = bottleneck_matching(n, Ap, Ai, Ax, row_of_col, &P.bottleneck);
  } else {
    row_of_col.assign(n, -1);
    P.struct_rank = max_matching(n, Ap, Ai, nullptr, 0.0, row_of_col);
  }
  if (P.struct_rank < n) { P.error = "structurally singular"; return -2; }
  // 2. BTF: strongly connected components
  std::vector<int32_t> perm0, blk0;
  if (opt.btf) {
    scc_order(n, Ap, Ai, row_of_col.data(), perm0, blk0);
  } else {
    perm0.resize(n);
    std::iota(perm0.begin(), perm0.end(), 0);
    blk0 = {0, n};
  }
  // 3. order every block; node space = column index c of A (row partner row_of_col[c])
  std::vector<int32_t> row_to_node(n);
  for (int c = 0; c < n; c++) row_to_node[row_of_col[c]] = c;
  std::vector<int32_t> pos_of(n, -1);
  std::vector<int32_t> final_perm;
  final_perm.reserve(n);
  P.blkptr.assign(1, 0);
  P.grpptr.assign(1, 0);
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  struct NdBlockInfo { int b; std::vector<int32_t> node_size, node_parent, node_level; std::vector<char> node_leaf; };
  std::vector<NdBlockInfo> ndinfo;
  for (size_t b = 0; b + 1 < blk0.size(); b++) {
    int s0 = blk0[b], s1 = blk0[b + 1], sz = s1 - s0;
    std::vector<int32_t> nodes(perm0.begin() + s0, perm0.begin() + s1);
    if (opt.nd_leaves > 1 && sz >= opt.nd_min_block) {
      // nested dissection with opt.nd_leaves leaves; every tree node becomes a group
      for (int a = 0; a < sz; a++) pos_of[nodes[a]] = a;
      local_graph(nodes, pos_of, Ap, Ai, row_to_node, xadj, adj);
      for (int a = 0; a < sz; a++) pos_of[nodes[a]] = -1;
      NdBuild B{xadj, adj, std::vector<int32_t>(sz, 0), std::vector<int32_t>(sz, -1), {}, 1};
      std::vector<int32_t> all(sz);
      std::iota(all.begin(), all.end(), 0);
      int levels = 0;
      while ((1 << levels) < opt.nd_leaves) levels++;
      std::vector<std::vector<int32_t>> nv;
      std::vector<int32_t> npar, nlev;
      std::vector<char> nleaf;
      nd_recurse(B, all, 0, levels, nv, npar, nlev, nleaf);
      NdBlockInfo info;
      info.b = (int)P.blkptr.size() - 1;
      std::vector<int32_t> sub_pos(sz, -1);
      for (size_t t = 0; t < nv.size(); t++) {
        auto& vs = nv[t];
        std::vector<int32_t> order_local = vs;
        if (opt.fill_order && vs.size() > 2) {
          // minimum degree on the node's induced subgraph
          std::vector<int32_t> gnodes(vs.size());
          for (size_t a = 0; a < vs.size(); a++) { gnodes[a] = nodes[vs[a]]; pos_of[gnodes[a]] = (int32_t)a; }
          std::vector<int64_t> sx;
          std::vector<int32_t> sa;
          local_graph(gnodes, pos_of, Ap, Ai, row_to_node, sx, sa);
          for (size_t a = 0; a < vs.size(); a++) pos_of[gnodes[a]] = -1;
          std::vector<int32_t> lp = min_degree_order((int)vs.size(), sx, sa);
          for (size_t a = 0; a < vs.size(); a++) order_local[a] = vs[lp[a]];
        }
        for (int v : order_local) final_perm.push_back(nodes[v]);
        if (!vs.empty()) P.grpptr.push_back((int32_t)final_perm.size());
        info.node_size.push_back((int32_t)vs.size());
        info.node_parent.push_back(npar[t]);
        info.node_leaf.push_back(nleaf[t]);
        info.node_level.push_back(nlev[t]);
      }
      ndinfo.push_back(std::move(info));
      P.n_nd_blocks++;
      P.blkptr.push_back((int32_t)final_perm.size());
      continue;
    }
    if (opt.fill_order && sz > 2) {
      for (int a = 0; a < sz; a++) pos_of[nodes[a]] = a;
      local_graph(nodes, pos_of, Ap, Ai, row_to_node, xadj, adj);
      std::vector<int32_t> lp = min_degree_order(sz, xadj, adj);
      for (int a = 0; a < sz; a++) pos_of[nodes[a]] = -1;
      for (int a = 0; a < sz; a++) final_perm.push_back(nodes[lp[a]]);
    } else {
      final_perm.insert(final_perm.end(), nodes.begin(), nodes.end());
    }
    P.blkptr.push_back((int32_t)final_perm.size());
    P.grpptr.push_back((int32_t)final_perm.size());
  }
  // 4. compose: R(k, l) = A(row_of_col[perm[k]], perm[l])
  P.prow.resize(n);
  P.qcol.resize(n);
  P.pinvrow.resize(n);
  for (int k = 0; k < n; k++) {
    P.qcol[k] = final_perm[k];
    P.prow[k] = row_of_col[final_perm[k]];
  }
  for (int k = 0; k < n; k++) P.pinvrow[P.prow[k]] = k;
  if (assemble_R(n, Ap, Ai, P) != 0) return -1;
  // 5. schedule.  Plain blocks: the column elimination tree of the block (George and
  // Ng: it bounds the dependencies of partial pivoting for any pivot sequence).  ND
  // blocks: pivots stay inside each node, so a leaf depends only on itself (the
  // column elimination tree of its own rows and columns), a separator's columns form
  // a chain, and every node's exit columns feed the first column of its nearest
  // non-empty ancestor.
  P.parent.assign(n, -1);
  std::vector<int32_t> prev(n), anc(n);
  std::vector<char> is_nd(P.blkptr.size(), 0);
  for (auto& info : ndinfo) is_nd[info.b] = 1;
  for (size_t b = 0; b + 1 < P.blkptr.size(); b++)
    if (!is_nd[b]) block_col_etree(P.blkptr[b], P.blkptr[b + 1], P.Rp, P.Ri, P.parent, prev, anc);
  for (auto& info : ndinfo) {
    const int nn = (int)info.node_size.size();
    std::vector<int32_t> c0(nn), c1(nn);
    int c = P.blkptr[info.b];
    for (int t = 0; t < nn; t++) { c0[t] = c; c += info.node_size[t]; c1[t] = c; }
    auto target_of = [&](int t) {
      int u = info.node_parent[t];
      while (u >= 0 && info.node_size[u] == 0) u = info.node_parent[u];
      return u < 0 ? -1 : c0[u];
    };
    for (int t = 0; t < nn; t++) {
      if (info.node_size[t] == 0) continue;
      const int tgt = target_of(t);
      if (info.node_leaf[t]) {
        block_col_etree(c0[t], c1[t], P.Rp, P.Ri, P.parent, prev, anc, c0[t], c1[t]);
        for (int k = c0[t]; k < c1[t]; k++)
          if (P.parent[k] < 0) P.parent[k] = tgt;
      } else {
        for (int k = c0[t]; k + 1 < c1[t]; k++) P.parent[k] = k + 1;
        P.parent[c1[t] - 1] = tgt;
      }
      NdNode nd;
      nd.g0 = c0[t]; nd.g1 = c1[t]; nd.parent = info.node_parent[t]; nd.level = 0; nd.leaf = info.node_leaf[t];
      P.nd_nodes.push_back(nd);
    }
  }
  finish_schedule(P);
  // ND tree over groups
  P.grp_parent.assign(P.grpptr.size() - 1, -1);
  for (auto& info : ndinfo) {
    const int nn = (int)info.node_size.size();
    std::vector<int32_t> c0(nn);
    int c = P.blkptr[info.b];
    for (int t = 0; t < nn; t++) { c0[t] = c; c += info.node_size[t]; }
    auto group_at = [&](int col) {
      return (int32_t)(std::upper_bound(P.grpptr.begin(), P.grpptr.end(), col) - P.grpptr.begin() - 1);
    };
    for (int t = 0; t < nn; t++) {
      if (info.node_size[t] == 0) continue;
      int u = info.node_parent[t];
      while (u >= 0 && info.node_size[u] == 0) u = info.node_parent[u];
      if (u >= 0) P.grp_parent[group_at(c0[t])] = group_at(c0[u]);
    }
  }
  // segments and levels
  {
    auto group_of = [&](int col) {
      return (int32_t)(std::upper_bound(P.grpptr.begin(), P.grpptr.end(), col) - P.grpptr.begin() - 1);
    };
    std::vector<int32_t> seg_of_block_level;  // level per segment
    std::vector<char> is_nd_b(P.blkptr.size(), 0);
    std::vector<const NdBlockInfo*> info_of(P.blkptr.size(), nullptr);
    for (auto& info : ndinfo) { is_nd_b[info.b] = 1; info_of[info.b] = &info; }
    for (size_t b = 0; b + 1 < P.blkptr.size(); b++) {
      if (!is_nd_b[b]) {
        P.seg_c0.push_back(P.blkptr[b]); P.seg_c1.push_back(P.blkptr[b + 1]); P.seg_level.push_back(0);
        continue;
      }
      const NdBlockInfo& info = *info_of[b];
      int c = P.blkptr[b];
      for (size_t t = 0; t < info.node_size.size(); t++) {
        if (info.node_size[t] == 0) continue;
        P.seg_c0.push_back(c); P.seg_c1.push_back(c + info.node_size[t]); P.seg_level.push_back(info.node_level[t]);
        c += info.node_size[t];
      }
    }
    P.seg_grp.resize(P.seg_c0.size());
    for (size_t sg = 0; sg < P.seg_c0.size(); sg++) P.seg_grp[sg] = group_of(P.seg_c0[sg]);
  }
  build_levels(P);
  return 0;
}

int build_plan_user(int n, const int32_t* Ap, const int32_t* Ai,
                    const int32_t* prow, const int32_t* qcol,
                    int nblk, const int32_t* blkptr, int ngrp, const int32_t* grpptr, Plan& P) {
  P = Plan();
  P.n = n;
  if (!validate_csc(n, Ap, Ai, P.error)) return -1;
  P.nnz = Ap[n];
  P.prow.assign(prow, prow + n);
  P.qcol.assign(qcol, qcol + n);
  P.pinvrow.assign(n, -1);
  std::vector<char> seen(n, 0);
  for (int k = 0; k < n; k++) {
    if (prow[k] < 0 || prow[k] >= n || P.pinvrow[prow[k]] >= 0) { P.error = "prow not a permutation"; return -1; }
    P.pinvrow[prow[k]] = k;
    if (qcol[k] < 0 || qcol[k] >= n || seen[qcol[k]]) { P.error = "qcol not a permutation"; return -1; }
    seen[qcol[k]] = 1;
  }
  if (nblk < 1 || ngrp < 1 || blkptr[0] != 0 || blkptr[nblk] != n || grpptr[0] != 0 || grpptr[ngrp] != n) {
    P.error = "bad block/group pointers";
    return -1;
  }
  P.blkptr.assign(blkptr, blkptr + nblk + 1);
  P.grpptr.assign(grpptr, grpptr + ngrp + 1);
  for (int b = 0; b < nblk; b++)
    if (blkptr[b + 1] <= blkptr[b]) { P.error = "empty block"; return -1; }
  {
    int b = 0;
    for (int g = 0; g < ngrp; g++) {
      if (grpptr[g + 1] <= grpptr[g]) { P.error = "empty group"; return -1; }
      while (blkptr[b + 1] <= grpptr[g]) b++;
      if (grpptr[g + 1] > blkptr[b + 1]) { P.error = "group crosses a block boundary"; return -1; }
    }
  }
  P.struct_rank = n;
  if (assemble_R(n, Ap, Ai, P) != 0) return -1;
  P.parent.assign(n, -1);
  std::vector<int32_t> prev(n), anc(n);
  for (int b = 0; b < nblk; b++) block_col_etree(P.blkptr[b], P.blkptr[b + 1], P.Rp, P.Ri, P.parent, prev, anc);
  finish_schedule(P);
  P.grp_parent.assign(P.grpptr.size() - 1, -1);
  for (int b = 0; b < nblk; b++) {
    P.seg_c0.push_back(P.blkptr[b]); P.seg_c1.push_back(P.blkptr[b + 1]); P.seg_level.push_back(0);
  }
  P.seg_grp.assign(P.seg_c0.size(), -1);
  build_levels(P);
  return 0;
}

// ---------------------------------------------------------------------------
// Level-0 cooperative schedule and the fill of a factorization without row exchanges.
//
// With the diagonal taken as pivot in every column (the matching puts large entries
// there, and the threshold rule keeps them unless an entry is over 1/tau times
// larger), the reach of column k is the closure of struct(R(:,k)) over the L columns
// of the rows before k (Alg. 1's reach with pivot row i for column i).  Its rows
// before k are U(:,k) -- the columns k waits for -- and the rest L(:,k).  Row
// exchanges can change these sets, which the device detects; the column elimination
// tree gives lists that hold for every pivot sequence (George and Ng).
// ---------------------------------------------------------------------------
void build_level0_items(Plan& P, int co_min_cols, int bin_edge) {
  const int n = P.n;
  P.co_item_lo.clear(); P.co_item_hi.clear(); P.co_item_cols.clear(); P.co_item_kind.clear();
  P.col_item.assign(n, -1);
  P.co_max_item_cols = 0;
  P.co_bin_edge = bin_edge;
  const int nlev = (int)P.lvl_ptr.size() - 1;
  if (nlev < 1 || n == 0) return;
  // bin of a segment: 2 = a 1 x 1 diagonal block (its column of R is the diagonal), 1 =
  // at most bin_edge columns (one wavefront factors it column by column), 0 = larger
  auto bin_of = [&](int sg) {
    const int c0 = P.seg_c0[sg], sz = P.seg_c1[sg] - c0;
    if (sz == 1 && P.Rp[c0 + 1] - P.Rp[c0] == 1 && P.Ri[P.Rp[c0]] == c0) {
      const int b = (int)(std::upper_bound(P.blkptr.begin(), P.blkptr.end(), c0) - P.blkptr.begin()) - 1;
      if (P.blkptr[b] == c0 && P.blkptr[b + 1] == c0 + 1) return 2;
    }
    return sz <= bin_edge ? 1 : 0;
  };
  // items over level 0 (lvl_seg is largest first inside a level); an item holds one bin
  const int q0 = P.lvl_ptr[0], q1 = P.lvl_ptr[1];
  int start = q0, acc = 0, kind = -1;
  auto close = [&](int q) {
    if (q > start) {
      P.co_item_lo.push_back(start); P.co_item_hi.push_back(q); P.co_item_cols.push_back(acc);
      P.co_item_kind.push_back(kind);
    }
    start = q;
    acc = 0;
  };
  for (int q = q0; q < q1; q++) {
    const int sg = P.lvl_seg[q];
    const int sz = P.seg_c1[sg] - P.seg_c0[sg];
    const int kq = bin_of(sg);
    if (kq != kind) {
      close(q);
      kind = kq;
    } else if (kq == 2 ? acc >= kBin1ItemCols : (acc > 0 && (acc >= co_min_cols || sz >= co_min_cols))) {
      close(q);
    }
    acc += sz;
  }
  close(q1);
  for (size_t it = 0; it < P.co_item_lo.size(); it++) {
    P.co_max_item_cols = std::max(P.co_max_item_cols, P.co_item_cols[it]);
    for (int q = P.co_item_lo[it]; q < P.co_item_hi[it]; q++)
      for (int k = P.seg_c0[P.lvl_seg[q]]; k < P.seg_c1[P.lvl_seg[q]]; k++) P.col_item[k] = (int32_t)it;
  }
}

void build_level0_schedule(Plan& P, int co_min_cols, int64_t visit_budget, int bin_edge) {
  const int n = P.n;
  const int nlev = (int)P.lvl_ptr.size() - 1;
  P.co_item_lo.clear(); P.co_item_hi.clear(); P.co_item_cols.clear(); P.co_item_kind.clear();
  P.col_item.assign(n, -1);
  P.dep_ptr.assign(n + 1, 0); P.dep_idx.clear();
  P.sdep_ptr.assign(n + 1, 0); P.sdep_idx.clear();
  P.co_max_item_cols = 0;
  P.sym_ok = false;
  P.sym_lnz = P.sym_unz = P.sym_cb = 0;
  P.sym_ws_max = 0;
  if (nlev < 1 || n == 0) {
    P.sym_ok = true;
    P.sfo.clear();
    build_solve_orders(P, nullptr, false);
    return;
  }
  // segment of every column, level of every segment
  std::vector<int32_t> col_seg(n, -1);
  for (size_t sg = 0; sg < P.seg_c0.size(); sg++)
    for (int k = P.seg_c0[sg]; k < P.seg_c1[sg]; k++) col_seg[k] = (int32_t)sg;
  build_level0_items(P, co_min_cols, bin_edge);
  // safe lists: children in the column elimination tree, inside the segment
  {
    std::vector<int32_t> cnt(n + 1, 0);
    for (int k = 0; k < n; k++) {
      const int p = P.parent[k];
      if (p >= 0 && P.col_item[k] >= 0 && col_seg[p] == col_seg[k]) cnt[p + 1]++;
    }
    for (int k = 0; k < n; k++) cnt[k + 1] += cnt[k];
    P.sdep_ptr = cnt;
    P.sdep_idx.assign(cnt[n], 0);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int k = 0; k < n; k++) {   // ascending children: k increases
      const int p = P.parent[k];
      if (p >= 0 && P.col_item[k] >= 0 && col_seg[p] == col_seg[k]) P.sdep_idx[fill[p]++] = k;
    }
  }
  // symbolic factorization without row exchanges, block by block.  The closure of
  // struct(R(:,k)) over L columns of rows i < k (pivotal); `pivlim` limits which rows
  // count as pivotal (the separator first step applies only descendants, rows < g0).
  std::vector<int32_t> blk_hi(n);
  for (size_t b = 0; b + 1 < P.blkptr.size(); b++)
    for (int k = P.blkptr[b]; k < P.blkptr[b + 1]; k++) blk_hi[k] = P.blkptr[b + 1];
  std::vector<int64_t> Lb(n, 0), Le(n, 0);   // L(:,k) rows: Lrows[Lb[k] .. Le[k])
  std::vector<int32_t> Lrows;
  std::vector<int32_t> mark(n, -1), queue;
  queue.reserve(1024);
  int64_t visits = 0;
  std::vector<int32_t> deps;
  bool within = true;
  // reach of column k with rows < pivlim pivotal; fills queue with the reach
  auto closure = [&](int k, int pivlim, int stamp) {
    queue.clear();
    const int b1 = blk_hi[k];
    for (int32_t p = P.Rp[k]; p < P.Rp[k + 1]; p++) {
      const int i = P.Ri[p];
      if (i >= b1) continue;
      if (mark[i] != stamp) { mark[i] = stamp; queue.push_back(i); }
    }
    for (size_t t = 0; t < queue.size(); t++) {
      const int i = queue[t];
      if (i >= pivlim) continue;
      for (int64_t q = Lb[i]; q < Le[i]; q++) {
        const int r = Lrows[q];
        if (mark[r] != stamp) { mark[r] = stamp; queue.push_back(r); }
      }
      visits += Le[i] - Lb[i];
    }
  };
  // pass 1: level-0 columns (their closures only touch their own segment's columns);
  // pass 2: separator columns, whose closures use every earlier column
  std::vector<int32_t> dcnt(n + 1, 0);
  std::vector<std::vector<int32_t>> dlist(n);
  int stamp = 0;
  bool deps_ok = true;
  for (int pass = 0; pass < 2 && within; pass++) {
    for (int k = 0; k < n; k++) {
      const int sg = col_seg[k];
      const int lvl = sg >= 0 ? P.seg_level[sg] : 0;
      if ((pass == 0) != (lvl == 0)) continue;
      if (visits > visit_budget) {
        within = false;
        if (pass == 0) deps_ok = false;
        break;
      }
      const int g0 = P.seg_c0[sg];
      if (lvl >= 1) {
        // the separator first step: descendants' pivots only (rows before the separator)
        closure(k, g0, ++stamp);
        P.sym_cb += (int64_t)queue.size();
        P.sym_ws_max = std::max<int64_t>(P.sym_ws_max, (int64_t)queue.size());
      }
      closure(k, k, ++stamp);
      P.sym_ws_max = std::max<int64_t>(P.sym_ws_max, (int64_t)queue.size());
      int64_t lc = 0, uc = 1;
      deps.clear();
      for (int i : queue) {
        if (i < k) {
          uc++;
          if (lvl == 0 && i >= g0) deps.push_back(i);
        } else if (i > k) {
          lc++;
        }
      }
      P.sym_lnz += lc;
      P.sym_unz += uc;
      // L(:,k) rows (columns are visited level 0 first, so offsets are kept per column)
      Lb[k] = (int64_t)Lrows.size();
      for (int i : queue)
        if (i > k) Lrows.push_back(i);
      Le[k] = (int64_t)Lrows.size();
      if (lvl == 0) {
        std::sort(deps.begin(), deps.end());
        dlist[k] = deps;
      }
    }
  }
  if (deps_ok) {
    for (int k = 0; k < n; k++) dcnt[k + 1] = dcnt[k] + (int32_t)dlist[k].size();
    P.dep_ptr = dcnt;
    P.dep_idx.clear();
    P.dep_idx.reserve(dcnt[n]);
    for (int k = 0; k < n; k++) P.dep_idx.insert(P.dep_idx.end(), dlist[k].begin(), dlist[k].end());
  } else {
    // the budget ran out: level-0 columns fall back to their safe lists
    P.dep_ptr = P.sdep_ptr;
    P.dep_idx = P.sdep_idx;
  }
  P.sym_ok = within;
  build_issue_order(P);
  if (deps_ok) {
    std::vector<std::vector<int32_t>> lr(n);
    for (int k = 0; k < n; k++)
      if (P.col_item[k] >= 0) lr[k].assign(Lrows.begin() + Lb[k], Lrows.begin() + Le[k]);
    build_solve_orders(P, &lr, true);
  } else {
    P.sfo.clear();
    build_solve_orders(P, nullptr, false);
  }
}

void build_solve_orders(Plan& P, const std::vector<std::vector<int32_t>>* lrows, bool backward) {
  const int n = P.n;
  const bool fresh = (int)P.sfo.size() != n;
  P.sfo.resize(n); P.sbo.resize(n); P.sfo_pos.resize(n); P.sbo_pos.resize(n);
  P.row_task0.assign(n, 0);
  std::vector<char> seen(n + 1, 0);
  std::vector<int32_t> fl(n, 0), bl(n, 0), ord;
  for (size_t q = 0; q < P.st_kind.size(); q++) {
    const int kind = P.st_kind[q], id = P.st_id[q];
    const int r0 = kind == 0 ? P.blkptr[id] : P.grpptr[id];
    const int r1 = kind == 0 ? P.blkptr[id + 1] : P.grpptr[id + 1];
    const int m = r1 - r0;
    if (m <= 0 || seen[r0]) continue;   // an ND node's forward and backward tasks share rows
    seen[r0] = 1;
    for (int k = r0; k < r1; k++) P.row_task0[k] = r0;
    // predictions exist for the first-level segments only; separators keep plain order
    const bool l0 = !P.col_item.empty() && P.col_item[r0] >= 0;
    ord.resize(m);
    if (lrows || fresh) {
      if (l0 && lrows)
        for (int j = r0; j < r1; j++)
          for (int r : (*lrows)[j])
            if (r < r1) fl[r] = std::max(fl[r], fl[j] + 1);
      std::iota(ord.begin(), ord.end(), r0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return fl[x] < fl[y]; });
      for (int i = 0; i < m; i++) { P.sfo[r0 + i] = ord[i]; P.sfo_pos[ord[i]] = i; }
    }
    if (l0 && backward)
      for (int j = r1 - 1; j >= r0; j--)
        for (int32_t e = P.dep_ptr[j]; e < P.dep_ptr[j + 1]; e++) {
          const int k = P.dep_idx[e];
          if (k >= r0 && k < j) bl[k] = std::max(bl[k], bl[j] + 1);
        }
    for (int i = 0; i < m; i++) ord[i] = r1 - 1 - i;   // plain backward order: descending
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return bl[x] < bl[y]; });
    for (int i = 0; i < m; i++) { P.sbo[r0 + i] = ord[i]; P.sbo_pos[ord[i]] = i; }
  }
}

void build_issue_order(Plan& P) {
  const int nco = (int)P.co_item_lo.size();
  P.co_item_off.assign(nco + 1, 0);
  for (int it = 0; it < nco; it++) P.co_item_off[it + 1] = P.co_item_off[it] + P.co_item_cols[it];
  P.co_issue.assign(3 * (size_t)P.co_item_off[nco], 0);
  std::vector<int32_t> col, ord, seg0, bot;
  for (int it = 0; it < nco; it++) {
    const int m = P.co_item_cols[it];
    col.resize(m);
    seg0.resize(m);
    int s = 0;
    for (int q = P.co_item_lo[it]; q < P.co_item_hi[it]; q++) {
      const int sg = P.lvl_seg[q];
      const int c0 = P.seg_c0[sg];
      for (int k = c0; k < P.seg_c1[sg]; k++, s++) {
        col[s] = k;
        seg0[s] = c0;
      }
    }
    // critical path first: by decreasing length of the longest dependency path from the
    // column to the end of its segment (every dependency lies on a longer path than its
    // dependents, so the order stays topological), then by slot.  On the batched-BTF
    // leaves a greedy schedule of 8 wavefronts finishes ~20% sooner than in level order.
    bot.assign(m, 1);
    for (int t = m - 1; t >= 0; t--) {
      const int k = col[t];
      for (int32_t e = P.dep_ptr[k]; e < P.dep_ptr[k + 1]; e++) {
        const int sj = t - (k - P.dep_idx[e]);
        bot[sj] = std::max(bot[sj], bot[t] + 1);
      }
    }
    ord.resize(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return bot[x] > bot[y]; });
    int32_t* out = P.co_issue.data() + 3 * (size_t)P.co_item_off[it];
    for (int i = 0; i < m; i++) {
      out[3 * i] = col[ord[i]];
      out[3 * i + 1] = ord[i];
      out[3 * i + 2] = seg0[ord[i]];
    }
  }
}

int64_t merge_learned_deps(Plan& P, const std::vector<int32_t>& items, const std::vector<int32_t>& Ubeg,
                           const std::vector<int32_t>& Ucnt, const std::vector<int32_t>& Ui) {
  const int n = P.n;
  std::vector<char> take(n, 0);
  for (int it : items)
    for (int q = P.co_item_lo[it]; q < P.co_item_hi[it]; q++)
      for (int k = P.seg_c0[P.lvl_seg[q]]; k < P.seg_c1[P.lvl_seg[q]]; k++) take[k] = 1;
  std::vector<int32_t> ptr(n + 1, 0), idx;
  idx.reserve(P.dep_idx.size());
  std::vector<int32_t> merged;
  int64_t added = 0;
  for (int k = 0; k < n; k++) {
    const int32_t* a0 = P.dep_idx.data() + P.dep_ptr[k];
    const int32_t* a1 = P.dep_idx.data() + P.dep_ptr[k + 1];
    if (take[k] && Ucnt[k] > 0) {
      // U(:,k) without its diagonal (last), ascending
      const int32_t* b0 = Ui.data() + Ubeg[k];
      const int32_t* b1 = b0 + (Ucnt[k] - 1);
      merged.clear();
      std::set_union(a0, a1, b0, b1, std::back_inserter(merged));
      added += (int64_t)merged.size() - (a1 - a0);
      idx.insert(idx.end(), merged.begin(), merged.end());
    } else {
      idx.insert(idx.end(), a0, a1);
    }
    ptr[k + 1] = (int32_t)idx.size();
  }
  P.dep_ptr = std::move(ptr);
  P.dep_idx = std::move(idx);
  build_issue_order(P);
  build_solve_orders(P, nullptr, true);
  return added;
}

}  // namespace basker
