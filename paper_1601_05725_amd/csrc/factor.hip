// Numeric factorization on gfx950.  One wavefront runs one column of the left-looking
// Gilbert-Peierls algorithm (Alg. 1) at a time:
//
//   reach     breadth-first closure of struct(R(:,k)) over the graph of L, with the
//             discovered rows kept in a per-wave LDS hash table (lanes expand the
//             L columns of a whole frontier at once, staging their entries for the
//             update when they fit);
//   order     the pivotal rows of the reach sorted by pivot index -- ascending pivot
//             index is a topological order because every edge of the graph of L runs
//             from a lower to a higher pivot index;
//   update    x_r = x_r - l_rj * x_j over L(:,j), lanes over the rows of L(:,j);
//   pivot     wavefront max-reduction over the candidates (non-pivotal rows of the
//             column's group), diagonal preference by threshold, smallest index on ties;
//   store     U(:,k) ascending with the diagonal last, L(:,k) compacted by ballot and
//             prefix count, both appended to device pools by bump allocation of
//             per-wave chunks.
//
// Scheduling follows the level sets of Alg. 4, one launch per level.  The first level
// (BTF blocks and ND leaves) runs on cooperative workgroups (factor_coop_kernel): a
// workgroup takes a work item (whole segments) from an atomic counter, and its waves
// take the item's columns in a level-ordered issue list, each column waiting for the
// columns of its dependency list through LDS done bits.  A speculative pass uses the
// dependency lists of the symbolic analysis without row exchanges; every column checks
// its reach against its list, and a pass over the results redoes any item whose
// speculation failed with the column elimination tree's safe lists.  Separator levels
// run one column per wavefront (factor_kernel), a separator's dense block on the dense
// kernel (sepdense.hip).  The kernel boundary between levels is the only
// synchronisation across workgroups.
//
// Arithmetic matches a serial run that updates in ascending pivot order: every update
// is a separately rounded multiply and subtract (built with -ffp-contract=off),
// L = x / pivot is an IEEE division, and each entry of x receives its updates in
// ascending pivot order.
#include "device.hpp"

#define COMMA ,

namespace basker {

namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// One workgroup is one wavefront.  Lanes exchange data through LDS and, across
// columns, through global memory; the lanes of one wavefront need no cache action to
// see each other's writes (one vector L1 per CU, memory instructions of a wavefront
// performed in order), so a wavefront-scope fence, which only keeps the compiler
// from moving memory operations across it, is all the ordering required.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rl_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// exclusive prefix sum of v over lanes [0, nb) (nb uniform, <= 64; v = 0 on lanes
// >= nb): scalar reads of the few lanes when nb is small, a shuffle scan otherwise
__device__ __forceinline__ int excl_scan(int v, int nb) {
  const int lane = lane_id();
  if (nb <= 16) {
    int acc = 0;
    for (int u = 0; u < nb; u++) {
      const int x = rl(v, u);
      if (u < lane) acc += x;
    }
    return acc;
  }
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(x, d, 64);
    if (lane >= d) x += t;
  }
  return x - v;
}

__device__ __forceinline__ int ld_relaxed(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-wave workspace: an open-addressing hash table keyed by R row (in LDS, or in a
// global fallback region for columns whose pattern does not fit in LDS).
struct Ws {
  int32_t* key;   // H, -1 empty
  double* val;    // H
  int32_t* pv;    // H: pivot column of the key's row when inserted, -1 if non-pivotal
  int32_t* ins;   // H: slots in insertion order
  int32_t* pj;    // H: pivotal list: pivot column j
  int32_t* ps;    //    slot of the pivotal row
  int32_t* pb;    //    L(:,j) offset
  int32_t* pc;    //    L(:,j) length
  unsigned long long* sk;  // H: sorted (j << 32 | list index)
  int32_t* cnt;   // [0] inserted, [1] pivotal, [2] overflow
  // staging of the update's L entries (always in LDS): workspace slot and value,
  // offsets and global starts of the staged columns
  int32_t* st_slot;
  double* st_val;
  int32_t* st_pre;
  int32_t* st_beg;
  // stage offset of every pivotal list entry's L column when the reach staged it (LDS
  // workspaces only; null: no staging during the reach)
  int32_t* pso;
  int H;
  int NP;         // capacity of the pivotal list
  int shift;      // 32 - log2(H)
  int SC;         // capacity of the stage (entries)
  int lim;        // rows a column may hold before it moves to the global workspace
};

// Per-wave pool allocator: a wave claims a chunk of the L and U pools with one atomic
// and hands out column storage from it, so the device-wide counters see one atomic
// per chunk instead of two per column.
struct Alloc {
  long long lcur, lend, ucur, uend, ccur, cend;
  long long lnz, unz;
  int offdiag;
};

constexpr int kStage = 512;   // staged L entries per pass of the update

// H hash slots; the pivotal list holds NP entries (a column overflows to the global
// workspace once more than H/2 rows are inserted, so NP = H/2 is always enough); SC
// staged L entries
template <int H, int NP, int SC = kStage>
struct LdsWs {
  int32_t key[H];
  double val[H];
  int32_t pv[H];
  int32_t ins[H];
  int32_t pj[NP];
  int32_t ps[NP];
  int32_t pb[NP];
  int32_t pc[NP];
  unsigned long long sk[NP];
  double st_val[SC];
  int32_t st_slot[SC];
  int32_t st_pre[72];
  int32_t st_beg[64];
  int32_t pso[NP];
  int32_t cnt[4];
};

// Speculation context of a column of the first level (cooperative kernel).  A
// speculative column counts rows pivoted by later columns as not pivotal, and every
// pivot column its reach uses must be in the dependency list it waited for; a pivot
// row must not have been claimed already.  Any other outcome is reported (return 3)
// and the column's work item is redone with safe dependencies.
struct ColCtx {
  int spec;
  const int32_t* deps;   // ascending
  int ndeps;
};

__device__ __forceinline__ unsigned hash_of(int32_t r, int shift) {
  return ((unsigned)r * 2654435761u) >> shift;
}

// insert r; returns the slot and whether it is new; -1 when the table is full.
// The overflow flag is raised once more than w.lim slots are in use.
__device__ __forceinline__ int ws_insert(const Ws& w, int32_t r, bool* isnew) {
  unsigned h = hash_of(r, w.shift);
  const unsigned mask = (unsigned)w.H - 1u;
  for (int t = 0; t < w.H; t++) {
    int old = atomicCAS(&w.key[h], -1, r);
    if (old == -1) {
      int pos = atomicAdd(&w.cnt[0], 1);
      w.ins[pos] = (int32_t)h;
      if (pos >= w.lim) w.cnt[2] = 1;
      *isnew = true;
      return (int)h;
    }
    if (old == r) { *isnew = false; return (int)h; }
    h = (h + 1u) & mask;
  }
  w.cnt[2] = 1;
  *isnew = false;
  return -1;
}

__device__ __forceinline__ int ws_lookup(const Ws& w, int32_t r) {
  unsigned h = hash_of(r, w.shift);
  const unsigned mask = (unsigned)w.H - 1u;
  for (int t = 0; t < w.H; t++) {
    int kk = w.key[h];
    if (kk == r) return (int)h;
    if (kk == -1) return -1;
    h = (h + 1u) & mask;
  }
  return -1;
}

// clear the slots the previous column used
__device__ __forceinline__ void ws_reset(const Ws& w) {
  const int lane = lane_id();
  wsync();
  int used = w.cnt[0];
  if (used > w.H) used = w.H;
  for (int t = lane; t < used; t += 64) w.key[w.ins[t]] = -1;
  wsync();
  if (lane == 0) { w.cnt[0] = 0; w.cnt[1] = 0; w.cnt[2] = 0; w.cnt[3] = 0; }
  wsync();
}

__device__ __forceinline__ void plist_push(const Ws& w, int32_t j, int slot) {
  int e = atomicAdd(&w.cnt[1], 1);
  if (e >= w.NP) {   // only past the overflow point; the column moves to the global workspace
    w.cnt[2] = 1;
    return;
  }
  w.pj[e] = j;
  w.ps[e] = slot;
  w.pb[e] = 0;
  w.pc[e] = 0;
}

// Sort the pivotal list [0, np) by pivot column: sk[t] = (j << 32 | list index),
// ascending.  Keys are distinct.  Bitonic network in registers (np <= 64) or LDS.
__device__ void plist_sort(const Ws& w, int np) {
  const int lane = lane_id();
  np = uniform(np);
  if (np <= 64) {
    // rank of every key among the np distinct keys, read lane by lane
    const unsigned key = lane < np ? (unsigned)w.pj[lane] : 0xffffffffu;
    int rank = 0;
    for (int u = 0; u < np; u++) rank += ((unsigned)rl((int)key, u) < key) ? 1 : 0;
    if (lane < np) w.sk[rank] = ((unsigned long long)key << 32) | (unsigned)lane;
    wsync();
    return;
  }
  int N = 1;
  while (N < np) N <<= 1;
  for (int t = lane; t < N; t += 64)
    w.sk[t] = t < np ? (((unsigned long long)(unsigned)w.pj[t] << 32) | (unsigned)t) : ~0ull;
  wsync();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < N; t += 64) {
        int l = t ^ j;
        if (l > t) {
          unsigned long long a = w.sk[t], b = w.sk[l];
          bool up = ((t & k) == 0);
          if ((a > b) == up) { w.sk[t] = b; w.sk[l] = a; }
        }
      }
      wsync();
    }
  }
}

// Expand the frontier entries [f0, f1) of the pivotal list: record each entry's
// L column and insert its rows.  New pivotal rows join the list (next frontier).
// plim: rows whose pivot column is >= plim count as not pivotal (see factor_column)
// sfill: entries staged so far (-1: staging abandoned); returns the new value.  While
// every expanded column fits in the stage, its L entries (workspace slot and value) are
// staged on the way, with the entry's stage offset in pso, for the update.
__device__ int expand_frontier(const FactorArgs& a, const Ws& w, int f0, int f1, int plim, int sfill) {
  const int lane = lane_id();
  for (int c0 = f0; c0 < f1; c0 += 64) {
    const int nb = uniform(f1 - c0 < 64 ? f1 - c0 : 64);
    const int e = c0 + lane;
    int beg = 0, cnt = 0;
    if (lane < nb) {
      const int j = w.pj[e];
      beg = a.Lbeg[j];
      cnt = a.Lcnt[j];
      w.pb[e] = beg;
      w.pc[e] = cnt;
    }
    const int excl = excl_scan(cnt, nb);
    const int total = rl(excl, nb - 1) + rl(cnt, nb - 1);
    if (sfill >= 0 && sfill + total > w.SC) sfill = -1;
    const bool stage = sfill >= 0;
    if (stage && lane < nb) w.pso[e] = sfill + excl;
    if (nb > 8) {
      if (lane < nb) {
        w.st_pre[lane] = excl;
        w.st_beg[lane] = beg;
      }
      wsync();
    }
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      // owner: the last list entry whose first position is <= t
      int ob = 0, oe = 0;
      if (nb <= 8) {
        for (int u = 0; u < nb; u++) {
          const int ex = rl(excl, u);
          const int bu = rl(beg, u);
          if (ex <= t) { ob = bu; oe = ex; }
        }
      } else {
        int lo = 0, hi = nb;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w.st_pre[mid] <= t) lo = mid; else hi = mid;
        }
        ob = w.st_beg[lo];
        oe = w.st_pre[lo];
      }
      if (t < total) {
        const int32_t r = a.Li[ob + (t - oe)];
        double lx = 0.0;
        if (stage) lx = a.Lx[ob + (t - oe)];
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0 && isnew) {
          w.val[slot] = 0.0;
          int32_t pvr = a.pinv[r];
          if (pvr >= plim) pvr = -1;
          w.pv[slot] = pvr;
          if (pvr >= 0) plist_push(w, pvr, slot);
        }
        if (stage) {
          w.st_slot[sfill + t] = slot;
          w.st_val[sfill + t] = lx;
        }
      }
    }
    if (stage) sfill += total;
  }
  wsync();
  return sfill;
}

// Factor (or refactor) column k with workspace w.  Returns 0 on success, 1 when the
// workspace overflowed (nothing was written), 2 on a numerical failure (status set).
// take n entries from [cur, end), claiming a new chunk from the device counter when
// the current one is short; returns the offset, or -1 when the pool is exhausted
__device__ __forceinline__ long long pool_take(long long* cur, long long* end, long long n,
                                               unsigned long long* counter, long long chunk, long long cap) {
  if (*cur + n > *end) {
    const long long want = n > chunk ? n : chunk;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, (unsigned long long)want);
    base = __shfl(base, 0, 64);
    if ((long long)base + want > cap) return -1;
    *cur = (long long)base;
    *end = (long long)base + want;
  }
  const long long off = *cur;
  *cur += n;
  return off;
}

// The next column's entries of R, loaded while the current column runs (a column of a
// segment in mode 0): offsets at the start, rows and values after the reach, and the
// rows' pivot columns after the update.  Between that last load and the next column only
// the current column's own pivot row changes its pivot column (no other wavefront
// pivots rows of this segment), so that one row is patched on use.
struct Pre {
  int k;        // column the data belongs to, -1 for none
  int b, e;     // R(:,k) = entries [b, e), at most 64
  int32_t r;    // the lane's row
  double x;     // the lane's value
  int32_t pv;   // pivot column of the lane's row when loaded
  int pp, pk;   // pivot row and index of the column during which pv was loaded
  int fresh;    // 1: pv was not loaded (rows and values only); read the pivot status on use
};

__device__ __forceinline__ int factor_column(const FactorArgs& a, const Ws& w, int k, Alloc& al, Pre& pre,
                                             int knext, const ColCtx& cx) {
  const int lane = lane_id();
  ws_reset(w);
  const int g0 = a.grp_lo[k], g1 = a.grp_hi[k];
  // The first step of a separator level (mode 1) applies only the pivots of the
  // separator's descendants, whose columns precede the separator's first column g0.  In
  // a factorization no other row is pivotal yet; a refactorization keeps the previous
  // pivots of every row, so later pivots (the separator's own and its ancestors') must
  // be read as not pivotal here.  A speculative column likewise ignores the pivots of
  // later columns that ran before it.
  const int plim = a.mode == 1 ? g0 : (cx.spec ? k : 0x7fffffff);
  const bool use_pre = a.mode == 0 && !a.refactor && pre.k == k;
  const Pre cur = pre;
  const bool do_pre = a.mode == 0 && !a.refactor && knext >= 0;
  pre.k = -1;
  if (do_pre) {
    pre.b = a.Rp[knext];
    pre.e = a.Rp[knext + 1];
    pre.fresh = 0;
    if (pre.e - pre.b <= 64) pre.k = knext;
  }

  int ub = 0, uc = 0, lb = 0, lc = 0, p = -1;
  // staging of the reach's L columns for the update (LDS workspaces, full factorization)
  int sfill = (w.pso != nullptr && !a.refactor) ? 0 : -1;
  if (!a.refactor || a.mode == 1) {
    if (use_pre) {
      // struct(R(:,k)) with values, loaded during the previous column
      if (lane < cur.e - cur.b) {
        const int32_t r = cur.r;
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0) {
          w.val[slot] = cur.x;
          int32_t pvr = cur.fresh ? a.pinv[r] : ((r == cur.pp) ? cur.pk : cur.pv);
          if (pvr >= plim) pvr = -1;
          w.pv[slot] = pvr;
          if (pvr >= 0) plist_push(w, pvr, slot);
        }
      }
    } else if (a.mode != 2) {
      // struct(R(:,k)) with values
      for (int q = a.Rp[k] + lane; q < a.Rp[k + 1]; q += 64) {
        const int32_t r = a.Ri[q];
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0) {
          w.val[slot] = a.Rx[q];
          int32_t pvr = a.pinv[r];
          if (pvr >= plim) pvr = -1;
          w.pv[slot] = pvr;
          if (pvr >= 0) plist_push(w, pvr, slot);
        }
      }
    } else {
      // the partial column left by mode 1: its non-pivotal rows with their values
      const int off = a.cb_off[k] + a.cb_np[k], nn = a.cb_nn[k];
      for (int t = lane; t < nn; t += 64) {
        const int32_t r = a.cbI[off + t];
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0) {
          w.val[slot] = a.cbX[off + t];
          const int32_t pvr = a.pinv[r];
          w.pv[slot] = pvr;
          if (pvr >= 0) plist_push(w, pvr, slot);
        }
      }
    }
    wsync();
    // reach: breadth-first over the graph of L
    int f0 = 0;
    int f1 = w.cnt[1];
    while (f0 < f1) {
      if (w.cnt[2]) break;
      sfill = expand_frontier(a, w, f0, f1, plim, sfill);
      f0 = f1;
      f1 = w.cnt[1];
    }
    wsync();
    if (w.cnt[2]) return 1;
  } else {
    // known pattern: U(:,k) rows (pivotal, ascending) and L(:,k) rows plus the pivot
    ub = a.Ubeg[k]; uc = a.Ucnt[k]; lb = a.Lbeg[k]; lc = a.Lcnt[k];
    p = a.piv[k];
    if (uc - 1 + lc + 1 > w.lim) return 1;
    for (int t = lane; t < uc - 1; t += 64) {
      const int32_t j = a.Ui[ub + t];
      bool isnew;
      int slot = ws_insert(w, a.piv[j], &isnew);
      if (slot < 0) continue;
      w.val[slot] = 0.0;
      w.pv[slot] = j;
      w.pj[t] = j;
      w.ps[t] = slot;
      w.pb[t] = a.Lbeg[j];
      w.pc[t] = a.Lcnt[j];
    }
    for (int t = lane; t < lc + 1; t += 64) {
      const int32_t r = t < lc ? a.Li[lb + t] : p;
      bool isnew;
      int slot = ws_insert(w, r, &isnew);
      if (slot < 0) continue;
      w.val[slot] = 0.0;
      w.pv[slot] = -1;
    }
    if (lane == 0) w.cnt[1] = uc - 1;
    wsync();
    int bad = 0;
    for (int q = a.Rp[k] + lane; q < a.Rp[k + 1]; q += 64) {
      int slot = ws_lookup(w, a.Ri[q]);
      if (slot < 0) bad = 1; else w.val[slot] = a.Rx[q];
    }
    if (__any(bad)) {
      if (lane == 0) {
        atomicMax(&a.status[ST_CODE], DEV_PATTERN);
        atomicMin(&a.status[ST_FAILCOL], k);
      }
      return 2;
    }
    wsync();
  }

  if (pre.k >= 0 && lane < pre.e - pre.b) {
    pre.r = a.Ri[pre.b + lane];
    pre.x = a.Rx[pre.b + lane];
  }
  // topological order: ascending pivot column
  const int np = w.cnt[1];
  if (!a.refactor || a.mode == 1) {
    plist_sort(w, np);
  } else {
    for (int t = lane; t < np; t += 64) w.sk[t] = ((unsigned long long)(unsigned)w.pj[t] << 32) | (unsigned)t;
    wsync();
  }
  if (cx.spec) {
    // every pivot column the reach used must be one this column waited for
    bool miss = false;
    for (int e = lane; e < np; e += 64) {
      const int32_t j = (int32_t)(w.sk[e] >> 32);
      int lo = 0, hi = cx.ndeps;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cx.deps[mid] < j) lo = mid + 1; else hi = mid;
      }
      if (lo >= cx.ndeps || cx.deps[lo] != j) miss = true;
    }
    if (__any(miss)) return 3;
  }

  // sparse triangular update, ascending pivot order.  When the reach staged every L
  // column it expanded, the update runs from the stage.  Otherwise the L(:,j) entries of
  // up to 64 list entries at a time are gathered into LDS in one wave-wide pass, their
  // rows resolved to workspace slots on the way, then applied column by column from LDS.
  const bool staged = sfill >= 0 && (!a.refactor || a.mode == 1);
  if (staged) {
    for (int t = 0; t < np; t++) {
      const int src = (int)(w.sk[t] & 0xffffffffu);
      const int o = w.pso[src], cj = w.pc[src];
      const double xj = w.val[w.ps[src]];
      for (int e = lane; e < cj; e += 64) {
        const int slot = w.st_slot[o + e];
        const double prod = w.st_val[o + e] * xj;
        if (slot >= 0) w.val[slot] = w.val[slot] - prod;
        else w.cnt[3] = 1;
      }
      wsync();
    }
  }
  for (int e0 = 0; e0 < (staged ? 0 : np); e0 += 64) {
    const int nb = uniform(np - e0 < 64 ? np - e0 : 64);
    int c = 0, beg = 0, sl = 0;
    if (lane < nb) {
      const int src = (int)(w.sk[e0 + lane] & 0xffffffffu);
      sl = w.ps[src];
      beg = w.pb[src];
      c = w.pc[src];
    }
    const int off = excl_scan(c, nb);
    int j0 = 0;
    while (j0 < nb) {
      const int off0 = rl(off, j0);
      const bool fit = lane >= j0 && lane < nb && off + c - off0 <= w.SC;
      const int nfit = __popcll(__ballot(fit));
      if (nfit == 0) {
        // a column longer than the stage: straight from global memory
        const int cj = rl(c, j0), bj = rl(beg, j0);
        const double xj = w.val[rl(sl, j0)];
        for (int t = lane; t < cj; t += 64) {
          const int slot = ws_lookup(w, a.Li[bj + t]);
          const double prod = a.Lx[bj + t] * xj;
          if (slot >= 0) w.val[slot] = w.val[slot] - prod;
          else w.cnt[3] = 1;
        }
        wsync();
        j0++;
        continue;
      }
      const int j1 = j0 + nfit;
      if (lane >= j0 && lane < j1) {
        w.st_pre[lane - j0] = off - off0;
        w.st_beg[lane - j0] = beg;
      }
      if (lane == j1 - 1) w.st_pre[j1 - j0] = off + c - off0;
      wsync();
      const int total = rl(off, j1 - 1) + rl(c, j1 - 1) - off0;
      const int nc = j1 - j0;
      for (int base = 0; base < total; base += 64 * 8) {
        int gi[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int q = base + u * 64 + lane;
          gi[u] = -1;
          if (q < total) {
            int lo = 0, hi = nc;
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (w.st_pre[mid] <= q) lo = mid; else hi = mid;
            }
            gi[u] = w.st_beg[lo] + (q - w.st_pre[lo]);
          }
        }
        int32_t rr[8];
        double xx[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          rr[u] = 0;
          xx[u] = 0.0;
          if (gi[u] >= 0) { rr[u] = a.Li[gi[u]]; xx[u] = a.Lx[gi[u]]; }
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int q = base + u * 64 + lane;
          if (gi[u] >= 0) { w.st_slot[q] = ws_lookup(w, rr[u]); w.st_val[q] = xx[u]; }
        }
      }
      wsync();
      for (int j = j0; j < j1; j++) {
        const int cj = rl(c, j);
        if (cj == 0) continue;
        const int o = rl(off, j) - off0;
        const double xj = w.val[rl(sl, j)];
        for (int t = lane; t < cj; t += 64) {
          const int slot = w.st_slot[o + t];
          const double prod = w.st_val[o + t] * xj;
          if (slot >= 0) w.val[slot] = w.val[slot] - prod;
          else w.cnt[3] = 1;
        }
        wsync();
      }
      j0 = j1;
    }
  }
  if (w.cnt[3]) {
    if (lane == 0) {
      atomicMax(&a.status[ST_CODE], DEV_PATTERN);
      atomicMin(&a.status[ST_FAILCOL], k);
    }
    return 2;
  }

  const int nins = w.cnt[0];
  if (a.mode == 1) {
    // park the partial column: descendant pivots (final U entries) ascending, then the
    // non-pivotal rows (separator and ancestor rows) with their partial values
    const long long off = pool_take(&al.ccur, &al.cend, nins, &a.pool_next[2], 0, a.cbcap);
    if (off < 0) {
      if (lane == 0) {
        atomicMax(&a.status[ST_CODE], DEV_POOL);
        a.status[ST_CBPOOL] = 1;
      }
      return 2;
    }
    for (int e = lane; e < np; e += 64) {
      const unsigned long long key = w.sk[e];
      a.cbI[off + e] = (int32_t)(key >> 32);
      a.cbX[off + e] = w.val[w.ps[(int)(key & 0xffffffffu)]];
    }
    int cnt = np;
    for (int base = 0; base < nins; base += 64) {
      const int t = base + lane;
      int s = 0;
      bool sel = false;
      if (t < nins) {
        s = w.ins[t];
        sel = w.pv[s] < 0;
      }
      const unsigned long long bm = __ballot(sel);
      const int pos = cnt + __popcll(bm & ((1ull << lane) - 1ull));
      if (sel) {
        a.cbI[off + pos] = w.key[s];
        a.cbX[off + pos] = w.val[s];
      }
      cnt += __popcll(bm);
    }
    if (lane == 0) {
      a.cb_off[k] = (int32_t)off;
      a.cb_np[k] = np;
      a.cb_nn[k] = nins - np;
    }
    return 0;
  }
  if (pre.k >= 0 && lane < pre.e - pre.b) pre.pv = a.pinv[pre.r];
  // pivot search over the candidates of the column's group
  double best = -1.0;
  int bidx = 0x7fffffff;
  int has_diag = 0;
  double xd = 0.0;
  for (int t = lane; t < nins; t += 64) {
    const int s = w.ins[t];
    const int32_t r = w.key[s];
    if (w.pv[s] < 0 && r >= g0 && r < g1) {
      const double v = fabs(w.val[s]);
      if (v > best || (v == best && r < bidx)) { best = v; bidx = r; }
      if (r == k) { has_diag = 1; xd = w.val[s]; }
    }
  }
  {
    // combine the lanes' partial results (only lanes below nins hold candidates)
    const int nl = uniform(nins < 64 ? nins : 64);
    if (nl <= 16) {
      double gb = -1.0;
      int gi = 0x7fffffff;
      for (int u = 0; u < nl; u++) {
        const double ob = rl_d(best, u);
        const int oi = rl(bidx, u);
        if (ob > gb || (ob == gb && oi < gi)) { gb = ob; gi = oi; }
      }
      best = gb;
      bidx = gi;
    } else {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) {
        const double ob = __shfl_xor(best, d, 64);
        const int oi = __shfl_xor(bidx, d, 64);
        if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
      }
    }
  }
  const unsigned long long dmask = __ballot(has_diag);
  if (dmask) xd = rl_d(xd, __ffsll((long long)dmask) - 1);
  const double m = best;   // -1 when there is no candidate

  if (!a.refactor) {
    if (!(m > 0.0)) {
      if (cx.spec) return 3;   // decided again with safe dependencies
      if (lane == 0) {
        atomicMax(&a.status[ST_CODE], DEV_SINGULAR);
        atomicMin(&a.status[ST_FAILCOL], k);
      }
      return 2;
    }
    p = (a.diag_pref && dmask && fabs(xd) >= a.tau * m) ? k : bidx;
  }
  const int sp = ws_lookup(w, p);
  if (sp < 0) {
    if (lane == 0) {
      atomicMax(&a.status[ST_CODE], DEV_PATTERN);
      atomicMin(&a.status[ST_FAILCOL], k);
    }
    return 2;
  }
  const double xp = w.val[sp];
  if (a.refactor) {
    const bool ok = (m > 0.0) && w.pv[sp] < 0 && p >= g0 && p < g1 && xp != 0.0 && fabs(xp) >= a.tau * m;
    if (!ok) {
      if (lane == 0) {
        atomicMax(&a.status[ST_CODE], DEV_REFACTOR_FAIL);
        atomicMin(&a.status[ST_FAILCOL], k);
      }
      return 2;
    }
  }

  // store U(:,k) and L(:,k)
  if (!a.refactor) {
    const int dnp = (a.mode == 2) ? a.cb_np[k] : 0;
    uc = dnp + np + 1;
    lc = nins - np - 1;
    const long long ubl = pool_take(&al.ucur, &al.uend, uc, &a.pool_next[1], a.chunk, a.Ucap);
    const long long lbl = pool_take(&al.lcur, &al.lend, lc, &a.pool_next[0], a.chunk, a.Lcap);
    if (ubl < 0 || lbl < 0) {
      if (lane == 0) {
        atomicMax(&a.status[ST_CODE], DEV_POOL);
        a.status[ST_POOL] = 1;
      }
      return 2;
    }
    ub = (int)ubl;
    lb = (int)lbl;
    al.unz += uc;
    al.lnz += lc;
    if (dnp) {
      // the descendant part the first step parked, four loads per lane in flight
      const int off = a.cb_off[k];
      for (int e0 = 0; e0 < dnp; e0 += 256) {
        int32_t ci[4];
        double cx[4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const int e = e0 + 64 * g + lane;
          ci[g] = e < dnp ? a.cbI[off + e] : 0;
          cx[g] = e < dnp ? a.cbX[off + e] : 0.0;
        }
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const int e = e0 + 64 * g + lane;
          if (e < dnp) {
            a.Ui[ub + e] = ci[g];
            a.Ux[ub + e] = cx[g];
          }
        }
      }
    }
    for (int e = lane; e < np; e += 64) {
      const unsigned long long key = w.sk[e];
      a.Ui[ub + dnp + e] = (int32_t)(key >> 32);
      a.Ux[ub + dnp + e] = w.val[w.ps[(int)(key & 0xffffffffu)]];
    }
    if (lane == 0) { a.Ui[ub + dnp + np] = k; a.Ux[ub + dnp + np] = xp; }
    int off = 0;
    for (int base = 0; base < nins; base += 64) {
      const int t = base + lane;
      int s = 0;
      bool sel = false;
      if (t < nins) {
        s = w.ins[t];
        sel = w.pv[s] < 0 && w.key[s] != p;
      }
      const unsigned long long bm = __ballot(sel);
      const int pos = off + __popcll(bm & ((1ull << lane) - 1ull));
      if (sel) {
        a.Li[lb + pos] = w.key[s];
        a.Lx[lb + pos] = w.val[s] / xp;
      }
      off += __popcll(bm);
    }
    if (lane == 0) {
      a.Lbeg[k] = lb; a.Lcnt[k] = lc; a.Ubeg[k] = ub; a.Ucnt[k] = uc;
      a.piv[k] = p;
    }
    if (p != k) al.offdiag++;
  } else {
    for (int e = lane; e < np; e += 64) a.Ux[ub + e] = w.val[w.ps[e]];
    if (lane == 0) a.Ux[ub + np] = xp;
    for (int t = lane; t < lc; t += 64) {
      const int s = ws_lookup(w, a.Li[lb + t]);
      if (s >= 0) a.Lx[lb + t] = w.val[s] / xp;
    }
  }
  if (a.refactor) {
    if (lane == 0) a.pinv[p] = k;
  } else {
    // claim the pivot row; a row can be claimed twice only by speculative columns.  A
    // speculative column stores its claim without waiting for the old value: the check
    // after the pass finds any row claimed twice (its pivot column is then not k).
    if (cx.spec) {
      if (lane == 0) __hip_atomic_store(&a.pinv[p], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int claimed = 1;
      if (lane == 0) claimed = atomicCAS(&a.pinv[p], -1, k) == -1;
      claimed = __shfl(claimed, 0, 64);
      if (!claimed) {
        if (lane == 0) {
          atomicMax(&a.status[ST_CODE], DEV_PATTERN);
          atomicMin(&a.status[ST_FAILCOL], k);
        }
        return 2;
      }
    }
  }
  pre.pp = p;
  pre.pk = k;
  return 0;
}

// HS hash slots and NPS pivotal-list entries per wave in LDS; a column moves to the
// global workspace past LQ quarters of the table (open addressing stays short at 3/4).
template <int HS, int NPS, int LQ = 2>
__global__ void __launch_bounds__(64) factor_kernel(FactorArgs a) {
  BASKER_SHARED(LdsWs<HS COMMA NPS>, lds);
  const int lane = lane_id();
  for (int t = lane; t < HS; t += 64) lds.key[t] = -1;
  if (lane == 0) { lds.cnt[0] = 0; lds.cnt[1] = 0; lds.cnt[2] = 0; lds.cnt[3] = 0; }
  Ws wl;
  wl.key = lds.key; wl.val = lds.val; wl.pv = lds.pv; wl.ins = lds.ins; wl.pj = lds.pj;
  wl.ps = lds.ps; wl.pb = lds.pb; wl.pc = lds.pc; wl.sk = lds.sk; wl.cnt = lds.cnt;
  wl.st_slot = lds.st_slot; wl.st_val = lds.st_val; wl.st_pre = lds.st_pre; wl.st_beg = lds.st_beg;
  wl.pso = lds.pso;
  wl.H = HS;
  wl.NP = NPS;
  wl.shift = 32 - __builtin_ctz(HS);
  wl.SC = kStage;
  wl.lim = HS / 4 * LQ;
  Ws wg;
  {
    const int H = a.gws_slots;
    char* base = a.gws + (int64_t)blockIdx.x * a.gws_stride;
    wg.key = (int32_t*)base;
    wg.val = (double*)(base + 4ll * H);
    wg.pv = (int32_t*)(base + 12ll * H);
    wg.ins = (int32_t*)(base + 16ll * H);
    wg.pj = (int32_t*)(base + 20ll * H);
    wg.ps = (int32_t*)(base + 24ll * H);
    wg.pb = (int32_t*)(base + 28ll * H);
    wg.pc = (int32_t*)(base + 32ll * H);
    wg.sk = (unsigned long long*)(base + 40ll * H);
    wg.cnt = (int32_t*)(base + 48ll * H);
    wg.st_slot = lds.st_slot; wg.st_val = lds.st_val; wg.st_pre = lds.st_pre; wg.st_beg = lds.st_beg;
    wg.pso = nullptr;
    wg.H = H;
    wg.NP = H;
    wg.shift = 32 - __builtin_ctz((unsigned)H);
    wg.SC = kStage;
    wg.lim = H >> 1;
  }
  wsync();
  const ColCtx cx0 = {0, nullptr, 0};
  Alloc al = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  Pre pre;
  pre.k = -1;
  pre.pp = -1;
  pre.pk = -1;
  pre.fresh = 0;
  if (a.mode == 1) {
    // one column at a time: every column of the level's separators is independent here
    const int ncols = a.col_end - a.col_begin;
    while (true) {
      int idx = 0;
      if (lane == 0) idx = atomicAdd(&a.lvl_ctr[a.level], 1);
      idx = __shfl(idx, 0, 64);
      if (idx >= ncols) break;
      if (ld_relaxed(&a.status[ST_CODE]) != DEV_OK) continue;
      const int k = a.col_list[a.col_begin + (a.reverse ? ncols - 1 - idx : idx)];
      int rc = factor_column(a, wl, k, al, pre, -1, cx0);
      if (rc == 1) {
        rc = factor_column(a, wg, k, al, pre, -1, cx0);
        if (rc == 1 && lane == 0) {
          atomicMax(&a.status[ST_CODE], DEV_WORKSPACE);
          atomicMin(&a.status[ST_FAILCOL], k);
          a.status[ST_WS] = 1;
        }
      }
      wsync();
    }
  } else {
    const int nitems = a.item_end - a.item_begin;
    while (true) {
      int idx = 0;
      if (lane == 0) idx = atomicAdd(&a.lvl_ctr[a.level], 1);
      idx = __shfl(idx, 0, 64);
      if (idx >= nitems) break;
      if (ld_relaxed(&a.status[ST_CODE]) != DEV_OK) continue;
      const int it = a.item_begin + (a.reverse ? nitems - 1 - idx : idx);
      for (int q = a.item_lo[it]; q < a.item_hi[it]; q++) {
        const int sg = a.lvl_seg[q];
        const int c0 = a.seg_c0[sg], c1 = a.seg_c1[sg];
        pre.k = -1;
        for (int k = c0; k < c1; k++) {
          const int knext = k + 1 < c1 ? k + 1 : -1;
          int rc = factor_column(a, wl, k, al, pre, knext, cx0);
          if (rc == 1) {
            rc = factor_column(a, wg, k, al, pre, knext, cx0);
            if (rc == 1 && lane == 0) {
              atomicMax(&a.status[ST_CODE], DEV_WORKSPACE);
              atomicMin(&a.status[ST_FAILCOL], k);
              a.status[ST_WS] = 1;
            }
          }
          if (rc != 0) break;
          // the next column reads this column's pinv/L/U entries written by other lanes
          wsync();
        }
      }
    }
  }
  if (lane == 0) {
    if (al.offdiag) atomicAdd(&a.status[ST_OFFDIAG], al.offdiag);
    if (!a.refactor && (al.lnz || al.unz)) {
      atomicAdd(&a.nnz_ctr[0], (unsigned long long)al.lnz);
      atomicAdd(&a.nnz_ctr[1], (unsigned long long)al.unz);
    }
  }
}

// ---------------------------------------------------------------------------
// First level on workgroups of NW wavefronts.  A workgroup takes one work item at a
// time (a large BTF block or ND leaf, or a run of small blocks); its waves take the
// item's columns in order from an LDS counter, and a wave starts column k once every
// column in k's dependency list is done (done bits in LDS, written with a release and
// read with an acquire at workgroup scope).  Columns are handed out in increasing
// order and every dependency precedes its column, so the earliest unfinished column
// can always run: the waits end.  A wait is still bounded (a stall is reported as an
// error, never a hang).
//
// With the dependencies of every pivot sequence (column elimination tree children) or
// the stored U pattern of a refactorization the result is the serial one.  With
// predicted dependencies (the U pattern without row exchanges, or one learned from an
// earlier factorization) the columns run speculatively: ColCtx's checks, the pivot
// claim and the check kernel after the launch flag every item whose result could
// differ from the serial one, and the redo pass factors those items again with the
// elimination-tree lists.  Accepted items are bit for bit the serial result: every
// row a column touched had the pivot status it has at that point of the serial order,
// and every L column it used was complete.
// ---------------------------------------------------------------------------
constexpr int kCoopStage = 256;
constexpr int kCoopDoneWords = kCoopMaxItemCols / 32;
constexpr unsigned kSpinLimit = 1u << 22;

template <int NW>
struct CoopCfg;
template <> struct CoopCfg<4> { static constexpr int H = 512; };
template <> struct CoopCfg<6> { static constexpr int H = 512; };
template <> struct CoopCfg<7> { static constexpr int H = 512; };   // the most 512-slot waves a CU's LDS holds
template <> struct CoopCfg<8> { static constexpr int H = 256; };

// dependency lists of up to this many columns are copied to LDS for the checks
constexpr int kCoopDepsLds = 64;

template <int NW>
struct CoopLds {
  LdsWs<CoopCfg<NW>::H, CoopCfg<NW>::H / 2, kCoopStage> ws[NW];
  unsigned done[kCoopDoneWords];
  int32_t deps[NW][kCoopDepsLds];
  int item, slot, bad, skip;
  unsigned long long ubase;
};

__device__ __forceinline__ bool done_bit(const unsigned* done, int slot) {
  const unsigned w = __hip_atomic_load(&done[slot >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return (w >> (slot & 31)) & 1u;
}

template <int NW>
__global__ void __launch_bounds__(64 * NW) factor_coop_kernel(FactorArgs a) {
  constexpr int HS = CoopCfg<NW>::H;
  BASKER_SHARED(CoopLds<NW>, sm);
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int lane = tid & 63;
  auto& L = sm.ws[wv];
  for (int t = lane; t < HS; t += 64) L.key[t] = -1;
  if (lane == 0) { L.cnt[0] = 0; L.cnt[1] = 0; L.cnt[2] = 0; L.cnt[3] = 0; }
  Ws wl;
  wl.key = L.key; wl.val = L.val; wl.pv = L.pv; wl.ins = L.ins; wl.pj = L.pj;
  wl.ps = L.ps; wl.pb = L.pb; wl.pc = L.pc; wl.sk = L.sk; wl.cnt = L.cnt;
  wl.st_slot = L.st_slot; wl.st_val = L.st_val; wl.st_pre = L.st_pre; wl.st_beg = L.st_beg;
  wl.pso = L.pso;
  wl.H = HS;
  wl.NP = HS / 2;
  wl.shift = 32 - __builtin_ctz(HS);
  wl.SC = kCoopStage;
  wl.lim = HS >> 1;
  Ws wg;
  {
    const int H = a.gws_slots;
    char* base = a.gws + ((int64_t)blockIdx.x * NW + wv) * a.gws_stride;
    wg.key = (int32_t*)base;
    wg.val = (double*)(base + 4ll * H);
    wg.pv = (int32_t*)(base + 12ll * H);
    wg.ins = (int32_t*)(base + 16ll * H);
    wg.pj = (int32_t*)(base + 20ll * H);
    wg.ps = (int32_t*)(base + 24ll * H);
    wg.pb = (int32_t*)(base + 28ll * H);
    wg.pc = (int32_t*)(base + 32ll * H);
    wg.sk = (unsigned long long*)(base + 40ll * H);
    wg.cnt = (int32_t*)(base + 48ll * H);
    wg.st_slot = L.st_slot; wg.st_val = L.st_val; wg.st_pre = L.st_pre; wg.st_beg = L.st_beg;
    wg.pso = nullptr;
    wg.H = H;
    wg.NP = H;
    wg.shift = 32 - __builtin_ctz((unsigned)H);
    wg.SC = kCoopStage;
    wg.lim = H >> 1;
  }
  Alloc al = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  long long sub_l = 0, sub_u = 0;
  int sub_off = 0;
  Pre pre;
  pre.k = -1; pre.pp = -1; pre.pk = -1; pre.fresh = 1;
  const int nitems = a.item_end - a.item_begin;
  while (true) {
    __syncthreads();
    if (tid == 0) {
      const int idx = atomicAdd(&a.lvl_ctr[a.level], 1);
      sm.item = idx < nitems ? a.item_begin + (a.reverse ? nitems - 1 - idx : idx) : -1;
      sm.slot = 0;
      sm.bad = 0;
      sm.skip = 0;
      if (sm.item >= 0 && a.redo) {
        sm.skip = __hip_atomic_load(&a.item_bad[sm.item], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        if (!sm.skip) atomicAdd(&a.status[ST_REDO], 1);
      }
    }
    __syncthreads();
    const int it = sm.item;
    if (it < 0) break;
    if (sm.skip) continue;
    const int kind = a.co_item_kind ? a.co_item_kind[it] : 0;
    if (kind == 2) {
      // 1 x 1 diagonal blocks, one thread each: the pivot is the block's only entry; U
      // takes one entry per column from one pool allocation for the item
      const int lo = a.co_item_lo[it], cnt = a.co_item_hi[it] - lo;
      if (!a.refactor) {
        if (tid == 0) {
          sm.ubase = atomicAdd(&a.pool_next[1], (unsigned long long)cnt);
          if ((long long)sm.ubase + cnt > a.Ucap) {
            atomicMax(&a.status[ST_CODE], DEV_POOL);
            a.status[ST_POOL] = 1;
          }
          al.unz += cnt;
        }
        __syncthreads();
        if ((long long)sm.ubase + cnt > a.Ucap) continue;
      }
      for (int i = tid; i < cnt; i += 64 * NW) {
        const int k = a.seg_c0[a.lvl_seg[lo + i]];
        const double x = a.Rx[a.Rp[k]];
        if (!a.refactor) {
          if (!(fabs(x) > 0.0)) {
            atomicMax(&a.status[ST_CODE], DEV_SINGULAR);
            atomicMin(&a.status[ST_FAILCOL], k);
            continue;
          }
          const int ub = (int)(sm.ubase + (unsigned long long)i);
          a.Ui[ub] = k;
          a.Ux[ub] = x;
          a.Ubeg[k] = ub;
          a.Ucnt[k] = 1;
          a.Lbeg[k] = 0;
          a.Lcnt[k] = 0;
          a.piv[k] = k;
          a.pinv[k] = k;
        } else {
          if (!(fabs(x) > 0.0) || a.Ucnt[k] != 1 || a.piv[k] != k) {
            atomicMax(&a.status[ST_CODE], DEV_REFACTOR_FAIL);
            atomicMin(&a.status[ST_FAILCOL], k);
            continue;
          }
          a.Ux[a.Ubeg[k]] = x;
          a.pinv[k] = k;
        }
      }
      continue;
    }
    if (kind == 1) {
      // segments of the small bin: one wavefront factors a whole segment column by
      // column (serial Gilbert-Peierls inside the segment; no waits between waves)
      const ColCtx cx0 = {0, nullptr, 0};
      const int lo = a.co_item_lo[it], nseg = a.co_item_hi[it] - lo;
      while (true) {
        int qi = 0;
        if (lane == 0) qi = atomicAdd(&sm.slot, 1);
        qi = __shfl(qi, 0, 64);
        if (qi >= nseg) break;
        if (ld_relaxed(&a.status[ST_CODE]) != DEV_OK) continue;
        const int sg = a.lvl_seg[lo + qi];
        const int c0 = a.seg_c0[sg], c1 = a.seg_c1[sg];
        pre.k = -1;
        pre.fresh = 0;
        for (int k = c0; k < c1; k++) {
          const int knext = k + 1 < c1 ? k + 1 : -1;
          const Pre pk = pre;
          int rc = factor_column(a, wl, k, al, pre, knext, cx0);
          if (rc == 1) {
            pre = pk;
            rc = factor_column(a, wg, k, al, pre, knext, cx0);
            if (rc == 1 && lane == 0) {
              atomicMax(&a.status[ST_CODE], DEV_WORKSPACE);
              atomicMin(&a.status[ST_FAILCOL], k);
              a.status[ST_WS] = 1;
            }
          }
          if (rc != 0) break;
          wsync();
        }
      }
      continue;
    }
    const int ncols = a.co_item_cols[it];
    for (int w = tid; w < ((ncols + 31) >> 5); w += 64 * NW) sm.done[w] = 0u;
    if (a.redo) {
      // clear what the failed speculation stored: pivots of the item's rows (the rows of
      // a diagonal block or ND leaf are its columns' indices), counts and offsets
      for (int q = a.co_item_lo[it]; q < a.co_item_hi[it]; q++) {
        const int sg = a.lvl_seg[q];
        for (int k = a.seg_c0[sg] + tid; k < a.seg_c1[sg]; k += 64 * NW) {
          a.pinv[k] = -1;
          if (a.Ucnt[k] > 0) {
            sub_u += a.Ucnt[k];
            sub_l += a.Lcnt[k];
            if (a.piv[k] != k) sub_off++;
          }
          a.Lcnt[k] = 0; a.Ucnt[k] = 0; a.Lbeg[k] = 0; a.Ubeg[k] = 0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
    __syncthreads();
    // this wave's cursor over the item's segments (slot order)
    int q = a.co_item_lo[it], base = 0;
    const int32_t* issue = a.use_issue ? a.co_issue + 3ll * a.co_item_off[it] : nullptr;
    while (true) {
      int i = 0;
      if (lane == 0) i = atomicAdd(&sm.slot, 1);
      i = __shfl(i, 0, 64);
      if (i >= ncols) break;
      int k, slot, sbase;
      if (issue) {
        k = issue[3 * i];
        slot = issue[3 * i + 1];
        sbase = slot - (k - issue[3 * i + 2]);
      } else {
        slot = i;
        while (slot >= base + (a.seg_c1[a.lvl_seg[q]] - a.seg_c0[a.lvl_seg[q]])) {
          base += a.seg_c1[a.lvl_seg[q]] - a.seg_c0[a.lvl_seg[q]];
          q++;
        }
        k = a.seg_c0[a.lvl_seg[q]] + (slot - base);
        sbase = base;
      }
      if (!a.refactor) {
        // R(:,k)'s rows and values do not depend on other columns: load them while
        // waiting (its rows' pivot status is read after the wait)
        const int rb = a.Rp[k], re = a.Rp[k + 1];
        pre.k = -1;
        if (re - rb <= 64) {
          pre.k = k;
          pre.b = rb;
          pre.e = re;
          pre.fresh = 1;
          if (lane < re - rb) {
            pre.r = a.Ri[rb + lane];
            pre.x = a.Rx[rb + lane];
          }
        }
      }
      const int32_t* dp;
      int nd;
      if (a.dep_src == 1) {
        dp = a.Ui + a.Ubeg[k];
        nd = a.Ucnt[k] - 1;
      } else {
        dp = a.dep_idx + a.dep_ptr[k];
        nd = a.dep_ptr[k + 1] - a.dep_ptr[k];
      }
      // wait for the dependencies (slots of the same segment: slot - (k - j)); a short
      // list is kept in LDS for the column's checks
      bool stalled = false;
      const bool deps_lds = nd <= kCoopDepsLds;
      for (int e = lane; e < nd; e += 64) {
        const int dj = dp[e];
        if (deps_lds) sm.deps[wv][e] = dj;
        const int js = slot - (k - dj);
        if (js < sbase || js >= slot) { stalled = true; break; }   // not an earlier column of the segment
        unsigned spins = 0;
        while (!done_bit(sm.done, js)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { stalled = true; break; }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      const bool any_stall = __any(stalled);
      int rc = 0;
      if (any_stall) {
        if (lane == 0) {
          atomicMax(&a.status[ST_CODE], DEV_STALL);
          atomicMin(&a.status[ST_FAILCOL], k);
        }
        rc = 2;
      } else if (__hip_atomic_load(&sm.bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) ||
                 ld_relaxed(&a.status[ST_CODE]) != DEV_OK) {
        rc = 2;   // the item is redone, or the factorization has failed: only release waiters
      } else {
        const ColCtx cx = {a.spec, deps_lds ? sm.deps[wv] : dp, nd};
        const Pre pk = pre;
        rc = factor_column(a, wl, k, al, pre, -1, cx);
        if (rc == 1) {
          pre = pk;
          rc = factor_column(a, wg, k, al, pre, -1, cx);
          if (rc == 1) {
            if (a.spec) {
              rc = 3;
            } else if (lane == 0) {
              atomicMax(&a.status[ST_CODE], DEV_WORKSPACE);
              atomicMin(&a.status[ST_FAILCOL], k);
              a.status[ST_WS] = 1;
            }
          }
        }
        if (rc == 3 && lane == 0) {
          sm.bad = 1;
          __hip_atomic_store(&a.item_bad[it], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // publish: the column's L, U, offsets and pivot before its done bit
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) atomicOr(&sm.done[slot >> 5], 1u << (slot & 31));
    }
  }
  // the wave's own columns (lane 0 holds the wave's tallies), and every thread's share
  // of what a redo took back (each thread cleared its own columns)
  long long dl = -sub_l, du = -sub_u;
  int doff = -sub_off;
  if (lane == 0) {
    dl += al.lnz;
    du += al.unz;
    doff += al.offdiag;
  }
  if (doff) atomicAdd(&a.status[ST_OFFDIAG], doff);
  if (!a.refactor && (dl || du)) {
    atomicAdd(&a.nnz_ctr[0], (unsigned long long)dl);
    atomicAdd(&a.nnz_ctr[1], (unsigned long long)du);
  }
}

// thread per first-level column (cols, or every column when cols is null): a row of
// L(:,k) whose pivot column is below k was pivotal when the serial order reaches k, so
// k's speculation was wrong
__global__ void factor_spec_check_kernel(FactorArgs a, int ncols, const int32_t* cols) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= ncols) return;
  const int k = cols ? cols[t] : t;
  const int it = a.col_item[k];
  if (it < 0 || a.item_bad[it]) return;
  // the column's pivot row holds its claim (no other column claimed it too)
  if (a.Ucnt[k] <= 0 || a.pinv[a.piv[k]] != k) {
    a.item_bad[it] = 1;
    return;
  }
  const int b = a.Lbeg[k], c = a.Lcnt[k];
  for (int e = 0; e < c; e++) {
    const int p = a.pinv[a.Li[b + e]];
    if (p >= 0 && p < k) {
      a.item_bad[it] = 1;
      return;
    }
  }
}

__global__ void factor_init_kernel(FactorArgs a, int32_t nlevels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n && !a.refactor) {
    a.pinv[i] = -1;
    a.Lbeg[i] = 0; a.Lcnt[i] = 0; a.Ubeg[i] = 0; a.Ucnt[i] = 0;
  }
  if (i < ST_WORDS) a.status[i] = (i == ST_FAILCOL) ? 0x7fffffff : 0;
  if (i < 2 * nlevels) a.lvl_ctr[i] = 0;
  // the separator partial-column buffer is refilled on every pass; the L/U pools keep
  // their columns in a refactorization
  if (i == 0) a.pool_next[2] = 0;
  if (i == 0 && !a.refactor) {
    a.pool_next[0] = 0; a.pool_next[1] = 0; a.nnz_ctr[0] = 0; a.nnz_ctr[1] = 0;
  }
}

__global__ void scatter_kernel(const double* __restrict__ vals, const int32_t* __restrict__ map,
                               double* __restrict__ out, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = vals[map[i]];
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = v;
}

}  // namespace

hipError_t launch_factor_init(const FactorArgs& a, int32_t nlevels, hipStream_t s) {
  int64_t cnt = a.n;
  if (cnt < ST_WORDS) cnt = ST_WORDS;
  if (cnt < nlevels) cnt = nlevels;
  const int blocks = (int)((cnt + 255) / 256);
  hipLaunchKernelGGL(factor_init_kernel, dim3(blocks), dim3(256), 0, s, a, nlevels);
  return hipGetLastError();
}

hipError_t launch_factor_level(const FactorArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((factor_kernel<kLdsSlots, kLdsSlots>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

int coop_lds_bytes(int waves) {
  if (waves == 4) return (int)sizeof(CoopLds<4>);
  if (waves == 6) return (int)sizeof(CoopLds<6>);
  if (waves == 7) return (int)sizeof(CoopLds<7>);
  if (waves == 8) return (int)sizeof(CoopLds<8>);
  return 0;
}

hipError_t launch_factor_coop(const FactorArgs& a, int waves, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (waves == 4)
    hipLaunchKernelGGL(factor_coop_kernel<4>, dim3(grid), dim3(64 * 4), 0, s, a);
  else if (waves == 8)
    hipLaunchKernelGGL(factor_coop_kernel<8>, dim3(grid), dim3(64 * 8), 0, s, a);
  else if (waves == 7)
    hipLaunchKernelGGL(factor_coop_kernel<7>, dim3(grid), dim3(64 * 7), 0, s, a);
  else
    hipLaunchKernelGGL(factor_coop_kernel<6>, dim3(grid), dim3(64 * 6), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_factor_spec_check(const FactorArgs& a, int ncols, const int32_t* cols, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(factor_spec_check_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s, a, ncols,
                     cols);
  return hipGetLastError();
}

hipError_t launch_factor_sep_step1(const FactorArgs& a, int grid, bool small, hipStream_t s) {
  if (small)
    hipLaunchKernelGGL((factor_kernel<kLdsSlotsStep1Small, kLdsSlotsStep1Small / 2, 3>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((factor_kernel<kLdsSlotsStep1, kLdsSlotsStep1 / 2>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_factor_sep_step2(const FactorArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((factor_kernel<kLdsSlotsSep, kLdsSlotsSep>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scatter(const double* vals, const int32_t* map, double* out, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, vals, map, out, cnt);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, v, cnt);
  return hipGetLastError();
}

}  // namespace basker
