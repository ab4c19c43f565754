// Numeric factorization on gfx950: a persistent kernel in which every wavefront
// repeatedly takes a ready column from a device queue and runs one column of the
// left-looking Gilbert-Peierls algorithm (Alg. 1) on it:
//
//   reach     breadth-first closure of struct(R(:,k)) over the graph of L, with the
//             discovered rows kept in a per-wave LDS hash table (lanes expand the
//             L columns of a whole frontier at once);
//   order     the pivotal rows of the reach sorted by pivot index -- ascending pivot
//             index is a topological order because every edge of the graph of L runs
//             from a lower to a higher pivot index;
//   update    x_r = x_r - l_rj * x_j over L(:,j), lanes over the rows of L(:,j);
//   pivot     wavefront max-reduction over the candidates (non-pivotal rows of the
//             column's group), diagonal preference by threshold, smallest index on ties;
//   store     U(:,k) ascending with the diagonal last, L(:,k) compacted by ballot and
//             prefix count, both appended to device pools by atomic bump allocation.
//
// Scheduling follows the level sets of Alg. 4: one launch per level, and in a level
// every wavefront takes whole segments (a BTF block, or one nested-dissection node)
// from an atomic counter and factors the segment's columns in order.  Segments of a
// level are independent (separate blocks, or ND nodes whose pivots stay inside the
// node), so no wavefront ever waits for another inside a launch; the kernel boundary
// between levels is the only synchronisation across workgroups.
//
// Arithmetic matches a serial run that updates in ascending pivot order: every update
// is a separately rounded multiply and subtract (built with -ffp-contract=off),
// L = x / pivot is an IEEE division, and each entry of x receives its updates in
// ascending pivot order.
#include "device.hpp"

namespace basker {

namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// One workgroup is one wavefront, so no hardware barrier is needed between lanes;
// what is needed is that every LDS and global access issued before this point has
// completed before any lane continues (lanes exchange data through LDS and, across
// columns, through the global arrays).  The fence keeps the compiler from moving
// memory operations across; the wait drains all outstanding memory counters.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
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
  int H;
  int shift;      // 32 - log2(H)
};

// Per-wave pool allocator: a wave claims a chunk of the L and U pools with one atomic
// and hands out column storage from it, so the device-wide counters see one atomic
// per chunk instead of two per column.
struct Alloc {
  long long lcur, lend, ucur, uend, ccur, cend;
  long long lnz, unz;
  int offdiag;
};

template <int H>
struct LdsWs {
  int32_t key[H];
  double val[H];
  int32_t pv[H];
  int32_t ins[H];
  int32_t pj[H];
  int32_t ps[H];
  int32_t pb[H];
  int32_t pc[H];
  unsigned long long sk[H];
  int32_t cnt[4];
};

__device__ __forceinline__ unsigned hash_of(int32_t r, int shift) {
  return ((unsigned)r * 2654435761u) >> shift;
}

// insert r; returns the slot and whether it is new; -1 when the table is full.
// The overflow flag is raised once more than half of the slots are in use.
__device__ __forceinline__ int ws_insert(const Ws& w, int32_t r, bool* isnew) {
  unsigned h = hash_of(r, w.shift);
  const unsigned mask = (unsigned)w.H - 1u;
  for (int t = 0; t < w.H; t++) {
    int old = atomicCAS(&w.key[h], -1, r);
    if (old == -1) {
      int pos = atomicAdd(&w.cnt[0], 1);
      w.ins[pos] = (int32_t)h;
      if (pos >= (w.H >> 1)) w.cnt[2] = 1;
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
  w.pj[e] = j;
  w.ps[e] = slot;
  w.pb[e] = 0;
  w.pc[e] = 0;
}

// Sort the pivotal list [0, np) by pivot column: sk[t] = (j << 32 | list index),
// ascending.  Keys are distinct.  Bitonic network in registers (np <= 64) or LDS.
__device__ void plist_sort(const Ws& w, int np) {
  const int lane = lane_id();
  if (np <= 64) {
    unsigned long long v = ~0ull;
    if (lane < np) v = ((unsigned long long)(unsigned)w.pj[lane] << 32) | (unsigned)lane;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        unsigned long long o = __shfl_xor(v, j, 64);
        bool up = ((lane & k) == 0);
        bool lower = ((lane & j) == 0);
        unsigned long long mn = v < o ? v : o, mx = v < o ? o : v;
        v = (lower == up) ? mn : mx;
      }
    }
    if (lane < np) w.sk[lane] = v;
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
__device__ void expand_frontier(const FactorArgs& a, const Ws& w, int f0, int f1) {
  const int lane = lane_id();
  for (int c0 = f0; c0 < f1; c0 += 64) {
    const int e = c0 + lane;
    int beg = 0, cnt = 0;
    if (e < f1) {
      const int j = w.pj[e];
      beg = a.Lbeg[j];
      cnt = a.Lcnt[j];
      w.pb[e] = beg;
      w.pc[e] = cnt;
    }
    const int incl = wave_incl_scan(cnt);
    const int excl = incl - cnt;
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      // owner lane: largest o with excl_o <= t
      int o = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        int cand = o + step;
        int ex = __shfl(excl, cand & 63, 64);
        if (cand < 64 && ex <= t) o = cand;
      }
      const int ob = __shfl(beg, o, 64);
      const int oe = __shfl(excl, o, 64);
      if (t < total) {
        const int32_t r = a.Li[ob + (t - oe)];
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0 && isnew) {
          w.val[slot] = 0.0;
          const int32_t pvr = a.pinv[r];
          w.pv[slot] = pvr;
          if (pvr >= 0) plist_push(w, pvr, slot);
        }
      }
    }
  }
  wsync();
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

__device__ int factor_column(const FactorArgs& a, const Ws& w, int k, Alloc& al) {
  const int lane = lane_id();
  ws_reset(w);
  const int g0 = a.grp_lo[k], g1 = a.grp_hi[k];

  int ub = 0, uc = 0, lb = 0, lc = 0, p = -1;
  if (!a.refactor || a.mode == 1) {
    if (a.mode != 2) {
      // struct(R(:,k)) with values
      for (int q = a.Rp[k] + lane; q < a.Rp[k + 1]; q += 64) {
        const int32_t r = a.Ri[q];
        bool isnew;
        int slot = ws_insert(w, r, &isnew);
        if (slot >= 0) {
          w.val[slot] = a.Rx[q];
          const int32_t pvr = a.pinv[r];
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
      expand_frontier(a, w, f0, f1);
      f0 = f1;
      f1 = w.cnt[1];
    }
    wsync();
    if (w.cnt[2]) return 1;
  } else {
    // known pattern: U(:,k) rows (pivotal, ascending) and L(:,k) rows plus the pivot
    ub = a.Ubeg[k]; uc = a.Ucnt[k]; lb = a.Lbeg[k]; lc = a.Lcnt[k];
    p = a.piv[k];
    if (uc - 1 + lc + 1 > (w.H >> 1)) return 1;
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

  // topological order: ascending pivot column
  const int np = w.cnt[1];
  if (!a.refactor || a.mode == 1) {
    plist_sort(w, np);
  } else {
    for (int t = lane; t < np; t += 64) w.sk[t] = ((unsigned long long)(unsigned)w.pj[t] << 32) | (unsigned)t;
    wsync();
  }

  // sparse triangular update
  for (int e = 0; e < np; e++) {
    const int src = (int)(w.sk[e] & 0xffffffffu);
    const int s = w.ps[src];
    const int beg = w.pb[src];
    const int c = w.pc[src];
    const double xj = w.val[s];
    for (int t = lane; t < c; t += 64) {
      const int32_t r = a.Li[beg + t];
      const double l = a.Lx[beg + t];
      const int slot = ws_lookup(w, r);
      const double prod = l * xj;
      if (slot >= 0) w.val[slot] = w.val[slot] - prod;
      else w.cnt[3] = 1;
    }
    wsync();
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
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const double ob = __shfl_xor(best, d, 64);
    const int oi = __shfl_xor(bidx, d, 64);
    if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
  }
  const unsigned long long dmask = __ballot(has_diag);
  if (dmask) xd = __shfl(xd, __ffsll((long long)dmask) - 1, 64);
  const double m = best;   // -1 when there is no candidate

  if (!a.refactor) {
    if (!(m > 0.0)) {
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
      const int off = a.cb_off[k];
      for (int e = lane; e < dnp; e += 64) {
        a.Ui[ub + e] = a.cbI[off + e];
        a.Ux[ub + e] = a.cbX[off + e];
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
  if (lane == 0) a.pinv[p] = k;
  return 0;
}

template <int HS>
__global__ void __launch_bounds__(64) factor_kernel(FactorArgs a) {
  BASKER_SHARED(LdsWs<HS>, lds);
  const int lane = lane_id();
  for (int t = lane; t < HS; t += 64) lds.key[t] = -1;
  if (lane == 0) { lds.cnt[0] = 0; lds.cnt[1] = 0; lds.cnt[2] = 0; lds.cnt[3] = 0; }
  Ws wl;
  wl.key = lds.key; wl.val = lds.val; wl.pv = lds.pv; wl.ins = lds.ins; wl.pj = lds.pj;
  wl.ps = lds.ps; wl.pb = lds.pb; wl.pc = lds.pc; wl.sk = lds.sk; wl.cnt = lds.cnt;
  wl.H = HS;
  wl.shift = 32 - __builtin_ctz(HS);
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
    wg.H = H;
    wg.shift = 32 - __builtin_ctz((unsigned)H);
  }
  wsync();
  Alloc al = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (a.mode == 1) {
    // one column at a time: every column of the level's separators is independent here
    const int ncols = a.col_end - a.col_begin;
    while (true) {
      int idx = 0;
      if (lane == 0) idx = atomicAdd(&a.lvl_ctr[a.level], 1);
      idx = __shfl(idx, 0, 64);
      if (idx >= ncols) break;
      if (ld_relaxed(&a.status[ST_CODE]) != DEV_OK) continue;
      const int k = a.col_list[a.col_begin + idx];
      int rc = factor_column(a, wl, k, al);
      if (rc == 1) {
        rc = factor_column(a, wg, k, al);
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
      const int it = a.item_begin + idx;
      for (int q = a.item_lo[it]; q < a.item_hi[it]; q++) {
        const int sg = a.lvl_seg[q];
        const int c0 = a.seg_c0[sg], c1 = a.seg_c1[sg];
        for (int k = c0; k < c1; k++) {
          int rc = factor_column(a, wl, k, al);
          if (rc == 1) {
            rc = factor_column(a, wg, k, al);
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

__global__ void factor_init_kernel(FactorArgs a, int32_t nlevels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n && !a.refactor) a.pinv[i] = -1;
  if (i < ST_WORDS) a.status[i] = (i == ST_FAILCOL) ? 0x7fffffff : 0;
  if (i < 2 * nlevels) a.lvl_ctr[i] = 0;
  if (i == 0 && !a.refactor) {
    a.pool_next[0] = 0; a.pool_next[1] = 0; a.pool_next[2] = 0; a.nnz_ctr[0] = 0; a.nnz_ctr[1] = 0;
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
  hipLaunchKernelGGL(factor_kernel<kLdsSlots>, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_factor_sep_step2(const FactorArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(factor_kernel<kLdsSlotsSep>, dim3(grid), dim3(64), 0, s, a);
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
