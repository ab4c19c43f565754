// Solve on gfx950: block back-substitution over the block triangular form (Sec. II).
//
// R = A(prow, qcol) is block upper triangular, so block b needs the solution of every
// later block it couples to: r_b = c_b - sum_{c > b} R_bc z_c, then L w = r(piv) and
// U z_b = w.  The work is cut into tasks that run in levels, one launch per level:
//   block task    : one block without an ND tree (residual, L rows, U rows);
//   forward task  : the L rows of one ND node (its rows depend on its own rows and on
//                   its descendants', which earlier levels finished);
//   backward task : the U rows of one ND node, root first (its rows depend on its own
//                   rows and on its ancestors', finished earlier).
// By default one launch runs every task (solve_flow_kernel): a workgroup takes the
// tasks in an issue order, waits on the done flags of the ND tasks it depends on, and
// waits for each coupled solution entry of a later block one by one (the solution
// vector holds a pending pattern until the entry is published); the launches per level
// remain as an option.
// A task is one workgroup of kSW wavefronts.  The waves take the task's rows round
// robin in an issue order, and a row waits only for the rows of the same task it reads
// (done bits in LDS, release/acquire at workgroup scope).  The issue order of a
// first-level task lists its rows by levels of the predicted dependency graph (rows
// with no dependency inside the task first), so independent rows do not queue behind
// a chain; after every factorization a check against the actual rows keeps an order
// only where every row's dependencies come before it, else the sweep's own order
// (ascending for L, descending for U) is used.  Either way a wave finishes a row before
// taking its next one and the first unfinished row in the order can always proceed.
//
// Each unknown is computed from one row of the factors, with the updates subtracted
// one at a time in the order the column sweep applies them: the coupling entries of
// the row (later blocks first, columns ascending inside a block), then L's entries in
// ascending column, or U's in descending column, each product rounded and subtracted
// separately, and z_k = w_k / u_kk.  The result is the column sweep's, bit for bit, and
// does not depend on the schedule.
#include "device.hpp"

#include <algorithm>
#include <map>
#include <mutex>

namespace basker {

// Work vectors of basker_solve_noalloc: W and Z of one solve.  Every device the
// library runs on holds its own copy until the process ends.  Host code never uses
// this name as an address: noalloc_scratch looks the device address up once per
// device and every launch takes that pointer.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ double rl_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Ordering between a row's value and its done bit.  In LDS a wavefront's LDS accesses
// are performed in program order, so only the compiler must keep them in order; in
// global memory the value is released and acquired at workgroup scope.
template <bool kLds>
__device__ __forceinline__ void publish_fence() {
  if (kLds) __atomic_signal_fence(__ATOMIC_SEQ_CST);
  else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}
template <bool kLds>
__device__ __forceinline__ void consume_fence() {
  if (kLds) __atomic_signal_fence(__ATOMIC_SEQ_CST);
  else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// done bit of task row i: in LDS, or in the global flag array (one word a row)
template <bool kLds>
struct Flags {
  unsigned* lds;       // m bits
  int32_t* glob;       // the task's rows of the global array
  __device__ __forceinline__ bool test(int i) const {
    if (kLds) return (__hip_atomic_load(&lds[i >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> (i & 31)) & 1u;
    return __hip_atomic_load(&glob[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
  }
  __device__ __forceinline__ void set(int i) const {
    if (kLds) atomicOr(&lds[i >> 5], 1u << (i & 31));
    else __hip_atomic_store(&glob[i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ void clear(int m, int tid) const {
    if (kLds) for (int w = tid; w < ((m + 31) >> 5); w += 64 * kSW) lds[w] = 0u;
    else for (int i = tid; i < m; i += 64 * kSW) glob[i] = 0;
  }
};

// acc - sum over entries, one at a time in entry order: lanes hold up to 64 products
__device__ __forceinline__ double subtract_in_order(double acc, double prod, int cnt) {
  for (int t = 0; t < cnt; t++) acc = acc - rl_d(prod, t);
  return acc;
}

// In the lane-per-row sweep a row's LDS value is its done flag: V holds kPending until
// the row's result is stored there with one 64-bit access.  kPending is a signaling NaN,
// which no arithmetic result equals; a result with exactly that bit pattern (only a
// copied input can have it) is stored quieted.
constexpr unsigned long long kPending = 0x7ff0dead5a5a5a5aull;

__device__ __forceinline__ bool pending_load(const double* V, int i, double& v) {
  const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(V) + i, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
  v = __longlong_as_double((long long)b);
  return b != kPending;
}

__device__ __forceinline__ void result_store(double* V, int i, double z) {
  unsigned long long b = (unsigned long long)__double_as_longlong(z);
  if (b == kPending) b |= 1ull << 51;
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(V) + i, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The solution vector Z is also a set of done flags, across workgroups: it holds
// kPending before the solve, and every unknown is stored there once, final, by the
// backward sweep that computes it, with one 64-bit store at agent scope (it reaches the
// memory every XCD reads); a row of another task reads it with agent-scope loads until
// the value is no longer kPending.  No fence is needed: the value is its own flag.
__device__ __forceinline__ void publish_store(double* Zp, int i, double z) {
  unsigned long long b = (unsigned long long)__double_as_longlong(z);
  if (b == kPending) b |= 1ull << 51;
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(Zp) + i, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool published_load(const double* Z, int j, double& v) {
  const unsigned long long b = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(Z) + j, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  v = __longlong_as_double((long long)b);
  return b != kPending;
}

// Bound of a wait for another task's results: 10 s of the 100 MHz real-time counter (a
// producing task can legitimately run for tens of milliseconds), or less once another
// wait of the launch has given up (status bit 8, read at a wait's first failed poll and
// every 256 polls after it).
constexpr unsigned long long kFlowWaitTicks = 1000000000ull;

// Wait until Z[j] is published; false (and status bit 8 set) when the wait gave up.
__device__ __forceinline__ bool wait_published(const SolveArgs& a, const double* Z, int j, double& v) {
  const unsigned long long w0 = __builtin_amdgcn_s_memrealtime();
  unsigned spins = 0;
  while (!published_load(Z, j, v)) {
    __builtin_amdgcn_s_sleep(2);
    if ((++spins & 255u) == 1 &&
        (__builtin_amdgcn_s_memrealtime() - w0 > kFlowWaitTicks ||
         (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8))) {
      __hip_atomic_fetch_or(a.status, 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v = 0.0;
      return false;
    }
  }
  return true;
}

// The first (up to) 64 entries of a sorted factor row, loaded ahead of their use: the
// lane's column and value, and the row's entry range.
struct RowPre {
  int e0, e1;
  int j;
  double x;
};

// ptr: the task's slice of the row pointers (in LDS, or global for tasks beyond LDS),
// kk the task-local row
__device__ __forceinline__ void row_prefetch(RowPre& r, const int32_t* ptr, const unsigned long long* keys,
                                             const double* vals, int kk, bool rev, int n, int lane) {
  r.e0 = ptr[kk];
  r.e1 = ptr[kk + 1];
  r.j = -1;
  r.x = 0.0;
  if (lane < r.e1 - r.e0) {
    const unsigned lo = (unsigned)keys[r.e0 + lane];
    r.j = rev ? n - 1 - (int)lo : (int)lo;
    r.x = vals[r.e0 + lane];
  }
}

// Subtract a sorted factor row from acc: columns inside the task's rows [r0, r0 + m)
// are read from V after their done bits, any other column is final and read from `fin`.
// Returns false on a stall.
// Subtract a sorted factor row from acc: columns inside the task's rows [r0, r0 + m)
// are read from V after their done bits, any other column is final and read from `fin`.
// A row longer than 64 entries is taken 64 at a time with two chunks of loads ahead:
// while chunk c is subtracted, the final values of chunk c + 1 and the entries of
// chunk c + 2 are in flight.  Returns false on a stall.
template <bool kLds>
__device__ __forceinline__ bool row_update(double& acc, const RowPre& r, const unsigned long long* keys,
                                           const double* vals, bool rev, int n, int r0, int m, const double* V,
                                           const Flags<kLds>& F, const double* fin, int lane) {
  bool stalled = false;
  // chunk c (j0, x0, v0: the final value of an outside column), chunk c + 1 (j1, x1)
  int j0 = r.j, j1 = -1;
  double x0 = r.x, x1 = 0.0;
  double v0 = (j0 >= 0 && (j0 < r0 || j0 >= r0 + m)) ? fin[j0] : 0.0;
  if (r.e0 + 64 + lane < r.e1) {
    const unsigned lo = (unsigned)keys[r.e0 + 64 + lane];
    j1 = rev ? n - 1 - (int)lo : (int)lo;
    x1 = vals[r.e0 + 64 + lane];
  }
  for (int b = r.e0; b < r.e1; b += 64) {
    const int cnt = (r.e1 - b < 64) ? r.e1 - b : 64;
    int j2 = -1;
    double x2 = 0.0, v1 = 0.0;
    if (b + 64 < r.e1) {   // uniform
      if (b + 128 + lane < r.e1) {
        const unsigned lo = (unsigned)keys[b + 128 + lane];
        j2 = rev ? n - 1 - (int)lo : (int)lo;
        x2 = vals[b + 128 + lane];
      }
      if (j1 >= 0 && (j1 < r0 || j1 >= r0 + m)) v1 = fin[j1];
    }
    double prod = 0.0;
    if (lane < cnt) {
      const int jj = j0 - r0;
      double v = v0;
      if (jj >= 0 && jj < m) {
        unsigned spins = 0;
        while (!F.test(jj)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { stalled = true; break; }
        }
        consume_fence<kLds>();
        v = V[jj];
      }
      prod = x0 * v;
    }
    acc = subtract_in_order(acc, prod, cnt);
    j0 = j1;
    x0 = x1;
    v0 = v1;
    j1 = j2;
    x1 = x2;
  }
  return !__any(stalled);
}

// Rows in flight per wavefront: each wave loads the entries of its next kPre rows while
// it works on the current one, so a row's global loads are issued kPre rows early.
constexpr int kPre = 4;

// One sweep of a task over its rows in issue order: row q of the order is taken by wave
// q mod kSW.  `P` holds the rows' entry ranges by task-local row, `O` the issue order
// (task-local rows, minus `ooff`), null for the plain order (ascending for L, descending
// for U).  The backward sweep divides by the diagonal.  Returns false on a stall.
template <bool kLds, bool kBack>
__device__ __forceinline__ bool sweep(const SolveArgs& a, double* V, const int32_t* P, const int32_t* O, int ooff,
                                      const unsigned long long* keys, const double* vals, const Flags<kLds>& F,
                                      const double* fin, double* Zp, int r0, int m, int wv, int lane) {
  const int n = a.n;
  RowPre pre[kPre];
  int kr[kPre];
  double dg[kPre];
#pragma unroll
  for (int i = 0; i < kPre; i++) {
    const int q = wv + i * kSW;
    kr[i] = 0;
    dg[i] = 1.0;
    if (q < m) {
      kr[i] = O ? O[q] - ooff : (kBack ? m - 1 - q : q);
      row_prefetch(pre[i], P, keys, vals, kr[i], kBack, n, lane);
      if (kBack) dg[i] = a.diag[r0 + kr[i]];
    }
  }
  bool ok = true;
  // the row in slot 0 is worked on; the others move down a slot after it, and the row
  // kPre rows later is prefetched into the last slot (every slot index is static)
  for (int q = wv; q < m; q += kSW) {
    double acc = V[kr[0]];
    ok &= row_update<kLds>(acc, pre[0], keys, vals, kBack, n, r0, m, V, F, fin, lane);
    if (kBack) acc = acc / dg[0];
    if (lane == 0) {
      V[kr[0]] = acc;
      if (kBack) publish_store(Zp, kr[0], acc);
    }
    publish_fence<kLds>();
    if (lane == 0) F.set(kr[0]);
#pragma unroll
    for (int i = 0; i + 1 < kPre; i++) {
      pre[i] = pre[i + 1];
      kr[i] = kr[i + 1];
      dg[i] = dg[i + 1];
    }
    const int qn = q + kPre * kSW;
    if (qn < m) {
      kr[kPre - 1] = O ? O[qn] - ooff : (kBack ? m - 1 - qn : qn);
      row_prefetch(pre[kPre - 1], P, keys, vals, kr[kPre - 1], kBack, n, lane);
      if (kBack) dg[kPre - 1] = a.diag[r0 + kr[kPre - 1]];
    }
  }
  return ok;
}

// Entries a thread holds in LDS for its current row (the lane-per-row sweep).
constexpr int kSlot = 8;

// LDS slots of the lane-per-row sweep: kSlot entries for each of the 64 kSW threads,
// entry t of thread i at t * 64 kSW + i: the task-local row of the entry's column (-1
// for a column outside the task, whose product the prefix pass already subtracted) and
// the entry's value.
struct Slots {
  int32_t* Sj;
  double* Sx;
};

// The coupling entries of a block task's row still to subtract, when the row-per-thread
// forward sweep takes them itself (Zr non-null): entries [q, qe) of the row in the
// off-diagonal part, the next one's column and value.  The row then starts from its
// right-hand side and needs none of its task's other rows' couplings to begin.
struct ResCur {
  int q, qe, j;
  double x;
};

__device__ __forceinline__ void res_open(ResCur& c, const SolveArgs& a, const double* Zr, int r0, int kk) {
  c.q = c.qe = 0;
  c.j = 0;
  c.x = 0.0;
  if (Zr != nullptr && kk >= 0) {
    const int i = a.piv[r0 + kk];
    c.q = a.OTp[i];
    c.qe = a.OTp[i + 1];
    if (c.q < c.qe) {
      c.j = a.OTj[c.q];
      c.x = a.OTx[c.q];
    }
  }
}

// Subtract the next coupling entry if its value is published; true on progress.
__device__ __forceinline__ bool res_step(ResCur& c, const SolveArgs& a, const double* Zr, double& acc) {
  double z;
  if (!published_load(Zr, c.j, z)) return false;
  acc = acc - c.x * z;
  c.q++;
  if (c.q < c.qe) {
    c.j = a.OTj[c.q];
    c.x = a.OTx[c.q];
  }
  return true;
}

// A row's first kSlot entries in registers (loaded a round before their use).
struct RowRegs {
  int k, e0, e1;
  double d;
  double acc;
  ResCur rc;
  int j[kSlot];
  double x[kSlot];
};

template <bool kBack>
__device__ __forceinline__ void load_row_regs(RowRegs& R, const SolveArgs& a, const int32_t* P, const int32_t* O,
                                              const unsigned long long* keys, const double* vals, const double* A0,
                                              const double* Zr, int r0, int m, int q) {
  R.k = -1;
  R.e0 = R.e1 = 0;
  R.d = 1.0;
  R.acc = 0.0;
  if (q < m) {
    R.k = O ? O[q] : (kBack ? m - 1 - q : q);
    R.e0 = P[R.k];
    R.e1 = P[R.k + 1];
    R.acc = A0[R.k];
    if (kBack) R.d = a.diag[r0 + R.k];
  }
  res_open(R.rc, a, Zr, r0, R.k);
#pragma unroll
  for (int t = 0; t < kSlot; t++) {
    R.j[t] = 0;
    R.x[t] = 0.0;
    if (R.e0 + t < R.e1) {
      const unsigned lo = (unsigned)keys[R.e0 + t];
      R.j[t] = kBack ? a.n - 1 - (int)lo : (int)lo;
      R.x[t] = vals[R.e0 + t];
    }
  }
}

__device__ __forceinline__ void store_slots(const Slots& S, int tid, const int* j, const double* x, int from, int e1,
                                            int r0, int m) {
  constexpr int T = 64 * kSW;
#pragma unroll
  for (int t = 0; t < kSlot; t++) {
    if (from + t < e1) {
      const int jj = j[t] - r0;
      S.Sj[t * T + tid] = (jj >= 0 && jj < m) ? jj : -1;
      S.Sx[t * T + tid] = x[t];
    }
  }
}

// The prefix of a row: its entries in columns outside the task come first in the
// sweep's order (columns of earlier tasks: descendants' before an ND node's own in L,
// ancestors' before them in U), and their values are final.  Thread per row, four
// entries' loads at a time; V[kk] -= the prefix, products subtracted one at a time.
template <bool kBack>
__device__ __forceinline__ void apply_prefixes(const SolveArgs& a, double* G, const int32_t* P,
                                               const unsigned long long* keys, const double* vals, const double* fin,
                                               int r0, int m, int tid) {
  const int n = a.n;
  for (int kk = tid; kk < m; kk += 64 * kSW) {
    int e = P[kk];
    const int e1 = P[kk + 1];
    double acc = G[kk];
    bool more = true;
    while (more && e < e1) {
      int j[4];
      double x[4], f[4];
      bool out[4];
#pragma unroll
      for (int t = 0; t < 4; t++) {
        j[t] = 0;
        x[t] = 0.0;
        if (e + t < e1) {
          const unsigned lo = (unsigned)keys[e + t];
          j[t] = kBack ? n - 1 - (int)lo : (int)lo;
          x[t] = vals[e + t];
        }
        out[t] = e + t < e1 && (j[t] < r0 || j[t] >= r0 + m);
      }
#pragma unroll
      for (int t = 0; t < 4; t++) f[t] = out[t] ? fin[j[t]] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        if (more && out[t]) acc = acc - x[t] * f[t];
        else more = false;
      }
      e += 4;
    }
    G[kk] = acc;
  }
}

// The sweep with one row per thread, for tasks in LDS whose rows are short: 64 kSW rows
// in flight.  The wavefronts work in rounds: in round r lane i of wave w takes position
// r 64 kSW + 64 w + i of the issue order, and the wave moves to its next round once all
// its rows are done.  A row's first entries are loaded into registers a round ahead and
// put into LDS slots when its round begins, so inside a round only rows longer than
// kSlot load from global memory.  A thread never blocks: every pass it subtracts the
// next entry of its row if that entry's row is done, so lanes waiting on one another
// still advance; entries are subtracted one at a time in the row's order.  Returns
// false on a stall.
template <bool kBack>
__device__ __forceinline__ bool sweep_lanes(const SolveArgs& a, double* V, const int32_t* P, const int32_t* O,
                                            const unsigned long long* keys, const double* vals, const double* A0,
                                            const Slots& S, double* Zp, const double* Zr, int r0, int m,
                                            int tid) {
  constexpr int T = 64 * kSW;
  const int n = a.n;
  RowRegs nx;
  load_row_regs<kBack>(nx, a, P, O, keys, vals, A0, Zr, r0, m, tid);
  unsigned idle = 0;
  bool stalled = false;
  for (int q = tid; __any(q < m); q += T) {
    const int kc = nx.k;
    int p = nx.e0, sb = nx.e0;
    const int e1 = nx.e1;
    const double dg = nx.d;
    double acc = nx.acc;
    ResCur rc = nx.rc;
    bool busy = kc >= 0;
    // the window: entries p and p + 1 of the row, the second only while it is in the
    // slots (lim: the last slot holding an entry)
    int j0 = -1, j1 = -1, lim = 0;
    double x0 = 0.0, x1 = 0.0;
    if (busy) {
      store_slots(S, tid, nx.j, nx.x, p, e1, r0, m);
      if (p < e1) {
        lim = (e1 - sb < kSlot ? e1 - sb : kSlot) - 1;
        j0 = nx.j[0] - r0;
        j0 = (j0 >= 0 && j0 < m) ? j0 : -1;
        x0 = nx.x[0];
        j1 = nx.j[1] - r0;
        j1 = (j1 >= 0 && j1 < m) ? j1 : -1;
        x1 = nx.x[1];
      }
    }
    load_row_regs<kBack>(nx, a, P, O, keys, vals, A0, Zr, r0, m, q + T);
    while (__any(busy)) {
      bool prog = false;
      if (busy && rc.q < rc.qe) {
        prog = res_step(rc, a, Zr, acc);
      } else if (busy) {
        if (p < e1) {
          double v0 = 0.0, v1 = 0.0;
          const bool c0 = pending_load(V, j0 >= 0 ? j0 : 0, v0) || j0 < 0;
          const bool c1 = c0 && (pending_load(V, j1 >= 0 ? j1 : 0, v1) || j1 < 0) && p - sb + 1 <= lim;
          double u = acc - x0 * v0;
          acc = (c0 && j0 >= 0) ? u : acc;
          u = acc - x1 * v1;
          acc = (c1 && j1 >= 0) ? u : acc;
          const int c = (int)c0 + (int)c1;
          p += c;
          if (c > 0 && p < e1) {
            if (p - sb >= kSlot) {
              // past the slots: the next kSlot entries from global memory
              int j[kSlot];
              double x[kSlot];
#pragma unroll
              for (int t = 0; t < kSlot; t++) {
                j[t] = 0;
                x[t] = 0.0;
                if (p + t < e1) {
                  const unsigned lo = (unsigned)keys[p + t];
                  j[t] = kBack ? n - 1 - (int)lo : (int)lo;
                  x[t] = vals[p + t];
                }
              }
              sb = p;
              lim = (e1 - sb < kSlot ? e1 - sb : kSlot) - 1;
              store_slots(S, tid, j, x, p, e1, r0, m);
            }
            const int u0 = p - sb, u1 = p - sb + 1 <= lim ? p - sb + 1 : lim;
            j0 = S.Sj[u0 * T + tid];
            x0 = S.Sx[u0 * T + tid];
            j1 = S.Sj[u1 * T + tid];
            x1 = S.Sx[u1 * T + tid];
          }
          prog = c > 0;
        }
        if (p >= e1) {
          const double z = kBack ? acc / dg : acc;
          result_store(V, kc, z);
          if (kBack) publish_store(Zp, kc, z);
          busy = false;
          prog = true;
        }
      }
      if (__any(prog)) {
        idle = 0;
      } else {
        __builtin_amdgcn_s_sleep(1);
        if (++idle > kSpinLimit) { stalled = true; break; }
      }
    }
    if (stalled) break;
  }
  return !stalled;
}

// Residual of task row kk: the right-hand side minus the coupling to later blocks, in
// the sweep's order; the entries' loads are issued four at a time, and an entry not yet
// published is waited for.  ok turns false when a wait gave up.
__device__ __forceinline__ double residual_row(const SolveArgs& a, const double* Bc, const double* Z, int i,
                                               bool& ok) {
  double acc = Bc[a.prow[i]];
  int q = a.OTp[i];
  const int qe = a.OTp[i + 1];
  for (; q < qe; q += 4) {
    const int c = qe - q;
    int j[4];
    double x[4], z[4];
    bool r[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      j[t] = t < c ? a.OTj[q + t] : 0;
      x[t] = t < c ? a.OTx[q + t] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; t++) r[t] = t >= c || published_load(Z, j[t], z[t]);
#pragma unroll
    for (int t = 0; t < 4; t++)
      if (!r[t]) ok &= wait_published(a, Z, j[t], z[t]);
#pragma unroll
    for (int t = 0; t < 4; t++)
      if (t < c) acc = acc - x[t] * z[t];
  }
  return acc;
}

// The sweep with one row per thread on a task whose entries are all in LDS: Ej holds the
// task-local row of every entry's column (-1 outside the task), Ex its value, entry e of
// the rows at e - e_base.  Rounds and the never-blocking loop as in sweep_lanes; a
// thread keeps the next four entries of its row in registers, and a pass polls the
// first two and subtracts the leading ones whose rows are done (one LDS round trip a
// pass).  Returns false on a stall.
template <bool kBack>
__device__ __forceinline__ bool sweep_staged(const SolveArgs& a, double* V, const int32_t* P, const int32_t* O,
                                             const int32_t* Ej, const double* Ex, int e_base, const double* A0,
                                             double* Zp, const double* Zr, int r0, int m, int tid) {
  constexpr int T = 64 * kSW;
  // the next round's row, a round ahead: task-local row, entry range, initial value,
  // diagonal, coupling entries
  int nk = -1, ne0 = 0, ne1 = 0;
  double nacc = 0.0, nd = 1.0;
  ResCur nrc;
  auto fetch = [&](int q) {
    nk = -1;
    if (q < m) {
      nk = O ? O[q] : (kBack ? m - 1 - q : q);
      ne0 = P[nk] - e_base;
      ne1 = P[nk + 1] - e_base;
      nacc = A0[nk];
      if (kBack) nd = a.diag[r0 + nk];
    }
    res_open(nrc, a, Zr, r0, nk);
  };
  fetch(tid);
  unsigned idle = 0;
  bool stalled = false;
  for (int q = tid; __any(q < m); q += T) {
    const int kc = nk, e1 = ne1;
    int p = ne0;
    double acc = nacc;
    ResCur rc = nrc;
    const double dg = nd;
    bool busy = kc >= 0;
    // the window: entries p .. p + 3 of the row (indices clamped into the row), in one
    // of two register sets.  A pass polls the rows of the first two, and the moved
    // window takes its first two entries from the old one and reads the other two into
    // the other set: those reads complete while the next pass's polls are in flight.
    struct Win {
      int j0, j1, j2, j3;
      double x0, x1, x2, x3;
    };
    auto at = [&](int e) { return e < e1 ? e : (e1 > 0 ? e1 - 1 : 0); };
    Win wa{-1, -1, -1, -1, 0.0, 0.0, 0.0, 0.0}, wb = wa;
    if (busy) {
      wa.j0 = Ej[at(p)];
      wa.x0 = Ex[at(p)];
      wa.j1 = Ej[at(p + 1)];
      wa.x1 = Ex[at(p + 1)];
      wa.j2 = Ej[at(p + 2)];
      wa.x2 = Ex[at(p + 2)];
      wa.j3 = Ej[at(p + 3)];
      wa.x3 = Ex[at(p + 3)];
    }
    fetch(q + T);
    auto pass = [&](const Win& cur, Win& nxt) {
      bool prog = false;
      if (busy && rc.q < rc.qe) {
        prog = res_step(rc, a, Zr, acc);
        nxt = cur;
      } else if (busy) {
        double v0 = 0.0, v1 = 0.0;
        const bool r0_ = pending_load(V, cur.j0 >= 0 ? cur.j0 : 0, v0) || cur.j0 < 0;
        const bool r1_ = pending_load(V, cur.j1 >= 0 ? cur.j1 : 0, v1) || cur.j1 < 0;
        const bool c0 = p < e1 && r0_;
        const bool c1 = c0 && p + 1 < e1 && r1_;
        double u = acc - cur.x0 * v0;
        acc = (c0 && cur.j0 >= 0) ? u : acc;
        u = acc - cur.x1 * v1;
        acc = (c1 && cur.j1 >= 0) ? u : acc;
        const int c = (int)c0 + (int)c1;
        p += c;
        nxt.j0 = c == 0 ? cur.j0 : (c == 1 ? cur.j1 : cur.j2);
        nxt.x0 = c == 0 ? cur.x0 : (c == 1 ? cur.x1 : cur.x2);
        nxt.j1 = c == 0 ? cur.j1 : (c == 1 ? cur.j2 : cur.j3);
        nxt.x1 = c == 0 ? cur.x1 : (c == 1 ? cur.x2 : cur.x3);
        // materialise the moved entries here, while the reads below are in flight (an
        // empty statement that only takes them as inputs)
        asm volatile("" ::"v"(nxt.j0), "v"(nxt.j1), "v"(nxt.x0), "v"(nxt.x1));
        nxt.j2 = Ej[at(p + 2)];
        nxt.x2 = Ex[at(p + 2)];
        nxt.j3 = Ej[at(p + 3)];
        nxt.x3 = Ex[at(p + 3)];
        prog = c > 0;
        if (p >= e1) {
          const double z = kBack ? acc / dg : acc;
          result_store(V, kc, z);
          if (kBack) publish_store(Zp, kc, z);
          busy = false;
          prog = true;
        }
      }
      if (__any(prog)) {
        idle = 0;
      } else {
        __builtin_amdgcn_s_sleep(1);
        if (++idle > kSpinLimit) stalled = true;
      }
    };
    while (__any(busy) && !stalled) {
      pass(wa, wb);
      if (!__any(busy) || stalled) break;
      pass(wb, wa);
    }
    if (stalled) break;
  }
  return !stalled;
}

// Copy the task's entries [e_base, e_base + E) into LDS: columns as task-local rows (-1
// outside the task), eight loads in flight per thread.
template <bool kBack>
__device__ __forceinline__ void stage_entries(int32_t* Ej, double* Ex, const unsigned long long* keys,
                                              const double* vals, int e_base, int E, int r0, int m, int n, int tid) {
  constexpr int T = 64 * kSW;
  for (int e = tid; e < E; e += 8 * T) {
    unsigned lo[8];
    double x[8];
#pragma unroll
    for (int t = 0; t < 8; t++) {
      lo[t] = 0u;
      x[t] = 0.0;
      if (e + t * T < E) {
        lo[t] = (unsigned)keys[e_base + e + t * T];
        x[t] = vals[e_base + e + t * T];
      }
    }
#pragma unroll
    for (int t = 0; t < 8; t++) {
      if (e + t * T < E) {
        const int jj = (kBack ? n - 1 - (int)lo[t] : (int)lo[t]) - r0;
        Ej[e + t * T] = (jj >= 0 && jj < m) ? jj : -1;
        Ex[e + t * T] = x[t];
      }
    }
  }
}

// A task in LDS whose rows hold at most this many entries on average runs its sweeps
// one row per thread; longer rows (ND separators) one row per wavefront.
constexpr int kLaneMeanMax = 24;

// LDS of a task: V (m doubles), row pointers (m + 1), issue order (m), then a region R
// of rbytes for the sweep: the done bits (row per wavefront), the entries (row per
// thread, all entries in LDS) or the entry slots (row per thread, kSlot entries each).
__host__ __device__ constexpr int64_t lds_base_bytes(int64_t m) { return (8 * m + 4 * (2 * m + 1) + 7) / 8 * 8; }
__host__ __device__ constexpr int64_t lds_flag_bytes(int64_t m) { return 4 * ((m + 31) / 32 + 1); }
__host__ __device__ constexpr int64_t lds_slot_bytes() { return 12 * (int64_t)kSlot * 64 * kSW; }

// One sweep (L forward, or U backward) of a task over its rows.  V holds the initial
// values and receives the results.  P / O: the row pointers and issue order (LDS for a
// task in LDS, else global with O offset by r0); `fin` the final values of columns
// outside the task; Zp the task's rows of Z, where the backward sweep publishes each
// result (null for the forward sweep); Zr non-null when V holds the right-hand sides
// and the row-per-thread sweep subtracts each row's couplings (read from Zr) itself.
// Whether a task in LDS sweeps one row per thread: E entries over m rows, rbytes of LDS
// for the sweep.
__device__ __forceinline__ bool lane_sweep(int E, int m, int64_t rbytes) {
  return E <= kLaneMeanMax * m && (12 * (int64_t)E <= rbytes || lds_slot_bytes() <= rbytes);
}

template <bool kLds, bool kBack>
__device__ __forceinline__ bool run_sweep(const SolveArgs& a, double* V, const int32_t* P, const int32_t* O, int ooff,
                                          char* R, int64_t rbytes, const Flags<kLds>& F, const unsigned long long* keys,
                                          const double* vals, const double* fin, double* G, bool prefix, double* Zp,
                                          const double* Zr, int r0, int m, int tid) {
  const int lane = tid & 63;
  const int wv = tid >> 6;
  if constexpr (kLds) {
    const int e_base = P[0];
    const int E = P[m] - e_base;
    if (lane_sweep(E, m, rbytes)) {
      // one row per thread: initial values to G (the task's rows of W, free until the
      // task's results), LDS values to pending
      for (int kk = tid; kk < m; kk += 64 * kSW) {
        G[kk] = V[kk];
        V[kk] = __longlong_as_double((long long)kPending);
      }
      __syncthreads();
      if (prefix) {
        apply_prefixes<kBack>(a, G, P, keys, vals, fin, r0, m, tid);
        __syncthreads();
      }
      if (12 * (int64_t)E <= rbytes) {
        double* Ex = reinterpret_cast<double*>(R);
        int32_t* Ej = reinterpret_cast<int32_t*>(Ex + E);
        stage_entries<kBack>(Ej, Ex, keys, vals, e_base, E, r0, m, a.n, tid);
        __syncthreads();
        return sweep_staged<kBack>(a, V, P, O, Ej, Ex, e_base, G, Zp, Zr, r0, m, tid);
      }
      double* Sx = reinterpret_cast<double*>(R);
      int32_t* Sj = reinterpret_cast<int32_t*>(Sx + kSlot * 64 * kSW);
      return sweep_lanes<kBack>(a, V, P, O, keys, vals, G, Slots{Sj, Sx}, Zp, Zr, r0, m, tid);
    }
  }
  return sweep<kLds, kBack>(a, V, P, O, ooff, keys, vals, F, fin, Zp, r0, m, wv, lane);
}

// Pl: LDS row pointers (m + 1), Po: LDS issue order (m), R: the LDS region of the
// sweeps, when the task is in LDS
template <bool kLds>
__device__ void run_task(const SolveArgs& a, double* V, int32_t* Pl, int32_t* Po, char* R, int64_t rbytes,
                         const Flags<kLds>& F, int kind, int id, int rhs, int tid) {
  int r0, r1;
  if (kind == 0) { r0 = a.blkptr[id]; r1 = a.blkptr[id + 1]; }
  else { r0 = a.grpptr[id]; r1 = a.grpptr[id + 1]; }
  const int m = r1 - r0;
  const int n = a.n;
  double* W = a.W + (int64_t)rhs * n;
  double* Z = a.Z + (int64_t)rhs * n;
  const double* Bc = a.B + (int64_t)rhs * a.ldb;
  const int obad = a.obad[r0];
  bool ok = true;
  if (kind != 2) {
    // residual of every row (independent of the task's other rows; it waits only for
    // the entries of later blocks it reads).  A block task swept one row per thread
    // leaves the couplings to the sweep, so that each row starts as soon as its own
    // are published; an ND node's rows subtract them before their prefix entries.
    const bool defer = kLds && kind == 0 && lane_sweep(a.LTp[r0 + m] - a.LTp[r0], m, rbytes);
    F.clear(m, tid);
    for (int kk = tid; kk < m; kk += 64 * kSW) {
      const int i = a.piv[r0 + kk];
      V[kk] = defer ? Bc[a.prow[i]] : residual_row(a, Bc, Z, i, ok);
    }
    // the task's L row pointers and forward order
    const int32_t* LP = a.LTp + r0;
    const int32_t* ord = (obad & 1) == 0 ? a.sfo + r0 : nullptr;
    int ooff = r0;
    if (kLds) {
      for (int kk = tid; kk <= m; kk += 64 * kSW) Pl[kk] = a.LTp[r0 + kk];
      LP = Pl;
      if (ord) {
        for (int kk = tid; kk < m; kk += 64 * kSW) Po[kk] = ord[kk] - r0;
        ord = Po;
        ooff = 0;
      }
    }
    __syncthreads();
    ok &= run_sweep<kLds, false>(a, V, LP, ord, ooff, R, rbytes, F, a.lkeys, a.lvals, W, W + r0, kind == 1, nullptr,
                                 defer ? Z : nullptr, r0, m, tid);
    __syncthreads();
    if (kind == 1) {
      for (int kk = tid; kk < m; kk += 64 * kSW) W[r0 + kk] = V[kk];
      if (!ok && tid == 0) atomicOr(a.status, 4);
      return;
    }
  } else if (V != W + r0) {
    for (int kk = tid; kk < m; kk += 64 * kSW) V[kk] = W[r0 + kk];
  }
  // U rows: z_k = (w_k - sum_{j > k} u_kj z_j) / u_kk
  F.clear(m, tid);
  __syncthreads();
  const int32_t* UP = a.UTp + r0;
  const int32_t* ord = (obad & 2) == 0 ? a.sbo + r0 : nullptr;
  int ooff = r0;
  if (kLds) {
    for (int kk = tid; kk <= m; kk += 64 * kSW) Pl[kk] = a.UTp[r0 + kk];
    UP = Pl;
    if (ord) {
      for (int kk = tid; kk < m; kk += 64 * kSW) Po[kk] = ord[kk] - r0;
      ord = Po;
      ooff = 0;
    }
  }
  __syncthreads();
  // every result is published to Z by the sweep as it is computed
  ok &= run_sweep<kLds, true>(a, V, UP, ord, ooff, R, rbytes, F, a.ukeys, a.uvals, Z, W + r0, kind == 2, Z + r0,
                              nullptr, r0, m, tid);
  if (!ok && tid == 0) atomicOr(a.status, 4);
}

// One task with the workgroup's dynamic LDS (smem_d, a.lds_bytes): every right-hand
// side in turn.
__device__ __forceinline__ void solve_task_body(const SolveArgs& a, double* smem_d, int t, int tid) {
  const int kind = a.st_kind[t], id = a.st_id[t];
  const int m = kind == 0 ? a.blkptr[id + 1] - a.blkptr[id] : a.grpptr[id + 1] - a.grpptr[id];
  const int64_t rbytes = (int64_t)a.lds_bytes - lds_base_bytes(m);
  const bool lds = rbytes >= lds_flag_bytes(m);
  for (int rhs = 0; rhs < a.nrhs; rhs++) {
    if (lds) {
      int32_t* Pl = reinterpret_cast<int32_t*>(smem_d + m);
      int32_t* Po = Pl + m + 1;
      char* R = reinterpret_cast<char*>(smem_d) + lds_base_bytes(m);
      Flags<true> F{reinterpret_cast<unsigned*>(R), nullptr};
      run_task<true>(a, smem_d, Pl, Po, R, rbytes, F, kind, id, rhs, tid);
    } else {
      const int r0 = kind == 0 ? a.blkptr[id] : a.grpptr[id];
      Flags<false> F{nullptr, a.sflag + r0};
      // work vector in place: the block's (or node's) part of W (Z receives only the
      // final values, which other tasks wait for)
      double* V = a.W + (int64_t)rhs * a.n + r0;
      run_task<false>(a, V, nullptr, nullptr, nullptr, 0, F, kind, id, rhs, tid);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64 * kSW) solve_task_kernel(SolveArgs a) {
  BASKER_DYN_SHARED(double, smem_d);
  solve_task_body(a, smem_d, a.t_begin + (int)blockIdx.x, (int)threadIdx.x);
}

// All tasks in one launch.  Workgroups take tasks from a counter in issue order (a
// topological order of the task graph) and wait for each task's predecessors' done
// flags before running it; the entries of later blocks that a residual reads are not
// flagged tasks but waited for one by one in Z (published as each is computed), so a
// task starts while the blocks it couples to are still finishing.  Every task a wait
// depends on sits earlier in the order, so it was taken by a workgroup that is already
// running, and the earliest unfinished task never waits: the waits end without any
// assumption about how many workgroups are resident.
// A task's results are released at agent scope before its flag (workgroups of one
// launch run on different XCDs, whose L2 caches are not coherent) and acquired at agent
// scope after the wait.  Waits are also bounded, by elapsed time (the 100 MHz real-time
// counter), not by a poll count: a predecessor can legitimately run for tens of
// milliseconds (the root separator of a 500k-row circuit does).  A wait that outlasts
// the bound sets bit 8 of the status, and every other wait sees that bit within 256
// polls and gives up too, so a launch whose flags never arrive still ends (the solve
// then reports the stall).
// s_waitcnt operand: vector memory count 0, the export and LDS counts left free
constexpr int kWaitVmcnt0 = 0x0F70;

__global__ void __launch_bounds__(64 * kSW) solve_flow_kernel(SolveArgs a) {
  BASKER_DYN_SHARED(double, smem_d);
  __shared__ int sh_t;
  const int tid = threadIdx.x;
  // The task index is read as a wave-uniform value (readfirstlane): with the loop's
  // exit provably uniform the compiler keeps one loop in which every thread passes
  // every barrier.  Read as a per-lane value, the exit looked divergent and the
  // structurizer moved thread 0's counter update out of the loop that holds the
  // barriers, so the other threads reran the previous task without end.
  if (tid == 0) sh_t = atomicAdd(a.qctr, 1);
  __syncthreads();
  int c = __builtin_amdgcn_readfirstlane(sh_t);
  while (c < a.ntasks) {
    const int t = __builtin_amdgcn_readfirstlane(a.issue[c]);
    if (tid < 64) {
      bool stalled = false;
      for (int e = a.dep_ptr[t] + tid; e < a.dep_ptr[t + 1]; e += 64) {
        const int d = a.dep[e];
        unsigned spins = 0;
        const unsigned long long w0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(&a.done[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          __builtin_amdgcn_s_sleep(2);
          if ((++spins & 255u) == 1 &&
              (__builtin_amdgcn_s_memrealtime() - w0 > kFlowWaitTicks ||
               (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8))) {
            stalled = true;
            break;
          }
        }
      }
      if (__any(stalled) && tid == 0) __hip_atomic_fetch_or(a.status, 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    solve_task_body(a, smem_d, t, tid);
    // every wave's result stores complete (acknowledged by L2) before the barrier, so
    // the one agent-scope release below (L2 write-back, then the flag) covers them:
    // the workgroup barrier alone does not wait for global stores
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (tid == 0) {
      if (a.succ[t]) __hip_atomic_store(&a.done[t], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      sh_t = atomicAdd(a.qctr, 1);
    }
    __syncthreads();
    c = __builtin_amdgcn_readfirstlane(sh_t);
  }
}

// Z before a solve: every unknown pending
__global__ void solve_pending_kernel(unsigned long long* Z, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) Z[i] = kPending;
}

__global__ void solve_unpermute_kernel(SolveArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n * a.nrhs;
  if (i < total) {
    const int rhs = (int)(i / a.n);
    const int k = (int)(i - (int64_t)rhs * a.n);
    a.B[(int64_t)rhs * a.ldb + a.qcol[k]] = a.Z[i];
  }
}

}  // namespace

size_t solve_lds_bytes(int32_t rows) {
  return (size_t)(lds_base_bytes(rows) + std::max(lds_flag_bytes(rows), lds_slot_bytes()));
}

hipError_t solve_lds_setup(size_t max_bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_task_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_flow_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes - kSolveFlowStaticLds);
}

hipError_t launch_solve_tasks(const SolveArgs& a, int ntasks, hipStream_t s) {
  if (ntasks > 0)
    hipLaunchKernelGGL(solve_task_kernel, dim3(ntasks), dim3(64 * kSW), (size_t)a.lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_flow(const SolveArgs& a, int grid, hipStream_t s) {
  if (a.ntasks > 0 && grid > 0)
    hipLaunchKernelGGL(solve_flow_kernel, dim3(grid), dim3(64 * kSW), (size_t)a.lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t noalloc_scratch(int device, double** ptr) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = addr.emplace(device, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

hipError_t launch_solve_pending(double* Z, int64_t cnt, hipStream_t s) {
  if (cnt > 0)
    hipLaunchKernelGGL(solve_pending_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(Z), cnt);
  return hipGetLastError();
}

hipError_t launch_solve_finish(const SolveArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)a.n * a.nrhs;
  if (total > 0)
    hipLaunchKernelGGL(solve_unpermute_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
