// C ABI of the library: symbolic analysis on the host, numeric factorization,
// refactorization and solve on the device (see include/basker.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/basker.h"
#include "device.hpp"
#include "symbolic.hpp"

using namespace basker;

namespace {

// device bytes are charged to the handle whose call is running on this thread; an
// allocation that would take the handle past its budget (0 = none) is refused
thread_local int64_t* t_acct = nullptr;
thread_local int64_t t_budget = 0;
struct AcctScope {
  int64_t* prev;
  int64_t prev_budget;
  AcctScope(int64_t* a, int64_t budget) : prev(t_acct), prev_budget(t_budget) {
    t_acct = a;
    t_budget = budget;
  }
  ~AcctScope() {
    t_acct = prev;
    t_budget = prev_budget;
  }
};

template <class T>
struct DBuf {
  T* p = nullptr;
  int64_t cap = 0;
  int64_t* acct = nullptr;   // device-byte counter of the owning handle
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    if (p && acct) *acct -= (int64_t)sizeof(T) * cap;
    p = nullptr;
    cap = 0;
  }
  hipError_t reserve(int64_t n) {
    if (n <= cap && p) return hipSuccess;
    release();
    int64_t m = n > 0 ? n : 1;
    if (t_acct && t_budget > 0 && *t_acct + (int64_t)sizeof(T) * m > t_budget) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc((void**)&p, sizeof(T) * (size_t)m);
    if (e != hipSuccess) { p = nullptr; return e; }
    cap = m;
    acct = t_acct;
    if (acct) *acct += (int64_t)sizeof(T) * cap;
    return hipSuccess;
  }
  hipError_t upload(const std::vector<T>& v, hipStream_t s) {
    hipError_t e = reserve((int64_t)v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
  }
};

}  // namespace

struct basker_ctx {
  int64_t dev_bytes = 0;     // declared first: buffers release into it when destroyed
  int device = 0;
  // refactorization graph: scatter + init + level launches, reading h->vals
  hipGraph_t rgraph = nullptr;
  hipGraphExec_t rgexec = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  basker_options opt{};
  Plan plan;
  std::string err;
  // plan on device
  DBuf<int32_t> Rp, Ri, Rmap, grp_lo, grp_hi, seg_c0, seg_c1, lvl_seg, lvl_ctr, item_lo, item_hi, lvl_col;
  // separator partial columns (first step of separator levels)
  DBuf<int32_t> cb_off, cb_np, cb_nn, cbI;
  DBuf<double> cbX;
  // dense separator panels
  DBuf<int32_t> dsep_seg, dsep_H, dsep_rng_ptr, dsep_rng_g0, dsep_rng_len, dsep_rng_loc, piv_local;
  DBuf<int64_t> dsep_poff, dsep_soff;
  DBuf<double> dpanel;
  DBuf<unsigned long long> dbits, dscratch;
  DBuf<int32_t> OTp, OTj, OTmap, prow, qcol, blkptr, grpptr;
  // first-level cooperative schedule
  DBuf<int32_t> co_item_lo, co_item_hi, co_item_cols, col_item, dep_ptr, dep_idx, sdep_ptr, sdep_idx, item_bad;
  DBuf<int32_t> co_item_off, co_issue, co_item_kind;
  bool coop = false;
  int coop_waves = 6;
  int coop_grid = 0;
  // autotuner: -2 = the first factorization (learning) runs before any trial; 0.. =
  // index of the next candidate to time; -1 = not tuning
  int tune_next = -1;
  std::vector<float> tune_ms;
  // solve tasks, row-wise factors (rebuilt after every factorization), done flags
  DBuf<int32_t> st_kind, st_id, s_status, sflag, LTp, UTp;
  DBuf<int32_t> st_dep_ptr, st_dep, st_succ, st_issue;   // the one-launch solve's task graph
  DBuf<int32_t> sfo, sbo, sfo_pos, sbo_pos, row_task0, obad, ocount;   // solve issue orders and their check
  DBuf<unsigned long long> lkeys, lkeys_out, ukeys, ukeys_out;
  DBuf<double> lvals, lvals_out, uvals, uvals_out, diag;
  DBuf<char> rows_temp;
  std::vector<int32_t> st_lvl_lds;   // LDS bytes of every solve level's launch
  int32_t flow_lds = 0, flow_grid = 0;   // the one-launch solve: LDS per workgroup, workgroups
  int32_t flow_grid_shared = 0;           // workgroups while other solves run on the device
  // numeric state
  DBuf<double> vals, Rx, OTx;
  DBuf<int32_t> pinv, piv, Lbeg, Lcnt, Ubeg, Ucnt, status;
  DBuf<int32_t> Li, Ui;
  DBuf<double> Lx, Ux;
  DBuf<unsigned long long> pool, nnz_ctr;
  int64_t Lused = 0, Uused = 0;   // allocated extents of the pools (chunks leave gaps)
  int64_t chunk = 0;
  DBuf<char> gws;
  int64_t gws_stride = 0;
  int gws_slots = 0;
  int grid = 0;
  // solve scratch

  DBuf<double> W, Z, Bdev;
  bool factored = false;
  int64_t lnz = 0, unz = 0;
  hipEvent_t ev[6] = {};
  basker_info_t info{};
};

static basker_status fail(basker_ctx* h, basker_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

static basker_status hip_fail(basker_ctx* h, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  if (h) h->err = m;
  return e == hipErrorOutOfMemory ? BASKER_ERR_OOM : BASKER_ERR_DEVICE;
}

#define HIPCHK(h, expr)                                   \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
  } while (0)

extern "C" basker_status basker_default_options(basker_options* o) {
  if (!o) return BASKER_ERR_INVALID;
  std::memset(o, 0, sizeof(*o));
  o->pivot_tol = 1e-3;
  o->diag_pref = 1;
  o->matching = 1;
  o->btf = 1;
  o->fill_order = 1;
  o->nd_leaves = 16;
  o->nd_min_block = 10000;
  o->capacity_factor = 0.0;
  o->device = 0;
  o->stream = nullptr;
  o->refactor_graph = 1;
  o->max_grid = 0;
  o->hbm_budget = 0;
  o->sched_flags = 0;
  o->item_cols = 0;
  o->coop_waves = 0;
  return BASKER_OK;
}

static bool options_valid(const basker_options& o) {
  if (!(o.pivot_tol > 0.0 && o.pivot_tol <= 1.0)) return false;   // also rejects NaN
  if (o.nd_leaves < 1 || (o.nd_leaves & (o.nd_leaves - 1)) != 0) return false;
  if (o.hbm_budget < 0 || o.max_grid < 0 || o.item_cols < 0 || o.capacity_factor < 0) return false;
  if (o.coop_waves != 0 && o.coop_waves != 4 && o.coop_waves != 6 && o.coop_waves != 7 && o.coop_waves != 8)
    return false;
  if (o.bin_edge < -1 || o.autotune < 0 || o.autotune > 1) return false;
  return true;
}

// work budget (visited pattern entries) of the symbolic factorization without row exchanges
constexpr int64_t kSymVisitBudget = 400000000LL;
constexpr int kLdsPerCu = 160 * 1024;

extern "C" const char* basker_status_string(basker_status s) {
  switch (s) {
    case BASKER_OK: return "ok";
    case BASKER_REFACTOR_FELL_BACK: return "refactor fell back to a full factorization";
    case BASKER_ERR_INVALID: return "invalid input";
    case BASKER_ERR_STRUCT_SINGULAR: return "structurally singular";
    case BASKER_ERR_NUM_SINGULAR: return "numerically singular";
    case BASKER_ERR_OOM: return "out of memory";
    case BASKER_ERR_PATTERN: return "no factorization to reuse";
    case BASKER_ERR_DEVICE: return "device error";
    case BASKER_ERR_WORKSPACE: return "column pattern exceeds the workspace";
  }
  return "unknown status";
}

extern "C" const char* basker_last_error(basker_handle h) { return h ? h->err.c_str() : ""; }

// workgroups of the persistent factor launches: the widest level, capped by the
// occupancy target and the caller's max_grid
static int plan_grid(const Plan& P, const basker_options& o) {
  const int nlev = (int)P.lvl_ptr.size() - 1;
  int maxitems = 1;
  for (int l = 0; l < nlev; l++) maxitems = std::max(maxitems, P.lvl_item_ptr[l + 1] - P.lvl_item_ptr[l]);
  int grid = std::min(maxitems, kNumCu * kWavesPerCu);
  if (o.max_grid > 0) grid = std::min(grid, o.max_grid);
  return grid;
}

constexpr int kGwsSlots = 1 << 14;   // hash slots of a workgroup's global fallback workspace
static int64_t gws_stride_bytes() { return ((48LL * kGwsSlots + 16 + 255) / 256) * 256; }


// separator first-step buffer: twice its entries without row exchanges, or a bound
// from the separator column count
static int64_t cb_capacity(const Plan& P) {
  if (P.sym_ok) return std::max<int64_t>(4096, 2 * P.sym_cb);
  const int64_t sepcols = P.lvl_col_ptr.back() - (P.lvl_col_ptr.size() > 1 ? P.lvl_col_ptr[1] : 0);
  return std::max<int64_t>(4096, 256 * sepcols);
}

// first-level workgroups: one per CU (the waves' LDS workspaces fill a CU's LDS)
static int coop_grid_of(const Plan& P, const basker_options& o, int waves) {
  const int per_cu = std::max(1, kLdsPerCu / std::max(1, coop_lds_bytes(waves)));
  int grid = std::min<int>((int)P.co_item_lo.size(), kNumCu * per_cu);
  if (o.max_grid > 0) grid = std::min(grid, o.max_grid);
  return grid;
}

static int coop_waves_of(const basker_options& o) { return o.coop_waves ? o.coop_waves : 6; }
constexpr int kDefaultBinEdge = 32;
static int bin_edge_of(const basker_options& o) { return o.bin_edge == 0 ? kDefaultBinEdge : (o.bin_edge < 0 ? 0 : o.bin_edge); }

// Every first-level column in exactly one item with a slot count that matches its
// segments, and every dependency list ascending inside the column's own segment
// before the column: what the cooperative kernel's waits and slot arithmetic assume.
static bool level0_schedule_valid(const Plan& P) {
  const int n = P.n;
  if ((int)P.col_item.size() != n || (int)P.dep_ptr.size() != n + 1 || (int)P.sdep_ptr.size() != n + 1) return false;
  std::vector<int32_t> seen(n, 0);
  for (size_t it = 0; it < P.co_item_lo.size(); it++) {
    int64_t cols = 0;
    for (int q = P.co_item_lo[it]; q < P.co_item_hi[it]; q++) {
      if (q < P.lvl_ptr[0] || q >= P.lvl_ptr[1]) return false;
      const int sg = P.lvl_seg[q];
      for (int k = P.seg_c0[sg]; k < P.seg_c1[sg]; k++) {
        if (P.col_item[k] != (int32_t)it || seen[k]++) return false;
        for (int pass = 0; pass < 2; pass++) {
          const std::vector<int32_t>& ptr = pass ? P.sdep_ptr : P.dep_ptr;
          const std::vector<int32_t>& idx = pass ? P.sdep_idx : P.dep_idx;
          int prev = P.seg_c0[sg] - 1;
          for (int32_t e = ptr[k]; e < ptr[k + 1]; e++) {
            if (idx[e] <= prev || idx[e] >= k) return false;
            prev = idx[e];
          }
        }
      }
      cols += P.seg_c1[sg] - P.seg_c0[sg];
    }
    if (cols != P.co_item_cols[it]) return false;
  }
  for (int k = 0; k < n; k++)
    if ((P.col_item[k] >= 0) != (seen[k] == 1)) return false;
  // issue lists: every slot of an item once, with its column and segment start, and every
  // predicted dependency issued before the column that waits for it
  if (P.co_item_off.size() != P.co_item_lo.size() + 1) return false;
  for (size_t it = 0; it < P.co_item_lo.size(); it++) {
    const int m = P.co_item_cols[it];
    if (P.co_item_off[it + 1] - P.co_item_off[it] != m) return false;
    const int32_t* e = P.co_issue.data() + 3 * (size_t)P.co_item_off[it];
    std::vector<int32_t> pos(m, -1);
    for (int i = 0; i < m; i++) {
      const int k = e[3 * i], sl = e[3 * i + 1], c0 = e[3 * i + 2];
      if (sl < 0 || sl >= m || pos[sl] >= 0 || k < c0 || k >= n || P.col_item[k] != (int32_t)it) return false;
      pos[sl] = i;
    }
    for (int i = 0; i < m; i++) {
      const int k = e[3 * i], sl = e[3 * i + 1];
      for (int32_t d = P.dep_ptr[k]; d < P.dep_ptr[k + 1]; d++) {
        const int js = sl - (k - P.dep_idx[d]);
        if (js < 0 || pos[js] >= i) return false;
      }
    }
  }
  return true;
}

static bool coop_usable(const Plan& P) {
  return !P.co_item_lo.empty() && P.co_max_item_cols <= kCoopMaxItemCols && P.co_valid;
}

// fallback-workspace regions (one per wavefront of the widest launch)
static int64_t gws_regions(const Plan& P, const basker_options& o) {
  int64_t r = plan_grid(P, o);
  if (coop_usable(P)) {
    const int w = coop_waves_of(o);
    r = std::max<int64_t>(r, (int64_t)coop_grid_of(P, o, w) * w);
  }
  return r;
}

// Wavefronts take pool space in chunks of at least kMinChunk entries, and a wave can
// leave one chunk partly used per launch: the chunk is 1/(kChunkDiv * waves) of the
// pool, and the pools add kMinChunk per wave and launch of a first level (its
// speculative and redo passes) and of the separator levels.
constexpr int64_t kMinChunk = 16;
constexpr int64_t kChunkDiv = 32;

static int64_t pool_waves(const Plan& P, const basker_options& o) { return gws_regions(P, o); }

// initial L or U pool entries (which = 0: L, 1: U): twice the fill of a factorization
// without row exchanges (room for row exchanges, chunk slack and first-level items
// redone after a failed speculation), or capacity_factor * nnz(diagonal blocks)
static int64_t pool_capacity(const Plan& P, const basker_options& o, int which) {
  int64_t cap;
  if (o.capacity_factor > 0 || !P.sym_ok)
    cap = (int64_t)((o.capacity_factor > 0 ? o.capacity_factor : 6.0) * (double)P.Ri.size());
  else
    cap = 2 * (which == 0 ? P.sym_lnz : P.sym_unz);
  const int64_t launches = 2 + (int64_t)P.lvl_ptr.size();
  cap += P.n + 64 + kMinChunk * pool_waves(P, o) * launches;
  return std::min<int64_t>(cap, 0x7fffffffLL);
}

// bytes of the radix sort's workspace for up to `items` pairs: the sort's own answer,
// or a bound when it cannot be asked
static int64_t rows_temp_estimate(int64_t items, int n) {
  size_t b = 0;
  if (rows_temp_bytes(std::max<int64_t>(items, 1), n, &b) == hipSuccess) return std::max<int64_t>((int64_t)b, 1);
  (void)hipGetLastError();
  return 16 * items + (8 << 20);
}

// Device bytes a handle holds after upload_plan, a factorization without pool growth
// and a solve of 8 host right-hand sides: the same reservations, added up.
static int64_t plan_device_bytes(const Plan& P, const basker_options& o) {
  int64_t b = 0;
  auto add = [&](size_t elem, int64_t cnt) { b += (int64_t)elem * std::max<int64_t>(cnt, 1); };
  const int64_t n = P.n, nnzd = (int64_t)P.Ri.size(), nnzo = (int64_t)P.Oi.size();
  const int64_t ns = (int64_t)P.seg_c0.size(), nitem = (int64_t)P.item_lo.size();
  const int64_t nd = (int64_t)P.dsep_seg.size(), nr = (int64_t)P.dsep_rng_g0.size();
  const int64_t nb = (int64_t)P.blkptr.size() - 1, ng = (int64_t)P.grpptr.size() - 1;
  const int64_t nt = (int64_t)P.st_kind.size(), nlev = (int64_t)P.lvl_ptr.size() - 1;
  add(4, n + 1); add(4, nnzd); add(4, nnzd);                       // Rp, Ri, Rmap
  add(4, n); add(4, n);                                            // grp_lo, grp_hi
  add(4, ns); add(4, ns); add(4, ns); add(4, nitem); add(4, nitem);  // segments, items
  add(4, (int64_t)P.lvl_col.size());
  add(4, nd); add(4, nd); add(4, nd + 1); add(4, nr); add(4, nr); add(4, nr);
  add(8, nd); add(8, nd);
  add(8, P.dsep_panel_total); add(8, P.dsep_bits_total);
  add(8, (int64_t)kMaxPanelWords * (1 + kMaxNb));
  add(4, n); add(4, n); add(4, n); add(4, n);                      // piv_local, cb_off/np/nn
  const int64_t cb = cb_capacity(P);
  add(4, cb); add(8, cb);
  add(8, 2); add(4, 2 * nlev);
  add(4, n + 1); add(4, nnzo); add(4, nnzo);                       // OTp, OTj, OTmap
  add(4, n); add(4, n); add(4, nb + 1); add(4, ng + 1);            // prow, qcol, blkptr, grpptr
  add(4, nt); add(4, nt); add(4, 2 + nt); add(4, n); add(4, n + 1); add(4, n + 1);   // tasks, status, flags, row pointers
  add(4, nt + 1); add(4, (int64_t)P.st_dep.size()); add(4, nt); add(4, nt);    // the one-launch solve's task graph
  add(8, n);                                                                     // U's diagonal
  for (int t = 0; t < 6; t++) add(4, n);                                         // solve issue orders
  add(4, 1);
  add(8, P.nnz); add(8, nnzd); add(8, nnzo);                       // vals, Rx, OTx
  for (int t = 0; t < 6; t++) add(4, n);                           // pinv, piv, Lbeg..Ucnt
  add(4, kStatusWords); add(8, 3);
  const int64_t capL = pool_capacity(P, o, 0), capU = pool_capacity(P, o, 1);
  add(4, capL); add(8, capL); add(4, capU); add(8, capU);
  b += gws_stride_bytes() * gws_regions(P, o);
  const int64_t nco = (int64_t)P.co_item_lo.size();
  add(4, nco); add(4, nco); add(4, nco); add(4, n); add(4, nco);   // items, col_item, item_bad
  add(4, n + 1); add(4, (int64_t)P.dep_idx.size()); add(4, n + 1); add(4, (int64_t)P.sdep_idx.size());
  add(4, (int64_t)P.co_item_off.size()); add(4, (int64_t)P.co_issue.size()); add(4, nco);
  const int64_t nrhs = 8;
  add(8, n * nrhs); add(8, n * nrhs); add(8, n * nrhs);            // W, Z, Bdev
  // row-wise factors: keys and values, sorted copies, sort workspace, over the fill
  // without row exchanges (the pools' used extents), or the pools when not counted
  const int64_t rl = P.sym_ok ? P.sym_lnz + P.sym_lnz / 4 + 4096 : capL;
  const int64_t ru = P.sym_ok ? P.sym_unz + P.sym_unz / 4 + 4096 : capU;
  add(32, rl); add(32, ru);
  b += rows_temp_estimate(std::max(rl, ru), (int)n);
  return b;
}

// Everything the device needs from the plan, plus the solve's row-wise coupling and
// block dependency lists.
// The solve kernel takes each task's rows from its issue orders: every task's slice of
// sfo and sbo must list exactly the task's rows, with *_pos the inverse.
static bool solve_orders_valid(const Plan& P) {
  const int n = P.n;
  if ((int)P.sfo.size() != n || (int)P.sbo.size() != n || (int)P.sfo_pos.size() != n ||
      (int)P.sbo_pos.size() != n || (int)P.row_task0.size() != n)
    return false;
  for (int k = 0; k < n; k++) {
    const int t0 = P.row_task0[k];
    if (t0 < 0 || t0 > k || P.row_task0[t0] != t0) return false;
    const int f = P.sfo[k], b = P.sbo[k];
    if (f < 0 || f >= n || b < 0 || b >= n || P.row_task0[f] != t0 || P.row_task0[b] != t0) return false;
    if (P.sfo_pos[f] != k - t0 || P.sbo_pos[b] != k - t0) return false;
  }
  return true;
}

static basker_status upload_plan(basker_ctx* h) {
  AcctScope acct(&h->dev_bytes, h->opt.hbm_budget);
  Plan& P = h->plan;
  const int n = P.n;
  hipStream_t s = h->stream;
  if (!solve_orders_valid(P)) {
    P.sfo.clear();
    build_solve_orders(P, nullptr, false);
    if (!solve_orders_valid(P)) return fail(h, BASKER_ERR_INVALID, "solve issue orders");
  }
  std::vector<int32_t> glo(n), ghi(n);
  for (size_t g = 0; g + 1 < P.grpptr.size(); g++)
    for (int k = P.grpptr[g]; k < P.grpptr[g + 1]; k++) { glo[k] = P.grpptr[g]; ghi[k] = P.grpptr[g + 1]; }
  // off-diagonal part by row (CSR), in the order the block back-substitution subtracts
  // it from a row: later blocks first, columns ascending inside a block
  std::vector<int32_t> OTp(n + 1, 0), OTj(P.Oi.size()), OTmap(P.Oi.size());
  for (size_t q = 0; q < P.Oi.size(); q++) OTp[P.Oi[q] + 1]++;
  for (int i = 0; i < n; i++) OTp[i + 1] += OTp[i];
  {
    std::vector<int32_t> fillp(OTp.begin(), OTp.end() - 1);
    for (int b = (int)P.blkptr.size() - 2; b >= 0; b--)
      for (int k = P.blkptr[b]; k < P.blkptr[b + 1]; k++)
        for (int32_t q = P.Op[k]; q < P.Op[k + 1]; q++) {
          int32_t i = P.Oi[q];
          OTj[fillp[i]] = k;
          OTmap[fillp[i]] = P.Omap[q];
          fillp[i]++;
        }
  }
  const int nb = (int)P.blkptr.size() - 1;
  const int nlev = (int)P.lvl_ptr.size() - 1;
  HIPCHK(h, h->Rp.upload(P.Rp, s));
  HIPCHK(h, h->Ri.upload(P.Ri, s));
  HIPCHK(h, h->Rmap.upload(P.Rmap, s));
  HIPCHK(h, h->grp_lo.upload(glo, s));
  HIPCHK(h, h->grp_hi.upload(ghi, s));
  HIPCHK(h, h->seg_c0.upload(P.seg_c0, s));
  HIPCHK(h, h->seg_c1.upload(P.seg_c1, s));
  HIPCHK(h, h->lvl_seg.upload(P.lvl_seg, s));
  HIPCHK(h, h->item_lo.upload(P.item_lo, s));
  HIPCHK(h, h->item_hi.upload(P.item_hi, s));
  HIPCHK(h, h->lvl_col.upload(P.lvl_col, s));
  HIPCHK(h, h->dsep_seg.upload(P.dsep_seg, s));
  HIPCHK(h, h->dsep_H.upload(P.dsep_H, s));
  HIPCHK(h, h->dsep_rng_ptr.upload(P.dsep_rng_ptr, s));
  HIPCHK(h, h->dsep_rng_g0.upload(P.dsep_rng_g0, s));
  HIPCHK(h, h->dsep_rng_len.upload(P.dsep_rng_len, s));
  HIPCHK(h, h->dsep_rng_loc.upload(P.dsep_rng_loc, s));
  HIPCHK(h, h->dsep_poff.upload(P.dsep_poff, s));
  HIPCHK(h, h->dsep_soff.upload(P.dsep_soff, s));
  HIPCHK(h, h->dpanel.reserve(std::max<int64_t>(P.dsep_panel_total, 1)));
  HIPCHK(h, h->dbits.reserve(std::max<int64_t>(P.dsep_bits_total, 1)));
  // pivotal set and block L structure handed between the launches of a separator factored
  // block by block
  HIPCHK(h, h->dscratch.reserve((int64_t)kMaxPanelWords * (1 + kMaxNb)));
  HIPCHK(h, h->piv_local.reserve(n));
  HIPCHK(h, h->cb_off.reserve(n));
  HIPCHK(h, h->cb_np.reserve(n));
  HIPCHK(h, h->cb_nn.reserve(n));
  HIPCHK(h, h->cbI.reserve(cb_capacity(P)));
  HIPCHK(h, h->cbX.reserve(cb_capacity(P)));
  HIPCHK(h, h->nnz_ctr.reserve(2));
  HIPCHK(h, h->lvl_ctr.reserve(std::max(2 * nlev, 1)));
  HIPCHK(h, h->OTp.upload(OTp, s));
  HIPCHK(h, h->OTj.upload(OTj, s));
  HIPCHK(h, h->OTmap.upload(OTmap, s));
  HIPCHK(h, h->prow.upload(P.prow, s));
  HIPCHK(h, h->qcol.upload(P.qcol, s));
  HIPCHK(h, h->blkptr.upload(P.blkptr, s));
  HIPCHK(h, h->grpptr.upload(P.grpptr, s));
  HIPCHK(h, h->st_kind.upload(P.st_kind, s));
  HIPCHK(h, h->st_id.upload(P.st_id, s));
  // solve status word, task counter and done flags of the one-launch solve
  HIPCHK(h, h->s_status.reserve(2 + (int64_t)P.st_kind.size()));
  HIPCHK(h, h->st_dep_ptr.upload(P.st_dep_ptr, s));
  HIPCHK(h, h->st_dep.upload(P.st_dep, s));
  HIPCHK(h, h->st_succ.upload(P.st_succ, s));
  HIPCHK(h, h->st_issue.upload(P.st_issue, s));
  HIPCHK(h, h->sflag.reserve(n));
  HIPCHK(h, h->LTp.reserve(n + 1));
  HIPCHK(h, h->UTp.reserve(n + 1));
  HIPCHK(h, h->diag.reserve(n));
  HIPCHK(h, h->sfo.upload(P.sfo, s));
  HIPCHK(h, h->sbo.upload(P.sbo, s));
  HIPCHK(h, h->sfo_pos.upload(P.sfo_pos, s));
  HIPCHK(h, h->sbo_pos.upload(P.sbo_pos, s));
  HIPCHK(h, h->row_task0.upload(P.row_task0, s));
  HIPCHK(h, h->obad.reserve(n));
  HIPCHK(h, h->ocount.reserve(1));
  {
    // LDS per solve launch: the device's whole workgroup LDS when the level has no more
    // tasks than compute units (one task per CU, so the rows' entries can be staged), else
    // what the level's largest task that fits needs, so several tasks share a CU
    int lds_max = 0, ncu = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess)
      lds_max = 65536;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) ncu = 0;
    lds_max = std::min(lds_max, 160 * 1024);
    if (lds_max > 65536 && solve_lds_setup((size_t)lds_max) != hipSuccess) lds_max = 65536;
    (void)hipGetLastError();
    HIPCHK(h, sepdense_setup());
    const int nsl = (int)P.st_lvl_ptr.size() - 1;
    h->st_lvl_lds.assign(std::max(nsl, 0), 0);
    for (int l = 0; l < nsl; l++) {
      const int nt = P.st_lvl_ptr[l + 1] - P.st_lvl_ptr[l];
      size_t need = solve_lds_bytes(0);
      for (int t = P.st_lvl_ptr[l]; t < P.st_lvl_ptr[l + 1]; t++) {
        const size_t b = solve_lds_bytes(P.st_need[t]);
        if (b <= (size_t)lds_max) need = std::max(need, b);
      }
      h->st_lvl_lds[l] = nt <= ncu ? lds_max : (int32_t)std::min<size_t>(need, (size_t)lds_max);
    }
    // one launch for every task: workgroups with the whole LDS of a CU (less the
    // kernel's own few static bytes), on every CU while the solve is the device's only
    // work, on half of them while other handles work (measured on the batched-BTF
    // workload: every CU takes the lone solve 15.4 -> 14.8 ms but costs a fifth of the
    // throughput of four handles in flight; 32 workgroups slowed the lone solve by a
    // third)
    h->flow_lds = lds_max - kSolveFlowStaticLds;
    h->flow_grid = std::min<int>((int)P.st_kind.size(), std::max(ncu, 1));
    h->flow_grid_shared = std::min<int>((int)P.st_kind.size(), std::max(ncu / 2, 1));
  }
  const int64_t nnzd = (int64_t)P.Ri.size();
  HIPCHK(h, h->vals.reserve(P.nnz));
  HIPCHK(h, h->Rx.reserve(nnzd));
  HIPCHK(h, h->OTx.reserve((int64_t)OTj.size()));
  HIPCHK(h, h->pinv.reserve(n));
  HIPCHK(h, h->piv.reserve(n));
  HIPCHK(h, h->Lbeg.reserve(n));
  HIPCHK(h, h->Lcnt.reserve(n));
  HIPCHK(h, h->Ubeg.reserve(n));
  HIPCHK(h, h->Ucnt.reserve(n));
  HIPCHK(h, h->status.reserve(kStatusWords));
  HIPCHK(h, h->pool.reserve(3));
  (void)nb;
  // L/U pools
  HIPCHK(h, h->Li.reserve(pool_capacity(P, h->opt, 0)));
  HIPCHK(h, h->Lx.reserve(pool_capacity(P, h->opt, 0)));
  HIPCHK(h, h->Ui.reserve(pool_capacity(P, h->opt, 1)));
  HIPCHK(h, h->Ux.reserve(pool_capacity(P, h->opt, 1)));
  // persistent grid and the global fallback workspace (one region per wavefront)
  const int grid = plan_grid(P, h->opt);
  h->grid = grid;
  h->gws_slots = kGwsSlots;
  h->gws_stride = gws_stride_bytes();
  const int64_t regions = gws_regions(P, h->opt);
  HIPCHK(h, h->gws.reserve(h->gws_stride * regions));
  HIPCHK(h, hipMemsetAsync(h->gws.p, 0xff, (size_t)(h->gws_stride * regions), s));
  // first-level cooperative schedule
  h->coop = coop_usable(P);
  h->coop_waves = coop_waves_of(h->opt);
  h->coop_grid = h->coop ? coop_grid_of(P, h->opt, h->coop_waves) : 0;
  HIPCHK(h, h->co_item_lo.upload(P.co_item_lo, s));
  HIPCHK(h, h->co_item_hi.upload(P.co_item_hi, s));
  HIPCHK(h, h->co_item_cols.upload(P.co_item_cols, s));
  HIPCHK(h, h->col_item.upload(P.col_item, s));
  HIPCHK(h, h->dep_ptr.upload(P.dep_ptr, s));
  HIPCHK(h, h->dep_idx.upload(P.dep_idx, s));
  HIPCHK(h, h->sdep_ptr.upload(P.sdep_ptr, s));
  HIPCHK(h, h->sdep_idx.upload(P.sdep_idx, s));
  HIPCHK(h, h->item_bad.reserve((int64_t)P.co_item_lo.size()));
  HIPCHK(h, h->co_item_off.upload(P.co_item_off, s));
  HIPCHK(h, h->co_issue.upload(P.co_issue, s));
  HIPCHK(h, h->co_item_kind.upload(P.co_item_kind, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return BASKER_OK;
}

static basker_status make_handle(const basker_options* o, basker_handle* out, basker_ctx** ph) {
  if (!out) return BASKER_ERR_INVALID;
  *out = nullptr;
  basker_ctx* h = new (std::nothrow) basker_ctx();
  if (!h) return BASKER_ERR_OOM;
  if (o) h->opt = *o; else basker_default_options(&h->opt);
  if (!options_valid(h->opt)) {
    delete h;
    return BASKER_ERR_INVALID;
  }
  h->tune_next = h->opt.autotune ? -2 : -1;
  h->device = h->opt.device;
  if (h->device < 0) {  // analysis only: no device work
    *ph = h;
    return BASKER_OK;
  }
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) { delete h; return BASKER_ERR_DEVICE; }
  if (h->opt.stream) {
    h->stream = (hipStream_t)h->opt.stream;
  } else {
    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete h; return BASKER_ERR_DEVICE; }
    h->own_stream = true;
  }
  for (auto& ev : h->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) { basker_free(h); return BASKER_ERR_DEVICE; }
  }
  *ph = h;
  return BASKER_OK;
}

static void fill_info_static(basker_ctx* h) {
  const Plan& P = h->plan;
  basker_info_t& I = h->info;
  I.n = P.n;
  I.nnz = P.nnz;
  I.nnz_diag = (int64_t)P.Ri.size();
  I.nnz_offdiag = (int64_t)P.Oi.size();
  I.nblocks = (int32_t)P.blkptr.size() - 1;
  I.ngroups = (int32_t)P.grpptr.size() - 1;
  I.struct_rank = P.struct_rank;
  I.max_depth = P.max_depth;
  I.bottleneck = P.bottleneck;
  I.nd_blocks = P.n_nd_blocks;
  I.crit_cols = P.crit_cols;
  I.nlevels = (int32_t)P.lvl_ptr.size() - 1;
  I.solve_levels = (int32_t)P.st_lvl_ptr.size() - 1;
  I.fail_col = -1;
  I.sparse_seps = 0;
  {
    std::vector<char> dense(P.seg_c0.size(), 0);
    for (int32_t sg : P.dsep_seg) dense[sg] = 1;
    for (size_t sg = 0; sg < P.seg_c0.size(); sg++)
      if (P.seg_level[sg] >= 1 && !dense[sg]) I.sparse_seps++;
  }
  I.device_bytes_plan = plan_device_bytes(P, h->opt);
  I.coop_items = coop_usable(P) ? (int32_t)P.co_item_lo.size() : 0;
  I.coop_waves = coop_waves_of(h->opt);
  I.sched_bin_edge = bin_edge_of(h->opt);
  I.fill_bound = P.sym_ok ? 1 : 0;
  I.sym_lnz = P.sym_ok ? P.sym_lnz : 0;
  I.sym_unz = P.sym_ok ? P.sym_unz : 0;
  I.sym_ws_rows = P.sym_ok ? (int32_t)std::min<int64_t>(P.sym_ws_max, INT32_MAX) : 0;
}

extern "C" basker_status basker_symbolic(int32_t n, const int32_t* colptr, const int32_t* rowind, const double* values,
                                         const basker_options* o, basker_handle* out) {
  if (!colptr || (n > 0 && !rowind) || !out) return BASKER_ERR_INVALID;
  basker_ctx* h = nullptr;
  basker_status st = make_handle(o, out, &h);
  if (st != BASKER_OK) return st;
  SymbolicOptions so;
  so.matching = h->opt.matching;
  so.btf = h->opt.btf;
  so.fill_order = h->opt.fill_order;
  so.nd_leaves = h->opt.nd_leaves;
  so.nd_min_block = h->opt.nd_min_block;
  int rc = build_plan(n, colptr, rowind, values, so, h->plan);
  if (rc != 0) {
    basker_status s = rc == -2 ? BASKER_ERR_STRUCT_SINGULAR : BASKER_ERR_INVALID;
    basker_free(h);
    return s;
  }
  build_level0_schedule(h->plan, h->opt.item_cols ? h->opt.item_cols : 256, kSymVisitBudget, bin_edge_of(h->opt));
  h->plan.co_valid = level0_schedule_valid(h->plan);
  if (h->device >= 0) {
    st = upload_plan(h);
    if (st != BASKER_OK) { basker_free(h); return st; }
  }
  fill_info_static(h);
  *out = h;
  return BASKER_OK;
}

extern "C" basker_status basker_symbolic_ordered(int32_t n, const int32_t* colptr, const int32_t* rowind,
                                                 const int32_t* prow, const int32_t* qcol, int32_t nblocks,
                                                 const int32_t* blkptr, int32_t ngroups, const int32_t* grpptr,
                                                 const basker_options* o, basker_handle* out) {
  if (!colptr || (n > 0 && (!rowind || !prow || !qcol)) || !blkptr || !grpptr || !out) return BASKER_ERR_INVALID;
  basker_ctx* h = nullptr;
  basker_status st = make_handle(o, out, &h);
  if (st != BASKER_OK) return st;
  int rc = build_plan_user(n, colptr, rowind, prow, qcol, nblocks, blkptr, ngroups, grpptr, h->plan);
  if (rc != 0) { basker_free(h); return BASKER_ERR_INVALID; }
  build_level0_schedule(h->plan, h->opt.item_cols ? h->opt.item_cols : 256, kSymVisitBudget, bin_edge_of(h->opt));
  h->plan.co_valid = level0_schedule_valid(h->plan);
  if (h->device >= 0) {
    st = upload_plan(h);
    if (st != BASKER_OK) { basker_free(h); return st; }
  }
  fill_info_static(h);
  *out = h;
  return BASKER_OK;
}

static FactorArgs factor_args(basker_ctx* h, int refactor) {
  FactorArgs a{};
  a.n = h->plan.n;
  a.Rp = h->Rp.p; a.Ri = h->Ri.p; a.Rx = h->Rx.p;
  a.grp_lo = h->grp_lo.p; a.grp_hi = h->grp_hi.p;
  a.seg_c0 = h->seg_c0.p; a.seg_c1 = h->seg_c1.p; a.lvl_seg = h->lvl_seg.p; a.lvl_ctr = h->lvl_ctr.p;
  a.item_lo = h->item_lo.p;
  a.item_hi = h->item_hi.p;
  a.nnz_ctr = h->nnz_ctr.p;
  a.col_list = h->lvl_col.p;
  a.cb_off = h->cb_off.p; a.cb_np = h->cb_np.p; a.cb_nn = h->cb_nn.p;
  a.cbI = h->cbI.p; a.cbX = h->cbX.p; a.cbcap = std::min(h->cbI.cap, h->cbX.cap);
  a.mode = 0;
  // chunk: a fraction of the pool per wave so that the waves' partly used chunks
  // cannot exhaust it
  {
    const int64_t waves = std::max<int64_t>(pool_waves(h->plan, h->opt), 1);
    int64_t c = std::min(std::min(h->Li.cap, h->Lx.cap), std::min(h->Ui.cap, h->Ux.cap)) / (kChunkDiv * waves);
    c = std::max<int64_t>(kMinChunk, std::min<int64_t>(c, 1 << 16));
    a.chunk = c;
  }
  a.pinv = h->pinv.p; a.piv = h->piv.p;
  a.Lbeg = h->Lbeg.p; a.Lcnt = h->Lcnt.p; a.Ubeg = h->Ubeg.p; a.Ucnt = h->Ucnt.p;
  a.Li = h->Li.p; a.Lx = h->Lx.p; a.Ui = h->Ui.p; a.Ux = h->Ux.p;
  a.pool_next = h->pool.p;
  // a pool's index and value arrays are grown together; after a failed growth the
  // smaller of the two bounds both
  a.Lcap = std::min(h->Li.cap, h->Lx.cap); a.Ucap = std::min(h->Ui.cap, h->Ux.cap);
  a.status = h->status.p;
  a.tau = h->opt.pivot_tol;
  a.diag_pref = h->opt.diag_pref;
  a.refactor = refactor;
  a.gws = h->gws.p; a.gws_stride = h->gws_stride; a.gws_slots = h->gws_slots;
  a.reverse = h->opt.sched_flags & 1;
  a.co_item_lo = h->co_item_lo.p; a.co_item_hi = h->co_item_hi.p; a.co_item_cols = h->co_item_cols.p;
  a.co_item_kind = h->co_item_kind.p;
  a.col_item = h->col_item.p;
  a.item_bad = h->item_bad.p;
  a.co_item_off = h->co_item_off.p;
  a.co_issue = h->co_issue.p;
  a.use_issue = 0;
  return a;
}

// values -> device copy (if on host) -> scattered into R's block storage
static basker_status stage_values(basker_ctx* h, const double* values, int32_t on_device) {
  const double* dv = values;
  hipStream_t s = h->stream;
  if (!on_device) {
    if (h->plan.nnz > 0)
      HIPCHK(h, hipMemcpyAsync(h->vals.p, values, sizeof(double) * (size_t)h->plan.nnz, hipMemcpyHostToDevice, s));
    dv = h->vals.p;
  }
  HIPCHK(h, hipEventRecord(h->ev[4], s));
  HIPCHK(h, launch_scatter(dv, h->Rmap.p, h->Rx.p, (int64_t)h->plan.Ri.size(), s));
  HIPCHK(h, launch_scatter(dv, h->OTmap.p, h->OTx.p, (int64_t)h->plan.Oi.size(), s));
  HIPCHK(h, hipEventRecord(h->ev[5], s));
  return BASKER_OK;
}

// the launches of one device pass (init, then every level); returns the first error
// BASKER_TRACE_LEVELS=1 in the environment: every factor level is waited for and its
// completion reported on stderr (level, elapsed time, status word), for following a long
// factorization as it runs.  Ignored while the stream is being captured.
static bool trace_levels() {
  static const bool on = [] {
    const char* v = std::getenv("BASKER_TRACE_LEVELS");
    return v != nullptr && v[0] != '\0' && v[0] != '0';
  }();
  return on;
}

static double now_ms() {
  return (double)std::chrono::duration_cast<std::chrono::microseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count() / 1000.0;
}
static thread_local double trace_t0 = 0.0;

static hipError_t trace_level_done(basker_ctx* h, int l, const char* what) {
  if (!trace_levels()) return hipSuccess;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return hipSuccess;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return e;
  int32_t code = 0;
  e = hipMemcpy(&code, h->status.p + ST_CODE, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  std::fprintf(stderr, "basker: factor level %d %s done at %.1f ms, status %d\n", l, what, now_ms() - trace_t0, code);
  std::fflush(stderr);
  return hipSuccess;
}

static hipError_t enqueue_factor(basker_ctx* h, int refactor) {
  hipStream_t s = h->stream;
  if (trace_levels()) trace_t0 = now_ms();
  FactorArgs a = factor_args(h, refactor);
  const Plan& P = h->plan;
  const int nlev = (int)P.lvl_ptr.size() - 1;
  hipError_t e = launch_factor_init(a, nlev, s);
  if (e != hipSuccess) return e;
  DenseSepArgs dA{};
  dA.dsep_seg = h->dsep_seg.p; dA.seg_c0 = h->seg_c0.p; dA.seg_c1 = h->seg_c1.p; dA.dsep_H = h->dsep_H.p;
  dA.rng_ptr = h->dsep_rng_ptr.p; dA.rng_g0 = h->dsep_rng_g0.p; dA.rng_len = h->dsep_rng_len.p;
  dA.rng_loc = h->dsep_rng_loc.p; dA.poff = h->dsep_poff.p; dA.soff = h->dsep_soff.p;
  dA.panel = h->dpanel.p; dA.bits = h->dbits.p; dA.piv_local = h->piv_local.p;
  dA.cb_off = h->cb_off.p; dA.cb_np = h->cb_np.p; dA.cb_nn = h->cb_nn.p; dA.cbI = h->cbI.p; dA.cbX = h->cbX.p;
  dA.pinv = h->pinv.p; dA.piv = h->piv.p;
  dA.Lbeg = h->Lbeg.p; dA.Lcnt = h->Lcnt.p; dA.Ubeg = h->Ubeg.p; dA.Ucnt = h->Ucnt.p;
  dA.Li = h->Li.p; dA.Lx = h->Lx.p; dA.Ui = h->Ui.p; dA.Ux = h->Ux.p;
  dA.pool_next = h->pool.p; dA.Lcap = a.Lcap; dA.Ucap = a.Ucap; dA.nnz_ctr = h->nnz_ctr.p;
  dA.status = h->status.p; dA.tau = h->opt.pivot_tol; dA.diag_pref = h->opt.diag_pref; dA.refactor = refactor;
  dA.pbits_g = h->dscratch.p; dA.lb_g = h->dscratch.p + kMaxPanelWords;
  for (int l = 0; l < nlev; l++) {
    a.item_begin = P.lvl_item_ptr[l];
    a.item_end = P.lvl_item_ptr[l + 1];
    if (l == 0) {
      a.mode = 0;
      a.level = l;
      if (h->coop) {
        // cooperative workgroups over the first level's items: refactorizations wait
        // for their stored U pattern; factorizations run the predicted lists
        // speculatively, check them, and redo the failed items with the safe lists
        const int nco = (int)P.co_item_lo.size();
        a.item_begin = 0;
        a.item_end = nco;
        a.spec = 0;
        a.redo = 0;
        if (refactor) {
          a.dep_src = 1;
          if ((e = launch_factor_coop(a, h->coop_waves, h->coop_grid, s)) != hipSuccess) return e;
        } else if (h->opt.sched_flags & 2) {
          a.dep_src = 0;
          a.dep_ptr = h->sdep_ptr.p;
          a.dep_idx = h->sdep_idx.p;
          if ((e = launch_factor_coop(a, h->coop_waves, h->coop_grid, s)) != hipSuccess) return e;
        } else {
          if ((e = launch_fill_i32(h->item_bad.p, 0, nco, s)) != hipSuccess) return e;
          a.dep_src = 0;
          a.dep_ptr = h->dep_ptr.p;
          a.dep_idx = h->dep_idx.p;
          a.spec = 1;
          a.use_issue = 1;
          if ((e = launch_factor_coop(a, h->coop_waves, h->coop_grid, s)) != hipSuccess) return e;
          if ((e = launch_factor_spec_check(a, P.n, nullptr, s)) != hipSuccess) return e;
          a.spec = 0;
          a.use_issue = 0;
          a.redo = 1;
          a.level = nlev;   // the redo pass pops from its own counter
          a.dep_ptr = h->sdep_ptr.p;
          a.dep_idx = h->sdep_idx.p;
          if ((e = launch_factor_coop(a, h->coop_waves, h->coop_grid, s)) != hipSuccess) return e;
          a.redo = 0;
        }
        if ((e = trace_level_done(h, 0, "first level")) != hipSuccess) return e;
        continue;
      }
      const int grid = std::min(a.item_end - a.item_begin, h->grid);
      if (grid > 0 && (e = launch_factor_level(a, grid, s)) != hipSuccess) return e;
      continue;
    }
    // separator level (Alg. 4): the descendant part of every separator column in
    // parallel, then each separator's own columns -- sparse and in order for small
    // separators, on a dense panel for the others
    a.mode = 1;
    a.level = nlev + l;
    a.col_begin = P.lvl_col_ptr[l];
    a.col_end = refactor ? P.lvl_col_ptr[l] + P.lvl_dcol_cnt[l] : P.lvl_col_ptr[l + 1];
    // one wave a column, as many as are resident: the 4,096-slot table takes a CU's LDS
    // for one wave, the 2,048-slot one fits two, for plans whose every column workspace
    // (the symbolic bound, first steps included) stays within 3/4 of it
    const bool s1small =
        !(h->opt.sched_flags & 8) && P.sym_ok && P.sym_ws_max <= (int64_t)kLdsSlotsStep1Small / 4 * 3;
    int grid = std::min(std::min(a.col_end - a.col_begin, h->grid), s1small ? 2 * kNumCu : kNumCu);
    if (grid > 0 && (e = launch_factor_sep_step1(a, grid, s1small, s)) != hipSuccess) return e;
    a.level = l;
    grid = std::min(a.item_end - a.item_begin, kNumCu * 3);
    if (h->opt.max_grid > 0) grid = std::min(grid, h->opt.max_grid);
    if (grid > 0) {
      if (refactor) {
        a.mode = 0;
        if ((e = launch_factor_level(a, std::min(grid, h->grid), s)) != hipSuccess) return e;
      } else {
        a.mode = 2;
        if ((e = launch_factor_sep_step2(a, grid, s)) != hipSuccess) return e;
      }
    }
    dA.d_begin = P.lvl_dsep_ptr[l];
    if ((e = launch_sepdense(dA, P.lvl_dsep_ptr[l + 1] - P.lvl_dsep_ptr[l], s)) != hipSuccess) return e;
    // separators of several blocks (the launch above skips them): block by block
    for (int d = P.lvl_dsep_ptr[l]; d < P.lvl_dsep_ptr[l + 1]; d++) {
      const int sg = P.dsep_seg[d], H = P.dsep_H[d], m = P.seg_c1[sg] - P.seg_c0[sg];
      if (sep_split(m, block_width(H, (H + 63) / 64, m, kSepDenseLds)) &&
          (e = launch_sepdense_split(dA, d, H, m, kNumCu, s)) != hipSuccess)
        return e;
    }
    if ((e = trace_level_done(h, l, "separator")) != hipSuccess) return e;
  }
  return hipSuccess;
}

// status words, pool extents and stored nnz counts of the pass just enqueued
static basker_status read_factor_status(basker_ctx* h, int32_t* st, unsigned long long* poolc,
                                        unsigned long long* nnzc) {
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(st, h->status.p, sizeof(int32_t) * ST_WORDS, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(poolc, h->pool.p, sizeof(unsigned long long) * 3, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(nnzc, h->nnz_ctr.p, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return BASKER_OK;
}

// one device pass; fills st[ST_WORDS], the pool extents and the stored nnz counts
static basker_status run_factor_kernel(basker_ctx* h, int refactor, int32_t* st, unsigned long long* poolc,
                                       unsigned long long* nnzc) {
  hipStream_t s = h->stream;
  HIPCHK(h, hipEventRecord(h->ev[0], s));
  HIPCHK(h, enqueue_factor(h, refactor));
  HIPCHK(h, hipEventRecord(h->ev[1], s));
  basker_status r = read_factor_status(h, st, poolc, nnzc);
  if (r != BASKER_OK) return r;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess) h->info.factor_kernel_ms = ms;
  if (hipEventElapsedTime(&ms, h->ev[4], h->ev[5]) == hipSuccess) h->info.scatter_kernel_ms = ms;
  return BASKER_OK;
}

static void drop_refactor_graph(basker_ctx* h) {
  if (h->rgexec) (void)hipGraphExecDestroy(h->rgexec);
  if (h->rgraph) (void)hipGraphDestroy(h->rgraph);
  h->rgexec = nullptr;
  h->rgraph = nullptr;
}

// capture the refactorization launches (value scatter from h->vals, init, levels)
static bool capture_refactor_graph(basker_ctx* h) {
  hipStream_t s = h->stream;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  hipError_t e = launch_scatter(h->vals.p, h->Rmap.p, h->Rx.p, (int64_t)h->plan.Ri.size(), s);
  if (e == hipSuccess) e = launch_scatter(h->vals.p, h->OTmap.p, h->OTx.p, (int64_t)h->plan.Oi.size(), s);
  if (e == hipSuccess) e = enqueue_factor(h, 1);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  h->rgraph = g;
  h->rgexec = x;
  return true;
}
// Row-wise copies of the factors for the solve (rows.hip), after every successful
// factorization or refactorization: buffers sized by the pools' used extents.
static basker_status build_rows(basker_ctx* h) {
  hipStream_t s = h->stream;
  const int64_t lu = std::max<int64_t>(h->Lused, 1), uu = std::max<int64_t>(h->Uused, 1);
  HIPCHK(h, h->lkeys.reserve(lu)); HIPCHK(h, h->lkeys_out.reserve(lu));
  HIPCHK(h, h->lvals.reserve(lu)); HIPCHK(h, h->lvals_out.reserve(lu));
  HIPCHK(h, h->ukeys.reserve(uu)); HIPCHK(h, h->ukeys_out.reserve(uu));
  HIPCHK(h, h->uvals.reserve(uu)); HIPCHK(h, h->uvals_out.reserve(uu));
  size_t tb = 0;
  HIPCHK(h, rows_temp_bytes(std::max(lu, uu), h->plan.n, &tb));
  HIPCHK(h, h->rows_temp.reserve(std::max<int64_t>((int64_t)tb, 1)));
  RowsArgs r{};
  r.n = h->plan.n;
  r.pinv = h->pinv.p;
  r.Lbeg = h->Lbeg.p; r.Lcnt = h->Lcnt.p; r.Li = h->Li.p; r.Lx = h->Lx.p;
  r.Ubeg = h->Ubeg.p; r.Ucnt = h->Ucnt.p; r.Ui = h->Ui.p; r.Ux = h->Ux.p;
  r.Lused = h->Lused; r.Uused = h->Uused;
  r.lkeys = h->lkeys.p; r.lvals = h->lvals.p; r.lkeys_out = h->lkeys_out.p; r.lvals_out = h->lvals_out.p;
  r.ukeys = h->ukeys.p; r.uvals = h->uvals.p; r.ukeys_out = h->ukeys_out.p; r.uvals_out = h->uvals_out.p;
  r.temp = h->rows_temp.p;
  r.temp_bytes = (size_t)h->rows_temp.cap;
  r.LTp = h->LTp.p; r.UTp = h->UTp.p;
  r.diag = h->diag.p;
  r.row_task0 = h->row_task0.p; r.sfo_pos = h->sfo_pos.p; r.sbo_pos = h->sbo_pos.p;
  r.obad = h->obad.p;
  r.ocount = h->ocount.p;
  HIPCHK(h, hipEventRecord(h->ev[4], s));
  HIPCHK(h, launch_rows_build(r, s));
  HIPCHK(h, hipEventRecord(h->ev[5], s));
  int32_t fallbacks = 0;
  HIPCHK(h, hipMemcpyAsync(&fallbacks, h->ocount.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  h->info.solve_order_fallbacks = fallbacks;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev[4], h->ev[5]) == hipSuccess) h->info.rows_kernel_ms = ms;
  return BASKER_OK;
}

// After first-level items were redone: merge their observed U patterns (the columns
// each column actually waited for) into the predicted dependency lists, so the next
// factorization with similar values runs them speculatively again.
static basker_status learn_deps(basker_ctx* h) {
  Plan& P = h->plan;
  const int n = P.n;
  const int nco = (int)P.co_item_lo.size();
  hipStream_t s = h->stream;
  std::vector<int32_t> bad(nco), ub(n), uc(n), ui(h->Uused);
  HIPCHK(h, hipMemcpyAsync(bad.data(), h->item_bad.p, sizeof(int32_t) * nco, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(ub.data(), h->Ubeg.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(uc.data(), h->Ucnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  if (h->Uused > 0)
    HIPCHK(h, hipMemcpyAsync(ui.data(), h->Ui.p, sizeof(int32_t) * h->Uused, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  std::vector<int32_t> items;
  for (int it = 0; it < nco; it++)
    if (bad[it]) items.push_back(it);
  merge_learned_deps(P, items, ub, uc, ui);
  P.co_valid = level0_schedule_valid(P);
  if (!P.co_valid) h->coop = false;
  HIPCHK(h, h->dep_ptr.upload(P.dep_ptr, s));
  HIPCHK(h, h->dep_idx.upload(P.dep_idx, s));
  HIPCHK(h, h->co_issue.upload(P.co_issue, s));
  HIPCHK(h, h->sbo.upload(P.sbo, s));
  HIPCHK(h, h->sbo_pos.upload(P.sbo_pos, s));
  HIPCHK(h, hipStreamSynchronize(s));
  h->info.learn_events++;
  return BASKER_OK;
}

// First-level schedule candidates of the autotuner (bin edge option, wavefronts per
// workgroup).  Every candidate gives the same factors; only the time differs.
struct TuneCand {
  int bin_edge;
  int waves;
};
constexpr TuneCand kTuneCands[] = {{32, 6}, {8, 6}, {128, 6}, {-1, 6}, {32, 7}, {128, 7}, {32, 8}, {128, 8}, {32, 4}};
constexpr int kNumTuneCands = (int)(sizeof(kTuneCands) / sizeof(kTuneCands[0]));

// Rebuild the first level's work items for a bin edge and wave count and upload them;
// the dependency lists stay.  The fallback workspace grows if the wider workgroups need
// more wavefront regions.
static basker_status apply_schedule(basker_ctx* h, int bin_edge, int waves) {
  Plan& P = h->plan;
  hipStream_t s = h->stream;
  h->opt.bin_edge = bin_edge;
  h->opt.coop_waves = waves;
  build_level0_items(P, h->opt.item_cols ? h->opt.item_cols : 256, bin_edge_of(h->opt));
  build_issue_order(P);
  P.co_valid = level0_schedule_valid(P);
  h->coop = coop_usable(P);
  h->coop_waves = coop_waves_of(h->opt);
  h->coop_grid = h->coop ? coop_grid_of(P, h->opt, h->coop_waves) : 0;
  HIPCHK(h, h->co_item_lo.upload(P.co_item_lo, s));
  HIPCHK(h, h->co_item_hi.upload(P.co_item_hi, s));
  HIPCHK(h, h->co_item_cols.upload(P.co_item_cols, s));
  HIPCHK(h, h->co_item_kind.upload(P.co_item_kind, s));
  HIPCHK(h, h->col_item.upload(P.col_item, s));
  HIPCHK(h, h->item_bad.reserve((int64_t)P.co_item_lo.size()));
  HIPCHK(h, h->co_item_off.upload(P.co_item_off, s));
  HIPCHK(h, h->co_issue.upload(P.co_issue, s));
  const int64_t bytes = h->gws_stride * gws_regions(P, h->opt);
  if (bytes > h->gws.cap) {
    HIPCHK(h, h->gws.reserve(bytes));
    HIPCHK(h, hipMemsetAsync(h->gws.p, 0xff, (size_t)bytes, s));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  h->info.coop_items = h->coop ? (int32_t)P.co_item_lo.size() : 0;
  h->info.coop_waves = h->coop_waves;
  h->info.sched_bin_edge = bin_edge_of(h->opt);
  return BASKER_OK;
}

static basker_status do_factor_pass(basker_ctx* h);

// A full factorization; with autotune on, the first ones time the schedule candidates
// (the first call, which learns dependencies, is not timed) and the fastest is kept.
static basker_status do_factor(basker_ctx* h) {
  if (h->tune_next >= 0) {
    const TuneCand c = kTuneCands[h->tune_next];
    basker_status r = apply_schedule(h, c.bin_edge, c.waves);
    if (r != BASKER_OK) return r;
  }
  basker_status r = do_factor_pass(h);
  if (r != BASKER_OK || h->tune_next == -1) return r;
  if (h->tune_next == -2) {
    h->tune_next = 0;
    h->tune_ms.assign(kNumTuneCands, 0.f);
    return r;
  }
  h->tune_ms[h->tune_next] = (float)h->info.factor_kernel_ms;
  h->info.autotune_trials = ++h->tune_next;
  if (h->tune_next == kNumTuneCands) {
    int best = 0;
    for (int c = 1; c < kNumTuneCands; c++)
      if (h->tune_ms[c] < h->tune_ms[best]) best = c;
    h->tune_next = -1;
    r = apply_schedule(h, kTuneCands[best].bin_edge, kTuneCands[best].waves);
  }
  return r;
}

static basker_status do_factor_pass(basker_ctx* h) {
  drop_refactor_graph(h);   // pools may move
  for (int attempt = 0; attempt < 8; attempt++) {
    int32_t st[ST_WORDS];
    unsigned long long poolc[3], nnzc[2];
    basker_status r = run_factor_kernel(h, 0, st, poolc, nnzc);
    if (r != BASKER_OK) return r;
    h->info.fail_col = st[ST_FAILCOL] == 0x7fffffff ? -1 : st[ST_FAILCOL];
    if (st[ST_CODE] == DEV_OK) {
      h->lnz = (int64_t)nnzc[0];
      h->unz = (int64_t)nnzc[1];
      h->Lused = std::min<int64_t>((int64_t)poolc[0], h->Li.cap);
      h->Uused = std::min<int64_t>((int64_t)poolc[1], h->Ui.cap);
      h->info.lnz = h->lnz;
      h->info.unz = h->unz;
      h->info.offdiag_pivots = st[ST_OFFDIAG];
      h->info.dense_seps = st[ST_DSEP];
      h->info.redo_items = st[ST_REDO];
      h->factored = true;
      h->info.factor_calls++;
      if (st[ST_REDO] > 0) {
        basker_status lr = learn_deps(h);
        if (lr != BASKER_OK) return lr;
      }
      basker_status rr = build_rows(h);
      if (rr != BASKER_OK) h->factored = false;
      return rr;
    }
    h->factored = false;
    if (st[ST_CODE] == DEV_POOL && st[ST_CBPOOL]) {
      int64_t need = std::max<int64_t>((int64_t)poolc[2] * 4, 4 * h->cbI.cap);
      if (need > 0x7fffffffLL) need = 0x7fffffffLL;
      if (need <= h->cbI.cap) return fail(h, BASKER_ERR_OOM, "separator buffer exceeds 2^31 entries");
      HIPCHK(h, h->cbI.reserve(need));
      HIPCHK(h, h->cbX.reserve(need));
      h->info.pool_regrows++;
      continue;
    }
    if (st[ST_CODE] == DEV_POOL) {
      // grow the pool(s) that ran out to four times the demand seen so far (every growth
      // repeats the pass, and the demand seen is only what the pass reached)
      bool grew = false;
      const bool l_over = (int64_t)poolc[0] > h->Li.cap, u_over = (int64_t)poolc[1] > h->Ui.cap;
      if (l_over || !u_over) {
        int64_t need = std::min<int64_t>(std::max<int64_t>((int64_t)poolc[0] * 4, 4 * h->Li.cap), 0x7fffffffLL);
        if (need > h->Li.cap) {
          HIPCHK(h, h->Li.reserve(need));
          HIPCHK(h, h->Lx.reserve(need));
          grew = true;
        }
      }
      if (u_over || !l_over) {
        int64_t need = std::min<int64_t>(std::max<int64_t>((int64_t)poolc[1] * 4, 4 * h->Ui.cap), 0x7fffffffLL);
        if (need > h->Ui.cap) {
          HIPCHK(h, h->Ui.reserve(need));
          HIPCHK(h, h->Ux.reserve(need));
          grew = true;
        }
      }
      if (!grew) return fail(h, BASKER_ERR_OOM, "L/U pool exceeds 2^31 entries");
      h->info.pool_regrows++;
      continue;
    }
    if (st[ST_CODE] == DEV_SINGULAR)
      return fail(h, BASKER_ERR_NUM_SINGULAR, "numerically singular at column " + std::to_string(h->info.fail_col));
    if (st[ST_CODE] == DEV_WORKSPACE)
      return fail(h, BASKER_ERR_WORKSPACE, "column pattern exceeds the workspace at column " + std::to_string(h->info.fail_col));
    return fail(h, BASKER_ERR_DEVICE, "factor kernel status " + std::to_string(st[ST_CODE]));
  }
  return fail(h, BASKER_ERR_OOM, "L/U pool growth did not converge");
}

// A plan the numeric kernels cannot run is refused before any device work: a column
// whose reach without row exchanges exceeds the per-wave global workspace (known when
// the symbolic analysis finished within its budget; otherwise the kernels detect an
// overflow as they go).
static basker_status plan_guard(basker_ctx* h) {
  const Plan& P = h->plan;
  if (P.sym_ok && P.sym_ws_max > kGwsSlots / 2)
    return fail(h, BASKER_ERR_WORKSPACE,
                "a column's reach without row exchanges (" + std::to_string(P.sym_ws_max) +
                    " rows) exceeds the per-wave workspace (" + std::to_string(kGwsSlots / 2) + " rows)");
  return BASKER_OK;
}

// Handles busy in a factorization, refactorization or solve on each device (those calls
// return after their work), to size the one-launch solve's grid: every CU for a solve
// that is the device's only work, half of them when other handles are working.
constexpr int kMaxDevices = 64;
static std::atomic<int> g_busy[kMaxDevices];

struct BusyScope {
  std::atomic<int>* c;
  explicit BusyScope(int dev) : c(dev >= 0 && dev < kMaxDevices ? &g_busy[dev] : nullptr) {
    if (c) c->fetch_add(1);
  }
  ~BusyScope() {
    if (c) c->fetch_sub(1);
  }
  bool alone() const { return !c || c->load() <= 1; }
};

extern "C" basker_status basker_factor(basker_handle h, const double* values, int32_t values_on_device) {
  if (!h || (!values && h->plan.nnz > 0)) return BASKER_ERR_INVALID;
  AcctScope acct(&h->dev_bytes, h->opt.hbm_budget);
  const basker_status g = plan_guard(h);
  if (g != BASKER_OK) return g;
  if (h->device < 0) return fail(h, BASKER_ERR_DEVICE, "handle was created for analysis only (device < 0)");
  HIPCHK(h, hipSetDevice(h->device));
  BusyScope busy(h->device);
  basker_status r = stage_values(h, values, values_on_device);
  if (r != BASKER_OK) return r;
  return do_factor(h);
}

extern "C" basker_status basker_refactor(basker_handle h, const double* values, int32_t values_on_device) {
  if (!h || (!values && h->plan.nnz > 0)) return BASKER_ERR_INVALID;
  AcctScope acct(&h->dev_bytes, h->opt.hbm_budget);
  if (h->device < 0) return fail(h, BASKER_ERR_DEVICE, "handle was created for analysis only (device < 0)");
  if (!h->factored) return fail(h, BASKER_ERR_PATTERN, "refactor before a successful factor");
  HIPCHK(h, hipSetDevice(h->device));
  BusyScope busy(h->device);
  int32_t st[ST_WORDS];
  unsigned long long poolc[3], nnzc[2];
  basker_status r = BASKER_OK;
  bool graphed = false;
  if (h->opt.refactor_graph) {
    // the graph reads the values from the handle's buffer
    hipStream_t s = h->stream;
    if (h->plan.nnz > 0 && values != h->vals.p)
      HIPCHK(h, hipMemcpyAsync(h->vals.p, values, sizeof(double) * (size_t)h->plan.nnz,
                               values_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (h->rgexec || capture_refactor_graph(h)) {
      HIPCHK(h, hipEventRecord(h->ev[0], s));
      HIPCHK(h, hipGraphLaunch(h->rgexec, s));
      HIPCHK(h, hipEventRecord(h->ev[1], s));
      r = read_factor_status(h, st, poolc, nnzc);
      if (r != BASKER_OK) return r;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess) h->info.factor_kernel_ms = ms;
      h->info.scatter_kernel_ms = 0.0;   // inside the graph, counted in factor_kernel_ms
      graphed = true;
    }
  }
  if (!graphed) {
    r = stage_values(h, values, values_on_device);
    if (r != BASKER_OK) return r;
    r = run_factor_kernel(h, 1, st, poolc, nnzc);
    if (r != BASKER_OK) return r;
  }
  h->info.refactor_calls++;
  if (st[ST_CODE] == DEV_OK) {
    r = build_rows(h);
    if (r != BASKER_OK) h->factored = false;
    return r;
  }
  h->info.fail_col = st[ST_FAILCOL] == 0x7fffffff ? -1 : st[ST_FAILCOL];
  if (st[ST_CODE] == DEV_REFACTOR_FAIL || st[ST_CODE] == DEV_WORKSPACE) {
    h->info.refactor_fallbacks++;
    r = do_factor(h);
    return r == BASKER_OK ? BASKER_REFACTOR_FELL_BACK : r;
  }
  h->factored = false;
  return fail(h, BASKER_ERR_DEVICE, "refactor kernel status " + std::to_string(st[ST_CODE]));
}

// The task launches of one solve on device-resident B (leading dimension ld) with the
// work vectors W and Z (n * nrhs doubles each) given by the caller; the status word,
// flags and row-wise factors are the handle's.  Enqueues only: allocates nothing.
static basker_status enqueue_solve(basker_ctx* h, int32_t nrhs, double* dB, int32_t ld, double* W, double* Z,
                                   bool alone) {
  hipStream_t s = h->stream;
  SolveArgs a{};
  a.n = h->plan.n;
  a.nrhs = nrhs;
  a.ldb = ld;
  a.blkptr = h->blkptr.p;
  a.grpptr = h->grpptr.p;
  a.st_kind = h->st_kind.p; a.st_id = h->st_id.p;
  a.piv = h->piv.p;
  a.diag = h->diag.p;
  a.LTp = h->LTp.p; a.lkeys = h->lkeys_out.p; a.lvals = h->lvals_out.p;
  a.UTp = h->UTp.p; a.ukeys = h->ukeys_out.p; a.uvals = h->uvals_out.p;
  a.OTp = h->OTp.p; a.OTj = h->OTj.p; a.OTx = h->OTx.p;
  a.sfo = h->sfo.p; a.sbo = h->sbo.p; a.obad = h->obad.p;
  a.prow = h->prow.p; a.qcol = h->qcol.p;
  a.B = dB; a.W = W; a.Z = Z;
  a.sflag = h->sflag.p;
  a.status = h->s_status.p;
  a.qctr = h->s_status.p + 1;
  a.done = h->s_status.p + 2;
  a.ntasks = (int32_t)h->plan.st_kind.size();
  a.dep_ptr = h->st_dep_ptr.p; a.dep = h->st_dep.p; a.succ = h->st_succ.p; a.issue = h->st_issue.p;
  const Plan& P = h->plan;
  const int nsl = (int)P.st_lvl_ptr.size() - 1;
  HIPCHK(h, launch_fill_i32(h->s_status.p, 0, 2 + (int64_t)a.ntasks, s));
  // sched_flags bit 4 (a check of the failure path): the launch starts as if a wait had
  // already given up, so every wait that has to wait gives up at its first failed poll
  if (h->opt.sched_flags & 16) HIPCHK(h, launch_fill_i32(h->s_status.p, 8, 1, s));
  HIPCHK(h, launch_solve_pending(Z, (int64_t)a.n * nrhs, s));
  HIPCHK(h, hipEventRecord(h->ev[2], s));
  if (h->opt.sched_flags & 4) {
    for (int l = 0; l < nsl; l++) {
      a.t_begin = P.st_lvl_ptr[l];
      a.lds_bytes = h->st_lvl_lds[l];
      HIPCHK(h, launch_solve_tasks(a, P.st_lvl_ptr[l + 1] - P.st_lvl_ptr[l], s));
    }
  } else {
    a.t_begin = 0;
    a.lds_bytes = h->flow_lds;
    HIPCHK(h, launch_solve_flow(a, alone ? h->flow_grid : h->flow_grid_shared, s));
  }
  HIPCHK(h, launch_solve_finish(a, s));
  HIPCHK(h, hipEventRecord(h->ev[3], s));
  return BASKER_OK;
}

// wait for the solve just enqueued, read its status word and timing
static basker_status finish_solve(basker_ctx* h) {
  int32_t sst = 0;
  HIPCHK(h, hipMemcpyAsync(&sst, h->s_status.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev[2], h->ev[3]) == hipSuccess) h->info.solve_kernel_ms = ms;
  if (sst != 0) return fail(h, BASKER_ERR_DEVICE, "solve: a row's wait for another row did not end");
  return BASKER_OK;
}

extern "C" basker_status basker_solve(basker_handle h, int32_t nrhs, double* B, int32_t ldb, int32_t B_on_device) {
  if (!h || nrhs < 0 || (nrhs > 0 && !B) || ldb < h->plan.n) return BASKER_ERR_INVALID;
  AcctScope acct(&h->dev_bytes, h->opt.hbm_budget);
  if (!h->factored) return fail(h, BASKER_ERR_PATTERN, "solve before a successful factor");
  if (nrhs == 0 || h->plan.n == 0) return BASKER_OK;
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  const int n = h->plan.n;
  const int64_t tot = (int64_t)n * nrhs;
  HIPCHK(h, h->W.reserve(tot));
  HIPCHK(h, h->Z.reserve(tot));
  double* dB = B;
  int32_t ld = ldb;
  if (!B_on_device) {
    HIPCHK(h, h->Bdev.reserve(tot));
    HIPCHK(h, hipMemcpy2DAsync(h->Bdev.p, sizeof(double) * n, B, sizeof(double) * (size_t)ldb, sizeof(double) * n,
                               nrhs, hipMemcpyHostToDevice, s));
    dB = h->Bdev.p;
    ld = n;
  }
  BusyScope busy(h->device);
  basker_status r = enqueue_solve(h, nrhs, dB, ld, h->W.p, h->Z.p, busy.alone());
  if (r != BASKER_OK) return r;
  if (!B_on_device)
    HIPCHK(h, hipMemcpy2DAsync(B, sizeof(double) * (size_t)ldb, h->Bdev.p, sizeof(double) * n, sizeof(double) * n,
                               nrhs, hipMemcpyDeviceToHost, s));
  return finish_solve(h);
}

extern "C" basker_status basker_solve_noalloc(basker_handle h, int32_t nrhs, double* B, int32_t ldb) {
  if (!h || nrhs < 0 || (nrhs > 0 && !B) || ldb < h->plan.n) return BASKER_ERR_INVALID;
  if (h->device < 0) return fail(h, BASKER_ERR_DEVICE, "handle was created for analysis only (device < 0)");
  if (!h->factored) return fail(h, BASKER_ERR_PATTERN, "solve before a successful factor");
  if (nrhs == 0 || h->plan.n == 0) return BASKER_OK;
  HIPCHK(h, hipSetDevice(h->device));
  double* sp = nullptr;
  HIPCHK(h, noalloc_scratch(h->device, &sp));
  const int64_t n = h->plan.n;
  const int64_t need = 2 * n * (int64_t)nrhs;
  if (need > kNoAllocScratchDoubles)
    return fail(h, BASKER_ERR_WORKSPACE,
                "solve needs " + std::to_string(need) + " doubles of scratch (2 n nrhs); the static scratch holds " +
                    std::to_string(kNoAllocScratchDoubles));
  BusyScope busy(h->device);
  basker_status r = enqueue_solve(h, nrhs, B, ldb, sp, sp + n * nrhs, busy.alone());
  if (r != BASKER_OK) return r;
  return finish_solve(h);
}

extern "C" basker_status basker_info(basker_handle h, basker_info_t* info) {
  if (!h || !info) return BASKER_ERR_INVALID;
  *info = h->info;
  info->device_bytes = h->dev_bytes;
  return BASKER_OK;
}

extern "C" basker_status basker_get_ordering(basker_handle h, int32_t* prow, int32_t* qcol, int32_t* blkptr,
                                             int32_t* grpptr, int32_t* grpparent) {
  if (!h) return BASKER_ERR_INVALID;
  const Plan& P = h->plan;
  if (prow) std::copy(P.prow.begin(), P.prow.end(), prow);
  if (qcol) std::copy(P.qcol.begin(), P.qcol.end(), qcol);
  if (blkptr) std::copy(P.blkptr.begin(), P.blkptr.end(), blkptr);
  if (grpptr) std::copy(P.grpptr.begin(), P.grpptr.end(), grpptr);
  if (grpparent) std::copy(P.grp_parent.begin(), P.grp_parent.end(), grpparent);
  return BASKER_OK;
}

extern "C" basker_status basker_extract(basker_handle h, int32_t* piv, int64_t* Lp, int32_t* Li, double* Lx,
                                        int64_t* Up, int32_t* Ui, double* Ux) {
  if (!h) return BASKER_ERR_INVALID;
  if (!h->factored) return fail(h, BASKER_ERR_PATTERN, "extract before a successful factor");
  HIPCHK(h, hipSetDevice(h->device));
  const int n = h->plan.n;
  hipStream_t s = h->stream;
  std::vector<int32_t> hpiv(n), lb(n), lc(n), ubg(n), ucn(n);
  std::vector<int32_t> li(h->Lused), ui(h->Uused);
  std::vector<double> lx(h->Lused), ux(h->Uused);
  if (n > 0) {
    HIPCHK(h, hipMemcpyAsync(hpiv.data(), h->piv.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(lb.data(), h->Lbeg.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(lc.data(), h->Lcnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(ubg.data(), h->Ubeg.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(ucn.data(), h->Ucnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  }
  if (h->Lused > 0) {
    HIPCHK(h, hipMemcpyAsync(li.data(), h->Li.p, sizeof(int32_t) * h->Lused, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(lx.data(), h->Lx.p, sizeof(double) * h->Lused, hipMemcpyDeviceToHost, s));
  }
  if (h->Uused > 0) {
    HIPCHK(h, hipMemcpyAsync(ui.data(), h->Ui.p, sizeof(int32_t) * h->Uused, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(ux.data(), h->Ux.p, sizeof(double) * h->Uused, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  std::vector<int32_t> pinv(n, -1);
  for (int k = 0; k < n; k++) pinv[hpiv[k]] = k;
  if (piv) std::copy(hpiv.begin(), hpiv.end(), piv);
  std::vector<std::pair<int32_t, double>> tmp;
  int64_t lo = 0, uo = 0;
  if (Lp) Lp[0] = 0;
  if (Up) Up[0] = 0;
  for (int k = 0; k < n; k++) {
    tmp.clear();
    for (int t = 0; t < lc[k]; t++) tmp.push_back({pinv[li[lb[k] + t]], lx[lb[k] + t]});
    std::sort(tmp.begin(), tmp.end(), [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
      return x.first < y.first;
    });
    for (auto& e : tmp) {
      if (Li) Li[lo] = e.first;
      if (Lx) Lx[lo] = e.second;
      lo++;
    }
    if (Lp) Lp[k + 1] = lo;
    for (int t = 0; t < ucn[k]; t++) {
      if (Ui) Ui[uo] = ui[ubg[k] + t];
      if (Ux) Ux[uo] = ux[ubg[k] + t];
      uo++;
    }
    if (Up) Up[k + 1] = uo;
  }
  return BASKER_OK;
}

extern "C" void basker_free(basker_handle h) {
  if (!h) return;
  if (h->device < 0) { delete h; return; }
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  drop_refactor_graph(h);
  for (auto& ev : h->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}
