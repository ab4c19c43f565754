// Device-side argument blocks and kernel launchers shared by the HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// LDS declaration used by the kernels (a CPU debug build of the sources may redefine
// it to give every emulated workgroup its own copy)
#ifndef BASKER_SHARED
#define BASKER_SHARED(type, name) __shared__ type name
#endif
#ifndef BASKER_DYN_SHARED
#define BASKER_DYN_SHARED(type, name) extern __shared__ type name[]
#endif

namespace basker {

constexpr int kWave = 64;
constexpr int kLdsSlots = 512;        // per-wave LDS hash slots (power of two)
constexpr int kLdsSlotsSep = 1024;    // larger table for separator columns (mode 2)
constexpr int kLdsSlotsStep1 = 4096;  // the column-parallel first step of separator levels
// its variant for workspaces of at most 3/4 of this table (two waves fit a CU's LDS)
constexpr int kLdsSlotsStep1Small = 2048;
                                      // (one workgroup per CU: ~135 KB of LDS)
constexpr int kWavesPerCu = 6;        // persistent-grid occupancy target
constexpr int kNumCu = 256;

// status words (device): [0] error code, [1] failing column (min), [2] pool overflow,
// [3] workspace overflow, [4] pivots off the diagonal, [5] separator buffer overflow,
// [6] separators completed by the dense kernel
enum { ST_CODE = 0, ST_FAILCOL = 1, ST_POOL = 2, ST_WS = 3, ST_OFFDIAG = 4, ST_CBPOOL = 5, ST_DSEP = 6,
       ST_WORDS = 8 };
constexpr int kStatusWords = ST_WORDS;
enum { DEV_OK = 0, DEV_SINGULAR = 3, DEV_REFACTOR_FAIL = 8, DEV_WORKSPACE = 7, DEV_POOL = 4, DEV_PATTERN = 5,
       DEV_STALL = 9 };
// status word 7: first-level work items redone after a failed speculation
constexpr int ST_REDO = 7;
// the cooperative kernel keeps one done bit per column of an item in LDS
constexpr int kCoopMaxItemCols = 65536;

struct FactorArgs {
  int32_t n;
  const int32_t* Rp;       // diagonal-block part of R (rows ascending)
  const int32_t* Ri;
  const double* Rx;
  const int32_t* grp_lo;   // candidate group of each column: [grp_lo, grp_hi)
  const int32_t* grp_hi;
  const int32_t* seg_c0;   // segments: column ranges factored by one wave in order
  const int32_t* seg_c1;
  const int32_t* lvl_seg;  // segments in level order (largest first inside a level)
  const int32_t* item_lo;  // work items: item i = segments lvl_seg[item_lo[i] .. item_hi[i])
  const int32_t* item_hi;
  int32_t item_begin;      // items of the launched level: [item_begin, item_end)
  int32_t item_end;
  int32_t* lvl_ctr;        // one pop counter per level (zeroed before the level)
  int32_t level;
  int64_t chunk;           // pool entries a wave claims at a time
  unsigned long long* nnz_ctr;  // [0] nnz(L), [1] nnz(U) actually stored
  // separator levels of a factorization run in two launches (Alg. 4): mode 1 applies
  // the descendant pivots to every separator column independently (U of the
  // off-diagonal blocks and the reduction into the separator and ancestor rows) and
  // parks the partial column in the column buffer; mode 2 then factors each
  // separator's columns in order from those partial columns.  Mode 0 is the whole
  // column in one pass.
  int32_t mode;
  const int32_t* col_list; // mode 1: columns of the launched level [col_begin, col_end)
  int32_t col_begin;
  int32_t col_end;
  int32_t* cb_off;         // per column: offset of its partial column in the buffer
  int32_t* cb_np;          //   descendant pivots (U entries, ascending pivot column)
  int32_t* cb_nn;          //   non-pivotal rows that follow them
  int32_t* cbI;            // column buffer: pivot column (U part) or row (rest)
  double* cbX;
  int64_t cbcap;
  int32_t* pinv;           // R row -> column it pivots (-1)
  int32_t* piv;            // column -> R row
  int32_t* Lbeg;           // per-column offsets/counts into the pools
  int32_t* Lcnt;
  int32_t* Ubeg;
  int32_t* Ucnt;
  int32_t* Li;             // L rows (R-row numbering), values divided by the pivot
  double* Lx;
  int32_t* Ui;             // U rows (column numbering, ascending, diagonal last)
  double* Ux;
  unsigned long long* pool_next;   // [0] L, [1] U, [2] column buffer
  int64_t Lcap;
  int64_t Ucap;
  int32_t* status;
  double tau;
  int32_t diag_pref;
  int32_t refactor;
  char* gws;               // global fallback workspace, one region per workgroup
  int64_t gws_stride;      // bytes per region
  int32_t gws_slots;       // hash slots per region (power of two)
  int32_t reverse;         // hand out work items last first (results do not depend on it)
  // first level, cooperative kernel: items of consecutive segments (into lvl_seg) with
  // their column counts, a dependency list per column (dep_src 0: dep_ptr/dep_idx,
  // ascending column indices inside the segment; 1: the stored U pattern of a
  // refactorization), speculation (spec) with a per-item failure flag, and the redo
  // pass (redo: only items whose flag is set, their state cleared first)
  const int32_t* co_item_lo;
  const int32_t* co_item_hi;
  const int32_t* co_item_cols;
  const int32_t* col_item;
  const int32_t* dep_ptr;
  const int32_t* dep_idx;
  int32_t dep_src;
  int32_t spec;
  int32_t redo;
  int32_t* item_bad;
  const int32_t* co_item_kind;  // size bin of every item: 0 shared columns, 1 wave per segment, 2 thread per 1 x 1 block
  const int32_t* co_item_off;   // first issue entry of every item
  const int32_t* co_issue;      // (column, slot, segment start) in the issue order of the speculative pass
  int32_t use_issue;            // 1: take columns from co_issue; 0: in slot order
};

// row-wise copies of the factors (rows.hip): sort keys and values of the L and U pool
// extents, the sorted copies, and the row pointers LTp / UTp (n + 1 each)
struct RowsArgs {
  int32_t n;
  const int32_t* pinv;
  const int32_t* Lbeg; const int32_t* Lcnt; const int32_t* Li; const double* Lx;
  const int32_t* Ubeg; const int32_t* Ucnt; const int32_t* Ui; const double* Ux;
  int64_t Lused, Uused;
  unsigned long long* lkeys; double* lvals; unsigned long long* lkeys_out; double* lvals_out;
  unsigned long long* ukeys; double* uvals; unsigned long long* ukeys_out; double* uvals_out;
  void* temp;
  size_t temp_bytes;
  int32_t* LTp;
  int32_t* UTp;
  double* diag;            // out: U's diagonal (the last entry of every U column)
  // solve issue orders to check against the rows: the first row of every row's solve
  // task, each row's rank in its task's forward and backward orders; out: per task
  // (indexed by its first row) bit 0 = forward order invalid, bit 1 = backward
  const int32_t* row_task0;
  const int32_t* sfo_pos;
  const int32_t* sbo_pos;
  int32_t* obad;
  int32_t* ocount;         // out: sweeps found invalid (one word)
};

hipError_t rows_temp_bytes(int64_t items, int n, size_t* bytes);
hipError_t launch_rows_build(const RowsArgs& a, hipStream_t s);

// solve tasks are workgroups of kSW wavefronts
constexpr int kSW = 8;

struct SolveArgs {
  int32_t n;
  int32_t nrhs;
  int32_t ldb;
  const int32_t* blkptr;
  const int32_t* grpptr;
  // tasks of the launched level: st_*[t_begin .. t_begin + grid)
  const int32_t* st_kind;
  const int32_t* st_id;
  int32_t t_begin;
  int32_t lds_bytes;       // dynamic LDS of the launch; a task whose rows' work arrays fit runs in it
  const int32_t* piv;
  const double* diag;      // U's diagonal by column
  // row-wise factors: L rows ascending in column, U rows descending (keys: row << 32 |
  // column, or n - 1 - column for U), first entry of every row
  const int32_t* LTp; const unsigned long long* lkeys; const double* lvals;
  const int32_t* UTp; const unsigned long long* ukeys; const double* uvals;
  // issue orders: the rows of every task in the order its wavefronts take them
  // (sfo forward, sbo backward, at the task's first row), used where `obad` of the task
  // has the sweep's bit clear
  const int32_t* sfo;
  const int32_t* sbo;
  const int32_t* obad;
  const int32_t* OTp;      // off-diagonal part by R row (CSR), later blocks first, columns ascending
  const int32_t* OTj;
  const double* OTx;
  const int32_t* prow;
  const int32_t* qcol;
  double* B;               // in/out, column-major (A numbering)
  double* W;               // n x nrhs: L-solve results (pivot order)
  double* Z;               // n x nrhs: solution in R-column numbering
  int32_t* sflag;          // n: done flags of tasks whose rows do not fit in LDS
  int32_t* status;         // nonzero on a stalled wait
  // one launch for all tasks: predecessors of every task (launch positions), whether a
  // later task waits for it, done flags and the task counter (zero before the launch)
  int32_t ntasks;
  const int32_t* issue;    // the order in which tasks are taken (launch positions)
  const int32_t* dep_ptr;
  const int32_t* dep;
  const int32_t* succ;
  int32_t* done;
  int32_t* qctr;
};

struct DenseSepArgs {
  const int32_t* dsep_seg;  // dense separators: segment, panel rows, row ranges, offsets
  const int32_t* seg_c0;
  const int32_t* seg_c1;
  const int32_t* dsep_H;
  const int32_t* rng_ptr;
  const int32_t* rng_g0;
  const int32_t* rng_len;
  const int32_t* rng_loc;
  const int64_t* poff;
  const int64_t* soff;
  int32_t d_begin;          // separators of the launched level: [d_begin, d_begin + grid)
  double* panel;
  unsigned long long* bits;
  int32_t* piv_local;       // per column: local pivot row inside its separator panel
  const int32_t* cb_off;    // partial columns from the first step
  const int32_t* cb_np;
  const int32_t* cb_nn;
  const int32_t* cbI;
  const double* cbX;
  int32_t* pinv;
  int32_t* piv;
  int32_t* Lbeg; int32_t* Lcnt; int32_t* Ubeg; int32_t* Ucnt;
  int32_t* Li; double* Lx; int32_t* Ui; double* Ux;
  unsigned long long* pool_next;
  int64_t Lcap, Ucap;
  unsigned long long* nnz_ctr;
  int32_t* status;
  double tau;
  int32_t diag_pref;
  int32_t refactor;
  // separators factored block by block: the pivotal set (kMaxPanelWords words) and the
  // current block's L structure (W x nb words), carried from launch to launch
  unsigned long long* pbits_g;
  unsigned long long* lb_g;
};

// dense separators: panel rows up to 64 * kMaxPanelWords (one LDS row bitmask), an LDS
// block of kSepDenseLds bytes (set once per process with sepdense_setup)
constexpr int kMaxPanelWords = 176;
constexpr int kMaxNb = 32;          // dense block width
// Rows whose block-column L memberships are kept as one 32-bit mask each (the trailing
// update then visits only the block columns that update a row).
constexpr int kRowMaskRows = 4096;

// dense block width for panel height H: the LDS block holds nb columns of H doubles and
// two bitmasks of W words each, after the row masks (H words when H <= kRowMaskRows)
__host__ __device__ inline int block_width(int H, int W, int m, int lds_bytes) {
  if (H <= kRowMaskRows) lds_bytes -= 4 * H;
  int nb = lds_bytes / (8 * H + 16 * W);
  if (nb > kMaxNb) nb = kMaxNb;
  if (nb > m) nb = m;
  return nb < 1 ? 1 : nb;
}

// a separator of at least this many blocks is factored block by block in separate
// launches, its trailing updates spread over many workgroups
constexpr int kSplitBlocks = 3;
__host__ __device__ inline bool sep_split(int m, int nb) { return (m + nb - 1) / nb >= kSplitBlocks; }
constexpr int kSepDenseLds = 128 * 1024;
hipError_t sepdense_setup();
hipError_t launch_sepdense(const DenseSepArgs& a, int nsep, hipStream_t s);
// one separator (sep_split) block by block; ncu = workgroups for the spread launches
hipError_t launch_sepdense_split(const DenseSepArgs& a, int d, int H, int m, int ncu, hipStream_t s);
hipError_t launch_factor_init(const FactorArgs& a, int32_t nlevels, hipStream_t s);
hipError_t launch_factor_level(const FactorArgs& a, int grid, hipStream_t s);
// first level on workgroups of `waves` wavefronts (4, 6, 7 or 8); grid workgroups
hipError_t launch_factor_coop(const FactorArgs& a, int waves, int grid, hipStream_t s);
// the speculation check after the first level: a row of L(:,k) pivoted by an earlier
// column marks k's item for the redo pass
hipError_t launch_factor_spec_check(const FactorArgs& a, int ncols_level0, const int32_t* cols, hipStream_t s);
int coop_lds_bytes(int waves);
// small: the kLdsSlotsStep1Small variant (two waves a CU), for plans whose column
// workspaces are bounded by 3/4 of its table
hipError_t launch_factor_sep_step1(const FactorArgs& a, int grid, bool small, hipStream_t s);
hipError_t launch_factor_sep_step2(const FactorArgs& a, int grid, hipStream_t s);
hipError_t launch_scatter(const double* vals, const int32_t* map, double* out, int64_t cnt, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t cnt, hipStream_t s);
size_t solve_lds_bytes(int32_t rows);   // LDS a task of `rows` rows needs
hipError_t solve_lds_setup(size_t max_bytes);
hipError_t launch_solve_tasks(const SolveArgs& a, int ntasks, hipStream_t s);
hipError_t launch_solve_flow(const SolveArgs& a, int grid, hipStream_t s);
// LDS the one-launch solve kernel declares itself; its dynamic LDS is the rest
constexpr int kSolveFlowStaticLds = 256;
// Z (cnt doubles) set to the pending pattern the solve's tasks wait on; before every solve
hipError_t launch_solve_pending(double* Z, int64_t cnt, hipStream_t s);
hipError_t launch_solve_finish(const SolveArgs& a, hipStream_t s);
// the static device scratch of the solve that allocates nothing: its size in doubles,
// and its address on a device (looked up once per device; the device must be current)
constexpr int64_t kNoAllocScratchDoubles = 4ll << 20;
hipError_t noalloc_scratch(int device, double** ptr);

}  // namespace basker
