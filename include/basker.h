/*
 * basker_mi355x -- threshold-pivoting sparse LU for gfx950 (MI355X), C ABI.
 *
 * The numeric method is the left-looking Gilbert-Peierls factorization (Alg. 1 of
 * Booth, Rajamanickam, Thornquist, "Basker", arXiv:1601.05725): for each column a
 * reach on the graph of L, a sparse triangular update, a pivot choice and a copy
 * into L and U.  It runs over the diagonal blocks of the block triangular form
 * (Sec. III-A/B) and over the nested-dissection nodes of large blocks (Sec. III-C),
 * with pivots confined to the column's own block or ND node.
 *
 * Conventions for every call:
 *   - Matrices are square, order n, compressed sparse column (CSC): colptr[n+1]
 *     (colptr[0] = 0), rowind[nnz] strictly increasing inside each column,
 *     values[nnz] in FP64.  Indices are 0-based int32; nnz < 2^31.
 *   - The permuted matrix is R = A(prow, qcol): R(i,k) = A(prow[i], qcol[k]).  It is
 *     block upper triangular with blocks blkptr[0..nblocks]; candidate groups
 *     grpptr[0..ngroups] refine the blocks.  The factorization computes, for every
 *     diagonal block B, B(piv, :) = L U with L unit lower triangular and pivots of
 *     column k taken from the rows of k's group.  Off-diagonal blocks are not
 *     factored; the solve uses them as they are.
 *   - Pivot rule (tau = pivot_tol): with m the largest candidate magnitude of the
 *     updated column k, take row k if diag_pref is set, row k is a candidate and
 *     |x_k| >= tau*m; else the smallest candidate row index attaining m.
 *   - All pointers are host pointers unless an argument says otherwise.  The caller
 *     owns every array it passes; the library copies what it keeps.  The handle owns
 *     its device memory until basker_free.  A handle is not re-entrant; distinct
 *     handles are independent and may be used from different host threads.
 *   - Errors are returned as basker_status codes; nothing is thrown across the ABI.
 *     basker_info reports the failing column, and basker_last_error a message.
 */
#ifndef BASKER_MI355X_H
#define BASKER_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct basker_ctx* basker_handle;

typedef enum {
  BASKER_OK = 0,
  BASKER_REFACTOR_FELL_BACK = 1,   /* refactor failed its threshold check; a full factor ran instead */
  BASKER_ERR_INVALID = -1,         /* malformed CSC, bad ordering, bad argument, not block triangular */
  BASKER_ERR_STRUCT_SINGULAR = -2, /* no perfect matching (structural rank < n) */
  BASKER_ERR_NUM_SINGULAR = -3,    /* a column with no nonzero candidate */
  BASKER_ERR_OOM = -4,             /* device or host allocation failed */
  BASKER_ERR_PATTERN = -5,         /* refactor/solve called before a successful factor */
  BASKER_ERR_DEVICE = -6,          /* HIP runtime error */
  BASKER_ERR_WORKSPACE = -7        /* a column's pattern exceeds the per-wave workspace */
} basker_status;

typedef struct {
  double pivot_tol;        /* tau in (0, 1]; default 0.001 */
  int32_t diag_pref;       /* prefer the matched diagonal row (default 1) */
  int32_t matching;        /* bottleneck matching before BTF (default 1) */
  int32_t btf;             /* split into strongly connected components (default 1) */
  int32_t fill_order;      /* minimum-degree order inside blocks (default 1) */
  int32_t nd_leaves;       /* leaves of the ND tree of large blocks, power of two (default 16) */
  int32_t nd_min_block;    /* blocks of at least this order use ND (default 10000) */
  double capacity_factor;  /* initial L/U pools: 0 (default) = twice the fill of a factorization
                              without row exchanges, counted by the symbolic analysis (6 * nnz of
                              the diagonal blocks if that count exceeds its work budget);
                              > 0 = this factor * nnz(diagonal blocks).  Pools grow on overflow */
  int32_t device;          /* HIP device ordinal (default 0); -1 = symbolic analysis only, no device work */
  void* stream;            /* hipStream_t to enqueue on; NULL = the handle's own stream */
  int32_t refactor_graph;  /* 1 (default): basker_refactor replays a HIP graph of its launches,
                              captured on the first call and dropped by every full factorization;
                              0: launch eagerly */
  int32_t max_grid;        /* cap on the workgroups of the factor launches (0 = the device's
                              occupancy target); results do not depend on it */
  int64_t hbm_budget;      /* bytes of device memory the handle may hold (0 = unlimited): an
                              allocation beyond it fails the call with BASKER_ERR_OOM */
  int32_t sched_flags;     /* bit 0: hand out the work items of every level in reverse order;
                              bit 1: no speculative schedule of the first level (every
                              column waits for its column-elimination-tree children);
                              bit 2: solve with one launch per level of the task graph
                              instead of one launch for all tasks;
                              bit 3: the separator first step on its 4,096-slot LDS table
                              even where the 2,048-slot one (two waves a CU) would do;
                              bit 4 (a check of the failure path): the one-launch solve
                              starts with its abort bit set, so each wait that has to
                              wait gives up at once and the solve reports
                              BASKER_ERR_DEVICE; the kernels still end normally;
                              bits 0-3 change no result (checks of determinism) */
  int32_t item_cols;       /* first-level work items hold at least this many columns unless a
                              block or ND leaf is larger (0 = 256) */
  int32_t coop_waves;      /* wavefronts per workgroup of the first level: 4, 6, 7 or 8 (0 = 6);
                              4 to 7 waves have 512-slot LDS tables, 8 waves 256-slot ones */
  int32_t bin_edge;        /* size bins of the first level (Sec. III-B's fine BTF blocks): 1 x 1
                              blocks take one thread each, segments of 2..bin_edge columns one
                              wavefront each, larger ones share a workgroup's wavefronts
                              (0 = 32; -1 = no wavefront bin) */
  int32_t autotune;        /* 1: the first factorizations try the bin edges and wavefront counts
                              and keep the fastest (basker_info reports the choice); results do
                              not depend on it (default 0) */
} basker_options;

typedef struct {
  int32_t n;
  int64_t nnz;               /* nnz(A) */
  int64_t nnz_diag;          /* entries inside the diagonal blocks of R */
  int64_t nnz_offdiag;       /* entries in off-diagonal blocks */
  int32_t nblocks;
  int32_t ngroups;
  int32_t struct_rank;
  int32_t max_depth;         /* height of the column dependency forest */
  int64_t lnz;               /* nnz(L) without the unit diagonal */
  int64_t unz;               /* nnz(U) with the diagonal */
  int32_t fail_col;          /* column of the last numerical failure, -1 if none */
  int32_t offdiag_pivots;    /* pivots that left the matched diagonal */
  double bottleneck;         /* min |diagonal| after the matching */
  double factor_kernel_ms;   /* device time of the last factor/refactor kernel (HIP events) */
  double solve_kernel_ms;    /* device time of the last solve kernel */
  double scatter_kernel_ms;  /* device time of the last value scatter */
  int32_t factor_calls;
  int32_t refactor_calls;
  int32_t refactor_fallbacks;
  int32_t pool_regrows;
  int32_t nd_blocks;
  int32_t nlevels;           /* factor level sets (ND tree height + 1, or 1 without ND) */
  int32_t solve_levels;      /* level sets of the block back-substitution */
  int64_t crit_cols;         /* columns on the factor's critical path: sum over levels of the largest segment */
  int64_t device_bytes;      /* device memory the handle holds now */
  int32_t dense_seps;        /* ND separators the last factorization ran on the dense kernel */
  int32_t sparse_seps;       /* ND separators of the plan factored column by column */
  int64_t device_bytes_plan; /* device memory the handle is expected to hold after its first
                                factorization and a solve with 8 right-hand sides (set by the
                                symbolic analysis, also for device = -1; pool growth on an
                                underestimated fill adds to it) */
  int32_t coop_items;        /* work items of the first level (cooperative workgroups; 0 = not used) */
  int32_t coop_waves;        /* wavefronts per first-level workgroup */
  int32_t redo_items;        /* first-level items the last factorization redid after a failed speculation */
  int32_t learn_events;      /* factorizations whose observed dependencies were merged into the schedule */
  int32_t solve_order_fallbacks; /* solve sweeps of first-level tasks (forward or backward) that the
                                    check after the last factorization sent back to plain row order */
  double rows_kernel_ms;     /* device time of the row-wise copies of L and U built after the last
                                successful factor/refactor (used by the solve) */
  int64_t sym_lnz;           /* nnz(L) and nnz(U) of a factorization without row exchanges, from the
                                symbolic analysis (0 when its budget ran out) */
  int64_t sym_unz;
  int32_t fill_bound;        /* 1 when the symbolic analysis finished within its budget, so the two
                                counts above and sym_ws_rows hold; 0 when the budget ran out */
  int32_t sym_ws_rows;       /* largest column workspace (rows of one column's reach, a separator's
                                first step included) without row exchanges */
  int32_t sched_bin_edge;    /* bin edge of the first level's schedule in use (see bin_edge) */
  int32_t autotune_trials;   /* schedule candidates the autotuner has timed (its choice is in
                                sched_bin_edge and coop_waves once all are done) */
} basker_info_t;

/* Fill *o with the defaults listed above. */
basker_status basker_default_options(basker_options* o);

/* Every call that takes options rejects pivot_tol outside (0, 1], nd_leaves < 1 or
 * not a power of two, and a negative hbm_budget or max_grid, with BASKER_ERR_INVALID. */

/* Symbolic analysis of A (Sec. III-A bottleneck matching and strongly connected
 * components for the BTF, Alg. 2 fill order per block, Sec. III-C nested dissection
 * of large blocks).  values are read only by the matching.  Copies the pattern and
 * uploads the plan to the device.  On success *out owns a new handle. */
basker_status basker_symbolic(int32_t n, const int32_t* colptr, const int32_t* rowind, const double* values,
                              const basker_options* o, basker_handle* out);

/* Symbolic analysis with a caller-supplied ordering: R = A(prow, qcol), BTF blocks
 * blkptr[0..nblocks] and candidate groups grpptr[0..ngroups] (both start at 0, end
 * at n, strictly increasing; every group inside one block).  Entries of R below the
 * diagonal blocks make this return BASKER_ERR_INVALID. */
basker_status basker_symbolic_ordered(int32_t n, const int32_t* colptr, const int32_t* rowind,
                                      const int32_t* prow, const int32_t* qcol,
                                      int32_t nblocks, const int32_t* blkptr,
                                      int32_t ngroups, const int32_t* grpptr,
                                      const basker_options* o, basker_handle* out);

/* Numeric factorization (Alg. 1 per column over the BTF blocks, Sec. III-B, and the
 * ND nodes, Alg. 4) with the values of A in the symbolic call's CSC order.
 * values is a host pointer, or a device pointer when values_on_device != 0.
 * Returns after the factorization is complete.  Before any device work (also on an
 * analysis-only handle), a plan in which a column's reach without row exchanges exceeds
 * the per-wave workspace (basker_info sym_ws_rows above 8,192 rows, known when
 * fill_bound is 1) fails with BASKER_ERR_WORKSPACE. */
basker_status basker_factor(basker_handle h, const double* values, int32_t values_on_device);

/* Refactorization with new values and the pattern and pivots of the last successful
 * factorization (the symbolic reuse over a matrix sequence of Sec. V-F).  Each
 * column checks |u_kk| >= tau * (largest candidate magnitude) and u_kk != 0; on the
 * first failure the call runs basker_factor and returns BASKER_REFACTOR_FELL_BACK. */
basker_status basker_refactor(basker_handle h, const double* values, int32_t values_on_device);

/* Solve A X = B in place for nrhs right-hand sides, column-major with leading
 * dimension ldb >= n (block back-substitution over the BTF form, Sec. II).  B is a
 * host pointer, or a device pointer when B_on_device != 0.  Returns after the solve.
 * The solve is one launch over every CU of the device while no other handle of the
 * process is inside basker_factor, basker_refactor or a solve on that device, over
 * half of them otherwise; the result does not depend on it. */
basker_status basker_solve(basker_handle h, int32_t nrhs, double* B, int32_t ldb, int32_t B_on_device);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): basker_solve on a device-resident B
 * (column-major, leading dimension ldb >= n) that calls no allocating routine.  Its
 * work vectors live in a static device array of 4,194,304 doubles (32 MiB), which
 * every GPU the library runs on holds until the process ends; a solve needing more
 * than 2 n nrhs of them fails with BASKER_ERR_WORKSPACE before any device work.  Calls on one GPU share that array, so calls that overlap
 * on one GPU (different handles, streams or threads) race and must be serialised by
 * the caller.  Same kernels and results as basker_solve. */
basker_status basker_solve_noalloc(basker_handle h, int32_t nrhs, double* B, int32_t ldb);

/* Counters and timings of the handle. */
basker_status basker_info(basker_handle h, basker_info_t* info);

/* The ordering chosen by the symbolic analysis: prow[n], qcol[n], blkptr[nblocks+1],
 * grpptr[ngroups+1] and grpparent[ngroups], the nested-dissection tree over the
 * groups (Sec. III-C, Fig. 3: parent group of each ND node, -1 for roots and for
 * groups outside ND blocks).  Any pointer may be NULL to skip it. */
basker_status basker_get_ordering(basker_handle h, int32_t* prow, int32_t* qcol, int32_t* blkptr, int32_t* grpptr,
                                  int32_t* grpparent);

/* Copy the factors of the last factor/refactor to the host, in pivot order:
 * piv[n] (row of R chosen for each column), L strictly lower (unit diagonal implicit)
 * as Lp[n+1], Li[lnz], Lx[lnz], U with its diagonal last in every column as Up[n+1],
 * Ui[unz], Ux[unz]; rows ascending inside each column.  Sizes from basker_info.
 * Any pointer may be NULL. */
basker_status basker_extract(basker_handle h, int32_t* piv, int64_t* Lp, int32_t* Li, double* Lx,
                             int64_t* Up, int32_t* Ui, double* Ux);

/* Release the handle and its device memory.  NULL is ignored. */
void basker_free(basker_handle h);

/* Static text for a status code. */
const char* basker_status_string(basker_status s);

/* Message of the handle's last error ("" if none); valid until the next call on h. */
const char* basker_last_error(basker_handle h);

#ifdef __cplusplus
}
#endif

#endif /* BASKER_MI355X_H */
