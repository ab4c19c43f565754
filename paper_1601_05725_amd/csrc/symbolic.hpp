// Host-side symbolic analysis: orderings and the static plan the GPU kernels run.
//
// Builds R = A(prow, qcol) in block upper triangular form (Sec. III-A: a bottleneck
// matching puts large entries on the diagonal, then strongly connected components
// give the diagonal blocks), orders every small block for fill (Alg. 2) and
// the large blocks by nested dissection with a fill order inside every node
// (Sec. III-C), and derives the candidate groups (pivots stay inside a BTF block or
// an ND node) and the column dependency forest the numeric kernels schedule on.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace basker {

struct SymbolicOptions {
  int matching = 1;        // bottleneck matching (else: structural matching only)
  int btf = 1;             // split into strongly connected components
  int fill_order = 1;      // minimum-degree order inside blocks / ND nodes
  int nd_leaves = 16;      // leaves of the ND tree (power of two)
  int nd_min_block = 10000;// blocks at least this large are ordered by ND
};

struct NdNode {            // one node of the ND tree of a large block (postorder)
  int g0, g1;              // columns (= rows) in R
  int parent;              // index into nodes, -1 at the root
  int level;               // 0 at leaves
  bool leaf;
};

struct Plan {
  int n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> prow, qcol, pinvrow;   // R(i,k) = A(prow[i], qcol[k]); pinvrow = inverse of prow
  std::vector<int32_t> blkptr;                // BTF blocks
  std::vector<int32_t> grpptr;                // candidate groups (contiguous, nested in blocks)
  std::vector<int32_t> col_grp;               // group of each column
  std::vector<int32_t> grp_parent;            // ND tree over groups (-1: root or not ND)
  // diagonal-block part of R (factored), rows ascending; map = position in A's value array
  std::vector<int32_t> Rp, Ri, Rmap;
  // strictly upper off-diagonal-block part of R (solve only)
  std::vector<int32_t> Op, Oi, Omap;
  // column dependency forest: parent[k] > k or -1, nchild[k]; initial ready columns by priority
  std::vector<int32_t> parent, nchild, ready;
  std::vector<int32_t> depth;
  std::vector<NdNode> nd_nodes;
  // segments: contiguous column ranges factored by one wavefront each, column by
  // column.  A non-ND block is one segment at level 0; an ND node is one segment at
  // its tree level (leaves 0).  Levels run one after another (Alg. 4's level sets);
  // segments of one level are independent.
  std::vector<int32_t> seg_c0, seg_c1, seg_level;
  std::vector<int32_t> lvl_ptr, lvl_seg;      // segments of level l: lvl_seg[lvl_ptr[l] .. lvl_ptr[l+1])
  // work items: consecutive segments of one level with at least kItemCols columns in
  // total (a large segment is an item by itself); items of level l are
  // [lvl_item_ptr[l], lvl_item_ptr[l+1]), item i covers lvl_seg[item_lo[i] .. item_hi[i])
  std::vector<int32_t> item_lo, item_hi, lvl_item_ptr;
  // columns of every level (for the column-parallel first step of separator levels);
  // in a level the columns of dense separators come first (lvl_dcol_cnt of them)
  std::vector<int32_t> lvl_col, lvl_col_ptr, lvl_dcol_cnt;
  // dense separators: ND separators of at least kDenseSepMin columns are factored
  // right-looking on a dense panel whose rows are the separator's own rows followed by
  // the rows of its ancestor separators (the only rows its columns can reach)
  std::vector<int32_t> dsep_seg, dsep_H, dsep_rng_ptr, dsep_rng_g0, dsep_rng_len, dsep_rng_loc, lvl_dsep_ptr;
  std::vector<int64_t> dsep_poff, dsep_soff;
  int64_t dsep_panel_total = 0, dsep_bits_total = 0;
  std::vector<int32_t> seg_grp;               // group of each segment (its first column's group)
  int64_t crit_cols = 0;                      // sum over levels of the largest segment
  // solve tasks in launch order: kind 0 = whole block (id = block), 1 = forward part of
  // an ND node, 2 = backward part of an ND node (id = group); tasks of level l are
  // [st_lvl_ptr[l], st_lvl_ptr[l+1]); st_need = doubles of work storage
  std::vector<int32_t> st_kind, st_id, st_need, st_lvl_ptr;
  // predecessors of every task in launch order (earlier positions, ascending):
  // st_dep[st_dep_ptr[q] .. st_dep_ptr[q + 1]); st_succ[q] = 1 when a later task waits
  // for q; st_issue: the order in which the one-launch solve takes the tasks (launch
  // positions, a topological order of the task graph with its couplings)
  std::vector<int32_t> st_dep_ptr, st_dep, st_succ, st_issue;
  // ND groups for the solve: first descendant group (postorder), ancestors root first
  // (sg_anc[sg_anc_ptr[g] .. sg_anc_ptr[g+1])), total rows of the strict ancestors
  // (sg_choff: also the offset of the group's rows in any descendant's buffer), and
  // the offset of the group's [own rows | ancestor-row buffer] area (sg_tbase)
  std::vector<int32_t> sg_fd, sg_anc_ptr, sg_anc, sg_choff;
  std::vector<int64_t> sg_tbase;
  std::vector<int32_t> s_rowpos;   // R row of an ND block -> sg_choff[its group] + offset in the group
  int64_t s_gbuf_total = 0;
  // Level-0 cooperative schedule.  The first level's segments (BTF blocks and ND
  // leaves) are cut into items for workgroups of several wavefronts (consecutive
  // segments of lvl_seg's level-0 range, largest first, at least co_min_cols columns
  // unless a segment is larger); inside an item the waves take columns in order and a
  // column waits for its dependency list.  Two lists per level-0 column, inside its
  // segment and ascending: the predicted one, dep_* (the U pattern of a factorization
  // without row exchanges, or learned from an earlier factorization), and the safe
  // one, sdep_* (its children in the column elimination tree, which bounds the
  // dependencies of every pivot sequence).
  // Items hold one size bin each (co_item_kind): 0 = segments above the bin edge, whose
  // columns the waves share as above; 1 = segments of at most co_bin_edge columns, one
  // wavefront factoring a whole segment; 2 = 1 x 1 diagonal blocks, one thread each.
  std::vector<int32_t> co_item_lo, co_item_hi, co_item_cols, co_item_kind;
  int32_t co_bin_edge = 0;
  std::vector<int32_t> col_item;              // level-0 column -> item (-1 elsewhere)
  std::vector<int32_t> dep_ptr, dep_idx, sdep_ptr, sdep_idx;
  int32_t co_max_item_cols = 0;
  // issue order of the speculative pass: per item (from co_item_off), (column, slot,
  // first column of its segment) triples, longest remaining dependency path first in
  // the predicted dependency graph (a topological order that keeps the critical path
  // busy while the other waves take independent columns)
  std::vector<int32_t> co_item_off, co_issue;
  bool co_valid = false;                      // set by the library after checking the lists
  // Solve issue orders: the rows of every solve task (a block without ND, or an ND
  // node) in the order its wavefronts take them, rows of one level of the task's
  // dependency graph together -- the L sweep by levels of the predicted L pattern, the U
  // sweep by levels of the predicted U pattern (the dependency lists) -- or plain
  // order (ascending for L, descending for U) where no prediction exists.  row_task0 is
  // the first row of the task holding each row; *_pos the rank of a row in its task's
  // order.  The device checks the orders against the actual patterns after every
  // factorization.
  std::vector<int32_t> sfo, sbo, sfo_pos, sbo_pos, row_task0;
  // fill of a factorization without row exchanges, from the host symbolic pass (sizes
  // the L/U pools and the separator buffer); sym_ok false when the pass was cut short
  bool sym_ok = false;
  int64_t sym_lnz = 0, sym_unz = 0, sym_cb = 0;
  int64_t sym_ws_max = 0;   // largest reach (rows of one column's workspace), separator first steps included
  int struct_rank = 0;
  double bottleneck = 0.0;
  int max_depth = 0;
  int n_nd_blocks = 0;
  std::string error;
};

// Full pipeline from a CSC matrix (values used by the matching).  Returns 0, or a
// negative status (-1 invalid input, -2 structurally singular).
int build_plan(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax,
               const SymbolicOptions& opt, Plan& plan);

// Plan from a caller-supplied ordering: R = A(prow, qcol), BTF blocks blkptr[0..nblk],
// candidate groups grpptr[0..ngrp] nested in the blocks.  Lower off-diagonal blocks
// must be empty.  The schedule is the column elimination tree of each block, which
// is safe for any pivot sequence.
int build_plan_user(int n, const int32_t* Ap, const int32_t* Ai,
                    const int32_t* prow, const int32_t* qcol,
                    int nblk, const int32_t* blkptr, int ngrp, const int32_t* grpptr,
                    Plan& plan);

// Level-0 items and dependency lists, and the fill of a factorization without row
// exchanges (within a budget of visited pattern entries).
void build_level0_schedule(Plan& P, int co_min_cols, int64_t visit_budget, int bin_edge);

// The first level's work items (bins and grouping) alone, for a new bin edge or item
// size: the dependency lists are kept; build_issue_order must follow.
void build_level0_items(Plan& P, int co_min_cols, int bin_edge);

// columns of a work item of 1 x 1 blocks (one thread each)
constexpr int kBin1ItemCols = 2048;

// Issue order of every item from the predicted lists (after they change).
void build_issue_order(Plan& P);

// Solve issue orders: forward from the predicted L rows `lrows` of the first-level
// columns (null: keep the current forward orders, or plain ones on the first call),
// backward from the dependency lists (or plain when `backward` is false).
void build_solve_orders(Plan& P, const std::vector<std::vector<int32_t>>* lrows, bool backward);

// Merge the dependencies observed in a factorization (U pattern of every level-0 column
// of the given items) into the predicted lists: returns entries added.
int64_t merge_learned_deps(Plan& P, const std::vector<int32_t>& items, const std::vector<int32_t>& Ubeg,
                           const std::vector<int32_t>& Ucnt, const std::vector<int32_t>& Ui);

// exposed for tests of the orderings
int max_matching(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax, double thresh,
                 std::vector<int32_t>& match_row_of_col);
int bottleneck_matching(int n, const int32_t* Ap, const int32_t* Ai, const double* Ax,
                        std::vector<int32_t>& match_row_of_col, double* bottleneck);
int scc_order(int n, const int32_t* Ap, const int32_t* Ai, const int32_t* row_of_col,
              std::vector<int32_t>& perm, std::vector<int32_t>& blkptr);
std::vector<int32_t> min_degree_order(int n, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj);

}  // namespace basker
