// Dense factorization of nested-dissection separators (Alg. 4, the separator's own
// part after the descendant contributions have been applied, Sec. III-C).
//
// Once the descendant pivots of every column of a separator s have been applied (the
// first step of a separator level), what remains is the block formed by s's own rows and
// the rows of its ancestor separators: the only rows these columns can reach.  In
// circuits with long-range branches this block is close to dense, and the
// left-looking sweep turns into |s|^2/2 dependent steps.  Here one workgroup factors it
// right-looking on a dense panel (column-major in HBM, rows = s's rows then each
// ancestor's rows), nb columns at a time:
//
//   block     nb columns are loaded into LDS and factored column by column: the pivot
//             of column k among s's non-pivotal structural rows, L(:,k) = x / x_p on the
//             column's structure, and the rank-1 update of the block's later columns
//             whose pivot-row entry is structural;
//   output    the block's U and L columns are written to the pools, one wave a column;
//   trailing  every later column c is brought up to date with the block: its entries
//             in the block's pivot rows follow the block's small triangular recurrence
//             (entry p_t of column c is u_t once the earlier block columns have updated
//             it, and it is structural if it was or if fill from an earlier block column
//             reached it), after which every row of c is updated independently,
//             a_ic = a_ic - l_it * u_t for t ascending.
//
// Same result as the column sweep, bit for bit: each entry receives its updates in
// ascending pivot order with separately rounded multiply and subtract, and an update
// is applied exactly where the sparse path applies it (row in L(:,k)'s structure,
// pivot-row entry structural), so structurally zero entries stay exactly zero.  The
// structure is carried as a bitmask per column (fill merges the L rows of every column
// that updates it), so the stored L and U patterns are exactly the sparse ones.
#include "device.hpp"

#include <algorithm>

namespace basker {

namespace {

constexpr int kDT = 1024;             // threads per workgroup
constexpr int kNW = kDT / 64;
constexpr int kMaxPivl = 4096;        // local pivots kept in LDS for separators up to this size

__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rl_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The panel's rows are the row ranges of the separator and its ancestors (one range a
// group, at most kMaxRanges of them), kept in LDS: r_g0[t] first global row, r_loc[t]
// first panel row, r_len[t] rows.
constexpr int kMaxRanges = 32;

struct Ranges {
  int n;
  int g0[kMaxRanges];
  int loc[kMaxRanges];
  int len[kMaxRanges];
};

__device__ __forceinline__ int local_row(const Ranges& rg, int32_t r) {
  for (int t = 0; t < rg.n; t++)
    if (r >= rg.g0[t] && r < rg.g0[t] + rg.len[t]) return rg.loc[t] + (r - rg.g0[t]);
  return -1;
}

__device__ __forceinline__ int32_t global_row(const Ranges& rg, int loc) {
  for (int t = 0; t < rg.n; t++)
    if (loc >= rg.loc[t] && loc < rg.loc[t] + rg.len[t]) return rg.g0[t] + (loc - rg.loc[t]);
  return -1;
}

__device__ __forceinline__ bool bit(const unsigned long long* b, int i) { return (b[i >> 6] >> (i & 63)) & 1ull; }


// LDS the dense kernels declare besides the block area
struct SepShared {
  unsigned long long piv_bits[kMaxPanelWords]; // rows already pivotal
  int pivl_s[kMaxPivl];                        // local pivot rows (m <= kMaxPivl, whole-separator role)
  double ush[kNW][kMaxNb];                     // per wave: u_t of its trailing column
  double red_v[kNW];
  int red_i[kNW];
  int sh_fail;
  Ranges rg;
};

// Roles: 0 = a whole separator in one workgroup (separators of a few blocks); for the
// others (sep_split) the host runs 1 = zero the panel and scatter the partial columns
// (columns spread over the workgroups), then per block 2 = factor the block and write its
// columns (one workgroup), 3 = bring the later columns up to date with the block (the
// columns spread over the workgroups).  The arithmetic of every entry, and its order, is
// the same in every role.
template <int kRole>
__device__ __forceinline__ void sep_run(const DenseSepArgs& a, int d, int lds_bytes, int k0_arg, double* blk,
                                        SepShared& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int sg = a.dsep_seg[d];
  const int c0 = a.seg_c0[sg];
  const int m = a.seg_c1[sg] - c0;
  const int H = a.dsep_H[d];
  const int W = (H + 63) / 64;
  const int nb = block_width(H, W, m, lds_bytes);
  if (kRole == 0 && sep_split(m, nb)) return;
  if (kRole != 0 && __hip_atomic_load(&a.status[ST_CODE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != DEV_OK)
    return;   // the factorization has failed: nothing more to do (uniform)
  double* P = a.panel + a.poff[d];
  unsigned long long* S = a.bits + a.soff[d];
  int32_t* pivl = a.piv_local + c0;   // local pivot row of each separator column
  const bool pl_lds = kRole == 0 && m <= kMaxPivl;
  const bool use_rm = H <= kRowMaskRows;
  double* Pb = blk;                                                                       // H x nb
  unsigned long long* Sb = reinterpret_cast<unsigned long long*>(blk + (size_t)H * nb);   // W x nb structure
  unsigned long long* Lb = Sb + (size_t)W * nb;                                           // W x nb L structure
  unsigned* rmask = reinterpret_cast<unsigned*>(Lb + (size_t)W * nb);                     // H row masks
  unsigned long long* piv_bits = sh.piv_bits;
  int* pivl_s = sh.pivl_s;
  double (*ush)[kMaxNb] = sh.ush;
  double* red_v = sh.red_v;
  int* red_i = sh.red_i;
  int& sh_fail = sh.sh_fail;
  Ranges& rg = sh.rg;

  // ranges into LDS (the trailing role does not map rows)
  if (kRole != 3) {
    if (tid == 0) {
      sh_fail = 0;
      const int r0 = a.rng_ptr[d], nr = a.rng_ptr[d + 1] - r0;
      rg.n = nr;
      if (nr > kMaxRanges) sh_fail = 1;
      for (int t = 0; t < nr && t < kMaxRanges; t++) {
        rg.g0[t] = a.rng_g0[r0 + t];
        rg.loc[t] = a.rng_loc[r0 + t];
        rg.len[t] = a.rng_len[r0 + t];
      }
    }
    __syncthreads();
    if (sh_fail) {
      if (tid == 0) { atomicMax(&a.status[ST_CODE], DEV_PATTERN); atomicMin(&a.status[ST_FAILCOL], c0); }
      return;
    }
  }
  if (kRole == 0 || kRole == 1) {
    // zero the panel (role 0: all of it first; role 1: each column by the wave that
    // scatters into it, just before)
    if (kRole == 0) {
      for (int64_t i = tid; i < (int64_t)H * m; i += kDT) P[i] = 0.0;
      __syncthreads();
    }
    // the partial columns from the first step: non-pivotal rows with their values; the
    // structure words of a column are gathered in the wave's part of the (still unused)
    // block area with LDS atomics, then stored whole
    const int kfirst = (kRole == 0 ? 0 : (int)blockIdx.x * kNW) + wv;
    const int kstep = (kRole == 0 ? 1 : (int)gridDim.x) * kNW;
    for (int k = kfirst; k < m; k += kstep) {
      unsigned long long* sw = Sb + (size_t)wv * W;
      for (int w = lane; w < W; w += 64) sw[w] = 0ull;
      if (kRole == 1) {
        for (int i = lane; i < H; i += 64) P[i + (int64_t)k * H] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int c = c0 + k;
      const int off = a.cb_off[c] + a.cb_np[c], nn = a.cb_nn[c];
      for (int t = lane; t < nn; t += 64) {
        const int loc = local_row(rg, a.cbI[off + t]);
        if (loc < 0) { sh_fail = 1; continue; }
        P[loc + (int64_t)k * H] = a.cbX[off + t];
        atomicOr(&sw[loc >> 6], 1ull << (loc & 63));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int w = lane; w < W; w += 64) S[(int64_t)k * W + w] = sw[w];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (sh_fail) {
      if (tid == 0) { atomicMax(&a.status[ST_CODE], DEV_PATTERN); atomicMin(&a.status[ST_FAILCOL], c0); }
      return;
    }
    if (kRole == 1) {
      // the pivotal set the block role carries from block to block starts empty
      if (blockIdx.x == 0)
        for (int i = tid; i < kMaxPanelWords; i += kDT) a.pbits_g[i] = 0ull;
      return;
    }
  }
  if (kRole == 0)
    for (int i = tid; i < kMaxPanelWords; i += kDT) piv_bits[i] = 0ull;
  if (kRole == 2)
    for (int i = tid; i < kMaxPanelWords; i += kDT) piv_bits[i] = a.pbits_g[i];
  // trailing columns of this workgroup
  const int tfirst = (kRole == 3 ? (int)blockIdx.x * kNW : 0) + wv;
  const int tstep = (kRole == 3 ? (int)gridDim.x : 1) * kNW;
  __syncthreads();

  long long lnz = 0, unz = 0;
  int offdiag = 0;
  const int kb0 = kRole == 0 ? 0 : k0_arg;
  const int kb1 = kRole == 0 ? m : (k0_arg + 1 < m ? k0_arg + 1 : m);
  for (int k0 = kb0; k0 < kb1; k0 += nb) {
    const int nbk = (m - k0 < nb) ? m - k0 : nb;
    if (kRole != 3) {
      // ---- load the block (its columns have every update from earlier blocks)
      for (int64_t i = tid; i < (int64_t)H * nbk; i += kDT) Pb[i] = P[i + (int64_t)k0 * H];
      for (int i = tid; i < W * nbk; i += kDT) Sb[i] = S[i + (int64_t)k0 * W];
      __syncthreads();
    // ---- factor the block column by column
    const int nsw = m > 256 * (kNW - 1) ? kNW : (m + 255) / 256 > 0 ? (m + 255) / 256 : 1;   // searching waves
    for (int t = 0; t < nbk; t++) {
      const int k = k0 + t;
      const int c = c0 + k;
      double* Pk = Pb + (size_t)t * H;
      const unsigned long long* Sk = Sb + (size_t)t * W;
      // pivot search over the separator's non-pivotal rows (a structurally zero row
      // holds an exact 0 and attains the maximum only in a singular column), on one
      // wave per 256 rows: the largest magnitude, the smallest row among equals, is the
      // same however the rows are split, and fewer partial results are combined
      if (wv < nsw) {
        double best = -1.0;
        int bidx = 0x7fffffff;
        for (int i = wv * 64 + lane; i < m; i += nsw * 64) {
          if (bit(piv_bits, i)) continue;
          const double v = fabs(Pk[i]);
          if (v > best || (v == best && i < bidx)) { best = v; bidx = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bidx, o, 64);
          if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
        }
        if (lane == 0) { red_v[wv] = best; red_i[wv] = bidx; }
      }
      __syncthreads();
      // every thread combines the searching waves' results in the same order: the same
      // decision
      double bm = -1.0;
      int bi = 0x7fffffff;
      for (int u = 0; u < nsw; u++)
        if (red_v[u] > bm || (red_v[u] == bm && red_i[u] < bi)) { bm = red_v[u]; bi = red_i[u]; }
      const bool dcand = !bit(piv_bits, k) && bit(Sk, k);
      int p;
      int fail = 0;
      if (!a.refactor) {
        if (!(bm > 0.0)) fail = DEV_SINGULAR;
        p = (a.diag_pref && dcand && fabs(Pk[k]) >= a.tau * bm) ? k : bi;
      } else {
        p = a.piv[c] - c0;
        const bool okp = p >= 0 && p < m && !bit(piv_bits, p) && bit(Sk, p);
        if (!(okp && (bm > 0.0) && Pk[p] != 0.0 && fabs(Pk[p]) >= a.tau * bm)) fail = DEV_REFACTOR_FAIL;
      }
      if (fail) {
        if (tid == 0) { atomicMax(&a.status[ST_CODE], fail); atomicMin(&a.status[ST_FAILCOL], c); }
        return;   // every thread took the same decision
      }
      const double xp = Pk[p];
      // L structure: structural, not pivotal, not the pivot
      unsigned long long* Lk = Lb + (size_t)t * W;
      for (int w = tid; w < W; w += kDT) {
        unsigned long long b = Sk[w] & ~piv_bits[w];
        if ((p >> 6) == w) b &= ~(1ull << (p & 63));
        Lk[w] = b;
      }
      if (tid == 0) {
        pivl[k] = p;
        if (pl_lds) pivl_s[k] = p;
      }
      __syncthreads();
      // L(:,k) = x / x_p
      for (int i = tid; i < H; i += kDT)
        if (bit(Lk, i)) Pk[i] = Pk[i] / xp;
      if (tid == 0) piv_bits[p >> 6] |= 1ull << (p & 63);
      __syncthreads();
      // rank-1 update of the block's later columns whose pivot-row entry is structural.
      // Row p is not in L(:,k), so no thread changes the value or the structure bit of
      // row p that the others test here.
      for (int t2 = t + 1 + wv; t2 < nbk; t2 += kNW) {
        unsigned long long* S2 = Sb + (size_t)t2 * W;
        if (!bit(S2, p)) continue;   // wave-uniform
        double* Pc = Pb + (size_t)t2 * H;
        const double u = Pc[p];
        for (int w = lane; w < W; w += 64) S2[w] |= Lk[w];
        for (int i = lane; i < H; i += 64)
          if (bit(Lk, i)) {
            const double prod = Pk[i] * u;
            Pc[i] = Pc[i] - prod;
          }
      }
      __syncthreads();
    }
    // ---- outputs of the block's columns, one wave a column
    for (int t = wv; t < nbk; t += kNW) {
      const int k = k0 + t;
      const int c = c0 + k;
      const int p = pl_lds ? pivl_s[k] : pivl[k];
      const double* Pk = Pb + (size_t)t * H;
      const unsigned long long* Sk = Sb + (size_t)t * W;
      const unsigned long long* Lk = Lb + (size_t)t * W;
      const int dnp = a.cb_np[c];
      // s-internal U entries: earlier pivots j < k whose row is in the structure of k
      int nu = 0;
      for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        bool in = false;
        if (j < k) in = bit(Sk, pl_lds ? pivl_s[j] : pivl[j]);
        nu += __popcll(__ballot(in));
      }
      int nl = 0;
      for (int w = lane; w < W; w += 64) nl += __popcll(Lk[w]);
      for (int o = 32; o > 0; o >>= 1) nl += __shfl_xor(nl, o, 64);
      int ub = 0, lb = 0, bad = 0;
      if (lane == 0) {
        if (!a.refactor) {
          ub = (int)atomicAdd(&a.pool_next[1], (unsigned long long)(dnp + nu + 1));
          lb = (int)atomicAdd(&a.pool_next[0], (unsigned long long)nl);
          if ((int64_t)ub + dnp + nu + 1 > a.Ucap || (int64_t)lb + nl > a.Lcap) {
            atomicMax(&a.status[ST_CODE], DEV_POOL);
            a.status[ST_POOL] = 1;
            bad = 1;
          }
        } else {
          ub = a.Ubeg[c];
          lb = a.Lbeg[c];
          if (a.Ucnt[c] != dnp + nu + 1 || a.Lcnt[c] != nl) {
            atomicMax(&a.status[ST_CODE], DEV_PATTERN);
            atomicMin(&a.status[ST_FAILCOL], c);
            bad = 1;
          }
        }
      }
      ub = __shfl(ub, 0, 64);
      lb = __shfl(lb, 0, 64);
      if (__shfl(bad, 0, 64)) continue;
      // U: descendant part from the first step, then s-internal ascending, then diagonal
      // (the descendant part copied 256 entries at a time: four loads per lane in flight)
      const int off = a.cb_off[c];
      for (int u0 = 0; u0 < dnp; u0 += 256) {
        int32_t ci[4];
        double cx[4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const int u = u0 + 64 * g + lane;
          ci[g] = 0;
          cx[g] = 0.0;
          if (u < dnp) {
            if (!a.refactor) ci[g] = a.cbI[off + u];
            cx[g] = a.cbX[off + u];
          }
        }
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const int u = u0 + 64 * g + lane;
          if (u < dnp) {
            if (!a.refactor) a.Ui[ub + u] = ci[g];
            a.Ux[ub + u] = cx[g];
          }
        }
      }
      int pos = dnp;
      for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        bool in = false;
        int pr = 0;
        if (j < k) {
          pr = pl_lds ? pivl_s[j] : pivl[j];
          in = bit(Sk, pr);
        }
        const unsigned long long bm = __ballot(in);
        if (in) {
          const int q = pos + __popcll(bm & ((1ull << lane) - 1ull));
          if (!a.refactor) a.Ui[ub + q] = c0 + j;
          a.Ux[ub + q] = Pk[pr];
        }
        pos += __popcll(bm);
      }
      if (lane == 0) {
        a.Ux[ub + pos] = Pk[p];
        if (!a.refactor) {
          a.Ui[ub + pos] = c;
          a.Ubeg[c] = ub;
          a.Ucnt[c] = dnp + nu + 1;
          a.Lbeg[c] = lb;
          a.Lcnt[c] = nl;
          a.piv[c] = c0 + p;
        }
        a.pinv[c0 + p] = c;
      }
      if (!a.refactor) {
        // L: structure rows in ascending local order, 64 rows (one word) at a time
        int q = 0;
        for (int w = 0; w < W; w++) {
          const unsigned long long b = Lk[w];
          if (!b) continue;
          if ((b >> lane) & 1ull) {
            const int r = (w << 6) + lane;
            const int qq = q + __popcll(b & ((1ull << lane) - 1ull));
            a.Li[lb + qq] = global_row(rg, r);
            a.Lx[lb + qq] = Pk[r];
          }
          q += __popcll(b);
        }
        unz += dnp + nu + 1;
        lnz += nl;
      } else {
        // stored row order: look every stored row up in the block
        for (int u = lane; u < nl; u += 64) {
          const int loc = local_row(rg, a.Li[lb + u]);
          if (loc >= 0) a.Lx[lb + u] = Pk[loc];
        }
      }
      if (p != k) offdiag++;
    }
    } else {
      // the block as the block role left it: factored values and L structure
      for (int64_t i = tid; i < (int64_t)H * nbk; i += kDT) Pb[i] = P[i + (int64_t)k0 * H];
      for (int i = tid; i < W * nbk; i += kDT) Lb[i] = a.lb_g[i];
      __syncthreads();
    }
    if (kRole == 2) {
      // hand the block to the trailing role: its values, L structure and the pivotal set
      __syncthreads();
      for (int64_t i = tid; i < (int64_t)H * nbk; i += kDT) P[i + (int64_t)k0 * H] = Pb[i];
      for (int i = tid; i < W * nbk; i += kDT) a.lb_g[i] = Lb[i];
      for (int i = tid; i < kMaxPanelWords; i += kDT) a.pbits_g[i] = piv_bits[i];
    }
    if (kRole == 0 || kRole == 3) {
    // ---- bring every later column up to date with the block, one wave a column
    if (k0 + nbk < m) {
      if (use_rm) {
        // row i's mask: bit t set when row i is in L(:, k0 + t)
        for (int i = tid; i < H; i += kDT) {
          unsigned mk = 0u;
          for (int t = 0; t < nbk; t++) mk |= (unsigned)bit(Lb + (size_t)t * W, i) << t;
          rmask[i] = mk;
        }
        __syncthreads();
      }
      const int p_l = lane < nbk ? (pl_lds ? pivl_s[k0 + lane] : pivl[k0 + lane]) : 0;
      for (int cc = k0 + nbk + tfirst; cc < m; cc += tstep) {
        double* Pc = P + (int64_t)cc * H;
        unsigned long long* Scol = S + (int64_t)cc * W;
        // lane t < nbk: the column's entry in pivot row p_t and whether it is structural
        double ut = 0.0;
        bool st = false;
        if (lane < nbk) {
          ut = Pc[p_l];
          st = bit(Scol, p_l);
        }
        // the block's recurrence, t ascending: a structural u_t updates (and fills) the
        // pivot rows of the later block columns that are in L(:, k0 + t)
        for (int t = 0; t < nbk; t++) {
          if (!rl((int)st, t)) continue;
          const double u = rl_d(ut, t);
          if (lane > t && lane < nbk && bit(Lb + (size_t)t * W, p_l)) {
            const double prod = Pb[(size_t)t * H + p_l] * u;
            ut = ut - prod;
            st = true;
          }
        }
        const unsigned long long smask = __ballot(st) & ((nbk >= 64) ? ~0ull : ((1ull << nbk) - 1ull));
        if (lane < nbk) ush[wv][lane] = ut;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // every row: a_ic = a_ic - l_it * u_t for every structural u_t, t ascending
        if (smask) {
          for (int i = lane; i < H; i += 64) {
            unsigned eff;
            if (use_rm) {
              eff = rmask[i] & (unsigned)smask;
            } else {
              eff = 0u;
              for (int t = 0; t < nbk; t++)
                if (((smask >> t) & 1ull) && bit(Lb + (size_t)t * W, i)) eff |= 1u << t;
            }
            if (!eff) continue;
            double x = Pc[i];
            while (eff) {
              const int t = __builtin_ctz(eff);
              eff &= eff - 1u;
              const double prod = Pb[(size_t)t * H + i] * ush[wv][t];
              x = x - prod;
            }
            Pc[i] = x;
          }
        }
        // structure: the L rows of every block column with a structural u_t
        if (smask) for (int w = lane; w < W; w += 64) {
          unsigned long long b = Scol[w];
          for (int t = 0; t < nbk; t++)
            if ((smask >> t) & 1ull) b |= Lb[(size_t)t * W + w];
          Scol[w] = b;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    }
    __syncthreads();
  }
  if (kRole == 0 || (kRole == 2 && k0_arg + nb >= m))
    if (tid == 0) atomicAdd(&a.status[ST_DSEP], 1);
  if (kRole == 0 || kRole == 2) {
    if (lane == 0) {
      if (offdiag) atomicAdd(&a.status[ST_OFFDIAG], offdiag);
      if (!a.refactor && (lnz || unz)) {
        atomicAdd(&a.nnz_ctr[0], (unsigned long long)lnz);
        atomicAdd(&a.nnz_ctr[1], (unsigned long long)unz);
      }
    }
  }
}

__global__ void __launch_bounds__(kDT) sepdense_kernel(DenseSepArgs a, int lds_bytes) {
  BASKER_DYN_SHARED(double, blk);
  BASKER_SHARED(SepShared, sh);
  sep_run<0>(a, a.d_begin + (int)blockIdx.x, lds_bytes, 0, blk, sh);
}

__global__ void __launch_bounds__(kDT) sepdense_prep_kernel(DenseSepArgs a, int lds_bytes) {
  BASKER_DYN_SHARED(double, blk);
  BASKER_SHARED(SepShared, sh);
  sep_run<1>(a, a.d_begin, lds_bytes, 0, blk, sh);
}

__global__ void __launch_bounds__(kDT) sepdense_block_kernel(DenseSepArgs a, int lds_bytes, int k0) {
  BASKER_DYN_SHARED(double, blk);
  BASKER_SHARED(SepShared, sh);
  sep_run<2>(a, a.d_begin, lds_bytes, k0, blk, sh);
}

__global__ void __launch_bounds__(kDT) sepdense_trail_kernel(DenseSepArgs a, int lds_bytes, int k0) {
  BASKER_DYN_SHARED(double, blk);
  BASKER_SHARED(SepShared, sh);
  sep_run<3>(a, a.d_begin, lds_bytes, k0, blk, sh);
}

}  // namespace

hipError_t sepdense_setup() {
  const void* ks[4] = {reinterpret_cast<const void*>(&sepdense_kernel),
                       reinterpret_cast<const void*>(&sepdense_prep_kernel),
                       reinterpret_cast<const void*>(&sepdense_block_kernel),
                       reinterpret_cast<const void*>(&sepdense_trail_kernel)};
  for (const void* k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kSepDenseLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sepdense(const DenseSepArgs& a, int nsep, hipStream_t s) {
  if (nsep <= 0) return hipSuccess;
  hipLaunchKernelGGL(sepdense_kernel, dim3(nsep), dim3(kDT), kSepDenseLds, s, a, kSepDenseLds);
  return hipGetLastError();
}

hipError_t launch_sepdense_split(const DenseSepArgs& a0, int d, int H, int m, int ncu, hipStream_t s) {
  DenseSepArgs a = a0;
  a.d_begin = d;
  const int W = (H + 63) / 64;
  const int nb = block_width(H, W, m, kSepDenseLds);
  hipError_t e;
  const int gp = std::max(1, std::min((m + kNW - 1) / kNW, ncu));
  hipLaunchKernelGGL(sepdense_prep_kernel, dim3(gp), dim3(kDT), kSepDenseLds, s, a, kSepDenseLds);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k0 = 0; k0 < m; k0 += nb) {
    hipLaunchKernelGGL(sepdense_block_kernel, dim3(1), dim3(kDT), kSepDenseLds, s, a, kSepDenseLds, k0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int rest = m - k0 - nb;
    if (rest > 0) {
      const int gt = std::max(1, std::min((rest + kNW - 1) / kNW, ncu));
      hipLaunchKernelGGL(sepdense_trail_kernel, dim3(gt), dim3(kDT), kSepDenseLds, s, a, kSepDenseLds, k0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace basker
