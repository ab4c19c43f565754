// Dense factorization of nested-dissection separators (Alg. 4, the separator's own
// part after the descendant contributions have been applied, Sec. III-C).
//
// Once the descendant pivots of every column of a separator s have been applied (the
// first step of a separator level), what remains is the block formed by s's own rows and
// the rows of its ancestor separators: the only rows these columns can reach.  In
// circuits with long-range branches this block is close to dense, and the
// left-looking sweep turns into |s|^2/2 dependent steps.  Here one workgroup factors it
// right-looking on a dense panel (column-major, rows = s's rows then each ancestor's
// rows): for k = 0..|s|-1 it picks the pivot of column k, forms L(:,k), and applies the
// rank-1 update to every later column whose pivot-row entry is structurally nonzero.
//
// Same result as the column sweep, bit for bit: each entry receives its updates in
// ascending pivot order with separately rounded multiply and subtract; structurally
// zero entries are exactly zero and never win the pivot search (unless the whole
// candidate set is zero, which is singular either way).  The structure is carried as a
// bitmask per column (fill merges the pivot column's rows into every column it
// updates), so the stored L and U patterns are exactly the sparse ones.
#include "device.hpp"

namespace basker {

namespace {

constexpr int kDT = 1024;          // threads per workgroup
constexpr int kMaxRowWords = 256;  // panel rows up to 16,384
constexpr int kMaxPivl = 4096;     // local pivots kept in LDS for separators up to this size

__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rl_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int local_row(const DenseSepArgs& a, int d, int32_t r) {
  for (int t = a.rng_ptr[d]; t < a.rng_ptr[d + 1]; t++) {
    const int32_t g0 = a.rng_g0[t];
    if (r >= g0 && r < g0 + a.rng_len[t]) return a.rng_loc[t] + (r - g0);
  }
  return -1;
}

__device__ __forceinline__ int32_t global_row(const DenseSepArgs& a, int d, int loc) {
  for (int t = a.rng_ptr[d]; t < a.rng_ptr[d + 1]; t++) {
    const int l0 = a.rng_loc[t];
    if (loc >= l0 && loc < l0 + a.rng_len[t]) return a.rng_g0[t] + (loc - l0);
  }
  return -1;
}

__global__ void __launch_bounds__(kDT) sepdense_kernel(DenseSepArgs a) {
  __shared__ unsigned long long piv_bits[kMaxRowWords];   // rows already pivotal
  __shared__ unsigned long long lbits[kMaxRowWords];      // rows of L(:,k)
  __shared__ unsigned long long sk_s[kMaxRowWords];       // structure of column k
  __shared__ int pivl_s[kMaxPivl];                        // local pivot rows (m <= kMaxPivl)
  __shared__ double red_v[kDT / 64];
  __shared__ int red_i[kDT / 64];
  __shared__ int sh_p, sh_fail, sh_hasdiag;
  __shared__ double sh_xp, sh_xd, sh_m;
  __shared__ int sh_ub, sh_lb, sh_nu, sh_nl;
  __shared__ int sh_cnt[kDT / 64];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int nw = kDT / 64;
  const int d = a.d_begin + blockIdx.x;
  const int sg = a.dsep_seg[d];
  const int c0 = a.seg_c0[sg];
  const int m = a.seg_c1[sg] - c0;
  const int H = a.dsep_H[d];
  const int W = (H + 63) / 64;
  double* P = a.panel + a.poff[d];
  unsigned long long* S = a.bits + a.soff[d];
  int32_t* pivl = a.piv_local + c0;   // local pivot row of each separator column

  // zero the panel and the structure, clear the pivotal set
  for (int64_t i = tid; i < (int64_t)H * m; i += kDT) P[i] = 0.0;
  for (int64_t i = tid; i < (int64_t)W * m; i += kDT) S[i] = 0ull;
  for (int i = tid; i < kMaxRowWords; i += kDT) piv_bits[i] = 0ull;
  if (tid == 0) sh_fail = 0;
  __syncthreads();
  // the partial columns from the first step: non-pivotal rows with their values
  for (int k = wv; k < m; k += nw) {
    const int c = c0 + k;
    const int off = a.cb_off[c] + a.cb_np[c], nn = a.cb_nn[c];
    for (int t = lane; t < nn; t += 64) {
      const int loc = local_row(a, d, a.cbI[off + t]);
      if (loc < 0) { sh_fail = 1; continue; }
      P[loc + (int64_t)k * H] = a.cbX[off + t];
      atomicOr(&S[(int64_t)k * W + (loc >> 6)], 1ull << (loc & 63));
    }
  }
  __syncthreads();
  if (sh_fail) {
    if (tid == 0) { atomicMax(&a.status[ST_CODE], DEV_PATTERN); atomicMin(&a.status[ST_FAILCOL], c0); }
    return;
  }

  long long lnz = 0, unz = 0;
  int offdiag = 0;
  for (int k = 0; k < m; k++) {
    const int c = c0 + k;
    const double* Pk = P + (int64_t)k * H;
    const unsigned long long* Sk = S + (int64_t)k * W;
    // ---- pivot search over the separator's non-pivotal rows
    double best = -1.0;
    int bidx = 0x7fffffff;
    for (int i = tid; i < m; i += kDT) {
      if ((piv_bits[i >> 6] >> (i & 63)) & 1ull) continue;
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
    __syncthreads();
    if (tid == 0) {
      double bm = -1.0;
      int bi = 0x7fffffff;
      for (int t = 0; t < nw; t++)
        if (red_v[t] > bm || (red_v[t] == bm && red_i[t] < bi)) { bm = red_v[t]; bi = red_i[t]; }
      // candidates are the structural, non-pivotal rows of the separator; a structurally
      // zero row holds an exact 0 in the panel, so it can only attain the maximum when the
      // column is singular, but the diagonal test must see its structure explicitly
      const bool dcand = !((piv_bits[k >> 6] >> (k & 63)) & 1ull) && ((Sk[k >> 6] >> (k & 63)) & 1ull);
      int p;
      int fail = 0;
      if (!a.refactor) {
        if (!(bm > 0.0)) fail = DEV_SINGULAR;
        p = (a.diag_pref && dcand && fabs(Pk[k]) >= a.tau * bm) ? k : bi;
      } else {
        p = a.piv[c] - c0;
        const bool okp = p >= 0 && p < m && !((piv_bits[p >> 6] >> (p & 63)) & 1ull) &&
                         ((Sk[p >> 6] >> (p & 63)) & 1ull);
        if (!(okp && (bm > 0.0) && Pk[p] != 0.0 && fabs(Pk[p]) >= a.tau * bm)) fail = DEV_REFACTOR_FAIL;
      }
      if (fail) {
        sh_fail = fail;
        atomicMax(&a.status[ST_CODE], fail);
        atomicMin(&a.status[ST_FAILCOL], c);
      } else {
        sh_p = p;
        sh_xp = Pk[p];
        pivl[k] = p;
        if (m <= kMaxPivl) pivl_s[k] = p;
      }
    }
    __syncthreads();
    if (sh_fail) return;
    const int p = sh_p;
    const double xp = sh_xp;
    // ---- rows of L(:,k): structural, not pivotal, not the pivot
    for (int w = tid; w < W; w += kDT) {
      sk_s[w] = Sk[w];
      unsigned long long b = Sk[w] & ~piv_bits[w];
      if ((p >> 6) == w) b &= ~(1ull << (p & 63));
      lbits[w] = b;
    }
    __syncthreads();
    // ---- outputs of column k (wave 0): counts, pool space, U and L entries
    if (wv == 0) {
      const int dnp = a.cb_np[c];
      // s-internal U entries: earlier pivots j < k whose row is in the structure of k
      int nu = 0;
      for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        bool in = false;
        if (j < k) {
          const int pr = m <= kMaxPivl ? pivl_s[j] : pivl[j];
          in = (sk_s[pr >> 6] >> (pr & 63)) & 1ull;
        }
        nu += __popcll(__ballot(in));
      }
      int nl = 0;
      for (int w = 0; w < W; w++) nl += __popcll(lbits[w]);
      int ub = 0, lb = 0;
      if (lane == 0) {
        if (!a.refactor) {
          ub = (int)atomicAdd(&a.pool_next[1], (unsigned long long)(dnp + nu + 1));
          lb = (int)atomicAdd(&a.pool_next[0], (unsigned long long)nl);
          if ((int64_t)ub + dnp + nu + 1 > a.Ucap || (int64_t)lb + nl > a.Lcap) {
            atomicMax(&a.status[ST_CODE], DEV_POOL);
            a.status[ST_POOL] = 1;
            sh_fail = DEV_POOL;
          }
        } else {
          ub = a.Ubeg[c];
          lb = a.Lbeg[c];
          if (a.Ucnt[c] != dnp + nu + 1 || a.Lcnt[c] != nl) {
            atomicMax(&a.status[ST_CODE], DEV_PATTERN);
            atomicMin(&a.status[ST_FAILCOL], c);
            sh_fail = DEV_PATTERN;
          }
        }
        sh_ub = ub;
        sh_lb = lb;
      }
      ub = __shfl(ub, 0, 64);
      lb = __shfl(lb, 0, 64);
      if (!__any(lane == 0 && sh_fail != 0)) {
        // U: descendant part from the first step, then s-internal ascending, then diagonal
        const int off = a.cb_off[c];
        for (int t = lane; t < dnp; t += 64) {
          a.Ui[ub + t] = a.cbI[off + t];
          a.Ux[ub + t] = a.cbX[off + t];
        }
        int pos = dnp;
        for (int j0 = 0; j0 < k; j0 += 64) {
          const int j = j0 + lane;
          bool in = false;
          int pr = 0;
          if (j < k) {
            pr = m <= kMaxPivl ? pivl_s[j] : pivl[j];
            in = (sk_s[pr >> 6] >> (pr & 63)) & 1ull;
          }
          const unsigned long long bm = __ballot(in);
          if (in) {
            const int q = pos + __popcll(bm & ((1ull << lane) - 1ull));
            a.Ui[ub + q] = c0 + j;
            a.Ux[ub + q] = Pk[pr];
          }
          pos += __popcll(bm);
        }
        if (lane == 0) {
          a.Ui[ub + pos] = c;
          a.Ux[ub + pos] = xp;
          a.Ubeg[c] = ub;
          a.Ucnt[c] = dnp + nu + 1;
          a.Lbeg[c] = lb;
          a.Lcnt[c] = nl;
          a.piv[c] = c0 + p;
          a.pinv[c0 + p] = c;
        }
        unz += dnp + nu + 1;
        lnz += nl;
        if (p != k) offdiag++;
      }
    }
    __syncthreads();
    if (sh_fail) return;
    // ---- L values (kept in the panel column for the update) and their storage
    {
      const int lb = sh_lb;
      // ascending local row order: prefix over words
      int base = 0;
      for (int w0 = 0; w0 < W; w0 += kDT) {
        const int w = w0 + tid;
        int cnt = (w < W) ? __popcll(lbits[w]) : 0;
        // block-wide exclusive scan of cnt over w (two levels: wave, then waves)
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int t = __shfl_up(incl, o, 64);
          if (lane >= o) incl += t;
        }
        if (lane == 63) sh_cnt[wv] = incl;
        __syncthreads();
        int wpre = 0;
        for (int t = 0; t < wv; t++) wpre += sh_cnt[t];
        int tot = 0;
        for (int t = 0; t < nw; t++) tot += sh_cnt[t];
        __syncthreads();
        if (w < W) {
          int q = base + wpre + incl - cnt;
          unsigned long long b = lbits[w];
          while (b) {
            const int bit = __builtin_ctzll(b);
            b &= b - 1;
            const int r = (w << 6) + bit;
            const double l = Pk[r] / xp;
            P[r + (int64_t)k * H] = l;
            if (!a.refactor) {
              a.Li[lb + q] = global_row(a, d, r);
              a.Lx[lb + q] = l;
            }
            q++;
          }
        }
        base += tot;
      }
      if (a.refactor) {
        // stored row order: look every stored row up in the panel
        __syncthreads();
        const int cnt = a.Lcnt[c];
        for (int t = tid; t < cnt; t += kDT) {
          const int loc = local_row(a, d, a.Li[lb + t]);
          if (loc >= 0) a.Lx[lb + t] = P[loc + (int64_t)k * H];
        }
      }
    }
    if (tid == 0) piv_bits[p >> 6] |= 1ull << (p & 63);
    __syncthreads();
    // ---- rank-1 update of every later column whose pivot-row entry is structural
    // (columns k and cc are distinct, so their panel columns do not overlap: the loads of
    // four words are issued together before the stores)
    const double* __restrict__ Lk = P + (int64_t)k * H;
    // this wave's later columns cc = k + 1 + wv + nw * t, 64 at a time: one lane per
    // column tests the pivot row's structure bit and loads the multiplier, then the
    // columns with the bit set are updated one after another by the whole wave
    for (int t0 = 0; k + 1 + wv + nw * t0 < m; t0 += 64) {
      const int ccl = k + 1 + wv + nw * (t0 + lane);
      bool on = false;
      double ul = 0.0;
      if (ccl < m) {
        on = (S[(int64_t)ccl * W + (p >> 6)] >> (p & 63)) & 1ull;
        if (on) ul = P[(int64_t)ccl * H + p];
      }
      unsigned long long act = __ballot(on);
      while (act) {
        const int j = __ffsll((long long)act) - 1;
        act &= act - 1;
        const int cc = rl(ccl, j);
        const double u = rl_d(ul, j);
        unsigned long long* __restrict__ Sc = S + (int64_t)cc * W;
        double* __restrict__ Pc = P + (int64_t)cc * H;
        for (int w = lane; w < W; w += 64) {
          const unsigned long long b = lbits[w];
          if (b) Sc[w] |= b;
        }
        for (int w0 = 0; w0 < W; w0 += 4) {
          double lv[4], cv[4];
          bool onw[4];
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const int w = w0 + t;
            onw[t] = w < W && ((lbits[w] >> lane) & 1ull);
            lv[t] = 0.0;
            cv[t] = 0.0;
            if (onw[t]) {
              lv[t] = Lk[(w << 6) + lane];
              cv[t] = Pc[(w << 6) + lane];
            }
          }
#pragma unroll
          for (int t = 0; t < 4; t++) {
            if (onw[t]) {
              const double prod = lv[t] * u;
              Pc[((w0 + t) << 6) + lane] = cv[t] - prod;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (wv == 0 && lane == 0) {
    atomicAdd(&a.status[ST_DSEP], 1);
    if (offdiag) atomicAdd(&a.status[ST_OFFDIAG], offdiag);
    if (!a.refactor) {
      atomicAdd(&a.nnz_ctr[0], (unsigned long long)lnz);
      atomicAdd(&a.nnz_ctr[1], (unsigned long long)unz);
    }
  }
}

}  // namespace

hipError_t launch_sepdense(const DenseSepArgs& a, int nsep, hipStream_t s) {
  if (nsep <= 0) return hipSuccess;
  hipLaunchKernelGGL(sepdense_kernel, dim3(nsep), dim3(kDT), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
