// Solve on gfx950: block back-substitution over the block triangular form.
//
// R = A(prow, qcol) is block upper triangular, so block b needs the solution of every
// later block it couples to: r_b = c_b - sum_{c > b} R_bc z_c, then L w = r(piv) and
// U z_b = w.  The work is cut into tasks (one 64-lane workgroup each) that run in
// levels, one launch per level:
//   block task    : one block without an ND tree (residual, L sweep, U sweep);
//   forward task  : one ND node; its L columns reach its own rows and the rows of its
//                   ancestors, the latter collected in a per-node buffer that every
//                   ancestor adds to its own rows, descendants in a fixed order;
//   backward task : one ND node, root first; it subtracts the products of its rows of
//                   the ancestors' U columns (a contiguous range, U columns are sorted)
//                   with the ancestors' solution, then runs its own U sweep.
// A task keeps its work vectors in LDS when they fit and streams the L and U entries
// of 64 columns at a time into LDS with one wave-wide gather, so a column step costs
// LDS latency rather than a global-memory round trip.  Entries are applied column by
// column in a fixed order, so results do not depend on scheduling.
#include "device.hpp"

#include <map>
#include <mutex>

namespace basker {

// Work vectors of basker_solve_noalloc: W, Z and the ND node buffers of one solve.
// Every device the library runs on holds its own copy until the process ends.  Host
// code never uses this name as an address: noalloc_scratch looks the device address
// up once per device and every launch takes that pointer.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kStage = 512;   // staged entries per sub-batch

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// lanes exchange data through global memory between steps: drain every outstanding
// memory operation and keep the compiler from moving accesses across
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

// lanes exchange data through LDS: the LDS unit executes one wave's instructions in
// issue order, so only the compiler has to be kept from moving accesses across
__device__ __forceinline__ void lsync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <bool kLds>
__device__ __forceinline__ void step_sync() {
  if (kLds) lsync(); else wsync();
}

__device__ __forceinline__ int rl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double rl_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane) {
  int x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x - v;
}

// first position p in [lo, hi) with idx[p] >= key (idx ascending on [lo, hi))
__device__ __forceinline__ int lower_bound_g(const int32_t* idx, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (idx[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

struct Smem {
  double* sx;      // staged values
  int32_t* si;     // staged targets (index into the task's work vector)
  int32_t* pre;    // staged offsets of the sub-batch's columns (65)
  int32_t* sbeg;   // global start of the sub-batch's columns (64)
  double* work;    // work vectors when they fit
};

// One batch of up to 64 columns, column t of the batch in lane t: its entries are
// idx/val[beg .. beg+cnt), each applied as S[xf(idx)] -= val * mult(t), columns in
// lane order.  mult(t) also performs the column's own step (it is called for every
// column, also one without entries, when all_cols is set).
template <bool kLds, class Xf, class Mult>
__device__ __forceinline__ void run_batch(const Smem& sm, double* S, int lane, int nb, int beg, int cnt,
                                          const int32_t* idx, const double* val, bool all_cols, Xf xf,
                                          Mult mult) {
  const int off = wave_excl_scan(lane < nb ? cnt : 0, lane);
  int j0 = 0;
  while (j0 < nb) {
    const int off0 = rl(off, j0);
    const bool fit = lane >= j0 && lane < nb && off + cnt - off0 <= kStage;
    const int nfit = __popcll(__ballot(fit));
    if (nfit == 0) {
      // a column with more entries than the stage holds: straight from global memory
      const int c = rl(cnt, j0), b = rl(beg, j0);
      const double m = mult(j0);
      for (int e = lane; e < c; e += 64) {
        const int t = xf(idx[b + e]);
        const double x = val[b + e];
        if (t >= 0) S[t] = S[t] - x * m;
      }
      step_sync<kLds>();
      j0++;
      continue;
    }
    const int j1 = j0 + nfit;
    // stage the entries of columns [j0, j1)
    if (lane >= j0 && lane < j1) {
      sm.pre[lane - j0] = off - off0;
      sm.sbeg[lane - j0] = beg;
    }
    if (lane == j1 - 1) sm.pre[j1 - j0] = off + cnt - off0;
    lsync();
    const int total = rl(off, j1 - 1) + rl(cnt, j1 - 1) - off0;
    const int nc = j1 - j0;
    for (int base = 0; base < total; base += 64 * 8) {
      int gi[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int s = base + u * 64 + lane;
        gi[u] = -1;
        if (s < total) {
          int lo = 0, hi = nc;
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sm.pre[mid] <= s) lo = mid; else hi = mid;
          }
          gi[u] = sm.sbeg[lo] + (s - sm.pre[lo]);
        }
      }
      int32_t ri[8];
      double rx[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        ri[u] = 0;
        rx[u] = 0.0;
        if (gi[u] >= 0) { ri[u] = idx[gi[u]]; rx[u] = val[gi[u]]; }
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int s = base + u * 64 + lane;
        if (gi[u] >= 0) { sm.si[s] = xf(ri[u]); sm.sx[s] = rx[u]; }
      }
    }
    lsync();
    // apply, column by column
    for (int j = j0; j < j1; j++) {
      const int c = rl(cnt, j);
      if (c == 0 && !all_cols) continue;
      const int o = rl(off, j) - off0;
      const double m = mult(j);
      for (int e = lane; e < c; e += 64) {
        const int t = sm.si[o + e];
        const double x = sm.sx[o + e];
        if (t >= 0) S[t] = S[t] - x * m;
      }
      step_sync<kLds>();
    }
    j0 = j1;
  }
}

// residual of rows [r0, r0 + m): S[i] = B(prow[r0+i]) - sum_c R(r0+i, c) z_c
template <bool kLds>
__device__ void residual_rows(const SolveArgs& a, double* S, int r0, int m, const double* Bc, const double* Z,
                              int lane) {
  for (int i = lane; i < m; i += 64) {
    const int r = r0 + i;
    double v = Bc[a.prow[r]];
    for (int q = a.OTp[r]; q < a.OTp[r + 1]; q++) {
      const double prod = a.OTx[q] * Z[a.OTj[q]];
      v = v - prod;
    }
    S[i] = v;
  }
  step_sync<kLds>();
}

// L sweep over columns [c0, c1) (rows of the task start at c0); the pivot rows are
// own rows.  xf maps an L row to its slot in S.
template <bool kLds, class Xf>
__device__ void l_sweep(const SolveArgs& a, const Smem& sm, double* S, int c0, int c1, int lane, Xf xf) {
  for (int kb = c0; kb < c1; kb += 64) {
    const int nb = c1 - kb < 64 ? c1 - kb : 64;
    int beg = 0, cnt = 0, pv = 0;
    if (lane < nb) {
      const int k = kb + lane;
      beg = a.Lbeg[k];
      cnt = a.Lcnt[k];
      pv = a.piv[k] - c0;
    }
    run_batch<kLds>(sm, S, lane, nb, beg, cnt, a.Li, a.Lx, false, xf,
                    [&](int j) -> double { return S[rl(pv, j)]; });
  }
}

// U sweep over columns [c0, c1), last first; entries with rows below c0 belong to
// descendants and are skipped (search set) or absent (block task)
template <bool kLds>
__device__ void u_sweep(const SolveArgs& a, const Smem& sm, double* S, int c0, int c1, int lane, bool search) {
  for (int kb = c1; kb > c0; kb -= 64) {
    const int nb = kb - c0 < 64 ? kb - c0 : 64;
    int beg = 0, cnt = 0, kl = 0;
    double d = 1.0;
    if (lane < nb) {
      const int k = kb - 1 - lane;
      const int b = a.Ubeg[k], ca = a.Ucnt[k];
      d = a.Ux[b + ca - 1];
      beg = search ? lower_bound_g(a.Ui, b, b + ca - 1, c0) : b;
      cnt = b + ca - 1 - beg;
      kl = k - c0;
    }
    run_batch<kLds>(sm, S, lane, nb, beg, cnt, a.Ui, a.Ux, true, [&](int j) { return j - c0; },
                    [&](int j) -> double {
                      const int kk = rl(kl, j);
                      const double zk = S[kk] / rl_d(d, j);
                      step_sync<kLds>();
                      if (lane == 0) S[kk] = zk;
                      return zk;
                    });
  }
}

template <bool kLds>
__device__ void block_task(const SolveArgs& a, const Smem& sm, int b, int rhs, int lane) {
  const int b0 = a.blkptr[b], b1 = a.blkptr[b + 1], m = b1 - b0;
  double* Z = a.Z + (int64_t)rhs * a.n;
  const double* Bc = a.B + (int64_t)rhs * a.ldb;
  double* Wl = kLds ? sm.work : a.W + (int64_t)rhs * a.n + b0;
  double* Zl = kLds ? sm.work + m : Z + b0;
  residual_rows<kLds>(a, Wl, b0, m, Bc, Z, lane);
  int32_t* status = a.status;
  l_sweep<kLds>(a, sm, Wl, b0, b1, lane, [&](int r) {
    const int t = r - b0;
    if ((unsigned)t >= (unsigned)m) { atomicOr(status, 1); return -1; }
    return t;
  });
  for (int k = lane; k < m; k += 64) Zl[k] = Wl[a.piv[b0 + k] - b0];
  step_sync<kLds>();
  u_sweep<kLds>(a, sm, Zl, b0, b1, lane, false);
  if (kLds) {
    for (int k = lane; k < m; k += 64) Z[b0 + k] = Zl[k];
  }
}

template <bool kLds>
__device__ void nd_forward_task(const SolveArgs& a, const Smem& sm, int g, int rhs, int lane) {
  const int c0 = a.grpptr[g], c1 = a.grpptr[g + 1], m = c1 - c0;
  const int choff = a.sg_choff[g];
  double* Z = a.Z + (int64_t)rhs * a.n;
  const double* Bc = a.B + (int64_t)rhs * a.ldb;
  double* gb = a.gbuf + (int64_t)rhs * a.gbuf_total;
  double* S = kLds ? sm.work : gb + a.sg_tbase[g];
  residual_rows<kLds>(a, S, c0, m, Bc, Z, lane);
  for (int p = lane; p < choff; p += 64) S[m + p] = 0.0;
  // buffers of the descendants (postorder: groups [fd, g)), lowest first
  for (int d = a.sg_fd[g]; d < g; d++) {
    const double* bd = gb + a.sg_tbase[d] + (a.grpptr[d + 1] - a.grpptr[d]) + choff;
    for (int i = lane; i < m; i += 64) S[i] = S[i] + bd[i];
  }
  step_sync<kLds>();
  const int32_t* rowpos = a.rowpos;
  int32_t* status = a.status;
  l_sweep<kLds>(a, sm, S, c0, c1, lane, [&](int r) {
    const int t = r - c0;
    if ((unsigned)t < (unsigned)m) return t;
    const int p = rowpos[r];
    if (p < 0 || p >= choff) { atomicOr(status, 2); return -1; }
    return m + p;
  });
  for (int k = lane; k < m; k += 64) Z[c0 + k] = S[a.piv[c0 + k] - c0];
  if (kLds) {
    double* out = gb + a.sg_tbase[g] + m;
    for (int p = lane; p < choff; p += 64) out[p] = S[m + p];
  }
}

template <bool kLds>
__device__ void nd_backward_task(const SolveArgs& a, const Smem& sm, int g, int rhs, int lane) {
  const int c0 = a.grpptr[g], c1 = a.grpptr[g + 1], m = c1 - c0;
  double* Z = a.Z + (int64_t)rhs * a.n;
  double* S = kLds ? sm.work : Z + c0;
  if (kLds) {
    for (int i = lane; i < m; i += 64) S[i] = Z[c0 + i];
    lsync();
  }
  // ancestors' columns, last first: rows [c0, c1) of each column
  for (int q = a.sg_anc_ptr[g + 1] - 1; q >= a.sg_anc_ptr[g]; q--) {
    const int an = a.sg_anc[q];
    const int a0 = a.grpptr[an], a1 = a.grpptr[an + 1];
    for (int kb = a1; kb > a0; kb -= 64) {
      const int nb = kb - a0 < 64 ? kb - a0 : 64;
      int beg = 0, cnt = 0;
      double zk = 0.0;
      if (lane < nb) {
        const int k = kb - 1 - lane;
        const int b = a.Ubeg[k], e = b + a.Ucnt[k] - 1;
        beg = lower_bound_g(a.Ui, b, e, c0);
        cnt = lower_bound_g(a.Ui, beg, e, c1) - beg;
        zk = Z[k];
      }
      run_batch<kLds>(sm, S, lane, nb, beg, cnt, a.Ui, a.Ux, false, [&](int j) { return j - c0; },
                      [&](int j) -> double { return rl_d(zk, j); });
    }
  }
  u_sweep<kLds>(a, sm, S, c0, c1, lane, true);
  if (kLds) {
    for (int i = lane; i < m; i += 64) Z[c0 + i] = S[i];
  }
}

__global__ void __launch_bounds__(64) solve_task_kernel(SolveArgs a) {
  BASKER_DYN_SHARED(double, smem_d);
  const int lane = lane_id();
  Smem sm;
  sm.sx = smem_d;
  sm.work = smem_d + kStage;
  sm.si = reinterpret_cast<int32_t*>(smem_d + kStage + a.lds_doubles);
  sm.pre = sm.si + kStage;
  sm.sbeg = sm.pre + 72;
  const int t = a.t_begin + (int)blockIdx.x;
  const int kind = a.st_kind[t], id = a.st_id[t];
  const bool lds = a.st_need[t] <= a.lds_doubles;
  for (int rhs = 0; rhs < a.nrhs; rhs++) {
    if (kind == 0) {
      if (lds) block_task<true>(a, sm, id, rhs, lane); else block_task<false>(a, sm, id, rhs, lane);
    } else if (kind == 1) {
      if (lds) nd_forward_task<true>(a, sm, id, rhs, lane); else nd_forward_task<false>(a, sm, id, rhs, lane);
    } else {
      if (lds) nd_backward_task<true>(a, sm, id, rhs, lane); else nd_backward_task<false>(a, sm, id, rhs, lane);
    }
    wsync();
  }
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

size_t solve_lds_bytes(int32_t work_doubles) {
  return sizeof(double) * ((size_t)kStage + (size_t)work_doubles) + sizeof(int32_t) * ((size_t)kStage + 72 + 64);
}

hipError_t solve_lds_setup(size_t max_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_task_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
}

hipError_t launch_solve_tasks(const SolveArgs& a, int ntasks, hipStream_t s) {
  if (ntasks > 0)
    hipLaunchKernelGGL(solve_task_kernel, dim3(ntasks), dim3(64), solve_lds_bytes(a.lds_doubles), s, a);
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

hipError_t launch_solve_finish(const SolveArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)a.n * a.nrhs;
  if (total > 0)
    hipLaunchKernelGGL(solve_unpermute_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
