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
// A task is one workgroup of kSW wavefronts.  The waves take the task's rows round
// robin in the sweep's order (ascending for L, descending for U), and a row waits only
// for the rows of the same task it reads (done bits in LDS, release/acquire at
// workgroup scope); a wave finishes a row before taking its next one, so the first
// unfinished row can always proceed.
//
// Each unknown is computed from one row of the factors, with the updates subtracted
// one at a time in the order the column sweep applies them: the coupling entries of
// the row (later blocks first, columns ascending inside a block), then L's entries in
// ascending column, or U's in descending column, each product rounded and subtracted
// separately, and z_k = w_k / u_kk.  The result is the column sweep's, bit for bit, and
// does not depend on the schedule.
#include "device.hpp"

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
template <bool kLds>
__device__ __forceinline__ bool row_update(double& acc, const RowPre& r, const unsigned long long* keys,
                                           const double* vals, bool rev, int n, int r0, int m, const double* V,
                                           const Flags<kLds>& F, const double* fin, int lane) {
  bool stalled = false;
  for (int b = r.e0; b < r.e1; b += 64) {
    const int cnt = (r.e1 - b < 64) ? r.e1 - b : 64;
    int j = r.j;
    double x = r.x;
    if (b != r.e0) {
      j = -1;
      if (lane < cnt) {
        const unsigned lo = (unsigned)keys[b + lane];
        j = rev ? n - 1 - (int)lo : (int)lo;
        x = vals[b + lane];
      }
    }
    double prod = 0.0;
    if (lane < cnt) {
      double v;
      const int jj = j - r0;
      if (jj >= 0 && jj < m) {
        unsigned spins = 0;
        while (!F.test(jj)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { stalled = true; break; }
        }
        consume_fence<kLds>();
        v = V[jj];
      } else {
        v = fin[j];
      }
      prod = x * v;
    }
    acc = subtract_in_order(acc, prod, cnt);
  }
  return !__any(stalled);
}

template <bool kLds>
__device__ void run_task(const SolveArgs& a, double* V, int32_t* Pl, const Flags<kLds>& F, int kind, int id, int rhs,
                         int tid) {
  const int lane = tid & 63;
  const int wv = tid >> 6;
  int r0, r1;
  if (kind == 0) { r0 = a.blkptr[id]; r1 = a.blkptr[id + 1]; }
  else { r0 = a.grpptr[id]; r1 = a.grpptr[id + 1]; }
  const int m = r1 - r0;
  const int n = a.n;
  double* W = a.W + (int64_t)rhs * n;
  double* Z = a.Z + (int64_t)rhs * n;
  const double* Bc = a.B + (int64_t)rhs * a.ldb;
  bool ok = true;
  if (kind != 2) {
    // residual of every row (independent of the task's other rows): the right-hand
    // side minus the coupling to finished later blocks, in the sweep's order
    F.clear(m, tid);
    for (int kk = tid; kk < m; kk += 64 * kSW) {
      const int i = a.piv[r0 + kk];
      double acc = Bc[a.prow[i]];
      for (int q = a.OTp[i]; q < a.OTp[i + 1]; q++) {
        const double prod = a.OTx[q] * Z[a.OTj[q]];
        acc = acc - prod;
      }
      V[kk] = acc;
    }
    // the task's L row pointers
    const int32_t* LP = a.LTp + r0;
    if (kLds) {
      for (int kk = tid; kk <= m; kk += 64 * kSW) Pl[kk] = a.LTp[r0 + kk];
      LP = Pl;
    }
    __syncthreads();
    // L rows, ascending
    RowPre cur, nxt;
    if (wv < m) row_prefetch(cur, LP, a.lkeys, a.lvals, wv, false, n, lane);
    for (int kk = wv; kk < m; kk += kSW) {
      if (kk + kSW < m) row_prefetch(nxt, LP, a.lkeys, a.lvals, kk + kSW, false, n, lane);
      double acc = V[kk];
      ok &= row_update<kLds>(acc, cur, a.lkeys, a.lvals, false, n, r0, m, V, F, W, lane);
      if (lane == 0) V[kk] = acc;
      publish_fence<kLds>();
      if (lane == 0) F.set(kk);
      cur = nxt;
    }
    __syncthreads();
    if (kind == 1) {
      for (int kk = tid; kk < m; kk += 64 * kSW) W[r0 + kk] = V[kk];
      if (!ok && tid == 0) atomicOr(a.status, 4);
      return;
    }
  } else {
    for (int kk = tid; kk < m; kk += 64 * kSW) V[kk] = W[r0 + kk];
  }
  // U rows, descending: z_k = (w_k - sum_{j > k} u_kj z_j) / u_kk
  F.clear(m, tid);
  __syncthreads();
  const int32_t* UP = a.UTp + r0;
  if (kLds) {
    for (int kk = tid; kk <= m; kk += 64 * kSW) Pl[kk] = a.UTp[r0 + kk];
    UP = Pl;
  }
  __syncthreads();
  {
    RowPre cur, nxt;
    double dcur = 1.0, dnxt = 1.0;
    if (wv < m) {
      row_prefetch(cur, UP, a.ukeys, a.uvals, m - 1 - wv, true, n, lane);
      dcur = a.diag[r1 - 1 - wv];
    }
    for (int q = wv; q < m; q += kSW) {
      const int kk = m - 1 - q;
      if (q + kSW < m) {
        row_prefetch(nxt, UP, a.ukeys, a.uvals, kk - kSW, true, n, lane);
        dnxt = a.diag[r0 + kk - kSW];
      }
      double acc = V[kk];
      ok &= row_update<kLds>(acc, cur, a.ukeys, a.uvals, true, n, r0, m, V, F, Z, lane);
      const double z = acc / dcur;
      if (lane == 0) V[kk] = z;
      publish_fence<kLds>();
      if (lane == 0) F.set(kk);
      cur = nxt;
      dcur = dnxt;
    }
  }
  __syncthreads();
  for (int kk = tid; kk < m; kk += 64 * kSW) Z[r0 + kk] = V[kk];
  if (!ok && tid == 0) atomicOr(a.status, 4);
}

__global__ void __launch_bounds__(64 * kSW) solve_task_kernel(SolveArgs a) {
  BASKER_DYN_SHARED(double, smem_d);
  const int tid = threadIdx.x;
  const int t = a.t_begin + (int)blockIdx.x;
  const int kind = a.st_kind[t], id = a.st_id[t];
  const int m = kind == 0 ? a.blkptr[id + 1] - a.blkptr[id] : a.grpptr[id + 1] - a.grpptr[id];
  const bool lds = m <= a.lds_doubles;
  for (int rhs = 0; rhs < a.nrhs; rhs++) {
    if (lds) {
      // LDS: work vector (lds_doubles), row pointers (lds_doubles + 1), done bits
      int32_t* Pl = reinterpret_cast<int32_t*>(smem_d + a.lds_doubles);
      Flags<true> F{reinterpret_cast<unsigned*>(Pl + a.lds_doubles + 1), nullptr};
      run_task<true>(a, smem_d, Pl, F, kind, id, rhs, tid);
    } else {
      const int r0 = kind == 0 ? a.blkptr[id] : a.grpptr[id];
      Flags<false> F{nullptr, a.sflag + r0};
      // work vector in place: the block's (or node's) part of Z, or of W for a forward task
      double* V = (kind == 1 ? a.W : a.Z) + (int64_t)rhs * a.n + r0;
      run_task<false>(a, V, nullptr, F, kind, id, rhs, tid);
    }
    __syncthreads();
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
  return sizeof(double) * (size_t)work_doubles + sizeof(int32_t) * ((size_t)work_doubles + 1) +
         sizeof(unsigned) * (((size_t)work_doubles + 31) / 32 + 1);
}

hipError_t solve_lds_setup(size_t max_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&solve_task_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_bytes);
}

hipError_t launch_solve_tasks(const SolveArgs& a, int ntasks, hipStream_t s) {
  if (ntasks > 0)
    hipLaunchKernelGGL(solve_task_kernel, dim3(ntasks), dim3(64 * kSW), solve_lds_bytes(a.lds_doubles), s, a);
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
