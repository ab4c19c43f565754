// Solve on gfx950: block back-substitution over the block triangular form.
//
// R = A(prow, qcol) is block upper triangular, so block b needs the solution of every
// later block it couples to: r_b = c_b - sum_{c > b} R_bc z_c, then L w = r(piv) and
// U z_b = w.  A persistent kernel takes ready blocks from a device queue, one
// wavefront per block; a block becomes ready when every later block it reads from
// has finished (completion counters, device-scope release/acquire).  The coupling
// sums are pulled row by row in a fixed order, and the triangular solves run column
// by column inside one wave, so results do not depend on scheduling.
#include "device.hpp"

namespace basker {

namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ void wsync() { __syncthreads(); }

__global__ void __launch_bounds__(64) solve_kernel(SolveArgs a) {
  const int lane = lane_id();
  const int n = a.n;
  while (true) {
    int pos = 0;
    if (lane == 0) pos = atomicAdd(&a.ctrs[0], 1);
    pos = __shfl(pos, 0, 64);
    if (pos >= a.nblk) break;
    int b = -1;
    if (lane == 0) {
      long long spins = 0;
      while ((b = __hip_atomic_load(&a.queue[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) < 0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicMax(&a.status[0], DEV_STALL);
          break;
        }
      }
    }
    b = __shfl(b, 0, 64);
    wsync();
    if (b < 0) break;
    const int b0 = a.blkptr[b], b1 = a.blkptr[b + 1];
    for (int rhs = 0; rhs < a.nrhs; rhs++) {
      double* W = a.W + (int64_t)rhs * n;
      double* Z = a.Z + (int64_t)rhs * n;
      const double* Bc = a.B + (int64_t)rhs * a.ldb;
      // residual of this block's rows (R-row numbering)
      for (int i = b0 + lane; i < b1; i += 64) {
        double v = Bc[a.prow[i]];
        for (int q = a.OTp[i]; q < a.OTp[i + 1]; q++) {
          const double prod = a.OTx[q] * Z[a.OTj[q]];
          v = v - prod;
        }
        W[i] = v;
      }
      wsync();
      // L solve, column by column (rows of L are R rows)
      for (int k = b0; k < b1; k++) {
        const double wk = W[a.piv[k]];
        const int beg = a.Lbeg[k], cnt = a.Lcnt[k];
        for (int t = lane; t < cnt; t += 64) {
          const int r = a.Li[beg + t];
          const double prod = a.Lx[beg + t] * wk;
          W[r] = W[r] - prod;
        }
        wsync();
      }
      // U solve, column by column from the last (rows of U are columns)
      for (int k = b0 + lane; k < b1; k += 64) Z[k] = W[a.piv[k]];
      wsync();
      for (int k = b1 - 1; k >= b0; k--) {
        const int beg = a.Ubeg[k], cnt = a.Ucnt[k];
        const double zk = Z[k] / a.Ux[beg + cnt - 1];
        wsync();
        for (int t = lane; t < cnt - 1; t += 64) {
          const int j = a.Ui[beg + t];
          const double prod = a.Ux[beg + t] * zk;
          Z[j] = Z[j] - prod;
        }
        if (lane == 0) Z[k] = zk;
        wsync();
      }
    }
    // release the earlier blocks that read from this one
    if (lane == 0) {
      for (int q = a.bdep_ptr[b]; q < a.bdep_ptr[b + 1]; q++) {
        const int d = a.bdep_idx[q];
        const int old = __hip_atomic_fetch_add(&a.bdone[d], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == a.bdep_cnt[d]) {
          const int slot = __hip_atomic_fetch_add(&a.ctrs[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.queue[slot], d, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
}

__global__ void solve_init_kernel(SolveArgs a, const int32_t* ready, int32_t nready) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.nblk) {
    a.bdone[i] = 0;
    a.queue[i] = i < nready ? ready[i] : -1;
  }
  if (i == 0) { a.ctrs[0] = 0; a.ctrs[1] = nready; a.status[0] = 0; }
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

hipError_t launch_solve(const SolveArgs& a, const int32_t* ready, int32_t nready, int grid, hipStream_t s) {
  const int nb = a.nblk > 1 ? a.nblk : 1;
  hipLaunchKernelGGL(solve_init_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, a, ready, nready);
  hipLaunchKernelGGL(solve_kernel, dim3(grid), dim3(64), 0, s, a);
  const int64_t total = (int64_t)a.n * a.nrhs;
  if (total > 0)
    hipLaunchKernelGGL(solve_unpermute_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
