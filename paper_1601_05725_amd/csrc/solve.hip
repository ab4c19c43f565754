// Solve on gfx950: block back-substitution over the block triangular form.
//
// R = A(prow, qcol) is block upper triangular, so block b needs the solution of every
// later block it couples to: r_b = c_b - sum_{c > b} R_bc z_c, then L w = r(piv) and
// U z_b = w.  Blocks are grouped in levels (a block's level is one more than the
// highest level of the later blocks it reads from), one launch per level; inside a
// launch every wavefront takes whole blocks from an atomic counter.  The coupling sums
// are pulled row by row in a fixed order and the triangular solves run column by
// column inside one wave, so results do not depend on scheduling.
#include "device.hpp"

namespace basker {

namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// lanes exchange data through global memory between steps: drain every outstanding
// memory operation and keep the compiler from moving accesses across
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(64) solve_kernel(SolveArgs a) {
  const int lane = lane_id();
  const int n = a.n;
  const int nb = a.lvl_end - a.lvl_begin;
  while (true) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(&a.lvl_ctr[a.level], 1);
    idx = __shfl(idx, 0, 64);
    if (idx >= nb) break;
    const int b = a.blvl_blk[a.lvl_begin + idx];
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

hipError_t launch_solve_level(const SolveArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(solve_kernel, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_finish(const SolveArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)a.n * a.nrhs;
  if (total > 0)
    hipLaunchKernelGGL(solve_unpermute_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
