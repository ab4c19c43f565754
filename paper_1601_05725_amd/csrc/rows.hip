// Row-wise copies of the factors for the solve.
//
// The factorization stores L and U by columns (Alg. 1 produces one column of each per
// step).  The solve computes each unknown from one row of a factor, and does it the way
// the column sweep of the back-substitution would: row k of L receives its updates
// from columns j < k in ascending order, row k of U from columns j > k in descending
// order.  So the entries of every row are gathered and sorted by column: a key
// (row << 32 | column) per entry of the pools (or the reversed column for U), a radix
// sort of (key, value) pairs, and the first entry of every row found by binary search.
// Pool slots between the columns' chunks, and U's diagonal entries, get the largest
// key and sort to the end.  Last, the solve's issue orders are checked against the
// rows' actual patterns.
#include <hipcub/hipcub.hpp>

#include "device.hpp"

namespace basker {

namespace {

constexpr unsigned long long kNoKey = ~0ull;

__global__ void fill_keys_kernel(unsigned long long* keys, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) keys[i] = kNoKey;
}

// one wavefront per column j: L entries -> (pivot position of the row, j); U entries
// except the diagonal (last) -> (row, n - 1 - j)
__global__ void col_keys_kernel(RowsArgs a) {
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (gw >= a.n) return;
  const int j = (int)gw;
  const int lb = a.Lbeg[j], lc = a.Lcnt[j];
  for (int t = lane; t < lc; t += 64) {
    const int p = lb + t;
    a.lkeys[p] = ((unsigned long long)(unsigned)a.pinv[a.Li[p]] << 32) | (unsigned)j;
    a.lvals[p] = a.Lx[p];
  }
  const int ub = a.Ubeg[j], uc = a.Ucnt[j] - 1;
  if (lane == 0) a.diag[j] = a.Ux[ub + uc];
  for (int t = lane; t < uc; t += 64) {
    const int p = ub + t;
    a.ukeys[p] = ((unsigned long long)(unsigned)a.Ui[p] << 32) | (unsigned)(a.n - 1 - j);
    a.uvals[p] = a.Ux[p];
  }
}

// ptr[k] = first sorted entry of row k (k = 0..n)
__global__ void row_ptr_kernel(const unsigned long long* keys, int64_t cnt, int32_t* ptr, int n) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k > n) return;
  const unsigned long long key = (unsigned long long)(unsigned)k << 32;
  int64_t lo = 0, hi = cnt;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < key) lo = mid + 1; else hi = mid;
  }
  ptr[k] = (int32_t)lo;
}

__global__ void clear_order_flags_kernel(int32_t* x, int n, int32_t* count) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) x[i] = 0;
  if (i == 0) *count = 0;
}

// one wavefront per row k: an issue order is valid when every entry of the row in
// another row of the same task comes earlier in the task's order (then the first
// unfinished row in the order can always proceed)
__global__ void order_check_kernel(RowsArgs a) {
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (gw >= a.n) return;
  const int k = (int)gw;
  const int t0 = a.row_task0[k];
  bool badf = false, badb = false;
  for (int p = a.LTp[k] + lane; p < a.LTp[k + 1]; p += 64) {
    const int j = (int)(unsigned)a.lkeys_out[p];
    badf |= a.row_task0[j] == t0 && a.sfo_pos[j] >= a.sfo_pos[k];
  }
  for (int p = a.UTp[k] + lane; p < a.UTp[k + 1]; p += 64) {
    const int j = a.n - 1 - (int)(unsigned)a.ukeys_out[p];
    badb |= a.row_task0[j] == t0 && a.sbo_pos[j] >= a.sbo_pos[k];
  }
  const bool f = __any(badf), b = __any(badb);
  if (lane == 0 && (f || b)) {
    const int bits = (f ? 1 : 0) | (b ? 2 : 0);
    const int old = atomicOr(&a.obad[t0], bits);
    const int fresh = bits & ~old;
    if (fresh) atomicAdd(a.ocount, __popc(fresh));
  }
}

int key_bits(int n) {
  int b = 1;
  while ((1ll << b) < (long long)n + 1) b++;
  return 32 + b;
}

}  // namespace

hipError_t rows_temp_bytes(int64_t items, int n, size_t* bytes) {
  *bytes = 0;
  if (items <= 0) return hipSuccess;
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const unsigned long long*)nullptr,
                                            (unsigned long long*)nullptr, (const double*)nullptr, (double*)nullptr,
                                            (int)items, 0, key_bits(n));
}

hipError_t launch_rows_build(const RowsArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipError_t e;
  const int64_t tot = a.Lused + a.Uused;
  (void)tot;
  if (a.Lused > 0) {
    hipLaunchKernelGGL(fill_keys_kernel, dim3((unsigned)((a.Lused + 255) / 256)), dim3(256), 0, s, a.lkeys, a.Lused);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (a.Uused > 0) {
    hipLaunchKernelGGL(fill_keys_kernel, dim3((unsigned)((a.Uused + 255) / 256)), dim3(256), 0, s, a.ukeys, a.Uused);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(col_keys_kernel, dim3((unsigned)(((int64_t)a.n * 64 + 255) / 256)), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int bits = key_bits(a.n);
  size_t tb = a.temp_bytes;
  if (a.Lused > 0) {
    if ((e = hipcub::DeviceRadixSort::SortPairs(a.temp, tb, a.lkeys, a.lkeys_out, a.lvals, a.lvals_out, (int)a.Lused,
                                                0, bits, s)) != hipSuccess)
      return e;
  }
  tb = a.temp_bytes;
  if (a.Uused > 0) {
    if ((e = hipcub::DeviceRadixSort::SortPairs(a.temp, tb, a.ukeys, a.ukeys_out, a.uvals, a.uvals_out, (int)a.Uused,
                                                0, bits, s)) != hipSuccess)
      return e;
  }
  hipLaunchKernelGGL(row_ptr_kernel, dim3((unsigned)((a.n + 1 + 255) / 256)), dim3(256), 0, s,
                     (const unsigned long long*)a.lkeys_out, a.Lused, a.LTp, a.n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(row_ptr_kernel, dim3((unsigned)((a.n + 1 + 255) / 256)), dim3(256), 0, s,
                     (const unsigned long long*)a.ukeys_out, a.Uused, a.UTp, a.n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(clear_order_flags_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a.obad, a.n,
                     a.ocount);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(order_check_kernel, dim3((unsigned)(((int64_t)a.n * 64 + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace basker
