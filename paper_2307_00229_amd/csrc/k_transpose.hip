// k_transpose.hip -- CSR transpose on the device.
//
// Used to form P = (R built on A^T)^T: the input A^T of the restriction
// setup, and the transpose of its result.  Rows of the output are sorted by
// column like every CSR array of the library.  Stages: column counts
// (integer atomics) -> exclusive scan (per-block scans, one workgroup over
// the block totals, offsets) -> scatter (a per-column cursor) -> sort of each
// output row (the scatter order within a column is arbitrary).  Values are
// copied, so the transpose is exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kTT = 256;            // threads per workgroup
constexpr int kTPer = 4;            // scan entries per thread
constexpr int kTBlk = kTT * kTPer;  // scan entries per workgroup

__global__ void k_t_zero(int32_t* a, int n) {
  for (int j = blockIdx.x * kTT + threadIdx.x; j < n; j += gridDim.x * kTT) a[j] = 0;
}

// cnt[j] = entries of column j (indices outside [0, ncol) are skipped and
// flagged in *bad)
__global__ void k_t_count(int m, int ncol, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          int32_t* cnt, int32_t* bad) {
  for (int i = blockIdx.x * kTT + threadIdx.x; i < m; i += gridDim.x * kTT) {
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = ci[e];
      if ((unsigned)j < (unsigned)ncol) atomicAdd(&cnt[j], 1);
      else atomicExch(bad, 1);
    }
  }
}

// exclusive scan of cnt[0..n) into out[0..n), per block of kTBlk entries;
// block totals to sums[b]
__global__ __launch_bounds__(kTT) void k_t_scan_blocks(const int32_t* cnt, int n, int32_t* out, int32_t* sums) {
  __shared__ int sh[kTT / 64];
  const int base = blockIdx.x * kTBlk + threadIdx.x * kTPer;
  int v[kTPer];
  int my = 0;
#pragma unroll
  for (int k = 0; k < kTPer; ++k) {
    v[k] = (base + k < n) ? cnt[base + k] : 0;
    my += v[k];
  }
  int tot;
  int pre = block_exclusive_scan(my, sh, &tot);
#pragma unroll
  for (int k = 0; k < kTPer; ++k) {
    if (base + k < n) out[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the block totals in place; sums[nb] = total
__global__ __launch_bounds__(kTT) void k_t_scan_sums(int32_t* sums, int nb) {
  __shared__ int sh[kTT / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += kTT) {
    const int b = b0 + threadIdx.x;
    const int v = (b < nb) ? sums[b] : 0;
    int tot;
    const int pre = block_exclusive_scan(v, sh, &tot);
    const int c = carry;
    if (b < nb) sums[b] = c + pre;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void k_t_scan_add(int32_t* out, int n, const int32_t* sums, int nb) {
  for (int j = blockIdx.x * kTT + threadIdx.x; j < n; j += gridDim.x * kTT) out[j] += sums[j / kTBlk];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

// scatter: entry (i, j) to out row j at trp[j] + the column's cursor
__global__ void k_t_fill(int m, int ncol, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const double* __restrict__ va, const int32_t* __restrict__ trp, int32_t* cursor,
                         int32_t* tci, double* tva) {
  for (int i = blockIdx.x * kTT + threadIdx.x; i < m; i += gridDim.x * kTT) {
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = ci[e];
      if ((unsigned)j >= (unsigned)ncol) continue;
      const int pos = trp[j] + atomicAdd(&cursor[j], 1);
      tci[pos] = i;
      tva[pos] = va[e];
    }
  }
}

// sort every output row by column (insertion sort; rows of a transpose of
// the matrices here are short)
__global__ void k_t_sort(int ncol, const int32_t* __restrict__ trp, int32_t* tci, double* tva) {
  for (int j = blockIdx.x * kTT + threadIdx.x; j < ncol; j += gridDim.x * kTT) {
    const int e0 = trp[j], e1 = trp[j + 1];
    for (int a = e0 + 1; a < e1; ++a) {
      const int k = tci[a];
      const double x = tva[a];
      int b = a - 1;
      while (b >= e0 && tci[b] > k) {
        tci[b + 1] = tci[b];
        tva[b + 1] = tva[b];
        --b;
      }
      tci[b + 1] = k;
      tva[b + 1] = x;
    }
  }
}

int grid_for(int n, int cus) { return std::max(1, std::min((n + kTT - 1) / kTT, cus * 8)); }

}  // namespace

size_t transpose_scratch_ints(int ncol) { return (size_t)ncol + (size_t)(ncol / kTBlk + 2) + 1; }

size_t scan_scratch_ints(int n) { return (size_t)(n / kTBlk + 2); }

hipError_t launch_exclusive_scan(const int32_t* cnt, int n, int32_t* out, int32_t* sums, int cus, hipStream_t s) {
  const int nb = (n + kTBlk - 1) / kTBlk;
  if (nb > 0) hipLaunchKernelGGL(k_t_scan_blocks, dim3(nb), dim3(kTT), 0, s, cnt, n, out, sums);
  hipLaunchKernelGGL(k_t_scan_sums, dim3(1), dim3(kTT), 0, s, sums, nb);
  hipLaunchKernelGGL(k_t_scan_add, dim3(grid_for(n, cus)), dim3(kTT), 0, s, out, n, sums, nb);
  return hipGetLastError();
}

hipError_t launch_transpose(int m, int ncol, const int32_t* rp, const int32_t* ci, const double* va, int32_t* trp,
                            int32_t* tci, double* tva, int32_t* scratch, int cus, hipStream_t s) {
  int32_t* cursor = scratch;
  int32_t* bad = scratch + ncol;
  int32_t* sums = scratch + ncol + 1;
  const int nb = (ncol + kTBlk - 1) / kTBlk;
  hipLaunchKernelGGL(k_t_zero, dim3(grid_for(ncol + 1, cus)), dim3(kTT), 0, s, cursor, ncol + 1);
  if (m > 0) hipLaunchKernelGGL(k_t_count, dim3(grid_for(m, cus)), dim3(kTT), 0, s, m, ncol, rp, ci, cursor, bad);
  if (nb > 0) hipLaunchKernelGGL(k_t_scan_blocks, dim3(nb), dim3(kTT), 0, s, cursor, ncol, trp, sums);
  hipLaunchKernelGGL(k_t_scan_sums, dim3(1), dim3(kTT), 0, s, sums, nb);
  hipLaunchKernelGGL(k_t_scan_add, dim3(grid_for(ncol, cus)), dim3(kTT), 0, s, trp, ncol, sums, nb);
  hipLaunchKernelGGL(k_t_zero, dim3(grid_for(ncol, cus)), dim3(kTT), 0, s, cursor, ncol);
  if (m > 0) hipLaunchKernelGGL(k_t_fill, dim3(grid_for(m, cus)), dim3(kTT), 0, s, m, ncol, rp, ci, va, trp, cursor, tci, tva);
  if (ncol > 0) hipLaunchKernelGGL(k_t_sort, dim3(grid_for(ncol, cus)), dim3(kTT), 0, s, ncol, trp, tci, tva);
  return hipGetLastError();
}

}  // namespace clair
