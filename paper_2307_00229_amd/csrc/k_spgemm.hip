// k_spgemm.hip -- sparse product C = X Y on the device (FP64 values, int32
// CSR), for the Galerkin coarse operator A_c = R A P (Section 1: the coarse
// level of the hierarchy; Section 4.2 forms P and R separately).
//
// One wavefront per output row.  The row's products x_ij y_jc are gathered
// into an open-addressing hash table in LDS (keys inserted with LDS
// compare-and-swap, values summed with LDS FP64 atomics).  A row uses the
// smallest power of two (at least 64) that is twice its number of products,
// so short rows clear and scan only a few slots.  The kernels are compiled
// for tables of 2^6 .. 2^11 slots per wavefront; the launch takes the size
// the longest row of the product needs (a first pass finds the largest
// product count), so LDS does not cap the number of wavefronts per CU when
// every row is short.
// then the occupied slots are compacted in place and every entry is written
// at its rank among the row's columns, so rows come out sorted.  A symbolic
// pass counts the columns of every row first; the caller scans the counts
// into C's row pointers.  The pattern is structural: a column stays even
// when its products cancel.  Summation order inside a row is not fixed, so
// values agree with a sequential product to rounding.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kLgH = 11;    // log2 of the largest table
constexpr int kH = 1 << kLgH;  // hash slots per wavefront at most
static_assert(kSpgemmMaxRow <= kH * 3 / 4, "row bound below the table size");
// wavefronts per workgroup for a table of 2^LG slots
constexpr int waves_for(int LG) { return LG <= 8 ? 4 : 2; }

// Inserts key c into a table of 2^lg slots; returns its slot, or -1 when the
// table holds its bound of keys already (the probe sequence is bounded by
// the table size, so the loop always ends).
__device__ __forceinline__ int hash_insert(int* keys, int* count, int c, int lg, int bound) {
  const int size = 1 << lg;
  if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= bound) return -1;  // row already over
  int h = (int)(((uint32_t)c * 2654435761u) >> (32 - lg));
  for (int probe = 0; probe < size; ++probe) {
    const int prev = atomicCAS(&keys[h], -1, c);
    if (prev == c) return h;
    if (prev == -1) {
      // over the bound the row is reported and its contents do not matter
      return atomicAdd(count, 1) >= bound ? -1 : h;
    }
    h = (h + 1) & (size - 1);
  }
  return -1;
}

// Table size of row i: the smallest power of two >= max(64, 2 * products),
// capped at 2^LG; *bound = the keys it may hold (below the cap a row never
// reaches it: it has at most half as many columns as slots)
template <int LG>
__device__ __forceinline__ int table_lg(const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci, int k,
                                        const int32_t* __restrict__ yrp, int i, int* bound) {
  const int lane = threadIdx.x & 63;
  long long prod = 0;
  for (int e = xrp[i] + lane; e < xrp[i + 1]; e += 64) {
    const int j = xci[e];
    if ((unsigned)j < (unsigned)k) prod += yrp[j + 1] - yrp[j];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) prod += __shfl_xor(prod, o, 64);
  int lg = 6;
  while (lg < LG && (1ll << lg) < 2 * prod) ++lg;
  *bound = (lg == kLgH) ? kSpgemmMaxRow : (1 << lg);
  return lg;
}

// largest number of products of a row (indices out of range skipped; the
// count pass reports them), into *maxprod
__global__ void k_sg_maxprod(int m, const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci, int k,
                             const int32_t* __restrict__ yrp, int32_t* maxprod) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    long long prod = 0;
    for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
      const int j = xci[e];
      if ((unsigned)j < (unsigned)k) prod += yrp[j + 1] - yrp[j];
    }
    atomicMax(maxprod, (int32_t)min(prod, (long long)(1 << 30)));
  }
}

template <int LG>
__global__ __launch_bounds__(64 * waves_for(LG)) void k_sg_count(int m, const int32_t* __restrict__ xrp,
                                                                   const int32_t* __restrict__ xci, int k,
                                                                   const int32_t* __restrict__ yrp,
                                                                   const int32_t* __restrict__ yci, int ny,
                                                                   int32_t* cnt, int32_t* flags) {
  constexpr int kSW = waves_for(LG);
  __shared__ int keys[kSW][1 << LG];
  __shared__ int count[kSW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* kt = keys[wv];
  for (int i = blockIdx.x * kSW + wv; i < m; i += gridDim.x * kSW) {
    int bound;
    const int lg = table_lg<LG>(xrp, xci, k, yrp, i, &bound);
    for (int t = lane; t < (1 << lg); t += 64) kt[t] = -1;
    if (lane == 0) count[wv] = 0;
    wave_sync();
    bool over = false;
    for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
      const int j = xci[e];
      if ((unsigned)j >= (unsigned)k) { if (lane == 0) atomicExch(&flags[1], 1); continue; }
      for (int f = yrp[j] + lane; f < yrp[j + 1]; f += 64) {
        const int c = yci[f];
        if ((unsigned)c >= (unsigned)ny) { atomicExch(&flags[1], 1); continue; }
        if (hash_insert(kt, &count[wv], c, lg, bound) < 0) over = true;
      }
    }
    wave_sync();
    const int n = count[wv];
    const bool any_over = __ballot(over) != 0 || n > bound;
    if (lane == 0) {
      cnt[i] = any_over ? 0 : n;
      if (any_over) atomicExch(&flags[0], 1);
    }
    wave_sync();
  }
}

template <int LG>
__global__ __launch_bounds__(64 * waves_for(LG)) void k_sg_fill(int m, const int32_t* __restrict__ xrp,
                                                                  const int32_t* __restrict__ xci,
                                                                  const double* __restrict__ xva,
                                                                  const int32_t* __restrict__ yrp,
                                                                  const int32_t* __restrict__ yci,
                                                                  const double* __restrict__ yva,
                                                                  const int32_t* __restrict__ crp, int32_t* cci,
                                                                  double* cva) {
  constexpr int kSW = waves_for(LG);
  __shared__ int keys[kSW][1 << LG];
  __shared__ double vals[kSW][1 << LG];
  __shared__ int count[kSW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* kt = keys[wv];
  double* vt = vals[wv];
  for (int i = blockIdx.x * kSW + wv; i < m; i += gridDim.x * kSW) {
    const int c0 = crp[i], c1 = crp[i + 1];
    if (c1 == c0) continue;  // empty row (or one the symbolic pass rejected)
    int bound;
    const int lg = table_lg<LG>(xrp, xci, 0x7fffffff, yrp, i, &bound);
    const int size = 1 << lg;
    for (int t = lane; t < size; t += 64) { kt[t] = -1; vt[t] = 0.0; }
    if (lane == 0) count[wv] = 0;
    wave_sync();
    for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
      const int j = xci[e];
      const double x = xva[e];
      for (int f = yrp[j] + lane; f < yrp[j + 1]; f += 64) {
        const int h = hash_insert(kt, &count[wv], yci[f], lg, bound);
        if (h >= 0) atomicAdd(&vt[h], x * yva[f]);
      }
    }
    wave_sync();
    // compact the occupied slots in place (a slot moves only to an index at
    // or below its own, after the whole run of 64 slots has been read)
    int base = 0;
    for (int t0 = 0; t0 < size; t0 += 64) {
      const int key = kt[t0 + lane];
      const double val = vt[t0 + lane];
      const bool occ = key >= 0;
      const uint64_t mask = __ballot(occ);
      const int pos = base + __popcll(mask & ((1ull << lane) - 1));
      wave_sync();
      if (occ) { kt[pos] = key; vt[pos] = val; }
      base += __popcll(mask);
      wave_sync();
    }
    // every entry at its rank among the row's columns
    const int n = min(base, c1 - c0);
    for (int q = lane; q < n; q += 64) {
      const int key = kt[q];
      int rank = 0;
      for (int s2 = 0; s2 < n; ++s2) rank += kt[s2] < key ? 1 : 0;
      cci[c0 + rank] = key;
      cva[c0 + rank] = vt[q];
    }
    wave_sync();
  }
}

int sg_grid(int m, int waves, int cus) { return std::max(1, std::min((m + waves - 1) / waves, cus * 8)); }

template <int LG>
void launch_count_lg(int m, const int32_t* xrp, const int32_t* xci, int k, const int32_t* yrp, const int32_t* yci,
                     int ny, int32_t* cnt, int32_t* flags, int cus, hipStream_t s) {
  constexpr int W = waves_for(LG);
  hipLaunchKernelGGL(k_sg_count<LG>, dim3(sg_grid(m, W, cus)), dim3(64 * W), 0, s, m, xrp, xci, k, yrp, yci, ny, cnt,
                     flags);
}

template <int LG>
void launch_fill_lg(int m, const int32_t* xrp, const int32_t* xci, const double* xva, const int32_t* yrp,
                    const int32_t* yci, const double* yva, const int32_t* crp, int32_t* cci, double* cva, int cus,
                    hipStream_t s) {
  constexpr int W = waves_for(LG);
  hipLaunchKernelGGL(k_sg_fill<LG>, dim3(sg_grid(m, W, cus)), dim3(64 * W), 0, s, m, xrp, xci, xva, yrp, yci, yva,
                     crp, cci, cva);
}

}  // namespace

hipError_t launch_spgemm_count(int m, const int32_t* xrp, const int32_t* xci, int k, const int32_t* yrp,
                               const int32_t* yci, int ny, int32_t* cnt, int32_t* flags, int* lg_out, int cus,
                               hipStream_t s) {
  *lg_out = 6;
  if (m <= 0) return hipSuccess;
  // the table size: twice the largest product count, as a power of two
  hipLaunchKernelGGL(k_sg_maxprod, dim3(std::max(1, std::min((m + 255) / 256, cus * 8))), dim3(256), 0, s, m, xrp,
                     xci, k, yrp, flags + 2);
  int32_t maxprod = 0;
  hipError_t e = hipMemcpyAsync(&maxprod, flags + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  int lg = 6;
  while (lg < kLgH && (1ll << lg) < 2ll * maxprod) ++lg;
  *lg_out = lg;
  switch (lg) {
    case 6: launch_count_lg<6>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
    case 7: launch_count_lg<7>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
    case 8: launch_count_lg<8>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
    case 9: launch_count_lg<9>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
    case 10: launch_count_lg<10>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
    default: launch_count_lg<11>(m, xrp, xci, k, yrp, yci, ny, cnt, flags, cus, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_spgemm_fill(int m, const int32_t* xrp, const int32_t* xci, const double* xva, const int32_t* yrp,
                              const int32_t* yci, const double* yva, const int32_t* crp, int32_t* cci, double* cva,
                              int lg, int cus, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  switch (lg) {
    case 6: launch_fill_lg<6>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
    case 7: launch_fill_lg<7>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
    case 8: launch_fill_lg<8>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
    case 9: launch_fill_lg<9>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
    case 10: launch_fill_lg<10>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
    default: launch_fill_lg<11>(m, xrp, xci, xva, yrp, yci, yva, crp, cci, cva, cus, s); break;
  }
  return hipGetLastError();
}

}  // namespace clair
