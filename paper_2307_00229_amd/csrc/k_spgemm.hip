// k_spgemm.hip -- sparse product C = X Y on the device (FP64 values, int32
// CSR), for the Galerkin coarse operator A_c = R A P (Section 1: the coarse
// level of the hierarchy; Section 4.2 forms P and R separately).
//
// A group of lanes per output row (16 for short rows, else a wavefront), one
// lane per entry x_ij of X's row (that lane walks row j of Y).  The row's products x_ij y_jc are gathered
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

// Table size for a row of `prod` products: the smallest power of two
// >= max(64, 2 * prod), capped at 2^LG; *bound = the keys it may hold (below
// the cap a row never reaches it: it has at most half as many columns as
// slots)
template <int LG>
__device__ __forceinline__ int table_lg(long long prod, int* bound) {
  int lg = 6;
  while (lg < LG && (1ll << lg) < 2 * prod) ++lg;
  *bound = (lg == kLgH) ? kSpgemmMaxRow : (1 << lg);
  return lg;
}

// largest number of products of a row (indices out of range skipped; the
// count pass reports them), into *maxprod
__global__ void k_sg_maxprod(int m, const int32_t* __restrict__ xrp, const int32_t* __restrict__ xci, int k,
                             const int32_t* __restrict__ yrp, int32_t* maxprod) {
  int best = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    long long prod = 0;
    const int x1 = xrp[i + 1];
    for (int e0 = xrp[i]; e0 < x1; e0 += 8) {  // eight entries' loads in flight together
      int j[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) j[t] = e0 + t < x1 ? xci[e0 + t] : -1;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if ((unsigned)j[t] < (unsigned)k) prod += yrp[j[t] + 1] - yrp[j[t]];
    }
    best = max(best, (int)min(prod, (long long)(1 << 30)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0 && best > 0) atomicMax(maxprod, best);
}

// lanes per row: a quarter wavefront for tables of up to 128 slots (short
// rows), the whole wavefront above
constexpr int lanes_for(int LG) { return LG <= 7 ? 16 : 64; }

// Symbolic pass: groups of GL lanes, one row each (lane t of a group takes X
// entries t, t + GL, ...; the first one's column and Y row bounds stay in
// registers); the wavefront's loop over its rows is uniform, so the ballots
// see every group
template <int LG>
__global__ __launch_bounds__(64 * waves_for(LG)) void k_sg_count(int m, const int32_t* __restrict__ xrp,
                                                                   const int32_t* __restrict__ xci, int k,
                                                                   const int32_t* __restrict__ yrp,
                                                                   const int32_t* __restrict__ yci, int ny,
                                                                   int32_t* cnt, int32_t* flags) {
  constexpr int kSW = waves_for(LG), GL = lanes_for(LG), GPW = 64 / GL, NG = kSW * GPW;
  constexpr uint64_t gmask = GL == 64 ? ~0ull : ((1ull << GL) - 1);
  __shared__ int keys[NG][1 << LG];
  __shared__ int count[NG];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / GL, tl = lane % GL, grp = wv * GPW + g;
  int* kt = keys[grp];
  for (int i0 = (blockIdx.x * kSW + wv) * GPW; i0 < m; i0 += gridDim.x * NG) {
    const int i = i0 + g;
    const bool live = i < m;
    const int x0 = live ? xrp[i] : 0, x1 = live ? xrp[i + 1] : 0;
    const bool mine = x0 + tl < x1;
    int j0 = -1, ya = 0, yb = 0;
    long long prod = 0;
    if (mine) {
      j0 = xci[x0 + tl];
      if ((unsigned)j0 < (unsigned)k) { ya = yrp[j0]; yb = yrp[j0 + 1]; prod = yb - ya; }
    }
    for (int e = x0 + GL + tl; e < x1; e += GL) {
      const int j = xci[e];
      if ((unsigned)j < (unsigned)k) prod += yrp[j + 1] - yrp[j];
    }
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) prod += __shfl_xor(prod, o, 64);
    int bound;
    const int lg = table_lg<LG>(prod, &bound);
    for (int t = tl; t < (1 << lg); t += GL) kt[t] = -1;
    if (tl == 0) count[grp] = 0;
    wave_sync();
    bool over = false, bad = false;
    if (mine) {
      if ((unsigned)j0 >= (unsigned)k) bad = true;
      for (int f = ya; f < yb; ++f) {
        const int c = yci[f];
        if ((unsigned)c >= (unsigned)ny) bad = true;
        else if (hash_insert(kt, &count[grp], c, lg, bound) < 0) over = true;
      }
    }
    for (int e = x0 + GL + tl; e < x1; e += GL) {
      const int j = xci[e];
      if ((unsigned)j >= (unsigned)k) { bad = true; continue; }
      for (int f = yrp[j]; f < yrp[j + 1]; ++f) {
        const int c = yci[f];
        if ((unsigned)c >= (unsigned)ny) bad = true;
        else if (hash_insert(kt, &count[grp], c, lg, bound) < 0) over = true;
      }
    }
    if (bad) atomicExch(&flags[1], 1);
    wave_sync();
    const int n = count[grp];
    const bool any_over = ((__ballot(over) >> (g * GL)) & gmask) != 0 || n > bound;
    if (live && tl == 0) {
      cnt[i] = any_over ? 0 : n;
      if (any_over) atomicExch(&flags[0], 1);
    }
    wave_sync();
  }
}

// Numeric pass, the same groups: products into the row's table, then the
// occupied slots compacted in place (a slot moves only to an index at or
// below its own, after the group has read the whole run of GL slots) and
// every entry written at its rank among the row's columns
template <int LG>
__global__ __launch_bounds__(64 * waves_for(LG)) void k_sg_fill(int m, const int32_t* __restrict__ xrp,
                                                                  const int32_t* __restrict__ xci,
                                                                  const double* __restrict__ xva,
                                                                  const int32_t* __restrict__ yrp,
                                                                  const int32_t* __restrict__ yci,
                                                                  const double* __restrict__ yva,
                                                                  const int32_t* __restrict__ crp, int32_t* cci,
                                                                  double* cva) {
  constexpr int kSW = waves_for(LG), GL = lanes_for(LG), GPW = 64 / GL, NG = kSW * GPW;
  constexpr uint64_t gmask = GL == 64 ? ~0ull : ((1ull << GL) - 1);
  __shared__ int keys[NG][1 << LG];
  __shared__ double vals[NG][1 << LG];
  __shared__ int count[NG];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / GL, tl = lane % GL, grp = wv * GPW + g;
  int* kt = keys[grp];
  double* vt = vals[grp];
  for (int i0 = (blockIdx.x * kSW + wv) * GPW; i0 < m; i0 += gridDim.x * NG) {
    const int i = i0 + g;
    const int c0 = i < m ? crp[i] : 0, c1 = i < m ? crp[i + 1] : 0;
    const bool act = c1 > c0;  // empty rows, and rows the symbolic pass rejected, are skipped
    const int x0 = act ? xrp[i] : 0, x1 = act ? xrp[i + 1] : 0;
    const bool mine = x0 + tl < x1;
    int ya = 0, yb = 0;
    double xv = 0.0;
    if (mine) {
      const int j = xci[x0 + tl];
      xv = xva[x0 + tl];
      ya = yrp[j];
      yb = yrp[j + 1];
    }
    long long prod = yb - ya;
    for (int e = x0 + GL + tl; e < x1; e += GL) {
      const int j = xci[e];
      prod += yrp[j + 1] - yrp[j];
    }
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) prod += __shfl_xor(prod, o, 64);
    int bound;
    const int lg = table_lg<LG>(prod, &bound);
    const int size = act ? 1 << lg : 0;
    for (int t = tl; t < size; t += GL) { kt[t] = -1; vt[t] = 0.0; }
    if (tl == 0) count[grp] = 0;
    wave_sync();
    for (int f = ya; f < yb; ++f) {
      const int h = hash_insert(kt, &count[grp], yci[f], lg, bound);
      if (h >= 0) atomicAdd(&vt[h], xv * yva[f]);
    }
    for (int e = x0 + GL + tl; e < x1; e += GL) {
      const int j = xci[e];
      const double x = xva[e];
      for (int f = yrp[j]; f < yrp[j + 1]; ++f) {
        const int h = hash_insert(kt, &count[grp], yci[f], lg, bound);
        if (h >= 0) atomicAdd(&vt[h], x * yva[f]);
      }
    }
    wave_sync();
    int base = 0;
    for (int t0 = 0; t0 < size; t0 += GL) {
      const int key = kt[t0 + tl];
      const double val = vt[t0 + tl];
      const bool occ = key >= 0;
      const uint64_t bits = (__ballot(occ) >> (g * GL)) & gmask;
      const int pos = base + __popcll(bits & ((1ull << tl) - 1));
      wave_sync();
      if (occ) { kt[pos] = key; vt[pos] = val; }
      base += __popcll(bits);
      wave_sync();
    }
    const int n = min(base, c1 - c0);
    for (int q = tl; q < n; q += GL) {
      const int key = kt[q];
      int rank = 0;
      for (int s2 = 0; s2 < n; ++s2) rank += kt[s2] < key ? 1 : 0;
      cci[c0 + rank] = key;
      cva[c0 + rank] = vt[q];
    }
    wave_sync();
  }
}

// workgroups for m rows at `rows` rows per workgroup
int sg_grid(int m, int rows, int cus) { return std::max(1, std::min((m + rows - 1) / rows, cus * 8)); }

template <int LG>
void launch_count_lg(int m, const int32_t* xrp, const int32_t* xci, int k, const int32_t* yrp, const int32_t* yci,
                     int ny, int32_t* cnt, int32_t* flags, int cus, hipStream_t s) {
  constexpr int W = waves_for(LG);
  hipLaunchKernelGGL(k_sg_count<LG>, dim3(sg_grid(m, W * (64 / lanes_for(LG)), cus)), dim3(64 * W), 0, s, m, xrp,
                     xci, k, yrp, yci, ny, cnt, flags);
}

template <int LG>
void launch_fill_lg(int m, const int32_t* xrp, const int32_t* xci, const double* xva, const int32_t* yrp,
                    const int32_t* yci, const double* yva, const int32_t* crp, int32_t* cci, double* cva, int cus,
                    hipStream_t s) {
  constexpr int W = waves_for(LG);
  hipLaunchKernelGGL(k_sg_fill<LG>, dim3(sg_grid(m, W * (64 / lanes_for(LG)), cus)), dim3(64 * W), 0, s, m, xrp,
                     xci, xva, yrp, yci, yva, crp, cci, cva);
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
