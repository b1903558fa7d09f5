// k_plain.hip -- the plain FP64 per-row form of the restriction setup.
//
// The straightforward GPU formulation, kept as the baseline the mixed,
// batched path is measured against: one matrix at a time, one thread per
// C-row, one kernel per stage, FP64 everywhere, local blocks in global
// scratch, Gaussian elimination with partial pivoting.  Stages:
//   C-point count per block -> scan -> C list -> |N(i)| per row -> scan ->
//   column indices -> gather + solve -> projection sums -> projection.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kPT = 256;
constexpr int kPlainCap = 64;  // neighbourhood capacity of one thread

enum { PF_STATUS = 0, PF_FIRST_BAD = 1, PF_MAX_BLOCK = 2, PF_UNCOVERED = 3 };

__device__ void pflag(int32_t* flags, int code, int row) {
  atomicCAS(&flags[PF_STATUS], 0, code);
  atomicMin(&flags[PF_FIRST_BAD], row);
}

// breadth-first search into a private array; returns |N(i)| (sorted) or -1.
// With p.literal the pattern of S^{ell-1} T is taken literally: from the
// second step on C-points may be interior vertices (those reached before the
// last step wait in the array with the F-points, counting against its
// capacity, and are dropped at the end), and the second step also expands i
// itself (T's identity part).
__device__ int plain_bfs(const PlainWork& p, int i, int* N) {
  int s = 0, lo = 0, hi = 0;
  for (int depth = 1; depth <= p.ell; ++depth) {
    const int start = s;
    const bool lit = p.literal && depth >= 2;
    const int ulo = (depth == 1) ? 0 : (lit && depth == 2 ? lo - 1 : lo);
    const int uhi = (depth == 1) ? 1 : hi;
    for (int t = ulo; t < uhi; ++t) {
      const int u = (depth == 1 || t < lo) ? i : N[t];
      for (int e = p.grp[u]; e < p.grp[u + 1]; ++e) {  // the search graph: A or a strength matrix
        const int k = p.gci[e];
        if (k == u || k == i || (unsigned)k >= (unsigned)p.n || p.gva[e] == 0.0) continue;
        if (p.cf[k] != 0 && !(lit && depth < p.ell)) continue;  // a C-point is kept only to be expanded
        if (p.theta != 0.0 && !(fabs(p.gva[e]) >= p.theta * p.cmax[k])) continue;  // strength of A^T
        bool seen = false;
        for (int q = 0; q < s && !seen; ++q) seen = (N[q] == k);
        if (seen) continue;
        if (s == kPlainCap) return -1;
        N[s++] = k;
      }
    }
    lo = start;
    hi = s;
    // literal: the second step also expands i itself (T's identity part), so
    // an empty first level does not end the search
    if (lo == hi && !(p.literal && depth == 1)) break;
  }
  if (p.literal) {  // C-points were interior vertices only
    int m = 0;
    for (int a = 0; a < s; ++a)
      if (p.cf[N[a]] == 0) N[m++] = N[a];
    s = m;
  }
  for (int a = 1; a < s; ++a) {  // insertion sort
    const int v = N[a];
    int b = a - 1;
    while (b >= 0 && N[b] > v) { N[b + 1] = N[b]; --b; }
    N[b + 1] = v;
  }
  return s;
}

// cmax[v] = max over w != v of |a_wv| (bit patterns of non-negative doubles
// order like their values)
__global__ void k_p_colmax_clear(PlainWork p) {
  const int j = blockIdx.x * kPT + threadIdx.x;
  if (j < p.n) p.cmax[j] = 0.0;
}

__global__ void k_p_colmax(PlainWork p) {
  const int u = blockIdx.x * kPT + threadIdx.x;
  if (u >= p.n) return;
  for (int e = p.grp[u]; e < p.grp[u + 1]; ++e) {
    const int v = p.gci[e];
    if (v != u && (unsigned)v < (unsigned)p.n)
      atomicMax(reinterpret_cast<unsigned long long*>(p.cmax + v),
                          (unsigned long long)__double_as_longlong(fabs(p.gva[e])));
  }
}

__global__ void k_p_count_c(PlainWork p) {
  __shared__ int sh[kPT];
  const int j = blockIdx.x * kPT + threadIdx.x;
  sh[threadIdx.x] = (j < p.n && p.cf[j] != 0) ? 1 : 0;
  __syncthreads();
  for (int o = kPT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.blk_cnt[blockIdx.x] = sh[0];
}

// single-workgroup exclusive scan of a[0..n), a[n] = total
__global__ __launch_bounds__(1024) void k_p_scan_single(int32_t* a, int n) {
  __shared__ int sh[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b = 0; b < n; b += 1024) {
    const int j = b + threadIdx.x;
    const int v = (j < n) ? a[j] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (j < n) a[j] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) a[n] = carry;
}

__global__ void k_p_clist(PlainWork p) {
  __shared__ int sh[kPT];
  const int j = blockIdx.x * kPT + threadIdx.x;
  const int isc = (j < p.n && p.cf[j] != 0) ? 1 : 0;
  sh[threadIdx.x] = isc;
  __syncthreads();
  for (int o = 1; o < kPT; o <<= 1) {
    const int t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (isc) p.clist[p.blk_cnt[blockIdx.x] + sh[threadIdx.x] - 1] = j;
}

__global__ void k_p_sizes(PlainWork p, int n_c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  int s = 0;
  if (r < n_c) {
    int N[kPlainCap];
    const int i = p.clist[r];
    s = plain_bfs(p, i, N);
    if (s < 0) {
      pflag(p.flags, ST_UNSUPPORTED, i);
      s = 0;
    }
    p.sizes[r] = s + 1;
  }
  // largest block: reduced over the workgroup, one atomic per workgroup
  __shared__ int smax;
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  atomicMax(&smax, s);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&p.flags[PF_MAX_BLOCK], smax);
}

// three-phase scan of sizes[0..n) into R.row_ptr
__global__ void k_p_blocksum(const int32_t* a, int n, int32_t* sums) {
  __shared__ int sh[kPT];
  const int j = blockIdx.x * kPT + threadIdx.x;
  sh[threadIdx.x] = (j < n) ? a[j] : 0;
  __syncthreads();
  for (int o = kPT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

__global__ void k_p_apply(const int32_t* a, int n, const int32_t* sums, int nblk, int32_t* out) {
  __shared__ int sh[kPT];
  const int j = blockIdx.x * kPT + threadIdx.x;
  const int v = (j < n) ? a[j] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kPT; o <<= 1) {
    const int t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (j < n) out[j] = sums[blockIdx.x] + sh[threadIdx.x] - v;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nblk];
}

__global__ void k_p_fill(PlainWork p, int n_c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_c) return;
  int N[kPlainCap];
  const int i = p.clist[r];
  const int s = plain_bfs(p, i, N);
  if (s < 0 || s + 1 != p.Rrp[r + 1] - p.Rrp[r]) return;
  int pos = p.Rrp[r];
  bool ins = false;
  for (int q = 0; q < s; ++q) {
    if (!ins && i < N[q]) { p.Rci[pos++] = i; ins = true; }
    p.Rci[pos++] = N[q];
  }
  if (!ins) p.Rci[pos] = i;
}

// thread per row: FP64 block in global scratch, GEPP, solve
__global__ void k_p_solve(PlainWork p, int n_c, int smax) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_c) return;
  const int i = p.clist[r];
  const int e0 = p.Rrp[r], e1 = p.Rrp[r + 1];
  const int s = e1 - e0 - 1;
  double* K = p.kbuf + (int64_t)r * ((int64_t)smax * smax + smax);  // s x s, row stride s
  double* f = K + (int64_t)s * s;                                     // s entries
  if (s <= 0) {
    for (int e = e0; e < e1; ++e) p.Rva[e] = 1.0;
    return;
  }
  const int* Rc = p.Rci + e0;
  // position of fine column k in the row's F-list (the row holds i as well)
  auto fpos = [&](int k) -> int {
    int lo = 0, hi = s + 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Rc[mid] < k) lo = mid + 1; else hi = mid;
    }
    if (lo > s || Rc[lo] != k || k == i) return -1;
    return (k > i) ? lo - 1 : lo;
  };
  for (int t = 0; t < s * s; ++t) K[t] = 0.0;
  for (int q = 0; q < s; ++q) f[q] = 0.0;
  int p_ = 0;
  for (int e = 0; e <= s; ++e) {
    const int u = Rc[e];
    if (u == i) continue;
    for (int a = p.rp[u]; a < p.rp[u + 1]; ++a) {
      const int q = fpos(p.ci[a]);
      if (q >= 0) K[q * s + p_] = p.va[a];
    }
    ++p_;
  }
  for (int a = p.rp[i]; a < p.rp[i + 1]; ++a) {
    const int q = fpos(p.ci[a]);
    if (q >= 0) f[q] = -p.va[a];
  }
  double amax = 0.0;
  for (int t = 0; t < s * s; ++t) amax = fmax(amax, fabs(K[t]));
  const double tiny = 1e-14 * amax;
  bool sing = false;
  for (int k = 0; k < s && !sing; ++k) {
    int piv = k;
    double best = fabs(K[k * s + k]);
    for (int q = k + 1; q < s; ++q) {
      const double v = fabs(K[q * s + k]);
      if (v > best) { best = v; piv = q; }
    }
    if (!(best > tiny)) { sing = true; break; }
    if (piv != k) {
      for (int c = 0; c < s; ++c) { const double t = K[k * s + c]; K[k * s + c] = K[piv * s + c]; K[piv * s + c] = t; }
      const double t = f[k]; f[k] = f[piv]; f[piv] = t;
    }
    const double pv = K[k * s + k];
    for (int q = k + 1; q < s; ++q) {
      const double l = K[q * s + k] / pv;
      for (int c = k + 1; c < s; ++c) K[q * s + c] -= l * K[k * s + c];
      f[q] -= l * f[k];
    }
  }
  if (sing) {
    pflag(p.flags, ST_SINGULAR, i);
    for (int q = 0; q < s; ++q) f[q] = 0.0;
  } else {
    for (int k = s - 1; k >= 0; --k) {
      double acc = f[k];
      for (int c = k + 1; c < s; ++c) acc -= K[k * s + c] * f[c];
      f[k] = acc / K[k * s + k];
    }
  }
  int q = 0;
  for (int e = 0; e <= s; ++e) {
    if (Rc[e] == i) p.Rva[e0 + e] = 1.0;
    else p.Rva[e0 + e] = f[q++];
  }
}

__global__ void k_p_colsum(PlainWork p, int n_c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_c) return;
  const int i = p.clist[r];
  const double bi = p.B[i];
  for (int e = p.Rrp[r]; e < p.Rrp[r + 1]; ++e) {
    const int j = p.Rci[e];
    if (j == i) continue;
    unsafeAtomicAdd(&p.dsum[j], bi * bi);
    unsafeAtomicAdd(&p.rsum[j], p.Rva[e] * bi);
  }
}

__global__ void k_p_project(PlainWork p, int n_c) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_c) {
    const int i = p.clist[r];
    const double bi = p.B[i];
    for (int e = p.Rrp[r]; e < p.Rrp[r + 1]; ++e) {
      const int j = p.Rci[e];
      if (j == i) continue;
      const double dj = p.dsum[j];
      if (dj > 0.0) p.Rva[e] -= bi * (p.rsum[j] - p.B[j]) / dj;
    }
  }
}

__global__ void k_p_uncovered(PlainWork p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int u = (j < p.n && p.cf[j] == 0 && !(p.dsum[j] > 0.0)) ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) u += __shfl_xor(u, o, 64);
  if ((threadIdx.x & 63) == 0 && u) atomicAdd(&p.flags[PF_UNCOVERED], u);
}

inline int nblk(int n) { return (n + kPT - 1) / kPT; }

}  // namespace

hipError_t plain_colmax(const PlainWork& p, hipStream_t s) {
  if (p.n > 0 && p.theta != 0.0) {
    hipLaunchKernelGGL(k_p_colmax_clear, dim3(nblk(p.n)), dim3(kPT), 0, s, p);
    hipLaunchKernelGGL(k_p_colmax, dim3(nblk(p.n)), dim3(kPT), 0, s, p);
  }
  return hipGetLastError();
}
hipError_t plain_count_c(const PlainWork& p, hipStream_t s) {
  if (p.n > 0) hipLaunchKernelGGL(k_p_count_c, dim3(nblk(p.n)), dim3(kPT), 0, s, p);
  return hipGetLastError();
}
hipError_t plain_scan_blocks(int32_t* a, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_p_scan_single, dim3(1), dim3(1024), 0, s, a, n);
  return hipGetLastError();
}
hipError_t plain_clist(const PlainWork& p, hipStream_t s) {
  if (p.n > 0) hipLaunchKernelGGL(k_p_clist, dim3(nblk(p.n)), dim3(kPT), 0, s, p);
  return hipGetLastError();
}
hipError_t plain_sizes(const PlainWork& p, int n_c, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_p_sizes, dim3(nblk(n_c)), dim3(kPT), 0, s, p, n_c);
  return hipGetLastError();
}
hipError_t plain_scan(const PlainWork& p, int n_c, hipStream_t s) {
  const int nb = nblk(n_c);
  if (n_c > 0) hipLaunchKernelGGL(k_p_blocksum, dim3(nb), dim3(kPT), 0, s, p.sizes, n_c, p.scan_tmp);
  hipLaunchKernelGGL(k_p_scan_single, dim3(1), dim3(1024), 0, s, p.scan_tmp, nb);
  hipLaunchKernelGGL(k_p_apply, dim3(nb > 0 ? nb : 1), dim3(kPT), 0, s, p.sizes, n_c, p.scan_tmp, nb, p.Rrp);
  return hipGetLastError();
}
hipError_t plain_fill(const PlainWork& p, int n_c, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_p_fill, dim3(nblk(n_c)), dim3(kPT), 0, s, p, n_c);
  return hipGetLastError();
}
hipError_t plain_solve(const PlainWork& p, int n_c, int smax, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_p_solve, dim3(nblk(n_c)), dim3(kPT), 0, s, p, n_c, smax);
  return hipGetLastError();
}
hipError_t plain_colsum(const PlainWork& p, int n_c, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_p_colsum, dim3(nblk(n_c)), dim3(kPT), 0, s, p, n_c);
  return hipGetLastError();
}
hipError_t plain_project(const PlainWork& p, int n_c, hipStream_t s) {
  if (n_c > 0) hipLaunchKernelGGL(k_p_project, dim3(nblk(n_c)), dim3(kPT), 0, s, p, n_c);
  if (p.n > 0) hipLaunchKernelGGL(k_p_uncovered, dim3(nblk(p.n)), dim3(kPT), 0, s, p);
  return hipGetLastError();
}

}  // namespace clair
