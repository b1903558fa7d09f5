// k_approx.hip -- Algorithm 1 with the diagonal block inverse (Section 3.1.2:
// a block-diagonal approximate inverse of A_ff^{(*)}; the footnote of the
// comparison with root-node names the local diagonal inverse), run for a given
// number of iterations on a pattern built beforehand.
//
// One thread per entry of R (row q, C-point i = clist[q], column j):
//   start: -a_ij (the tentative operator), or with B the minimum-norm fit of
//          each F-column's constraint, z_ij = B_i B_j / d_j;
//   per iteration:
//     u_ij = -(R A)_ij / a_jj on the F-entries: column j of A is read from
//            A^T and each a_lj is paired with R's entry (q, l), found by a
//            binary search of row q (sorted; it holds the C-point's 1 too);
//            with B, s_j += u_ij B_i (FP64 atomics);
//     z_ij += u_ij - B_i s_j / d_j (the projection; Q Q^T is diagonal).
// The residual reads only the old R, so each iteration is one residual
// launch and one update launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kAT = 256;

int agrid(int64_t m, int cus) { return (int)std::max<int64_t>(1, std::min<int64_t>((m + kAT - 1) / kAT, cus * 16)); }

// diag[j] = a_jj (duplicates summed); erow[e] = q for the entries of row q of R
__global__ __launch_bounds__(kAT) void k_ap_prep(int n, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci, const double* __restrict__ va,
                                                double* diag, int n_c, const int32_t* __restrict__ Rrp,
                                                int32_t* erow) {
  for (int r = blockIdx.x * kAT + threadIdx.x; r < max(n, n_c); r += gridDim.x * kAT) {
    if (r < n) {
      double d = 0.0;
      for (int e = rp[r]; e < rp[r + 1]; ++e)
        if (ci[e] == r) d += va[e];
      diag[r] = d;
    }
    if (r < n_c)
      for (int e = Rrp[r]; e < Rrp[r + 1]; ++e) erow[e] = r;
  }
}

// tentative weights; column sums d_j = sum B_i^2 and entry counts; a zero
// diagonal on an F-column of the pattern reports the row's C-point
__global__ __launch_bounds__(kAT) void k_ap_start(int64_t nnz, const int32_t* __restrict__ erow,
                                                 const int32_t* __restrict__ clist, const int32_t* __restrict__ Rci,
                                                 double* Rva, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double* __restrict__ va,
                                                 const double* __restrict__ B, const double* __restrict__ diag,
                                                 double* d, int32_t* cnt, int32_t* bad_row) {
  for (int64_t e = blockIdx.x * (int64_t)kAT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kAT) {
    const int i = clist[erow[e]];
    const int j = Rci[e];
    if (j == i) {
      Rva[e] = 1.0;
      continue;
    }
    if (diag[j] == 0.0) atomicMin(bad_row, i);
    atomicAdd(&cnt[j], 1);
    if (B) {
      unsafeAtomicAdd(&d[j], B[i] * B[i]);
    } else {
      double a = 0.0;
      for (int t = rp[i]; t < rp[i + 1]; ++t)
        if (ci[t] == j) a += va[t];
      Rva[e] = -a;
    }
  }
}

// with B: the minimum-norm fit of every F-column's constraint
__global__ __launch_bounds__(kAT) void k_ap_fit(int64_t nnz, const int32_t* __restrict__ erow,
                                               const int32_t* __restrict__ clist, const int32_t* __restrict__ Rci,
                                               double* Rva, const double* __restrict__ B,
                                               const double* __restrict__ d) {
  for (int64_t e = blockIdx.x * (int64_t)kAT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kAT) {
    const int i = clist[erow[e]];
    const int j = Rci[e];
    if (j == i) continue;
    Rva[e] = d[j] > 0.0 ? B[i] * B[j] / d[j] : 0.0;
  }
}

__global__ __launch_bounds__(kAT) void k_ap_resid(int64_t nnz, const int32_t* __restrict__ erow,
                                                 const int32_t* __restrict__ clist, const int32_t* __restrict__ Rrp,
                                                 const int32_t* __restrict__ Rci, const double* __restrict__ Rva,
                                                 const int32_t* __restrict__ trp, const int32_t* __restrict__ tci,
                                                 const double* __restrict__ tva, const double* __restrict__ diag,
                                                 const double* __restrict__ B, double* u, double* sj) {
  for (int64_t e = blockIdx.x * (int64_t)kAT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kAT) {
    const int q = erow[e];
    const int i = clist[q];
    const int j = Rci[e];
    if (j == i) {
      u[e] = 0.0;
      continue;
    }
    const int r0 = Rrp[q], len = Rrp[q + 1] - r0;
    double acc = 0.0;
    for (int t = trp[j]; t < trp[j + 1]; ++t) {
      const int l = tci[t];  // a_lj, l a row of A
      int lo = 0, hi = len;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Rci[r0 + mid] < l) lo = mid + 1; else hi = mid;
      }
      if (lo < len && Rci[r0 + lo] == l) acc += Rva[r0 + lo] * tva[t];
    }
    const double x = -acc / diag[j];
    u[e] = x;
    if (B) unsafeAtomicAdd(&sj[j], x * B[i]);
  }
}

__global__ __launch_bounds__(kAT) void k_ap_update(int64_t nnz, const int32_t* __restrict__ erow,
                                                  const int32_t* __restrict__ clist, const int32_t* __restrict__ Rci,
                                                  double* Rva, const double* __restrict__ u,
                                                  const double* __restrict__ B, const double* __restrict__ d,
                                                  const double* __restrict__ sj) {
  for (int64_t e = blockIdx.x * (int64_t)kAT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kAT) {
    const int i = clist[erow[e]];
    const int j = Rci[e];
    if (j == i) continue;
    double x = u[e];
    if (B && d[j] > 0.0) x -= B[i] * sj[j] / d[j];
    Rva[e] += x;
  }
}

// F-points no row reaches
__global__ __launch_bounds__(kAT) void k_ap_uncovered(int n, const int8_t* __restrict__ cf,
                                                     const int32_t* __restrict__ cnt, unsigned long long* out) {
  for (int j = blockIdx.x * kAT + threadIdx.x; j < n; j += gridDim.x * kAT)
    if (cf[j] == 0 && cnt[j] == 0) atomicAdd(out, 1ull);
}

}  // namespace

hipError_t launch_diag_start(const DiagWork& w, hipStream_t s) {
  const int m = std::max(w.n, w.n_c);
  if (m > 0)
    hipLaunchKernelGGL(k_ap_prep, dim3(agrid(m, w.cus)), dim3(kAT), 0, s, w.n, w.rp, w.ci, w.va, w.diag, w.n_c,
                       w.Rrp, w.erow);
  if (w.nnz > 0) {
    hipLaunchKernelGGL(k_ap_start, dim3(agrid(w.nnz, w.cus)), dim3(kAT), 0, s, w.nnz, w.erow, w.clist, w.Rci, w.Rva,
                       w.rp, w.ci, w.va, w.B, w.diag, w.d, w.cnt, w.bad_row);
    if (w.B)
      hipLaunchKernelGGL(k_ap_fit, dim3(agrid(w.nnz, w.cus)), dim3(kAT), 0, s, w.nnz, w.erow, w.clist, w.Rci, w.Rva,
                         w.B, w.d);
  }
  if (w.n > 0)
    hipLaunchKernelGGL(k_ap_uncovered, dim3(agrid(w.n, w.cus)), dim3(kAT), 0, s, w.n, w.cf, w.cnt, w.uncovered);
  return hipGetLastError();
}

hipError_t launch_diag_iteration(const DiagWork& w, hipStream_t s) {
  if (w.nnz == 0) return hipSuccess;
  if (w.B) {
    hipError_t e = hipMemsetAsync(w.sj, 0, sizeof(double) * (size_t)std::max(1, w.n), s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ap_resid, dim3(agrid(w.nnz, w.cus)), dim3(kAT), 0, s, w.nnz, w.erow, w.clist, w.Rrp, w.Rci,
                     w.Rva, w.trp, w.tci, w.tva, w.diag, w.B, w.u, w.sj);
  hipLaunchKernelGGL(k_ap_update, dim3(agrid(w.nnz, w.cus)), dim3(kAT), 0, s, w.nnz, w.erow, w.clist, w.Rci, w.Rva,
                     w.u, w.B, w.d, w.sj);
  return hipGetLastError();
}

}  // namespace clair
