// k_constraints.hip -- k > 1 constraint vectors (Section 2.3 allows a block
// of constraint vectors; with k of them Section 3.1's Q holds k rows per
// F-point and Q Q^T is block diagonal with k x k blocks).
//
// Applied to an R built without constraints: for each F-column j with
// contributing rows I_j, G_j = sum_i B_i B_i^T and r_j = sum_i z_ij B_i - B_j,
// lambda_j = pinv(G_j) r_j, then z_ij -= B_i^T lambda_j: the Euclidean
// projection onto {R^T B_c = B}.  Three passes: sums (one thread per row of
// R, FP64 atomics into the column's packed Gram matrix and right-hand side),
// a k x k pseudo-inverse solve per column (one thread each: Jacobi
// eigen-decomposition in registers, eigenvalues at or below rcond times the
// largest dropped), the update (one thread per row).  B is n x k, row-major;
// k <= 4.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kKT = 256;
constexpr int kKMax = 4;
constexpr int kPack = kKMax * (kKMax + 1) / 2;

__device__ __forceinline__ int packed(int a, int b) {  // a <= b, row-major upper triangle
  return a * kKMax - a * (a - 1) / 2 + (b - a);
}

// the C-point of row q (its only entry in a C-column); -1 with *bad set when
// an index lies outside [0, n)
__device__ __forceinline__ int row_cpoint(int n, const int32_t* rp, const int32_t* ci, const int8_t* cf, int q,
                                          unsigned long long* bad) {
  int i = -1;
  for (int e = rp[q]; e < rp[q + 1]; ++e) {
    const int j = ci[e];
    if (j < 0 || j >= n) {
      atomicAdd(bad, 1ull);
      return -1;
    }
    if (cf[j] != 0) i = j;
  }
  return i;
}

__global__ void k_pk_sums(int n, int n_c, int k, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ va, const int8_t* __restrict__ cf, const double* __restrict__ B,
                          double* G, double* r, int32_t* cnt, unsigned long long* bad) {
  for (int q = blockIdx.x * kKT + threadIdx.x; q < n_c; q += gridDim.x * kKT) {
    const int i = row_cpoint(n, rp, ci, cf, q, bad);
    if (i < 0) continue;
    double bi[kKMax];
    for (int t = 0; t < kKMax; ++t) bi[t] = t < k ? B[(int64_t)i * k + t] : 0.0;
    for (int e = rp[q]; e < rp[q + 1]; ++e) {
      const int j = ci[e];
      if (cf[j] != 0) continue;
      atomicAdd(&cnt[j], 1);
      const double z = va[e];
      for (int a = 0; a < k; ++a) {
        unsafeAtomicAdd(&r[(int64_t)j * kKMax + a], z * bi[a]);
        for (int b = a; b < k; ++b) unsafeAtomicAdd(&G[(int64_t)j * kPack + packed(a, b)], bi[a] * bi[b]);
      }
    }
  }
}

// lambda_j = pinv(G_j) (r_j - B_j) in place of r_j; counts the columns no row reaches
__global__ void k_pk_solve(int n, int k, double rcond, const int8_t* __restrict__ cf, const double* __restrict__ B,
                           const double* __restrict__ G, double* r, const int32_t* __restrict__ cnt,
                           unsigned long long* uncovered) {
  for (int j = blockIdx.x * kKT + threadIdx.x; j < n; j += gridDim.x * kKT) {
    if (cf[j] != 0) continue;
    if (cnt[j] == 0) {
      atomicAdd(uncovered, 1ull);
      continue;
    }
    double a[kKMax][kKMax], v[kKMax][kKMax], rhs[kKMax];
    for (int p = 0; p < kKMax; ++p) {
      rhs[p] = p < k ? r[(int64_t)j * kKMax + p] - B[(int64_t)j * k + p] : 0.0;
      for (int q = 0; q < kKMax; ++q) {
        a[p][q] = (p < k && q < k) ? G[(int64_t)j * kPack + (p <= q ? packed(p, q) : packed(q, p))] : 0.0;
        v[p][q] = p == q ? 1.0 : 0.0;
      }
    }
    // cyclic Jacobi: rotate (p, q) pairs until the off-diagonal part is negligible
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0, on = 0.0;
      for (int p = 0; p < k; ++p) {
        on += a[p][p] * a[p][p];
        for (int q = p + 1; q < k; ++q) off += a[p][q] * a[p][q];
      }
      if (!(off > 1e-40 * on)) break;
      for (int p = 0; p < k; ++p) {
        for (int q = p + 1; q < k; ++q) {
          if (a[p][q] == 0.0) continue;
          const double h = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
          const double t = copysign(1.0, h) / (fabs(h) + sqrt(h * h + 1.0));
          const double c = rsqrt(t * t + 1.0), s = t * c;
          for (int m = 0; m < kKMax; ++m) {
            const double x = a[m][p], y = a[m][q];
            a[m][p] = c * x - s * y;
            a[m][q] = s * x + c * y;
          }
          for (int m = 0; m < kKMax; ++m) {
            const double x = a[p][m], y = a[q][m];
            a[p][m] = c * x - s * y;
            a[q][m] = s * x + c * y;
          }
          for (int m = 0; m < kKMax; ++m) {
            const double x = v[m][p], y = v[m][q];
            v[m][p] = c * x - s * y;
            v[m][q] = s * x + c * y;
          }
        }
      }
    }
    double wmax = 0.0;
    for (int p = 0; p < k; ++p) wmax = fmax(wmax, fabs(a[p][p]));
    double lam[kKMax] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m < k; ++m) {
      const double wm = a[m][m];
      if (!(fabs(wm) > rcond * wmax)) continue;
      double proj = 0.0;
      for (int p = 0; p < k; ++p) proj += v[p][m] * rhs[p];
      for (int p = 0; p < k; ++p) lam[p] += v[p][m] * proj / wm;
    }
    for (int p = 0; p < k; ++p) r[(int64_t)j * kKMax + p] = lam[p];
  }
}

__global__ void k_pk_apply(int n, int n_c, int k, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           double* va, const int8_t* __restrict__ cf, const double* __restrict__ B,
                           const double* __restrict__ lam, const int32_t* __restrict__ cnt, unsigned long long* bad) {
  for (int q = blockIdx.x * kKT + threadIdx.x; q < n_c; q += gridDim.x * kKT) {
    const int i = row_cpoint(n, rp, ci, cf, q, bad);
    if (i < 0) continue;
    for (int e = rp[q]; e < rp[q + 1]; ++e) {
      const int j = ci[e];
      if (cf[j] != 0 || cnt[j] == 0) continue;
      double dz = 0.0;
      for (int t = 0; t < k; ++t) dz += B[(int64_t)i * k + t] * lam[(int64_t)j * kKMax + t];
      va[e] -= dz;
    }
  }
}

int kgrid(int m, int cus) { return std::max(1, std::min((m + kKT - 1) / kKT, cus * 8)); }

}  // namespace

size_t constraint_scratch_bytes(int n) {
  return (size_t)n * (sizeof(double) * (kPack + kKMax) + sizeof(int32_t)) + 64;
}

hipError_t launch_project_k(int n, int n_c, const int32_t* rp, const int32_t* ci, double* va, const int8_t* cf,
                            const double* B, int k, double rcond, void* scratch, unsigned long long* counters,
                            int cus, hipStream_t s) {
  unsigned long long* uncovered = counters;
  unsigned long long* bad = counters + 1;
  double* G = static_cast<double*>(scratch);
  double* r = G + (size_t)n * kPack;
  int32_t* cnt = reinterpret_cast<int32_t*>(r + (size_t)n * kKMax);
  hipError_t e = hipMemsetAsync(scratch, 0, (size_t)n * (sizeof(double) * (kPack + kKMax) + sizeof(int32_t)), s);
  if (e != hipSuccess) return e;
  if (n_c > 0) hipLaunchKernelGGL(k_pk_sums, dim3(kgrid(n_c, cus)), dim3(kKT), 0, s, n, n_c, k, rp, ci, va, cf, B, G, r, cnt,
                                bad);
  if (n > 0) hipLaunchKernelGGL(k_pk_solve, dim3(kgrid(n, cus)), dim3(kKT), 0, s, n, k, rcond, cf, B, G, r, cnt, uncovered);
  if (n_c > 0) hipLaunchKernelGGL(k_pk_apply, dim3(kgrid(n_c, cus)), dim3(kKT), 0, s, n, n_c, k, rp, ci, va, cf, B, r, cnt,
                                 bad);
  return hipGetLastError();
}

}  // namespace clair
