// k_constraints.hip -- k > 1 constraint vectors (Section 2.3 allows a block
// of constraint vectors; with k of them Section 3.1's Q holds k rows per
// F-point and Q Q^T is block diagonal with k x k blocks).
//
// Applied to an R built without constraints: for each F-column j with
// contributing rows I_j, G_j = sum_i B_i B_i^T and r_j = sum_i z_ij B_i - B_j,
// lambda_j = pinv(G_j) r_j, then z_ij -= B_i^T lambda_j: the Euclidean
// projection onto {R^T B_c = B}.  Row q of R belongs to the q-th C-point.
//
// Gather form, no floating-point atomics: R is transposed on the device
// (columns sorted by row, so every column is summed in ascending row order),
// one thread per F-column forms G_j and r_j from its column of R^T and solves
// the k x k system in registers (Jacobi eigen-decomposition; eigenvalues at or
// below rcond times the largest are dropped), one thread per row of R applies
// the update.  The row -> C-point map comes from a scan of the C/F marker.
// B is n x k, row-major; k <= 8, a template parameter: up to 4 the k x k
// matrices of a thread stay in registers, from 5 to 8 they live in LDS (64
// threads per workgroup, thread index fastest, so the banks do not clash).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kKT = 256;

__global__ __launch_bounds__(kKT) void k_pk_marks(int n, int n_rows, const int8_t* __restrict__ cf, int32_t* flag,
                                                 int32_t* rowc) {
  for (int i = blockIdx.x * kKT + threadIdx.x; i < max(n, n_rows); i += gridDim.x * kKT) {
    if (i < n) flag[i] = cf[i] != 0;
    if (i < n_rows) rowc[i] = -1;
  }
}

// rowc[q] = the q-th C-point (rows beyond the C-points keep -1)
__global__ __launch_bounds__(kKT) void k_pk_rowc(int n, int n_rows, const int8_t* __restrict__ cf,
                                                const int32_t* __restrict__ pos, int32_t* rowc) {
  for (int i = blockIdx.x * kKT + threadIdx.x; i < n; i += gridDim.x * kKT)
    if (cf[i] != 0 && pos[i] < n_rows) rowc[pos[i]] = i;
}

// lambda_j = pinv(G_j) r_j for every F-column j, from column j of R^T
template <int K>
__global__ __launch_bounds__(kKT) void k_pk_solve(int n, int n_rows, double rcond, const int8_t* __restrict__ cf,
                                                 const double* __restrict__ B, const int32_t* __restrict__ trp,
                                                 const int32_t* __restrict__ tci, const double* __restrict__ tva,
                                                 const int32_t* __restrict__ rowc, double* lam,
                                                 unsigned long long* uncovered) {
  for (int j = blockIdx.x * kKT + threadIdx.x; j < n; j += gridDim.x * kKT) {
    if (cf[j] != 0) continue;
    double a[K][K], v[K][K], rhs[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      rhs[p] = 0.0;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        a[p][q] = 0.0;
        v[p][q] = p == q ? 1.0 : 0.0;
      }
    }
    int used = 0;
    for (int e = trp[j]; e < trp[j + 1]; ++e) {
      const int q = tci[e];
      const int i = (unsigned)q < (unsigned)n_rows ? rowc[q] : -1;
      if (i < 0) continue;
      ++used;
      const double z = tva[e];
      double bi[K];
#pragma unroll
      for (int t = 0; t < K; ++t) bi[t] = B[(int64_t)i * K + t];
#pragma unroll
      for (int p = 0; p < K; ++p) {
        rhs[p] += z * bi[p];
#pragma unroll
        for (int t = p; t < K; ++t) a[p][t] += bi[p] * bi[t];
      }
    }
    if (used == 0) {
      atomicAdd(uncovered, 1ull);
#pragma unroll
      for (int p = 0; p < K; ++p) lam[(int64_t)j * K + p] = 0.0;
      continue;
    }
#pragma unroll
    for (int p = 0; p < K; ++p) {
      rhs[p] -= B[(int64_t)j * K + p];
#pragma unroll
      for (int t = 0; t < p; ++t) a[p][t] = a[t][p];
    }
    // cyclic Jacobi; each rotation sets its pair to zero exactly, so the
    // off-diagonal part falls quadratically to nothing
    for (int sweep = 0; sweep < 30; ++sweep) {
      double off = 0.0, on = 0.0;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        on += a[p][p] * a[p][p];
#pragma unroll
        for (int q = p + 1; q < K; ++q) off += a[p][q] * a[p][q];
      }
      if (!(off > 1e-40 * on)) break;
#pragma unroll
      for (int p = 0; p < K; ++p) {
#pragma unroll
        for (int q = p + 1; q < K; ++q) {
          const double apq = a[p][q];
          const double h = (a[q][q] - a[p][p]) / (2.0 * (apq != 0.0 ? apq : 1.0));
          double t = copysign(1.0, h) / (fabs(h) + sqrt(h * h + 1.0));
          if (apq == 0.0) t = 0.0;
          const double c = rsqrt(t * t + 1.0), s = t * c;
#pragma unroll
          for (int m = 0; m < K; ++m) {
            const double x = a[m][p], y = a[m][q];
            a[m][p] = c * x - s * y;
            a[m][q] = s * x + c * y;
          }
#pragma unroll
          for (int m = 0; m < K; ++m) {
            const double x = a[p][m], y = a[q][m];
            a[p][m] = c * x - s * y;
            a[q][m] = s * x + c * y;
          }
          a[p][q] = 0.0;
          a[q][p] = 0.0;
#pragma unroll
          for (int m = 0; m < K; ++m) {
            const double x = v[m][p], y = v[m][q];
            v[m][p] = c * x - s * y;
            v[m][q] = s * x + c * y;
          }
        }
      }
    }
    double wmax = 0.0;
#pragma unroll
    for (int p = 0; p < K; ++p) wmax = fmax(wmax, fabs(a[p][p]));
    double l[K];
#pragma unroll
    for (int p = 0; p < K; ++p) l[p] = 0.0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double wm = a[m][m];
      if (!(fabs(wm) > rcond * wmax)) continue;
      double proj = 0.0;
#pragma unroll
      for (int p = 0; p < K; ++p) proj += v[p][m] * rhs[p];
#pragma unroll
      for (int p = 0; p < K; ++p) l[p] += v[p][m] * proj / wm;
    }
#pragma unroll
    for (int p = 0; p < K; ++p) lam[(int64_t)j * K + p] = l[p];
  }
}

// the same for K = 5..8 with the two K x K matrices of each thread in LDS
constexpr int kKL = 64;
template <int K>
__global__ __launch_bounds__(kKL) void k_pk_solve_lds(int n, int n_rows, double rcond, const int8_t* __restrict__ cf,
                                                     const double* __restrict__ B, const int32_t* __restrict__ trp,
                                                     const int32_t* __restrict__ tci, const double* __restrict__ tva,
                                                     const int32_t* __restrict__ rowc, double* lam,
                                                     unsigned long long* uncovered) {
  __shared__ double sa[K * K * kKL], sv[K * K * kKL];
  const int tid = threadIdx.x;
  auto a = [&](int p, int q) -> double& { return sa[(p * K + q) * kKL + tid]; };
  auto v = [&](int p, int q) -> double& { return sv[(p * K + q) * kKL + tid]; };
  for (int j = blockIdx.x * kKL + tid; j < n; j += gridDim.x * kKL) {
    if (cf[j] != 0) continue;
    double rhs[K];
    for (int p = 0; p < K; ++p) {
      rhs[p] = 0.0;
      for (int q = 0; q < K; ++q) {
        a(p, q) = 0.0;
        v(p, q) = p == q ? 1.0 : 0.0;
      }
    }
    int used = 0;
    for (int e = trp[j]; e < trp[j + 1]; ++e) {
      const int q = tci[e];
      const int i = (unsigned)q < (unsigned)n_rows ? rowc[q] : -1;
      if (i < 0) continue;
      ++used;
      const double z = tva[e];
      for (int p = 0; p < K; ++p) {
        const double bp = B[(int64_t)i * K + p];
        rhs[p] += z * bp;
        for (int t = p; t < K; ++t) a(p, t) += bp * B[(int64_t)i * K + t];
      }
    }
    if (used == 0) {
      atomicAdd(uncovered, 1ull);
      for (int p = 0; p < K; ++p) lam[(int64_t)j * K + p] = 0.0;
      continue;
    }
    for (int p = 0; p < K; ++p) {
      rhs[p] -= B[(int64_t)j * K + p];
      for (int t = 0; t < p; ++t) a(p, t) = a(t, p);
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
      double off = 0.0, on = 0.0;
      for (int p = 0; p < K; ++p) {
        on += a(p, p) * a(p, p);
        for (int q = p + 1; q < K; ++q) off += a(p, q) * a(p, q);
      }
      if (!(off > 1e-40 * on)) break;
      for (int p = 0; p < K; ++p) {
        for (int q = p + 1; q < K; ++q) {
          const double apq = a(p, q);
          const double h = (a(q, q) - a(p, p)) / (2.0 * (apq != 0.0 ? apq : 1.0));
          double t = copysign(1.0, h) / (fabs(h) + sqrt(h * h + 1.0));
          if (apq == 0.0) t = 0.0;
          const double c = rsqrt(t * t + 1.0), sn = t * c;
          for (int m = 0; m < K; ++m) {
            const double x = a(m, p), y = a(m, q);
            a(m, p) = c * x - sn * y;
            a(m, q) = sn * x + c * y;
          }
          for (int m = 0; m < K; ++m) {
            const double x = a(p, m), y = a(q, m);
            a(p, m) = c * x - sn * y;
            a(q, m) = sn * x + c * y;
          }
          a(p, q) = 0.0;
          a(q, p) = 0.0;
          for (int m = 0; m < K; ++m) {
            const double x = v(m, p), y = v(m, q);
            v(m, p) = c * x - sn * y;
            v(m, q) = sn * x + c * y;
          }
        }
      }
    }
    double wmax = 0.0;
    for (int p = 0; p < K; ++p) wmax = fmax(wmax, fabs(a(p, p)));
    double l[K];
    for (int p = 0; p < K; ++p) l[p] = 0.0;
    for (int m = 0; m < K; ++m) {
      const double wm = a(m, m);
      if (!(fabs(wm) > rcond * wmax)) continue;
      double proj = 0.0;
      for (int p = 0; p < K; ++p) proj += v(p, m) * rhs[p];
      for (int p = 0; p < K; ++p) l[p] += v(p, m) * proj / wm;
    }
    for (int p = 0; p < K; ++p) lam[(int64_t)j * K + p] = l[p];
  }
}

// z_ij -= B_i^T lambda_j on the F-entries of every row
template <int K>
__global__ __launch_bounds__(kKT) void k_pk_apply(int n, int n_rows, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, double* va,
                                                 const int8_t* __restrict__ cf, const double* __restrict__ B,
                                                 const int32_t* __restrict__ rowc, const double* __restrict__ lam) {
  for (int q = blockIdx.x * kKT + threadIdx.x; q < n_rows; q += gridDim.x * kKT) {
    const int i = rowc[q];
    if (i < 0) continue;
    double bi[K];
#pragma unroll
    for (int t = 0; t < K; ++t) bi[t] = B[(int64_t)i * K + t];
    for (int e = rp[q]; e < rp[q + 1]; ++e) {
      const int j = ci[e];
      if ((unsigned)j >= (unsigned)n || cf[j] != 0) continue;
      double dz = 0.0;
#pragma unroll
      for (int t = 0; t < K; ++t) dz += bi[t] * lam[(int64_t)j * K + t];
      va[e] -= dz;
    }
  }
}

int kgrid(int m, int cus) { return std::max(1, std::min((m + kKT - 1) / kKT, cus * 8)); }

template <int K>
void launch_k(int n, int n_rows, const int32_t* rp, const int32_t* ci, double* va, const int8_t* cf, const double* B,
              double rcond, const ProjectScratch& w, unsigned long long* uncovered, int cus, hipStream_t s) {
  if constexpr (K <= 4) {
    if (n > 0)
      hipLaunchKernelGGL(k_pk_solve<K>, dim3(kgrid(n, cus)), dim3(kKT), 0, s, n, n_rows, rcond, cf, B, w.trp, w.tci,
                         w.tva, w.rowc, w.lam, uncovered);
  } else {
    if (n > 0)
      hipLaunchKernelGGL(k_pk_solve_lds<K>, dim3(std::max(1, std::min((n + kKL - 1) / kKL, cus * 16))), dim3(kKL), 0,
                         s, n, n_rows, rcond, cf, B, w.trp, w.tci, w.tva, w.rowc, w.lam, uncovered);
  }
  if (n_rows > 0)
    hipLaunchKernelGGL(k_pk_apply<K>, dim3(kgrid(n_rows, cus)), dim3(kKT), 0, s, n, n_rows, rp, ci, va, cf, B, w.rowc,
                       w.lam);
}

}  // namespace

hipError_t launch_project_k(int n, int n_rows, const int32_t* rp, const int32_t* ci, double* va, const int8_t* cf,
                            const double* B, int k, double rcond, const ProjectScratch& w,
                            unsigned long long* uncovered, int cus, hipStream_t s) {
  if (n > 0 || n_rows > 0)
    hipLaunchKernelGGL(k_pk_marks, dim3(kgrid(std::max(n, n_rows), cus)), dim3(kKT), 0, s, n, n_rows, cf, w.flag,
                       w.rowc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n > 0) {
    e = launch_exclusive_scan(w.flag, n, w.pos, w.scan_sums, cus, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pk_rowc, dim3(kgrid(n, cus)), dim3(kKT), 0, s, n, n_rows, cf, w.pos, w.rowc);
  }
  e = launch_transpose(n_rows, n, rp, ci, va, w.trp, w.tci, w.tva, w.t_scratch, cus, s);
  if (e != hipSuccess) return e;
  switch (k) {
    case 1: launch_k<1>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 2: launch_k<2>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 3: launch_k<3>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 4: launch_k<4>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 5: launch_k<5>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 6: launch_k<6>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 7: launch_k<7>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    case 8: launch_k<8>(n, n_rows, rp, ci, va, cf, B, rcond, w, uncovered, cus, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clair
