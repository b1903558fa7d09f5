// k_smooth.hip -- smoothing of the constraint vector B (Section 4: B = 1 is
// pre-smoothed on every level with CFF-weighted Jacobi: per iteration one
// weighted Jacobi sweep on the C-points, then two on the F-points, for the
// homogeneous system M x = 0, M = A or A^T).
//
// A sweep on the points with cf == which reads the old vector x and writes
// y: y_i = x_i - omega (M x)_i / m_ii there, y_i = x_i elsewhere; one thread
// per row of M (the caller passes A^T's rows for M = A^T).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kST = 256;

__global__ void k_jacobi_sweep(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const double* __restrict__ va, const int8_t* __restrict__ cf, int which_c,
                               double omega, const double* __restrict__ x, double* __restrict__ y, int32_t* flag) {
  for (int i = blockIdx.x * kST + threadIdx.x; i < n; i += gridDim.x * kST) {
    if ((cf[i] != 0) != (which_c != 0)) {
      y[i] = x[i];
      continue;
    }
    double mx = 0.0, d = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int c = ci[e];
      if ((unsigned)c >= (unsigned)n) { atomicExch(flag, 2); continue; }
      mx += va[e] * x[c];
      if (c == i) d = va[e];
    }
    if (d == 0.0) {
      atomicMax(flag, 1);
      y[i] = x[i];
    } else {
      y[i] = x[i] - omega * mx / d;
    }
  }
}

}  // namespace

hipError_t launch_jacobi_sweep(int n, const int32_t* rp, const int32_t* ci, const double* va, const int8_t* cf,
                               int which_c, double omega, const double* x, double* y, int32_t* flag, int cus,
                               hipStream_t s) {
  if (n > 0) {
    const int blocks = std::max(1, std::min((n + kST - 1) / kST, cus * 8));
    hipLaunchKernelGGL(k_jacobi_sweep, dim3(blocks), dim3(kST), 0, s, n, rp, ci, va, cf, which_c, omega, x, y, flag);
  }
  return hipGetLastError();
}

}  // namespace clair
