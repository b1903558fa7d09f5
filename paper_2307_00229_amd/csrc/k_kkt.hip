// k_kkt.hip -- the exact constrained minimiser in the normal-equations metric
// (Section 3.1.1: minimise |a_fc + A_ff w| subject to Q w = B|_F, solved
// there by a KKT system whose (1,1) block is A_ff^T A_ff), for comparison
// with Algorithm 1's Euclidean projection.
//
// For restriction (Algorithm 1 on A^T) row r of R, C-point i, F-columns N,
// has the block K = A[N,N]^T, a = A[i,N]^T and the energy |a + K z|^2.  With
// Abar = K^T K, stationarity gives z = z0 - Abar^{-1} B_i lambda|_N (z0 the
// unconstrained minimiser, the exact l-AIR row) and lambda solves the sparse
// SPD system M lambda = Q z0 - B_F, M = Q Abar^{-1} Q^T, over the covered
// F-points.  Here: the Cholesky factor of every Abar (one thread per row,
// interleaved over rows so a wavefront's accesses are consecutive), then
// conjugate gradients on M applied matrix-free (gather lambda on N, two
// triangular solves, scatter B_i^2 times the result with FP64 atomics), then
// the correction of every row.  The CG scalars stay on the device: the step
// lengths are read from device memory, a one-thread kernel tests convergence
// and sets a flag after which every step kernel returns at once, so the host
// can queue several steps between reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kQT = 256;

int qgrid(int64_t m, int cus) { return (int)std::max<int64_t>(1, std::min<int64_t>((m + kQT - 1) / kQT, cus * 16)); }

__global__ __launch_bounds__(kQT) void k_q_marks(int n, int n_rows, const int8_t* __restrict__ cf, int32_t* flag,
                                                int32_t* rowc) {
  for (int i = blockIdx.x * kQT + threadIdx.x; i < max(n, n_rows); i += gridDim.x * kQT) {
    if (i < n) flag[i] = cf[i] != 0;
    if (i < n_rows) rowc[i] = -1;
  }
}

// rowc[q] = the q-th C-point
__global__ __launch_bounds__(kQT) void k_q_rowc(int n, int n_rows, const int8_t* __restrict__ cf,
                                               const int32_t* __restrict__ pos, int32_t* rowc) {
  for (int i = blockIdx.x * kQT + threadIdx.x; i < n; i += gridDim.x * kQT)
    if (cf[i] != 0 && pos[i] < n_rows) rowc[pos[i]] = i;
}

// position of the C-point's own entry in row [e0, e0 + len) (len if absent)
__device__ __forceinline__ int cpos(const int32_t* Rci, int e0, int len, int i) {
  int pc = 0;
  while (pc < len && Rci[e0 + pc] != i) ++pc;
  return pc;
}

// K of row r, then Abar = K^T K and its lower Cholesky factor in place of
// Abar; entry (a, b) of row r at [(a * smax + b) * n_rows + r].  bad[0] = 1
// for a row without its C-point entry or an index out of range, bad[1] = the
// smallest C-point whose Abar is not positive definite (INT32_MAX beforehand)
__global__ __launch_bounds__(kQT) void k_q_chol(int n, int n_rows, const int32_t* __restrict__ Rrp,
                                               const int32_t* __restrict__ Rci, const int32_t* __restrict__ rowc,
                                               const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                               const double* __restrict__ va, double* Kb, double* Lb, int smax,
                                               int32_t* bad) {
  const int64_t nr = n_rows;
  for (int r = blockIdx.x * kQT + threadIdx.x; r < n_rows; r += gridDim.x * kQT) {
    const int i = rowc[r];
    if (i < 0) continue;
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int pc = cpos(Rci, e0, len, i);
    if (pc == len || len - 1 > smax) {
      atomicExch(&bad[0], 1);
      continue;
    }
    const int s = len - 1;
    auto K = [&](int a, int b) -> double& { return Kb[((int64_t)a * smax + b) * nr + r]; };
    auto L = [&](int a, int b) -> double& { return Lb[((int64_t)a * smax + b) * nr + r]; };
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) K(a, b) = 0.0;
    bool oob = false;
    for (int p2 = 0; p2 < s; ++p2) {
      const int row = Rci[e0 + p2 + (p2 >= pc)];
      if ((unsigned)row >= (unsigned)n) { oob = true; break; }
      for (int t = rp[row]; t < rp[row + 1]; ++t) {
        const int col = ci[t];
        int lo = 0, hi = len;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Rci[e0 + mid] < col) lo = mid + 1; else hi = mid;
        }
        if (lo < len && Rci[e0 + lo] == col && col != i) K(col > i ? lo - 1 : lo, p2) += va[t];
      }
    }
    if (oob) {
      atomicExch(&bad[0], 1);
      continue;
    }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b <= a; ++b) {
        double acc = 0.0;
        for (int c = 0; c < s; ++c) acc += K(c, a) * K(c, b);
        L(a, b) = acc;
      }
    bool spd = true;
    for (int a = 0; a < s && spd; ++a) {
      double d = L(a, a);
      for (int c = 0; c < a; ++c) d -= L(a, c) * L(a, c);
      if (!(d > 0.0)) { spd = false; break; }
      const double la = sqrt(d);
      L(a, a) = la;
      for (int b = a + 1; b < s; ++b) {
        double v = L(b, a);
        for (int c = 0; c < a; ++c) v -= L(b, c) * L(a, c);
        L(b, a) = v / la;
      }
    }
    if (!spd) atomicMin(&bad[1], i);
  }
}

// x <- Abar^{-1} x with the row's Cholesky factor (x in T, interleaved)
__device__ __forceinline__ void chol_solve(const double* Lb, double* Tb, int smax, int64_t nr, int r, int s) {
  auto L = [&](int a, int b) { return Lb[((int64_t)a * smax + b) * nr + r]; };
  auto T = [&](int a) -> double& { return Tb[(int64_t)a * nr + r]; };
  for (int a = 0; a < s; ++a) {
    double v = T(a);
    for (int c = 0; c < a; ++c) v -= L(a, c) * T(c);
    T(a) = v / L(a, a);
  }
  for (int a = s - 1; a >= 0; --a) {
    double v = T(a);
    for (int c = a + 1; c < s; ++c) v -= L(c, a) * T(c);
    T(a) = v / L(a, a);
  }
}

// rhs_j += B_i z0_ij, cnt_j += 1 over the F-entries
__global__ __launch_bounds__(kQT) void k_q_rhs(int n, int n_rows, const int32_t* __restrict__ Rrp,
                                              const int32_t* __restrict__ Rci, const double* __restrict__ Rva,
                                              const int32_t* __restrict__ rowc, const double* __restrict__ B,
                                              double* rhs, int32_t* cnt) {
  for (int r = blockIdx.x * kQT + threadIdx.x; r < n_rows; r += gridDim.x * kQT) {
    const int i = rowc[r];
    if (i < 0) continue;
    const double bi = B[i];
    for (int e = Rrp[r]; e < Rrp[r + 1]; ++e) {
      const int j = Rci[e];
      if (j == i || (unsigned)j >= (unsigned)n) continue;  // an index out of range is reported by k_q_chol
      unsafeAtomicAdd(&rhs[j], bi * Rva[e]);
      atomicAdd(&cnt[j], 1);
    }
  }
}

// covered F-points: rhs_j -= B_j (and residual and direction start there);
// every other point holds 0
__global__ __launch_bounds__(kQT) void k_q_rhs_fin(int n, const int8_t* __restrict__ cf,
                                                  const double* __restrict__ B, const int32_t* __restrict__ cnt,
                                                  double* rhs, double* res, double* p, double* x, double* Ap) {
  for (int j = blockIdx.x * kQT + threadIdx.x; j < n; j += gridDim.x * kQT) {
    const double v = (cf[j] == 0 && cnt[j] > 0) ? rhs[j] - B[j] : 0.0;
    rhs[j] = v;
    res[j] = v;
    p[j] = v;
    x[j] = 0.0;
    Ap[j] = 0.0;
  }
}

// y += M p, M = sum over rows of B_i^2 Abar^{-1} on N (y zeroed beforehand)
__global__ __launch_bounds__(kQT) void k_q_matvec(int n_rows, const int32_t* __restrict__ Rrp,
                                                 const int32_t* __restrict__ Rci, const int32_t* __restrict__ rowc,
                                                 const double* __restrict__ Lb, int smax, double* Tb,
                                                 const double* __restrict__ B, const double* __restrict__ p,
                                                 double* y, const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t nr = n_rows;
  for (int r = blockIdx.x * kQT + threadIdx.x; r < n_rows; r += gridDim.x * kQT) {
    const int i = rowc[r];
    if (i < 0) continue;
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int pc = cpos(Rci, e0, len, i);
    const int s = len - 1;
    if (s <= 0 || pc == len) continue;
    for (int a = 0; a < s; ++a) Tb[(int64_t)a * nr + r] = p[Rci[e0 + a + (a >= pc)]];
    chol_solve(Lb, Tb, smax, nr, r, s);
    const double b2 = B[i] * B[i];
    for (int a = 0; a < s; ++a) unsafeAtomicAdd(&y[Rci[e0 + a + (a >= pc)]], b2 * Tb[(int64_t)a * nr + r]);
  }
}

// *out += x . y
__global__ __launch_bounds__(kQT) void k_q_dot(int n, const double* __restrict__ x, const double* __restrict__ y,
                                              double* out, const int32_t* __restrict__ done) {
  __shared__ double part[kQT / 64];
  if (done && *done) return;
  double acc = 0.0;
  for (int j = blockIdx.x * kQT + threadIdx.x; j < n; j += gridDim.x * kQT) acc += x[j] * y[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kQT / 64; ++w) t += part[w];
    unsafeAtomicAdd(out, t);
  }
}

// sc: [0] res.res, [1] p.Ap, [2] the new res.res, [3] the stop level,
// [4] beta; *done set once the step cannot or need not go on
// x += alpha p, res -= alpha Ap, and the new res.res into sc[2]
__global__ __launch_bounds__(kQT) void k_q_axpy(int n, double* sc, const double* __restrict__ p,
                                               const double* __restrict__ Ap, double* x, double* res, int32_t* done) {
  __shared__ double part[kQT / 64];
  if (*done) return;
  if (!(sc[1] > 0.0)) {  // breakdown (lambda is as good as it gets)
    if (blockIdx.x == 0 && threadIdx.x == 0) *done = 1;
    return;
  }
  const double alpha = sc[0] / sc[1];
  double acc = 0.0;
  for (int j = blockIdx.x * kQT + threadIdx.x; j < n; j += gridDim.x * kQT) {
    x[j] += alpha * p[j];
    const double r = res[j] - alpha * Ap[j];
    res[j] = r;
    acc += r * r;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kQT / 64; ++w) t += part[w];
    unsafeAtomicAdd(&sc[2], t);
  }
}

// one thread: convergence test, beta, the step count; clears [1] and [2] for
// the next step
__global__ void k_q_scalars(double* sc, int32_t* done, int32_t* steps) {
  if (*done) return;
  *steps += 1;
  if (!(sc[2] > sc[3])) {
    *done = 1;
    return;
  }
  sc[4] = sc[2] / sc[0];
  sc[0] = sc[2];
  sc[1] = 0.0;
  sc[2] = 0.0;
}

// p = res + beta p, and Ap cleared for the next step's product
__global__ __launch_bounds__(kQT) void k_q_dir(int n, const double* __restrict__ sc, const double* __restrict__ res,
                                              double* p, double* Ap, const int32_t* __restrict__ done) {
  if (*done) return;
  const double beta = sc[4];
  for (int j = blockIdx.x * kQT + threadIdx.x; j < n; j += gridDim.x * kQT) {
    p[j] = res[j] + beta * p[j];
    Ap[j] = 0.0;
  }
}

// z_ij -= B_i (Abar^{-1} lambda|_N)_j
__global__ __launch_bounds__(kQT) void k_q_apply(int n_rows, const int32_t* __restrict__ Rrp,
                                                const int32_t* __restrict__ Rci, double* Rva,
                                                const int32_t* __restrict__ rowc, const double* __restrict__ Lb,
                                                int smax, double* Tb, const double* __restrict__ B,
                                                const double* __restrict__ lam) {
  const int64_t nr = n_rows;
  for (int r = blockIdx.x * kQT + threadIdx.x; r < n_rows; r += gridDim.x * kQT) {
    const int i = rowc[r];
    if (i < 0) continue;
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int pc = cpos(Rci, e0, len, i);
    const int s = len - 1;
    if (s <= 0 || pc == len) continue;
    for (int a = 0; a < s; ++a) Tb[(int64_t)a * nr + r] = lam[Rci[e0 + a + (a >= pc)]];
    chol_solve(Lb, Tb, smax, nr, r, s);
    const double bi = B[i];
    for (int a = 0; a < s; ++a) Rva[e0 + a + (a >= pc)] -= bi * Tb[(int64_t)a * nr + r];
  }
}

}  // namespace

hipError_t launch_kkt_setup(const KktWork& w, hipStream_t s) {
  const int m = std::max(w.n, w.n_rows);
  if (m > 0)
    hipLaunchKernelGGL(k_q_marks, dim3(qgrid(m, w.cus)), dim3(kQT), 0, s, w.n, w.n_rows, w.cf, w.flag, w.rowc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (w.n > 0) {
    e = launch_exclusive_scan(w.flag, w.n, w.pos, w.scan_sums, w.cus, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_q_rowc, dim3(qgrid(w.n, w.cus)), dim3(kQT), 0, s, w.n, w.n_rows, w.cf, w.pos, w.rowc);
  }
  if (w.n_rows > 0) {
    hipLaunchKernelGGL(k_q_chol, dim3(qgrid(w.n_rows, w.cus)), dim3(kQT), 0, s, w.n, w.n_rows, w.Rrp, w.Rci, w.rowc,
                       w.rp, w.ci, w.va, w.K, w.L, w.smax, w.bad);
    hipLaunchKernelGGL(k_q_rhs, dim3(qgrid(w.n_rows, w.cus)), dim3(kQT), 0, s, w.n, w.n_rows, w.Rrp, w.Rci, w.Rva,
                       w.rowc, w.B, w.rhs, w.cnt);
  }
  if (w.n > 0)
    hipLaunchKernelGGL(k_q_rhs_fin, dim3(qgrid(w.n, w.cus)), dim3(kQT), 0, s, w.n, w.cf, w.B, w.cnt, w.rhs, w.res,
                       w.p, w.x, w.Ap);
  return hipGetLastError();
}

hipError_t launch_kkt_dot(const KktWork& w, const double* x, const double* y, double* out, hipStream_t s) {
  if (w.n > 0)
    hipLaunchKernelGGL(k_q_dot, dim3(std::max(1, std::min((w.n + kQT - 1) / kQT, w.cus))), dim3(kQT), 0, s, w.n, x,
                       y, out, w.done);  // one workgroup per CU: few atomics on the one sum
  return hipGetLastError();
}

hipError_t launch_kkt_step(const KktWork& w, hipStream_t s) {
  if (w.n <= 0) return hipSuccess;
  const int g = qgrid(w.n, w.cus);
  if (w.n_rows > 0)
    hipLaunchKernelGGL(k_q_matvec, dim3(qgrid(w.n_rows, w.cus)), dim3(kQT), 0, s, w.n_rows, w.Rrp, w.Rci, w.rowc,
                       w.L, w.smax, w.T, w.B, w.p, w.Ap, w.done);
  hipError_t e = launch_kkt_dot(w, w.p, w.Ap, w.sc + 1, s);
  if (e != hipSuccess) return e;
  // one workgroup per CU: few atomics on the residual's sum
  hipLaunchKernelGGL(k_q_axpy, dim3(std::max(1, std::min((w.n + kQT - 1) / kQT, w.cus))), dim3(kQT), 0, s, w.n, w.sc,
                     w.p, w.Ap, w.x, w.res, w.done);
  hipLaunchKernelGGL(k_q_scalars, dim3(1), dim3(1), 0, s, w.sc, w.done, w.steps);
  hipLaunchKernelGGL(k_q_dir, dim3(g), dim3(kQT), 0, s, w.n, w.sc, w.res, w.p, w.Ap, w.done);
  return hipGetLastError();
}

hipError_t launch_kkt_apply(const KktWork& w, hipStream_t s) {
  if (w.n_rows > 0)
    hipLaunchKernelGGL(k_q_apply, dim3(qgrid(w.n_rows, w.cus)), dim3(kQT), 0, s, w.n_rows, w.Rrp, w.Rci, w.Rva,
                       w.rowc, w.L, w.smax, w.T, w.B, w.x);
  return hipGetLastError();
}

}  // namespace clair
