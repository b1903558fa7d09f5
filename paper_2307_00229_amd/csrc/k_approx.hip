// k_approx.hip -- Algorithm 1 with approximate block inverses (Section 3.1.2:
// a block-diagonal approximate inverse of A_ff^{(*)}, e.g. diagonal or ILU;
// the footnote of the comparison with root-node names the local diagonal
// inverse), run for a given number of iterations on a pattern built
// beforehand.  Three inverses: the diagonal of each block K_i = A[N,N]^T,
// its incomplete LU factorisation without fill (ILU(0)), or m steps of GMRES
// on the local system from zero.
//
// One thread per entry of R (row q, C-point i = clist[q], column j):
//   start: -a_ij (the tentative operator), or with B the minimum-norm fit of
//          each F-column's constraint, z_ij = B_i B_j / d_j;
//   per iteration:
//     rho_ij = -(R A)_ij on the F-entries: column j of A is read from A^T
//            and each a_lj is paired with R's entry (q, l), found by a binary
//            search of row q (sorted; it holds the C-point's 1 too);
//     u_i = Khat_i^{-1} rho_i: rho_ij / a_jj (diagonal, same kernel), the
//            two triangular solves with the row's ILU(0) factors, or GMRES
//            with the row's block (one thread per row, in place on the row's
//            entries);
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
    if (bad_row && diag[j] == 0.0) atomicMin(bad_row, i);
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
                                                 const double* __restrict__ B, double* u, double* sj, int scale) {
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
    if (scale) {  // the diagonal inverse
      const double x = -acc / diag[j];
      u[e] = x;
      if (B) unsafeAtomicAdd(&sj[j], x * B[i]);
    } else {
      u[e] = -acc;
    }
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

// ILU(0) of every row's block K = A[N,N]^T (N = the row's F-columns, in
// order), interleaved over rows so that the lanes of a wavefront touch
// consecutive addresses: K[a][b] of row r at fac[(a * smax + b) * n_c + r].
// Row-oriented elimination touching only pattern positions, unit lower
// factor: row a is eliminated against the final rows above it, and its
// pattern (a bit mask, s <= 64) is read just before, while it still holds K's
// values.  A zero pivot reports the row's C-point.
// (factor = 0: the block only, for GMRES)
__global__ __launch_bounds__(kAT) void k_ap_block(int n_c, const int32_t* __restrict__ Rrp,
                                                 const int32_t* __restrict__ Rci, const int32_t* __restrict__ clist,
                                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const double* __restrict__ va, double* fac, int smax, int factor,
                                                 int32_t* bad_row) {
  for (int r = blockIdx.x * kAT + threadIdx.x; r < n_c; r += gridDim.x * kAT) {
    const int i = clist[r];
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int s = len - 1;
    if (s <= 0) continue;
    auto K = [&](int a, int b) -> double& { return fac[((int64_t)a * smax + b) * n_c + r]; };
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) K(a, b) = 0.0;
    // F-entry p of the row is R entry e0 + p before the C-point, e0 + p + 1 after
    int pc = 0;
    while (pc < len && Rci[e0 + pc] != i) ++pc;
    for (int p2 = 0; p2 < s; ++p2) {
      const int row = Rci[e0 + p2 + (p2 >= pc ? 1 : 0)];
      for (int t = rp[row]; t < rp[row + 1]; ++t) {
        const int col = ci[t];
        int lo = 0, hi = len;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Rci[e0 + mid] < col) lo = mid + 1; else hi = mid;
        }
        if (lo < len && Rci[e0 + lo] == col && col != i) {
          const int q = col > i ? lo - 1 : lo;
          K(q, p2) += va[t];
        }
      }
    }
    if (!factor) continue;
    bool zero = false;
    for (int a = 0; a < s && !zero; ++a) {
      uint64_t ma = 0;
      for (int b = 0; b < s; ++b)
        if (K(a, b) != 0.0) ma |= 1ull << b;
      for (int b = 0; b < a; ++b) {
        if (!((ma >> b) & 1ull)) continue;
        const double mult = K(a, b) / K(b, b);
        K(a, b) = mult;
        for (int c = b + 1; c < s; ++c)
          if ((ma >> c) & 1ull) K(a, c) -= mult * K(b, c);
      }
      zero = K(a, a) == 0.0;
    }
    if (zero) atomicMin(bad_row, i);
  }
}

// u_i = (L U)^{-1} rho_i on the row's F-entries, in place; with B the column
// sums s_j += u_ij B_i
__global__ __launch_bounds__(kAT) void k_ap_ilu_solve(int n_c, const int32_t* __restrict__ Rrp,
                                                     const int32_t* __restrict__ Rci,
                                                     const int32_t* __restrict__ clist,
                                                     const double* __restrict__ fac, int smax,
                                                     const double* __restrict__ B, double* u, double* sj) {
  for (int r = blockIdx.x * kAT + threadIdx.x; r < n_c; r += gridDim.x * kAT) {
    const int i = clist[r];
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int s = len - 1;
    if (s <= 0) continue;
    // the C-point's position in the row; F-entry a is u[e0 + a + (a >= pc)]
    int pc = 0;
    while (pc < len && Rci[e0 + pc] != i) ++pc;
    double* x = u + e0;
    auto K = [&](int a, int b) { return fac[((int64_t)a * smax + b) * n_c + r]; };
    for (int a = 1; a < s; ++a) {
      double v = x[a + (a >= pc)];
      for (int b = 0; b < a; ++b) v -= K(a, b) * x[b + (b >= pc)];
      x[a + (a >= pc)] = v;
    }
    for (int a = s - 1; a >= 0; --a) {
      double v = x[a + (a >= pc)];
      for (int c = a + 1; c < s; ++c) v -= K(a, c) * x[c + (c >= pc)];
      x[a + (a >= pc)] = v / K(a, a);
    }
    if (B) {
      const double bi = B[i];
      for (int a = 0; a < s; ++a) {
        const int e = e0 + a + (a >= pc);
        unsafeAtomicAdd(&sj[Rci[e]], x[a + (a >= pc)] * bi);
      }
    }
  }
}

// GMRES(m) on the row's block from zero: u_i = the vector of the Krylov space
// span{rho, K rho, ..., K^{m-1} rho} with the least residual |rho - K u|
// (Arnoldi with modified Gram-Schmidt, Givens rotations; it stops when the
// new basis vector's norm is at most 1e-12 of K v_j's).  Basis V ((m + 1) x
// smax), Hessenberg H ((m + 1) x m), rotations and right-hand side g (3 (m +
// 1)) per row, interleaved over rows in gw; with B the column sums
// s_j += u_ij B_i.
__global__ __launch_bounds__(kAT) void k_ap_gmres(int n_c, const int32_t* __restrict__ Rrp,
                                                 const int32_t* __restrict__ Rci, const int32_t* __restrict__ clist,
                                                 const double* __restrict__ fac, int smax, int m, double* gw,
                                                 const double* __restrict__ B, double* u, double* sj) {
  const int64_t nc = n_c;
  double* Vb = gw;
  double* Hb = Vb + (int64_t)(m + 1) * smax * nc;
  double* cb = Hb + (int64_t)(m + 1) * m * nc;
  double* sb = cb + (int64_t)(m + 1) * nc;
  double* gb = sb + (int64_t)(m + 1) * nc;
  for (int r = blockIdx.x * kAT + threadIdx.x; r < n_c; r += gridDim.x * kAT) {
    const int i = clist[r];
    const int e0 = Rrp[r], len = Rrp[r + 1] - e0;
    const int s = len - 1;
    if (s <= 0) continue;
    int pc = 0;
    while (pc < len && Rci[e0 + pc] != i) ++pc;
    double* x = u + e0;  // rho in, u out; F-entry a at x[a + (a >= pc)]
    auto X = [&](int a) -> double& { return x[a + (a >= pc)]; };
    auto K = [&](int a, int c) { return fac[((int64_t)a * smax + c) * nc + r]; };
    auto V = [&](int k, int a) -> double& { return Vb[((int64_t)k * smax + a) * nc + r]; };
    auto H = [&](int a, int c) -> double& { return Hb[((int64_t)a * m + c) * nc + r]; };
    auto CS = [&](int k) -> double& { return cb[(int64_t)k * nc + r]; };
    auto SN = [&](int k) -> double& { return sb[(int64_t)k * nc + r]; };
    auto G = [&](int k) -> double& { return gb[(int64_t)k * nc + r]; };
    double beta = 0.0;
    for (int a = 0; a < s; ++a) beta += X(a) * X(a);
    beta = sqrt(beta);
    if (beta == 0.0) continue;  // u = 0
    for (int a = 0; a < s; ++a) V(0, a) = X(a) / beta;
    for (int t = 0; t <= m; ++t) G(t) = 0.0;
    G(0) = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      for (int a = 0; a < s; ++a) {
        double acc = 0.0;
        for (int c = 0; c < s; ++c) acc += K(a, c) * V(j, c);
        V(j + 1, a) = acc;
      }
      double w0 = 0.0;
      for (int a = 0; a < s; ++a) w0 += V(j + 1, a) * V(j + 1, a);
      w0 = sqrt(w0);
      for (int q = 0; q <= j; ++q) {
        double h = 0.0;
        for (int a = 0; a < s; ++a) h += V(j + 1, a) * V(q, a);
        H(q, j) = h;
        for (int a = 0; a < s; ++a) V(j + 1, a) -= h * V(q, a);
      }
      double hn = 0.0;
      for (int a = 0; a < s; ++a) hn += V(j + 1, a) * V(j + 1, a);
      hn = sqrt(hn);
      for (int q = 0; q < j; ++q) {
        const double h0 = H(q, j), h1 = H(q + 1, j);
        H(q, j) = CS(q) * h0 + SN(q) * h1;
        H(q + 1, j) = -SN(q) * h0 + CS(q) * h1;
      }
      const double hjj = H(j, j);
      const double rr = sqrt(hjj * hjj + hn * hn);
      CS(j) = rr > 0.0 ? hjj / rr : 1.0;
      SN(j) = rr > 0.0 ? hn / rr : 0.0;
      H(j, j) = rr;
      G(j + 1) = -SN(j) * G(j);
      G(j) = CS(j) * G(j);
      k = j + 1;
      if (!(hn > 1e-12 * w0)) break;  // the Krylov space is invariant: exact
      for (int a = 0; a < s; ++a) V(j + 1, a) /= hn;
    }
    for (int q = k - 1; q >= 0; --q) {
      double v = G(q);
      for (int c = q + 1; c < k; ++c) v -= H(q, c) * G(c);
      G(q) = H(q, q) != 0.0 ? v / H(q, q) : 0.0;
    }
    for (int a = 0; a < s; ++a) {
      double v = 0.0;
      for (int q = 0; q < k; ++q) v += G(q) * V(q, a);
      X(a) = v;
    }
    if (B) {
      const double bi = B[i];
      for (int a = 0; a < s; ++a) unsafeAtomicAdd(&sj[Rci[e0 + a + (a >= pc)]], X(a) * bi);
    }
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
                       w.rp, w.ci, w.va, w.B, w.diag, w.d, w.cnt, (w.ilu || w.gmres) ? nullptr : w.bad_row);
    if (w.ilu || w.gmres)
      hipLaunchKernelGGL(k_ap_block, dim3(agrid(w.n_c, w.cus)), dim3(kAT), 0, s, w.n_c, w.Rrp, w.Rci, w.clist, w.rp,
                         w.ci, w.va, w.fac, w.smax, w.ilu, w.bad_row);
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
                     w.Rva, w.trp, w.tci, w.tva, w.diag, w.B, w.u, w.sj, (w.ilu || w.gmres) ? 0 : 1);
  if (w.ilu)
    hipLaunchKernelGGL(k_ap_ilu_solve, dim3(agrid(w.n_c, w.cus)), dim3(kAT), 0, s, w.n_c, w.Rrp, w.Rci, w.clist, w.fac,
                       w.smax, w.B, w.u, w.sj);
  if (w.gmres)
    hipLaunchKernelGGL(k_ap_gmres, dim3(agrid(w.n_c, w.cus)), dim3(kAT), 0, s, w.n_c, w.Rrp, w.Rci, w.clist, w.fac,
                       w.smax, w.krylov, w.gw, w.B, w.u, w.sj);
  hipLaunchKernelGGL(k_ap_update, dim3(agrid(w.nnz, w.cus)), dim3(kAT), 0, s, w.nnz, w.erow, w.clist, w.Rci, w.Rva,
                     w.u, w.B, w.d, w.sj);
  return hipGetLastError();
}

}  // namespace clair
