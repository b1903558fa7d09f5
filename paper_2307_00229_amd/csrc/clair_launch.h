// clair_launch.h -- host-side launchers of the libclair kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "clair_device.h"

namespace clair {

constexpr int kMaxChunk = 2048;   // fine points per symbolic-pass workgroup (upper bound)
constexpr int kLdsBlockMax = 64;  // workgroup FP64 solver keeps blocks up to this size in LDS

// mixed (default) path
// empties the projection's column lists and writes R.row_ptr[n_c] (plan execute)
hipError_t launch_clear_sums(const Work& w, int64_t n_total, int blocks, hipStream_t s);
hipError_t launch_validate(const Work& w, int blocks, hipStream_t s);
// member lists of the aggregates of the matrices given with them (w.agg_*)
hipError_t launch_agg_lists(const Work& w, int64_t n_total, int blocks, int cus, hipStream_t s);
// column maxima of every matrix with theta > 0 (w.cmax, batch-wide fine numbering)
hipError_t launch_colmax(const Work& w, int64_t n_total, int blocks, hipStream_t s);
hipError_t launch_adj(const Work& w, hipStream_t s);
hipError_t launch_count(const Work& w, hipStream_t s);
hipError_t launch_count_mid(const Work& w, int blocks, hipStream_t s);
hipError_t launch_count_big(const Work& w, int blocks, hipStream_t s);
hipError_t launch_scan(const Work& w, hipStream_t s);
// which = 0: bin A with group = GA; which = 1: bin B with group = 32
hipError_t launch_numeric(const Work& w, int which, int group, int sm, int wg_threads, int cus, hipStream_t s);
// group lanes per row with rows_per_lane block rows each (bins A and B)
hipError_t launch_lanes(const Work& w, int which, int group, int rows_per_lane, int sm, int wg_threads, int cus,
                        hipStream_t s);
// one thread per row with |N| <= 8 (GA == 1); four lanes per row (GA == 4)
hipError_t launch_quad8(const Work& w, int wg_threads, int cus, hipStream_t s);
hipError_t launch_rows8(const Work& w, int wg_threads, int cus, hipStream_t s);
hipError_t launch_rows_wg(const Work& w, int blocks, hipStream_t s);
// the constraint projection over the column lists (one workgroup per chunk)
hipError_t launch_project(const Work& w, hipStream_t s);

// CSR transpose of an m x ncol matrix: trp[ncol+1], tci/tva[nnz]; scratch of
// transpose_scratch_ints(ncol) ints (column cursors, a flag set to 1 for an
// index outside [0, ncol), block totals)
size_t transpose_scratch_ints(int ncol);
hipError_t launch_transpose(int m, int ncol, const int32_t* rp, const int32_t* ci, const double* va, int32_t* trp,
                            int32_t* tci, double* tva, int32_t* scratch, int cus, hipStream_t s);

// out[0..n) = exclusive prefix of cnt, out[n] = total; sums: scan_scratch_ints(n)
size_t scan_scratch_ints(int n);
hipError_t launch_exclusive_scan(const int32_t* cnt, int n, int32_t* out, int32_t* sums, int cus, hipStream_t s);

// sparse product C = X Y (X: m rows, Y: k x ny), one wavefront per row of C.
// Symbolic: cnt[i] = distinct columns of row i; flags (4 ints, zeroed by the
// caller): [0] = 1 for a row above kSpgemmMaxRow columns, [1] = 1 for an index
// out of range, [2] the largest product count of a row.  It synchronises the
// stream once (to size the hash tables) and returns the table size in
// *lg_out, which the numeric pass takes.  Numeric: sorted rows at crp[i]
// (crp from the scan of cnt).
constexpr int kSpgemmMaxRow = 1536;
hipError_t launch_spgemm_count(int m, const int32_t* xrp, const int32_t* xci, int k, const int32_t* yrp,
                               const int32_t* yci, int ny, int32_t* cnt, int32_t* flags, int* lg_out, int cus,
                               hipStream_t s);
hipError_t launch_spgemm_fill(int m, const int32_t* xrp, const int32_t* xci, const double* xva, const int32_t* yrp,
                              const int32_t* yci, const double* yva, const int32_t* crp, int32_t* cci, double* cva,
                              int lg, int cus, hipStream_t s);

// one weighted Jacobi sweep for M x = 0 on the points with (cf != 0) == which_c
// (M's rows given); flag: 1 = zero diagonal on a swept row, 2 = bad index
hipError_t launch_jacobi_sweep(int n, const int32_t* rp, const int32_t* ci, const double* va, const int8_t* cf,
                               int which_c, double omega, const double* x, double* y, int32_t* flag, int cus,
                               hipStream_t s);

// k constraint vectors (k <= 4) imposed on an R built without constraints.
// Device work arrays (sizes for n fine points, n_rows rows, nnz entries):
// R^T (trp n + 1, tci nnz, tva nnz), the transpose's t_scratch
// (transpose_scratch_ints(n)), the C/F flags (flag n), their scan (pos n + 1,
// scan_sums scan_scratch_ints(n)), row -> C-point (rowc n_rows), lambda
// (lam n * k).  *uncovered (device, zeroed by the caller) counts the
// F-columns no row reaches; an index outside [0, n) sets t_scratch[n] to 1
// (the transpose's flag) and is skipped everywhere; pos[n] is the number of
// C-points, which the caller compares with n_rows.
struct ProjectScratch {
  int32_t *trp, *tci;
  double* tva;
  int32_t* t_scratch;
  int32_t *flag, *pos, *scan_sums, *rowc;
  double* lam;
};
hipError_t launch_project_k(int n, int n_rows, const int32_t* rp, const int32_t* ci, double* va, const int8_t* cf,
                            const double* B, int k, double rcond, const ProjectScratch& w,
                            unsigned long long* uncovered, int cus, hipStream_t s);

// Algorithm 1 with approximate block inverses, on R's pattern (rows sorted,
// the C-point's own entry included).  A^T in trp/tci/tva; clist[q] = the
// C-point of row q; work arrays: diag, d, sj (n), cnt (n, zeroed), u and erow
// (nnz), *bad_row (INT32_MAX beforehand), *uncovered (zeroed).  ilu: ILU(0)
// of every block instead of its diagonal; gmres: `krylov` GMRES steps on
// every local system; fac holds the blocks (factors for ILU(0)), smax^2 * n_c
// doubles (smax >= the largest block, <= 64), interleaved over rows; gw the
// GMRES work, ((krylov + 1) (smax + krylov + 3)) * n_c doubles.
struct DiagWork {
  int ilu, gmres, krylov;
  double *fac, *gw;
  int smax;
  int n, n_c;
  int64_t nnz;
  int cus;
  const int32_t *rp, *ci;
  const double* va;
  const int32_t *trp, *tci;
  const double* tva;
  const int8_t* cf;
  const double* B;
  const int32_t *Rrp, *Rci, *clist;
  double* Rva;
  double *diag, *d, *sj, *u;
  int32_t *cnt, *erow, *bad_row;
  unsigned long long* uncovered;
};
hipError_t launch_diag_start(const DiagWork& w, hipStream_t s);
hipError_t launch_diag_iteration(const DiagWork& w, hipStream_t s);

// the normal-equations (KKT) minimiser on an unconstrained R (rows sorted,
// the C-point's entry included; n_rows = the number of C-points).  Device
// arrays: flag (n), pos (n + 1), scan_sums (scan_scratch_ints(n)), rowc
// (n_rows), K and L (smax^2 * n_rows), T (smax * n_rows), rhs, res, p, x, Ap
// (n), cnt (n, zeroed), rhs zeroed, bad (2 ints: 0 and INT32_MAX); CG state
// sc (5 doubles: res.res, p.Ap, new res.res, stop level, beta), done and
// steps (ints, zeroed).
struct KktWork {
  double* sc;
  int32_t *done, *steps;
  int n, n_rows, smax, cus;
  const int32_t *rp, *ci;
  const double* va;
  const int8_t* cf;
  const double* B;
  const int32_t *Rrp, *Rci;
  double* Rva;
  int32_t *flag, *pos, *scan_sums, *rowc, *cnt, *bad;
  double *K, *L, *T, *rhs, *res, *p, *x, *Ap;
};
hipError_t launch_kkt_setup(const KktWork& w, hipStream_t s);
// *out += x . y (skipped once done)
hipError_t launch_kkt_dot(const KktWork& w, const double* x, const double* y, double* out, hipStream_t s);
// one CG step with the scalars on the device; a no-op once *done
hipError_t launch_kkt_step(const KktWork& w, hipStream_t s);
hipError_t launch_kkt_apply(const KktWork& w, hipStream_t s);               // z -= B_i Abar^{-1} x|_N

// plain FP64 per-row form: one matrix, one thread per row, one kernel per stage
struct PlainWork {
  const int32_t* rp;
  const int32_t* ci;
  const double* va;
  // the graph of the neighbourhood search (A, or a strength matrix)
  const int32_t* grp;
  const int32_t* gci;
  const double* gva;
  int32_t literal;  // 1: the pattern of S^{ell-1} T taken literally (C-points as interior vertices)
  const int8_t* cf;
  const double* B;
  int32_t n;
  int32_t ell;
  double theta;       // strength threshold of the search (0: every stored nonzero)
  double* cmax;       // [n] largest off-diagonal |a_wv| of column v (when theta > 0)
  int32_t* blk_cnt;   // [nblk + 1]
  int32_t* clist;     // [n]   C-points in ascending order
  int32_t* sizes;     // [n+1] |N(i)| then exclusive scan of |N(i)|+1
  int32_t* scan_tmp;  // [n/256 + 2]
  double* kbuf;       // [n_c * (smax * smax + smax)]
  double* dsum;       // [n]
  double* rsum;       // [n]
  int32_t* flags;     // [8]: status, first_bad, max_block, ...
  int32_t* Rrp;
  int32_t* Rci;
  double* Rva;
};

hipError_t plain_colmax(const PlainWork& p, hipStream_t s);                  // cmax
hipError_t plain_count_c(const PlainWork& p, hipStream_t s);                 // blk_cnt
hipError_t plain_scan_blocks(int32_t* a, int n, hipStream_t s);             // exclusive, a[n] = total
hipError_t plain_clist(const PlainWork& p, hipStream_t s);                   // clist
hipError_t plain_sizes(const PlainWork& p, int n_c, hipStream_t s);          // sizes, flags
hipError_t plain_scan(const PlainWork& p, int n_c, hipStream_t s);           // sizes -> offsets, Rrp
hipError_t plain_fill(const PlainWork& p, int n_c, hipStream_t s);           // Rci
hipError_t plain_solve(const PlainWork& p, int n_c, int smax, hipStream_t s);  // Rva
hipError_t plain_colsum(const PlainWork& p, int n_c, hipStream_t s);         // dsum, rsum
hipError_t plain_project(const PlainWork& p, int n_c, hipStream_t s);        // Rva

}  // namespace clair
