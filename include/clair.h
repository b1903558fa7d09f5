/*
 * clair.h -- C ABI of libclair: the restriction setup of constrained l-AIR
 * (C-l-AIR) on AMD Instinct MI355X (gfx950).
 *
 * Method (Ali, Brannick, Kahl, Krzysik, Schroder, Southworth, "Constrained
 * Local Approximate Ideal Restriction for Advection-Diffusion Problems"):
 *
 *   R = [Z I] in reduction form (Section 2, eq. basicsplit): one row per
 *   C-point, the C-point itself injected with weight 1.  Row i is built by
 *   Algorithm 1 applied to A^T (Section 3.1.3) with exact local inverses, for
 *   which one iteration suffices (Remark 2):
 *
 *   1. pattern: N(i) = F-points reachable from C-point i by a walk of at most
 *      `ell` edges of A's graph whose interior vertices are F-points (the
 *      sparsity pattern (S^{m-1} T)|_F of Algorithm 1 with m = ell, classical
 *      strength with threshold 0, i.e. every stored nonzero off-diagonal entry
 *      is an edge);
 *   2. local l-AIR system (Section 2.1, eq. system):
 *      (A[N,N])^T z = -A[i,N]^T;
 *   3. mode constraint R^T B_c = B on the F-points (Section 2.3,
 *      eq. global_const1 and Section 3.1, eq. Qdef) imposed by the Euclidean
 *      projection I - Q^T (Q Q^T)^{-1} Q of Algorithm 1.  Q Q^T is diagonal:
 *      for F-column j with contributing rows I_j,
 *        d_j = sum_{i in I_j} B_i^2,  r_j = sum_{i in I_j} z_ij B_i - B_j,
 *        z_ij <- z_ij - B_i r_j / d_j.
 *      Columns no row reaches (d_j = 0) are left alone and counted as
 *      "uncovered".  B = NULL skips step 3: the rows are plain l-AIR (Remark 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array pointers are DEVICE pointers (memory of the current HIP device),
 *   owned by the caller.  Inputs are read only.  The library never frees or
 *   reallocates caller memory.
 * - A is square n x n CSR with int32 indices: row_ptr[n+1] (row_ptr[0] = 0),
 *   col_idx[nnz] strictly ascending within each row (no duplicates), val[nnz]
 *   float64.  A stored zero is not an edge.
 * - cf_marker: int8[n], nonzero = C-point, 0 = F-point.
 * - R (output) is n_c x n CSR, n_c = number of C-points.  Row r belongs to the
 *   r-th C-point in ascending fine index.  Column indices are fine indices,
 *   ascending within each row; the C-point's own column holds exactly 1.0.
 *   row_ptr must hold n_c + 1 entries; col_idx and val must hold nnz(R).
 * - Precision: CLAIR_PREC_MIXED (default) gathers the local blocks and
 *   factorises them in FP32 and refines the solution with FP64 residuals
 *   until the FP64 backward error is at rounding level; the projection is
 *   FP64.  Rows whose FP32 factorisation is unreliable are redone in FP64.
 *   CLAIR_PREC_FP64 is the plain per-row FP64 form (one thread per row, one
 *   kernel per stage, one matrix at a time).  CLAIR_PREC_MIXED_BF16 is the
 *   mixed form whose workgroup solver (blocks of 33 to 128 points) takes the
 *   L21 and U12 tiles of its blocked LU's trailing updates rounded to
 *   bfloat16 (matrix cores, FP32 accumulation), refines in FP64 for up to 10
 *   steps, and redoes a row that does not converge with FP32 updates
 *   (clair_info_t.n_bf16_retries); smaller blocks are solved as in
 *   CLAIR_PREC_MIXED.  clair_build_R_batched / _ex and clair_build_R_agg
 *   accept it; graphs and plans use CLAIR_PREC_MIXED.
 * - Errors: every entry point returns a clair_status (0 = CLAIR_OK).  Nothing
 *   aborts and no C++ exception crosses the ABI.  Per-matrix details land in
 *   clair_info_t.
 * - Thread safety: one clair_ctx_t must not be used by two host threads at
 *   once.  Different contexts are independent.
 */
#ifndef CLAIR_H
#define CLAIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum clair_status {
  CLAIR_OK = 0,
  CLAIR_ERR_INVALID = 1,     /* bad argument, unsorted/duplicate CSR, ell < 1, ... */
  CLAIR_ERR_CAPACITY = 2,    /* R does not fit: required sizes are in clair_info_t / R_out */
  CLAIR_ERR_SINGULAR = 3,    /* a local block is singular (first fine row in info.first_bad_row) */
  CLAIR_ERR_HIP = 4,         /* a HIP runtime call failed */
  CLAIR_ERR_UNSUPPORTED = 5, /* a neighbourhood exceeds CLAIR_MAX_BLOCK, or an input or option the entry point does not take */
  CLAIR_ERR_NOMEM = 6        /* workspace allocation failed */
} clair_status;

enum { CLAIR_PREC_MIXED = 0, CLAIR_PREC_FP64 = 1, CLAIR_PREC_MIXED_BF16 = 2 };

/* Largest local block (|N(i)|) any path accepts. */
#define CLAIR_MAX_BLOCK 1024

/* Input matrix.  Device pointers; see conventions above. */
typedef struct clair_csr {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;
} clair_csr_t;

/* Output restriction.  Capacities are inputs; sizes are outputs. */
typedef struct clair_csr_out {
  int32_t n_rows;        /* out: n_c */
  int32_t n_cols;        /* out: n */
  int64_t nnz;           /* out: nnz(R), also reported with CLAIR_ERR_CAPACITY */
  int32_t row_capacity;  /* in: entries available in row_ptr (needs n_c + 1) */
  int32_t pad_;
  int64_t nnz_capacity;  /* in: entries available in col_idx and val */
  int32_t* row_ptr;      /* device */
  int32_t* col_idx;      /* device */
  double* val;           /* device */
} clair_csr_out_t;

/* Per-matrix result details. */
typedef struct clair_info {
  int32_t status;           /* clair_status of this matrix */
  int32_t first_bad_row;    /* fine index of a singular / oversized row, or -1 */
  int32_t n_c;              /* number of C-points (rows of R) */
  int32_t max_block;        /* largest |N(i)| */
  int64_t nnz;              /* nnz(R) */
  int64_t n_uncovered;      /* F-points no row reaches (only when B != NULL) */
  int32_t refine_iters_max; /* most FP64 refinement steps any row needed (mixed) */
  int32_t n_fp64_rows;      /* rows solved by the FP64 fallback (mixed) */
  int32_t n_bf16_retries;   /* rows of more than 32 points whose BF16-update factorisation did not
                               converge and was redone with FP32 updates (CLAIR_PREC_MIXED_BF16) */
  int32_t reserved;         /* 0 */
} clair_info_t;

/* Options for the _ex entry points.  Zero-initialised = defaults. */
typedef struct clair_opts {
  void* stream;       /* hipStream_t to run on; NULL = null stream */
  int32_t precision;  /* CLAIR_PREC_MIXED (0), CLAIR_PREC_FP64 (1) or CLAIR_PREC_MIXED_BF16 (2) */
  int32_t async;      /* 1: only enqueue; read results later with clair_ctx_info */
  int32_t validate;   /* 1: check CSR order / index range on the device first */
  int32_t timing;     /* 1: record per-stage HIP events (see clair_ctx_stage_times) */
} clair_opts_t;

/* Opaque library context: owns device workspace and a pinned staging area. */
typedef struct clair_ctx clair_ctx_t;

/* Create a context on the current HIP device.  Returns CLAIR_ERR_HIP if no
 * device is usable. */
int clair_ctx_create(clair_ctx_t** ctx);
void clair_ctx_destroy(clair_ctx_t* ctx);

/*
 * clair_build_R -- one matrix, synchronous, mixed precision, library-owned
 * default context of the current device, null stream.
 *   A          input matrix (device arrays)
 *   cf_marker  device int8[n]
 *   B          device float64[n] constraint vector, or NULL (plain l-AIR rows)
 *   ell        pattern degree m of Algorithm 1, >= 1
 *   R_out      capacities in, sizes out.  If the capacities are too small
 *              (or col_idx == NULL) nothing is written except the sizes and
 *              CLAIR_ERR_CAPACITY is returned: a size query.
 */
int clair_build_R(const clair_csr_t* A, const int8_t* cf_marker, const double* B, int32_t ell,
                  clair_csr_out_t* R_out);

/*
 * clair_build_R_agg -- clair_build_R_batched with the aggregation-based base
 * pattern (Section 3.1.3: with aggregation-based coarsening, T is the
 * aggregation operator).  agg[k]: device int32[n], the root C-point of every
 * point's aggregate, or -1; an F-point j belongs to root r = agg[k][j] when r
 * is a C-point index in range (any other value: to no aggregate).  Row i of
 * R starts from the F-points of i's aggregate and adds ell - 1 steps of the
 * search (with the context's strength threshold); at ell = 1 it is the
 * aggregate.  agg[k] may be NULL for a matrix that keeps the classical
 * pattern.  Mixed precision only (CLAIR_PREC_FP64 returns
 * CLAIR_ERR_UNSUPPORTED); plans and graphs take the classical pattern.
 * Sizes and capacities as clair_build_R_batched (a synchronous call with too
 * small capacities reports the sizes).
 */
int clair_build_R_agg(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf_marker,
                      const int32_t* const* agg, const double* const* B, const int32_t* ell, clair_csr_out_t* R_out,
                      const clair_opts_t* opts, clair_info_t* info);

/* Same for one matrix with explicit context, options and info (info may be NULL). */
int clair_build_R_ex(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker,
                     const double* B, int32_t ell, clair_csr_out_t* R_out, const clair_opts_t* opts,
                     clair_info_t* info);

/*
 * clair_build_R_batched -- nmat independent setups in one pass: every stage
 * is one kernel launch over the rows of all matrices.  Arrays of length nmat:
 * A[k], cf[k], B[k] (entries may be NULL), ell[k], R_out[k], info[k] (info may
 * be NULL).  Equivalent to nmat calls of clair_build_R_ex.  The return value
 * is the first non-OK per-matrix status (CLAIR_OK if all succeeded).
 * With opts->async = 1 the call only enqueues work on opts->stream (no host
 * synchronisation, so it can be captured into a hipGraph); R_out sizes and
 * info are then obtained with clair_ctx_info after the stream has finished.
 * In async mode the capacities must already be large enough: a matrix that
 * does not fit reports CLAIR_ERR_CAPACITY in its info and its R is not written.
 */
int clair_build_R_batched(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A,
                          const int8_t* const* cf_marker, const double* const* B, const int32_t* ell,
                          clair_csr_out_t* R_out, const clair_opts_t* opts, clair_info_t* info);

/*
 * clair_build_R_approx -- Algorithm 1 with approximate block inverses
 * (Section 3.1.2 allows a diagonal, GMRES or ILU approximation of each block
 * A_ff^{(i)}; the footnote of the comparison with root-node names the
 * diagonal one), run for `iterations` steps.  Same pattern as clair_build_R
 * (distance-ell F-neighbourhoods, the context's strength threshold), no exact
 * local solves.  With K_i = A[N,N]^T the block of C-point i:
 *   inverse = CLAIR_INVERSE_DIAG: K_i replaced by its diagonal (a_jj);
 *   inverse = CLAIR_INVERSE_ILU0: by its incomplete LU factors without fill
 *             (ILU(0): unit lower L and upper U on K_i's nonzero pattern,
 *             L U = K_i there; row-oriented elimination);
 *   inverse = CLAIR_INVERSE_GMRES: u_i = `krylov` (1..32) steps of GMRES on
 *             K_i u = rho_i from u = 0 (the least residual over the Krylov
 *             space; it stops early once the space is invariant, a new basis
 *             vector at most 1e-12 of K v_j).  krylov is ignored otherwise.
 *   start: z_ij = -a_ij (the tentative operator); with B, every F-column is
 *          replaced by the minimum-norm solution of its constraint,
 *          z_ij = B_i B_j / d_j with d_j = sum over the column's rows of B_i^2;
 *   each iteration: rho_i = -(R A) on row i's F-entries (the block
 *          residual), u_i = Khat_i^{-1} rho_i, projected with B
 *          (u_ij -= B_i sum_i(u_ij B_i) / d_j), then z += u.
 * Every iterate meets the constraint where B is given.  One iteration gives
 * clair_build_R's result when the approximate inverse is exact for every
 * block (Remark 2): diagonal blocks for the diagonal, blocks whose
 * factorisation has no fill for ILU(0), krylov >= the block size for GMRES.  FP64 throughout; per-column sums by
 * FP64 atomics (rounding order not fixed).
 *   R_out     as for clair_build_R (n_rows, n_cols, nnz set; too small
 *             capacities return CLAIR_ERR_CAPACITY, a size query)
 *   info      n_c, nnz, max_block, n_uncovered (with B), first_bad_row
 * A zero diagonal on a pattern F-column (diagonal) or a zero pivot (ILU(0))
 * returns CLAIR_ERR_SINGULAR, first_bad_row = the smallest C-point concerned.
 * Blocks above 64 points return CLAIR_ERR_UNSUPPORTED; an unknown `inverse`
 * or krylov outside 1..32 for GMRES CLAIR_ERR_INVALID.  cf_marker may be NULL
 * only when A->n = 0.  ILU(0) and GMRES keep n_c x s^2 doubles of blocks (s
 * the largest block) in the context, GMRES n_c x (krylov + 1)(s + krylov + 3)
 * more.
 * Synchronises `stream`.
 */
enum { CLAIR_INVERSE_DIAG = 1, CLAIR_INVERSE_ILU0 = 2, CLAIR_INVERSE_GMRES = 3 };
int clair_build_R_approx(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker, const double* B,
                         int32_t ell, int32_t inverse, int32_t krylov, int32_t iterations, clair_csr_out_t* R_out,
                         clair_info_t* info, void* stream);

/*
 * clair_build_R_kkt -- for comparison with Algorithm 1: the exact solution of
 * Section 3.1.1's constrained problem in the normal-equations metric (its
 * KKT system has the (1,1) block A_ff^T A_ff; Algorithm 1 projects in the
 * Euclidean norm instead).  For restriction, row i (C-point i, F-columns N)
 * has K_i = A[N,N]^T, a_i = A[i,N]^T and the energy |a_i + K_i z_i|^2; R
 * minimises the sum over the rows subject to R^T B_c = B.  Same pattern as
 * clair_build_R (the context's strength threshold).  Computed as
 * z_i = z0_i - Abar_i^{-1} B_i lambda|_N with z0 the exact unconstrained rows,
 * Abar_i = K_i^T K_i (Cholesky per row) and lambda from conjugate gradients
 * on Q Abar^{-1} Q^T lambda = Q z0 - B_F (SPD over the covered F-points;
 * stopped at a residual of 1e-14 of the right-hand side, at most 10000
 * steps).  B = NULL gives the unconstrained rows.
 *   R_out     as for clair_build_R (a size query with too small capacities)
 *   info      as clair_build_R's; refine_iters_max = the CG steps taken
 * An Abar_i that is not positive definite returns CLAIR_ERR_SINGULAR with
 * first_bad_row = the smallest such C-point; blocks above 64 points
 * CLAIR_ERR_UNSUPPORTED.  cf_marker may be NULL only when A->n = 0.
 * Synchronises `stream` (the host reads the CG convergence flag every 8
 * steps; the step scalars stay on the device).
 */
int clair_build_R_kkt(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker, const double* B,
                      int32_t ell, clair_csr_out_t* R_out, clair_info_t* info, void* stream);

/* clair_build_R_diag -- clair_build_R_approx with CLAIR_INVERSE_DIAG. */
int clair_build_R_diag(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker, const double* B,
                       int32_t ell, int32_t iterations, clair_csr_out_t* R_out, clair_info_t* info, void* stream);

/*
 * clair_transpose -- AT = A^T for an A of A->n rows and ncol columns (sorted
 * CSR in, sorted CSR out; values copied exactly).  AT_out: n_rows = ncol,
 * n_cols = A->n, nnz = A->nnz are set; with too small capacities (row_ptr
 * needs ncol + 1 entries) nothing else is written and CLAIR_ERR_CAPACITY is
 * returned.  A column index outside [0, ncol), or A->row_ptr[0] != 0 or
 * A->row_ptr[A->n] != A->nnz (read from the device), returns
 * CLAIR_ERR_INVALID; the calls built on the transpose (clair_build_P,
 * clair_smooth_B on A^T, clair_build_R_approx) check the same.
 * Synchronises `stream`.
 */
int clair_transpose(clair_ctx_t* ctx, const clair_csr_t* A, int32_t ncol, clair_csr_out_t* AT_out, void* stream);

/*
 * clair_build_P -- interpolation by the same method: P = W(A), Algorithm 1
 * applied to A itself (Section 3.1.3; R is the same algorithm applied to
 * A^T).  Computed as P = (restriction of A^T)^T on the device: A^T is formed
 * in library buffers, its restriction built with opts (precision; the
 * context's strength threshold, which then measures strength in A), and
 * transposed into P_out.  B is the constraint vector for P (a near-null
 * vector of A), or NULL.  P is n x n_c: row f holds the C-columns (coarse
 * indices 0..n_c-1) whose pattern reaches f; a C-point's row is its own
 * injection.  P_out: n_rows = n, n_cols = n_c, nnz are set; too small
 * capacities return CLAIR_ERR_CAPACITY (a size query).  info describes the
 * restriction of A^T (n_c, max_block, refinement).  Synchronous: opts->async
 * and opts->timing are ignored.
 */
int clair_build_P(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker, const double* B, int32_t ell,
                  clair_csr_out_t* P_out, const clair_opts_t* opts, clair_info_t* info);

/*
 * clair_spgemm -- C = X Y for X of X->n rows and x_cols columns and Y of
 * Y->n = x_cols rows and y_cols columns (sorted CSR in and out, FP64).  The
 * pattern is structural: every column that some product x_ij y_jc reaches,
 * also where the products cancel.  Each row's sum is formed in no fixed
 * order, so values agree with a sequential product to rounding.  C_out:
 * n_rows, n_cols, nnz are set; too small capacities return
 * CLAIR_ERR_CAPACITY (a size query).  A row of C with more than 1536 columns
 * returns CLAIR_ERR_UNSUPPORTED; an index out of range CLAIR_ERR_INVALID.
 * Synchronises `stream`.
 */
int clair_spgemm(clair_ctx_t* ctx, const clair_csr_t* X, int32_t x_cols, const clair_csr_t* Y, int32_t y_cols,
                 clair_csr_out_t* C_out, void* stream);

/*
 * clair_galerkin -- the coarse operator A_c = R A P of the next level
 * (Section 1), R: n_c x n, A: n x n, P: n x n_c, as R (A P) with the
 * intermediate A P in library buffers.  Same pattern, rounding, capacity and
 * error rules as clair_spgemm.  Synchronises `stream`.
 */
int clair_galerkin(clair_ctx_t* ctx, const clair_csr_t* R, const clair_csr_t* A, const clair_csr_t* P, int32_t n_c,
                   clair_csr_out_t* Ac_out, void* stream);

/*
 * clair_smooth_B -- the constraint vector after `iterations` of
 * CFF-weighted Jacobi for M x = 0 (Section 4 pre-smooths B = 1 with 5 such
 * iterations on every level): per iteration one weighted Jacobi sweep on the
 * C-points (cf != 0), then two on the F-points; a sweep on a set S sets
 * x_i <- x_i - omega (M x)_i / m_ii for every i in S from the same old x.
 * M = A (transpose = 0: the vector for P) or A^T (transpose = 1: the vector
 * for R, which is built from A^T).  omega is the caller's (the paper uses
 * 1 / rho(D^{-1} A)).  B_in and B_out: device float64[n]; they may be the
 * same array.  A zero diagonal on a swept point returns CLAIR_ERR_SINGULAR
 * (B_out then holds the result with those points left unchanged); an index
 * out of range returns CLAIR_ERR_INVALID.  Synchronises `stream`.
 */
int clair_smooth_B(clair_ctx_t* ctx, const clair_csr_t* A, const int8_t* cf_marker, const double* B_in,
                   double* B_out, int32_t iterations, double omega, int32_t transpose, void* stream);

/*
 * clair_project_constraints -- k constraint vectors (Section 2.3 allows a
 * block of them; Section 3.1's Q then holds k rows per F-point): imposes
 * R^T B_c = B, for every column of B, on an R built with B = NULL, in place.
 * For each F-column j with contributing rows: G_j = sum_i B_i B_i^T (k x k),
 * r_j = sum_i z_ij B_i - B_j, z_ij -= B_i^T pinv(G_j) r_j -- the Euclidean
 * projection onto the constraints (k = 1 gives what clair_build_R computes
 * with B).  pinv drops eigenvalues at or below rcond times the largest (a
 * column reached by fewer rows than k gets the least-squares fit).
 *   R          R from this library (n_rows = n_c, nnz, device arrays); its
 *              values are updated
 *   n, cf      fine size and the C/F marker R was built with
 *   B          device float64[n * k], row-major (B[j * k + t])
 *   k          1 <= k <= 8
 * Row q of R belongs to the q-th C-point; n_rows must equal the number of
 * C-points.  *n_uncovered (may be NULL): F-points no row reaches (left
 * unchanged).  A column index outside [0, n), a row count that differs
 * from the number of C-points, or R's row_ptr[0] != 0 or row_ptr[n_rows] !=
 * nnz gives CLAIR_ERR_INVALID (R may then be partly updated).  Deterministic: every column is summed in ascending row order.
 * Synchronises `stream`.
 */
int clair_project_constraints(clair_ctx_t* ctx, clair_csr_out_t* R, int32_t n, const int8_t* cf_marker,
                              const double* B, int32_t k, double rcond, int64_t* n_uncovered, void* stream);

/* Results of the last call on ctx (synchronises its stream).  Fills nmat info
 * entries and the sizes in R_out (may be NULL).  Returns the first non-OK status. */
int clair_ctx_info(clair_ctx_t* ctx, int32_t nmat, clair_csr_out_t* R_out, clair_info_t* info);

/* Sizes only (symbolic phase, synchronous): n_c and nnz(R) of each matrix. */
int clair_size_R(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf_marker,
                 const int32_t* ell, int32_t* n_c, int64_t* nnz, void* stream);

/* Per-stage device time of the last call made with opts.timing = 1, in ms.
 * names/ms arrays of length cap; returns the number of stages written. */
int clair_ctx_stage_times(clair_ctx_t* ctx, const char** names, float* ms, int32_t cap);

/*
 * Tuning: kernel shape of the mixed path.  group = lanes that solve one row
 * of |N| <= 8 (1, 4 or 8) or the largest |N| the lane-group solver takes
 * (16 or 32, one lane per block row); rows with larger blocks go to the
 * workgroup-per-row path.  wg_threads = threads per workgroup (64, 128 or
 * 256), chunk = fine points per workgroup in the symbolic pass (multiple of
 * 256, at most 2048).  0 keeps the current value; defaults 8, 256, 1024.
 * Invalid values return CLAIR_ERR_INVALID and change nothing.  clair_autotune picks them by timing
 * candidates on the given inputs (and stores the result in ctx).
 */
int clair_ctx_set_tuning(clair_ctx_t* ctx, int32_t group, int32_t wg_threads, int32_t chunk);
int clair_ctx_get_tuning(clair_ctx_t* ctx, int32_t* group, int32_t* wg_threads, int32_t* chunk);

/*
 * Lane layout of the bin-B solver (rows whose |N| lies above the bin-A bound
 * and at most 32): binB_lanes = 8, 16 or 32 lanes per row, each lane holding
 * ceil(b / binB_lanes) rows of the block, where b = 16, 20, 24 or 32 is the
 * smallest bound that holds the largest block the last synchronous call read
 * back (8 lanes become 16 at b = 32, 32 lanes become 16 at b = 16).  0 keeps
 * the current value; default 32.  Other values return CLAIR_ERR_INVALID and
 * change nothing.
 */
int clair_ctx_set_bin_shape(clair_ctx_t* ctx, int32_t binB_lanes);
int clair_ctx_get_bin_shape(clair_ctx_t* ctx, int32_t* binB_lanes);

/*
 * clair_build_R_noalloc -- clair_build_R_ex for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one matrix, mixed precision, default tuning, synchronous on
 * `stream` (NULL = null stream), allocating no device or host memory.  The
 * whole workspace sits in a static device array of
 * CLAIR_NOALLOC_SCRATCH_BYTES (96 MiB), one copy per device the library runs
 * on, held until the process ends: the descriptors, per-point arrays of about
 * 270 bytes per fine point of A, and the projection's listed records (8 bytes
 * per entry of R_out's nnz capacity when B != NULL), which fit a 512 x 512
 * five-point matrix.  An input that does not fit returns
 * CLAIR_ERR_UNSUPPORTED (clair_last_error states the sizes) before any device
 * work; rows whose neighbourhood exceeds 64 points are reported the same way
 * (first_bad_row).  Arguments, size query and results as clair_build_R_ex.
 * Every call on one device shares that device's array and host staging, so
 * calls that overlap on one device (other threads, other streams) race; the
 * array keeps the last call's contents, and every call re-initialises what it
 * reads.
 */
#define CLAIR_NOALLOC_SCRATCH_BYTES (96 * 1024 * 1024)
int clair_build_R_noalloc(const clair_csr_t* A, const int8_t* cf_marker, const double* B, int32_t ell,
                          clair_csr_out_t* R_out, void* stream, clair_info_t* info);

/* Bytes of device memory ctx holds for the FP64 blocks of rows above 64
 * points (one slot per workgroup of the FP64 solver, each the square of the
 * largest block a synchronous call has read back, rounded up to a multiple
 * of 8 points; 0 until such a row occurs).  Grows, never shrinks, until
 * clair_ctx_destroy.  NULL arguments return CLAIR_ERR_INVALID. */
int clair_ctx_scratch_bytes(clair_ctx_t* ctx, int64_t* bytes);

/*
 * Strength threshold theta of the neighbourhood search.  Algorithm 1
 * (Section 3.1.3) grows the pattern from a classical strength-of-connection
 * matrix S; Section 4 uses thresholds between 0.05 and 0.5.  R is Algorithm 1
 * applied to A^T, so the walk from C-point i takes the step u -> v when u != v,
 * a_uv is stored and nonzero, and |a_uv| >= theta * max_{w != v} |a_wv| (in
 * A^T, v depends strongly on u).  theta = 0 (the default) keeps every stored
 * nonzero.  The values of A are compared in FP64.
 * The setting applies to later calls on ctx (both precisions), to graphs
 * captured and to plans created after it; a plan keeps the pattern of its
 * creation (rows of more than 32 points are searched again at execute, and a
 * row whose pattern the new values change is reported as CLAIR_ERR_INVALID).
 * theta outside [0, 1], or NaN, returns CLAIR_ERR_INVALID and changes nothing.
 */
int clair_ctx_set_strength(clair_ctx_t* ctx, double theta);

/*
 * How the symbolic phase of the mixed form finds N(i) (Section 3.1.3, the
 * pattern of Algorithm 1) for matrices with ell >= 2.  By default (mode -1) a
 * prepass first lists, for every point u, the F-points that one step from u
 * reaches (the edge test above), in 4 slots per point when every such matrix
 * has at most five stored entries per row on average, else 8; the search then
 * takes each level's whole frontier from that list in one round of loads.
 * Points with more such neighbours than slots are expanded from the rows of
 * A (or of the strength matrix), as are matrices with more than nine stored
 * entries per row on average, aggregates and every call of
 * clair_build_R_noalloc.  Mode 0 searches every row from A directly; 4 or 8
 * forces that width.  The pattern and R are identical in every mode; the
 * setting changes only the work (mode 4 on a nine-point stencil sends most
 * points down the row path).  Any other mode returns CLAIR_ERR_INVALID.
 * Applies to later calls on ctx, graphs captured and plans created after it.
 */
int clair_ctx_set_search_adjacency(clair_ctx_t* ctx, int32_t mode);

/*
 * A strength matrix of the caller's as the graph of the neighbourhood search
 * (Algorithm 1 takes the strength matrix S as an input, Section 3.1.3): one n
 * x n CSR per matrix of the batches that follow (device arrays, rows sorted,
 * same n as the matrix; the arrays must stay valid while ctx uses them).  The
 * search then steps u -> v along S's stored nonzero entries u != v instead of
 * A's, in A's orientation (row u of S lists the v that u reaches), and theta
 * filters S's entries against S's column maxima; the local systems always use
 * A.  nmat = 0 or S = NULL returns to A's graph.  The setting applies to
 * clair_size_R, clair_build_R / _ex / _batched (both precisions), clair_build_R_agg,
 * clair_autotune, clair_build_R_approx and clair_build_R_kkt (one matrix),
 * graphs and plans created after it; a batch whose size or matrix sizes
 * differ returns CLAIR_ERR_INVALID, and clair_build_P (which would need a
 * strength matrix of A^T) CLAIR_ERR_UNSUPPORTED.  With opts->validate the
 * mixed path checks S's order and index range as well; otherwise indices
 * outside [0, n) are skipped by the search.
 */
int clair_ctx_set_graph(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* S);

/*
 * on = 1: the pattern of Algorithm 1's expansion S^{ell-1} T taken literally
 * (T = [S_fc, I]): C-points may then be interior vertices of a walk (the
 * first step reaches i's F-neighbours and i itself, every later step any
 * vertex; only F-points join N(i)).  The default (on = 0) keeps F-points as
 * interior vertices; the two agree for ell <= 2.  Both forms, the size
 * query, graphs, plans and the approximate-inverse build follow the setting
 * for any ell.  The searches hold the C-points they pass through before the
 * last step too: the mixed form's register search moves a row to its
 * workgroup search beyond 32 such vertices, which holds up to
 * CLAIR_MAX_BLOCK; the FP64 form's search holds 64, and a row that does not
 * fit fails as an oversized neighbourhood does.  The mixed form builds no
 * compact adjacency for such matrices at ell >= 3.  The classical base
 * pattern only (not the aggregation-based one).  on outside {0, 1} returns
 * CLAIR_ERR_INVALID.
 */
int clair_ctx_set_literal_pattern(clair_ctx_t* ctx, int32_t on);
int clair_ctx_get_strength(clair_ctx_t* ctx, double* theta);
/*
 * clair_autotune -- picks the tuning (clair_ctx_set_tuning) and the bin-B
 * layout (clair_ctx_set_bin_shape) for a batch by timing candidates on it
 * (reps setups each, after one warm-up), and stores them in ctx.  The
 * candidates follow the batch's histogram of block sizes (read back after
 * one synchronous setup): bin-A bounds of 16 and 32 are tried only when rows
 * above 8 (16) points exist, the bin-B layouts only when rows fall between
 * the bin-A bound and 32.  The pick is cached per process by (device,
 * histogram signature, the number of matrices, the strength setting): a
 * batch whose histogram has, size by size, the same binary order of
 * magnitude of rows reuses it with no timing runs.  Leaves R_out as one
 * setup with the chosen tuning writes it.
 */
int clair_autotune(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf_marker,
                   const double* const* B, const int32_t* ell, clair_csr_out_t* R_out, void* stream,
                   int32_t reps);
/* Timing runs of the last clair_autotune on ctx (0 when the cache held it). */
int clair_ctx_autotune_runs(clair_ctx_t* ctx, int32_t* timed);

/* hipGraph replay of a batched setup on fixed buffers (values of A and B may
 * change between launches; the pattern may change as long as R still fits).
 * clair_graph_create captures clair_build_R_batched (async) on `stream`. */
typedef struct clair_graph clair_graph_t;
int clair_graph_create(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A,
                       const int8_t* const* cf_marker, const double* const* B, const int32_t* ell,
                       clair_csr_out_t* R_out, void* stream, clair_graph_t** graph);
int clair_graph_launch(clair_graph_t* graph, void* stream);
void clair_graph_destroy(clair_graph_t* graph);
/* Results of the last launch of `graph` (synchronises its stream), as clair_ctx_info. */
int clair_graph_info(clair_graph_t* graph, int32_t nmat, clair_csr_out_t* R_out, clair_info_t* info);

/*
 * Symbolic/numeric split for repeated setups on one sparsity pattern (for
 * instance a time-dependent operator whose values change while its graph
 * does not).  The neighbourhoods N(i) and the layout of R depend only on the
 * pattern of A (Algorithm 1, pattern expansion), the local solves and the
 * constraint projection on its values and on B.
 *
 * clair_plan_create runs the symbolic phase of a batch once (C/F indexing,
 * N(i), sizes of R) and keeps its state in a private context copied from
 * ctx's tuning.  R_out[k] gives the capacities; on return n_rows and nnz hold
 * the sizes.  If a matrix does not fit, or its input is invalid, no plan is
 * made and the first non-OK status is returned (CLAIR_ERR_CAPACITY: a size
 * query).  The cf_marker arrays must stay valid and unchanged while the plan
 * exists.
 *
 * clair_plan_execute runs the numeric phase: block gather, FP32 factorisation
 * with FP64 refinement, R write and projection.  A[k] must have the pattern
 * the plan was made with: the same n, row_ptr and col_idx contents, and the
 * same set of stored entries that are nonzero (a value that becomes exactly
 * zero removes an edge and needs a new plan); the arrays themselves may be
 * other buffers.  B[k] may change (NULL: unconstrained rows).  R_out[k] must
 * hold the sizes the plan reported.  opts->precision must be MIXED; with
 * opts->async = 1 the call only enqueues (results by clair_plan_info).
 * Returns the first non-OK per-matrix status.
 */
typedef struct clair_plan clair_plan_t;
int clair_plan_create(clair_ctx_t* ctx, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf_marker,
                      const int32_t* ell, clair_csr_out_t* R_out, void* stream, clair_plan_t** plan);
int clair_plan_execute(clair_plan_t* plan, int32_t nmat, const clair_csr_t* A, const double* const* B,
                       clair_csr_out_t* R_out, const clair_opts_t* opts, clair_info_t* info);
/* Results of the last execute of `plan` (synchronises its stream), as clair_ctx_info. */
int clair_plan_info(clair_plan_t* plan, int32_t nmat, clair_csr_out_t* R_out, clair_info_t* info);
void clair_plan_destroy(clair_plan_t* plan);

const char* clair_strerror(int status);

/* Text of the last HIP failure seen by this host thread inside the library
 * (empty if none): the failing call and the runtime's message. */
const char* clair_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLAIR_H */
