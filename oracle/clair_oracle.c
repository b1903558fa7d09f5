/*
 * clair_oracle.c -- plain, slow, FP64 reference implementation of the
 * constrained l-AIR (C-l-AIR) restriction setup.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or helper with the GPU
 * path; only tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  Nothing in the product path calls it.
 *
 * What it computes (Ali, Brannick, Kahl, Krzysik, Schroder, Southworth,
 * "Constrained Local Approximate Ideal Restriction for Advection-Diffusion
 * Problems"):
 *
 *   R = [Z I] in reduction form (Section 2, eq. basicsplit), C-points
 *   injected.  Row i of R (i a C-point) is obtained from Algorithm 1 applied to
 *   A^T (Section 3.1.3): the pattern of the row is the distance-ell
 *   F-neighbourhood N(i) of i (Algorithm 1, pattern expansion S^{m-1} T with
 *   m = ell, interior vertices F, S the classical strength matrix of A^T with
 *   threshold theta; T = S_fc for classical C/F coarsening, or the
 *   aggregation operator when aggregates are given), the local l-AIR system is
 *   (A[N,N])^T z = -A[i,N]^T (Section 2.1, eq. system), and the mode
 *   constraint R^T B_c = B on the F-points (Section 2.3, eq. global_const1;
 *   Section 3.1, eq. Qdef) is imposed by the Euclidean projection
 *   I - Q^T (Q Q^T)^{-1} Q of Algorithm 1 (projection step).
 *
 * With exact local inverses and k = 1 (Remark 2) the algorithm reduces to:
 *   1. z0 = local l-AIR solution of every C-row (Remark 1);
 *   2. for every F-column j with contributing C-rows I_j:
 *        d_j = sum_{i in I_j} B_i^2,   r_j = sum_{i in I_j} z0_ij B_i - B_j,
 *        z_ij = z0_ij - B_i r_j / d_j          (if d_j > 0).
 *   Q's rows are the F-rows of W = R^T, so Q Q^T is diagonal with entries d_j.
 *   Columns with d_j = 0 (no C-row reaches them) cannot be constrained; the
 *   pseudo-inverse leaves them untouched and they are counted as uncovered.
 *
 * Everything is FP64.  Local systems are solved by Gaussian elimination with
 * partial pivoting; a pivot with |pivot| <= 1e-14 * max|block| is reported as
 * singular.  Rows are independent and may run in parallel (OpenMP); the
 * projection sums every column in ascending row order, serially.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID 1
#define ORC_ERR_CAPACITY 2
#define ORC_ERR_SINGULAR 3
#define ORC_ERR_NOMEM 4

/* ------------------------------------------------------------------------ */
/* Neighbourhood: the F-points reachable from C-point i by a walk of at most  */
/* ell edges of A's graph whose interior vertices are all F-points.  An edge  */
/* u -> v exists when u != v, a_uv is stored and nonzero, and                 */
/* |a_uv| >= theta * cmax[v] with cmax[v] = max_{w != v} |a_wv|.              */
/* Breadth-first search, expanding F vertices only.                           */
/*                                                                            */
/* Why a column maximum: Algorithm 1 runs on M = A^T, whose classical         */
/* strength matrix has S_xy != 0 when |m_xy| >= theta max_{w != x} |m_xw|,    */
/* i.e. |a_yx| >= theta max_{w != x} |a_wx|.  A pattern entry (f, c) of       */
/* S^{m-1} T is a chain f -> ... -> c of such entries; walking it backwards   */
/* from c, each step from u to v uses S_vu, the test above.  theta = 0 keeps  */
/* every stored nonzero.                                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t* mark;  /* length n, stamp per vertex */
  int32_t stamp;
  int32_t* list;  /* growing list of found F-points */
  int32_t cap;
} bfs_ws;

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static int ws_push(bfs_ws* w, int32_t len, int32_t v) {
  if (len >= w->cap) {
    int32_t nc = w->cap ? 2 * w->cap : 64;
    int32_t* nl = (int32_t*)realloc(w->list, sizeof(int32_t) * (size_t)nc);
    if (!nl) return -1;
    w->list = nl;
    w->cap = nc;
  }
  w->list[len] = v;
  return 0;
}

/* Is u -> v (entry e of row u) an edge of the search? */
static int is_edge(int32_t u, int32_t e, const int32_t* ci, const double* va, double theta,
                   const double* cmax) {
  const int32_t v = ci[e];
  if (v == u || va[e] == 0.0) return 0;
  return theta == 0.0 || fabs(va[e]) >= theta * cmax[v];
}

/* cmax[v] = max over the off-diagonal entries of column v of |a_wv|. */
static void column_max(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, double* cmax) {
  for (int32_t v = 0; v < n; ++v) cmax[v] = 0.0;
  for (int32_t w = 0; w < n; ++w)
    for (int32_t e = rp[w]; e < rp[w + 1]; ++e)
      if (ci[e] != w) cmax[ci[e]] = fmax(cmax[ci[e]], fabs(va[e]));
}

/* Aggregates (may be NULL): agg[j] = the root C-point of j's aggregate or
 * -1.  The base pattern T is then the aggregation operator (Section 3.1.3,
 * aggregation-based coarsening): column c holds the F-points of c's
 * aggregate, and the expansion S^{m-1} T adds m-1 steps from them.  Members
 * of root c are listed in mem[mrp[c] .. mrp[c+1]). */
typedef struct {
  const int32_t* mrp;
  const int32_t* mem;
} agg_lists;

/* Returns s = |N(i)| (>= 0), N(i) sorted ascending in w->list[0..s), or -1 on OOM.
 * literal != 0: the pattern of S^{ell-1} T taken literally, where C-points
 * may be interior vertices: the first step (T = [S_fc, I]) reaches i's
 * F-neighbours and i itself, every later step any vertex; only F-points join
 * N(i).  The same as the default for ell <= 2. */
static int32_t neighbourhood(int32_t i, int ell, const int32_t* rp, const int32_t* ci,
                             const double* va, const int8_t* cf, double theta, const double* cmax,
                             const agg_lists* ag, bfs_ws* w, int literal) {
  w->stamp++;
  w->mark[i] = w->stamp;
  int32_t len = 0;
  int32_t lo = 0, hi = 0; /* current frontier = list[lo..hi); level 0 frontier is {i} */
  for (int depth = 1; depth <= ell; ++depth) {
    if (literal && depth >= 2) {
      /* the frontier holds F- and C-points; at depth 2 it also holds i (T's
         identity part), whose C-neighbours become interior vertices */
      int32_t before = len;
      for (int32_t t = (depth == 2 ? lo - 1 : lo); t < hi; ++t) {
        int32_t u = (t < lo) ? i : w->list[t];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
          int32_t k = ci[e];
          if (!is_edge(u, e, ci, va, theta, cmax) || w->mark[k] == w->stamp) continue;
          w->mark[k] = w->stamp;
          if (ws_push(w, len, k)) return -1;
          ++len;
        }
      }
      lo = before;
      hi = len;
      if (lo == hi) break;
      continue;
    }
    int32_t before = len;
    if (depth == 1 && ag) {
      /* the aggregate's F-points */
      for (int32_t t = ag->mrp[i]; t < ag->mrp[i + 1]; ++t) {
        int32_t k = ag->mem[t];
        if (cf[k] != 0 || w->mark[k] == w->stamp) continue;
        w->mark[k] = w->stamp;
        if (ws_push(w, len, k)) return -1;
        ++len;
      }
    } else if (depth == 1) {
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        int32_t k = ci[e];
        if (!is_edge(i, e, ci, va, theta, cmax) || cf[k] != 0 || w->mark[k] == w->stamp) continue;
        w->mark[k] = w->stamp;
        if (ws_push(w, len, k)) return -1;
        ++len;
      }
    } else {
      for (int32_t t = lo; t < hi; ++t) {
        int32_t u = w->list[t];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
          int32_t k = ci[e];
          if (!is_edge(u, e, ci, va, theta, cmax) || cf[k] != 0 || w->mark[k] == w->stamp) continue;
          w->mark[k] = w->stamp;
          if (ws_push(w, len, k)) return -1;
          ++len;
        }
      }
    }
    lo = before;
    hi = len;
    /* literal: the second step also expands i itself (T's identity part),
       so an empty first level does not end the search */
    if (lo == hi && !(literal && depth == 1)) break;
  }
  if (literal) { /* C-points were interior vertices only */
    int32_t m = 0;
    for (int32_t t = 0; t < len; ++t)
      if (cf[w->list[t]] == 0) w->list[m++] = w->list[t];
    len = m;
  }
  qsort(w->list, (size_t)len, sizeof(int32_t), cmp_i32);
  return len;
}

static int32_t find_sorted(const int32_t* a, int32_t len, int32_t key) {
  int32_t l = 0, h = len;
  while (l < h) {
    int32_t m = (l + h) >> 1;
    if (a[m] < key) l = m + 1; else h = m;
  }
  return (l < len && a[l] == key) ? l : -1;
}

/* Solve K x = f (K is s x s row-major, overwritten) by Gaussian elimination with
 * partial pivoting.  Returns 0 on success, 1 if a pivot is negligible. */
static int gepp_solve(double* K, double* f, int32_t s) {
  double amax = 0.0;
  for (int64_t t = 0; t < (int64_t)s * s; ++t) amax = fmax(amax, fabs(K[t]));
  const double tiny = 1e-14 * amax;
  for (int32_t k = 0; k < s; ++k) {
    int32_t p = k;
    double best = fabs(K[(int64_t)k * s + k]);
    for (int32_t q = k + 1; q < s; ++q) {
      double v = fabs(K[(int64_t)q * s + k]);
      if (v > best) { best = v; p = q; }
    }
    if (!(best > tiny)) return 1;
    if (p != k) {
      for (int32_t c = 0; c < s; ++c) {
        double t = K[(int64_t)k * s + c];
        K[(int64_t)k * s + c] = K[(int64_t)p * s + c];
        K[(int64_t)p * s + c] = t;
      }
      double t = f[k]; f[k] = f[p]; f[p] = t;
    }
    double piv = K[(int64_t)k * s + k];
    for (int32_t q = k + 1; q < s; ++q) {
      double l = K[(int64_t)q * s + k] / piv;
      if (l == 0.0) continue;
      for (int32_t c = k + 1; c < s; ++c) K[(int64_t)q * s + c] -= l * K[(int64_t)k * s + c];
      f[q] -= l * f[k];
    }
  }
  for (int32_t k = s - 1; k >= 0; --k) {
    double acc = f[k];
    for (int32_t c = k + 1; c < s; ++c) acc -= K[(int64_t)k * s + c] * f[c];
    f[k] = acc / K[(int64_t)k * s + k];
  }
  return 0;
}

static int check_csr(int32_t n, const int32_t* rp, const int32_t* ci) {
  if (n < 0 || !rp) return 1;
  if (rp[0] != 0) return 1;
  for (int32_t r = 0; r < n; ++r) {
    if (rp[r + 1] < rp[r]) return 1;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= n) return 1;
      if (e > rp[r] && ci[e] <= ci[e - 1]) return 1; /* ascending, no duplicates */
    }
  }
  return 0;
}

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) return nthreads;
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* Member lists of the aggregates: mrp[n+1], mem[n]; an F-point j joins the
 * aggregate of agg[j] when that is a C-point index in range. */
static int build_agg_lists(int32_t n, const int8_t* cf, const int32_t* agg, int32_t** mrp_out, int32_t** mem_out) {
  int32_t* mrp = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!mrp || !mem) { free(mrp); free(mem); return ORC_ERR_NOMEM; }
  for (int32_t j = 0; j < n; ++j) {
    int32_t r = agg[j];
    if (cf[j] == 0 && r >= 0 && r < n && cf[r] != 0) mrp[r + 1]++;
  }
  for (int32_t r = 0; r < n; ++r) mrp[r + 1] += mrp[r];
  int32_t* fill = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  if (!fill) { free(mrp); free(mem); return ORC_ERR_NOMEM; }
  for (int32_t j = 0; j < n; ++j) { /* ascending j: each list comes out sorted */
    int32_t r = agg[j];
    if (cf[j] == 0 && r >= 0 && r < n && cf[r] != 0) mem[mrp[r] + fill[r]++] = j;
  }
  free(fill);
  *mrp_out = mrp;
  *mem_out = mem;
  return ORC_OK;
}

/* Number of C-points and nnz(R) = sum_i (|N(i)| + 1).  Also the per-row sizes
 * when `sizes` (length n_c) is given. */
/* The search runs on the graph G (g_rp, g_ci, g_va: n x n CSR): A itself, or
   a strength matrix the caller gives, whose stored entries u -> v are the
   edges (filtered by theta against G's column maxima, as for A). */
int orc_pattern_size_g(int32_t n, const int32_t* g_rp, const int32_t* g_ci, const double* g_va,
                       const int8_t* cf, const int32_t* agg, int32_t ell, double theta, int32_t literal,
                       int32_t nthreads, int32_t* n_c_out, int64_t* nnz_out, int32_t* sizes) {
  const int32_t* rp = g_rp;
  const int32_t* ci = g_ci;
  const double* va = g_va;
  if (ell < 1 || !(theta >= 0.0 && theta <= 1.0) || check_csr(n, rp, ci)) return ORC_ERR_INVALID;
  double* cmax = NULL;
  if (theta > 0.0) {
    cmax = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!cmax) return ORC_ERR_NOMEM;
    column_max(n, rp, ci, va, cmax);
  }
  agg_lists ag = {NULL, NULL};
  if (agg) {
    int32_t *mrp = NULL, *mem = NULL;
    if (build_agg_lists(n, cf, agg, &mrp, &mem)) { free(cmax); return ORC_ERR_NOMEM; }
    ag.mrp = mrp;
    ag.mem = mem;
  }
  int32_t n_c = 0;
  for (int32_t j = 0; j < n; ++j) n_c += (cf[j] != 0);
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
  if (!clist) { free(cmax); free((void*)ag.mrp); free((void*)ag.mem); return ORC_ERR_NOMEM; }
  for (int32_t j = 0, r = 0; j < n; ++j) if (cf[j]) clist[r++] = j;
  int64_t total = 0;
  int err = 0;
  int nt = set_threads(nthreads);
#pragma omp parallel num_threads(nt) reduction(+ : total)
  {
    bfs_ws w;
    w.mark = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    w.stamp = 0; w.list = NULL; w.cap = 0;
    if (!w.mark) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(static)
      for (int32_t r = 0; r < n_c; ++r) {
        int32_t s = neighbourhood(clist[r], ell, rp, ci, va, cf, theta, cmax, agg ? &ag : NULL, &w, literal);
        if (s < 0) {
#pragma omp atomic write
          err = 1;
          continue;
        }
        if (sizes) sizes[r] = s;
        total += s + 1;
      }
    }
    free(w.mark);
    free(w.list);
  }
  free(clist);
  free(cmax);
  free((void*)ag.mrp);
  free((void*)ag.mem);
  if (err) return ORC_ERR_NOMEM;
  *n_c_out = n_c;
  *nnz_out = total;
  return ORC_OK;
}

int orc_pattern_size(int32_t n, const int32_t* rp, const int32_t* ci, const double* va,
                     const int8_t* cf, const int32_t* agg, int32_t ell, double theta, int32_t nthreads,
                     int32_t* n_c_out, int64_t* nnz_out, int32_t* sizes) {
  return orc_pattern_size_g(n, rp, ci, va, cf, agg, ell, theta, 0, nthreads, n_c_out, nnz_out, sizes);
}

/*
 * Build R.  B may be NULL (unconstrained: plain l-AIR rows, Remark 1).
 * R_rp has n_c+1 entries; R_ci/R_va have `cap` entries.  Statistics (may be
 * NULL): n_uncovered = F-points with d_j = 0 (only when B is given);
 * bad_row = fine index of the first C-row whose local block is singular.
 */
int orc_build_R_g(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, const int32_t* g_rp,
                  const int32_t* g_ci, const double* g_va, const int8_t* cf, const int32_t* agg, const double* B,
                  int32_t ell, double theta, int32_t literal, int32_t nthreads, int32_t* R_rp, int32_t* R_ci,
                  double* R_va, int64_t cap, int64_t* n_uncovered, int32_t* bad_row);

int orc_build_R(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, const int8_t* cf,
                const int32_t* agg, const double* B, int32_t ell, double theta, int32_t nthreads, int32_t* R_rp,
                int32_t* R_ci, double* R_va, int64_t cap, int64_t* n_uncovered, int32_t* bad_row) {
  return orc_build_R_g(n, rp, ci, va, rp, ci, va, cf, agg, B, ell, theta, 0, nthreads, R_rp, R_ci, R_va, cap,
                       n_uncovered, bad_row);
}

/* The same with the search on the graph G (A, or a strength matrix); the
   local systems always use A. */
int orc_build_R_g(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, const int32_t* g_rp,
                  const int32_t* g_ci, const double* g_va, const int8_t* cf, const int32_t* agg, const double* B,
                  int32_t ell, double theta, int32_t literal, int32_t nthreads, int32_t* R_rp, int32_t* R_ci,
                  double* R_va, int64_t cap, int64_t* n_uncovered, int32_t* bad_row) {
  if (ell < 1 || !(theta >= 0.0 && theta <= 1.0) || check_csr(n, rp, ci) || check_csr(n, g_rp, g_ci))
    return ORC_ERR_INVALID;
  int32_t n_c = 0;
  int64_t nnz = 0;
  for (int32_t j = 0; j < n; ++j) n_c += (cf[j] != 0);
  int32_t* sizes = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
  if (!sizes || !clist) { free(sizes); free(clist); return ORC_ERR_NOMEM; }
  int rc = orc_pattern_size_g(n, g_rp, g_ci, g_va, cf, agg, ell, theta, literal, nthreads, &n_c, &nnz, sizes);
  if (rc) { free(sizes); free(clist); return rc; }
  if (nnz > cap) { free(sizes); free(clist); return ORC_ERR_CAPACITY; }
  double* cmax = NULL;
  if (theta > 0.0) {
    cmax = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!cmax) { free(sizes); free(clist); return ORC_ERR_NOMEM; }
    column_max(n, g_rp, g_ci, g_va, cmax);
  }
  agg_lists ag = {NULL, NULL};
  if (agg) {
    int32_t *mrp = NULL, *mem = NULL;
    if (build_agg_lists(n, cf, agg, &mrp, &mem)) { free(sizes); free(clist); free(cmax); return ORC_ERR_NOMEM; }
    ag.mrp = mrp;
    ag.mem = mem;
  }
  for (int32_t j = 0, r = 0; j < n; ++j) if (cf[j]) clist[r++] = j;
  R_rp[0] = 0;
  for (int32_t r = 0; r < n_c; ++r) R_rp[r + 1] = R_rp[r] + sizes[r] + 1;

  /* Step 1: per-row local l-AIR solves, (A[N,N])^T z = -A[i,N]^T. */
  int32_t first_bad = -1;
  int err = 0;
  int nt = set_threads(nthreads);
#pragma omp parallel num_threads(nt)
  {
    bfs_ws w;
    w.mark = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    w.stamp = 0; w.list = NULL; w.cap = 0;
    double* K = NULL;
    double* f = NULL;
    int64_t kcap = 0;
    if (!w.mark) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(dynamic, 64)
      for (int32_t r = 0; r < n_c; ++r) {
        int32_t i = clist[r];
        int32_t s = neighbourhood(i, ell, g_rp, g_ci, g_va, cf, theta, cmax, agg ? &ag : NULL, &w, literal);
        if (s < 0) {
#pragma omp atomic write
          err = 1;
          continue;
        }
        if ((int64_t)s * s > kcap || !K) {
          kcap = (int64_t)s * s + 64;
          free(K); free(f);
          K = (double*)malloc(sizeof(double) * (size_t)kcap);
          f = (double*)malloc(sizeof(double) * (size_t)(s + 8));
          if (!K || !f) {
#pragma omp atomic write
            err = 1;
            kcap = 0;
            continue;
          }
        }
        const int32_t* N = w.list;
        /* K = (A[N,N])^T : K[q][p] = a_{N_p, N_q};  f = -A[i, N]. */
        memset(K, 0, sizeof(double) * (size_t)s * (size_t)s);
        for (int32_t p = 0; p < s; ++p) {
          int32_t row = N[p];
          for (int32_t e = rp[row]; e < rp[row + 1]; ++e) {
            int32_t q = find_sorted(N, s, ci[e]);
            if (q >= 0) K[(int64_t)q * s + p] = va[e];
          }
        }
        for (int32_t q = 0; q < s; ++q) f[q] = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
          int32_t q = find_sorted(N, s, ci[e]);
          if (q >= 0) f[q] = -va[e];
        }
        if (s > 0 && gepp_solve(K, f, s)) {
#pragma omp critical
          {
            if (first_bad < 0 || i < first_bad) first_bad = i;
          }
          for (int32_t q = 0; q < s; ++q) f[q] = 0.0;
        }
        /* Row r of R: the F-entries of N(i) and the injected C-point i (= 1). */
        int32_t pos = R_rp[r];
        int inserted = 0;
        for (int32_t p = 0; p < s; ++p) {
          if (!inserted && i < N[p]) { R_ci[pos] = i; R_va[pos] = 1.0; ++pos; inserted = 1; }
          R_ci[pos] = N[p]; R_va[pos] = f[p]; ++pos;
        }
        if (!inserted) { R_ci[pos] = i; R_va[pos] = 1.0; ++pos; }
      }
    }
    free(K); free(f); free(w.mark); free(w.list);
  }
  free(sizes);
  free(cmax);
  free((void*)ag.mrp);
  free((void*)ag.mem);
  if (err) { free(clist); return ORC_ERR_NOMEM; }
  if (bad_row) *bad_row = first_bad;

  /* Step 2: Euclidean projection onto {Q w = B|_F}, column by column. */
  int64_t uncovered = 0;
  if (B) {
    double* d = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* rs = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!d || !rs) { free(d); free(rs); free(clist); return ORC_ERR_NOMEM; }
    for (int32_t r = 0; r < n_c; ++r) {
      double bi = B[clist[r]];
      for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) {
        int32_t j = R_ci[e];
        if (j == clist[r]) continue;
        d[j] += bi * bi;
        rs[j] += R_va[e] * bi;
      }
    }
    for (int32_t j = 0; j < n; ++j) {
      if (cf[j]) continue;
      if (d[j] > 0.0) rs[j] -= B[j]; else ++uncovered;
    }
    for (int32_t r = 0; r < n_c; ++r) {
      double bi = B[clist[r]];
      for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) {
        int32_t j = R_ci[e];
        if (j == clist[r] || !(d[j] > 0.0)) continue;
        R_va[e] -= bi * rs[j] / d[j];
      }
    }
    free(d);
    free(rs);
  }
  if (n_uncovered) *n_uncovered = uncovered;
  free(clist);
  return first_bad >= 0 ? ORC_ERR_SINGULAR : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* k constraint vectors (Section 2.3 allows a block of constraint vectors;    */
/* Section 3.1's Q then has k rows per F-point).  B is n x k, row-major.      */
/* For each F-column j with contributing rows I_j:                            */
/*   G_j = sum_i B_i B_i^T (k x k),  r_j = sum_i z_ij B_i - B_j,              */
/*   lambda_j = pinv(G_j) r_j,       z_ij -= B_i^T lambda_j,                  */
/* the Euclidean projection onto {Q w = B_F}; Q Q^T is block diagonal with    */
/* the G_j.  pinv drops eigenvalues <= rcond * the largest (symmetric         */
/* Jacobi eigen-decomposition).  Applied in place to R's F-entries.           */
/* ------------------------------------------------------------------------ */

/* eigen-decomposition of the symmetric k x k matrix a (destroyed): values w,
 * vectors in the columns of v (row-major k x k); cyclic Jacobi rotations */
static void sym_eig(int k, double* a, double* w, double* v) {
  for (int p = 0; p < k; ++p)
    for (int q = 0; q < k; ++q) v[p * k + q] = (p == q) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < k; ++p) {
      diag += a[p * k + p] * a[p * k + p];
      for (int q = p + 1; q < k; ++q) off += a[p * k + q] * a[p * k + q];
    }
    if (off <= 1e-40 * diag || off == 0.0) break;
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        const double apq = a[p * k + q];
        if (apq == 0.0) continue;
        /* rotation angle that zeroes a_pq */
        const double theta = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int m = 0; m < k; ++m) { /* columns p, q */
          const double amp = a[m * k + p], amq = a[m * k + q];
          a[m * k + p] = c * amp - sn * amq;
          a[m * k + q] = sn * amp + c * amq;
        }
        for (int m = 0; m < k; ++m) { /* rows p, q */
          const double apm = a[p * k + m], aqm = a[q * k + m];
          a[p * k + m] = c * apm - sn * aqm;
          a[q * k + m] = sn * apm + c * aqm;
        }
        for (int m = 0; m < k; ++m) {
          const double vmp = v[m * k + p], vmq = v[m * k + q];
          v[m * k + p] = c * vmp - sn * vmq;
          v[m * k + q] = sn * vmp + c * vmq;
        }
      }
    }
  }
  for (int p = 0; p < k; ++p) w[p] = a[p * k + p];
}

int orc_project_k(int32_t n, int32_t n_c, const int32_t* R_rp, const int32_t* R_ci, double* R_va, const int8_t* cf,
                  const double* B, int32_t k, double rcond, int64_t* n_uncovered) {
  if (n < 0 || n_c < 0 || k < 1 || k > 8 || !(rcond >= 0.0)) return ORC_ERR_INVALID;
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
  double* G = (double*)calloc((size_t)(n > 0 ? n : 1) * (size_t)(k * k), sizeof(double));
  double* r = (double*)calloc((size_t)(n > 0 ? n : 1) * (size_t)k, sizeof(double));
  char* cov = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!clist || !G || !r || !cov) { free(clist); free(G); free(r); free(cov); return ORC_ERR_NOMEM; }
  for (int32_t j = 0, q = 0; j < n && q < n_c; ++j) if (cf[j]) clist[q++] = j;
  for (int32_t q = 0; q < n_c; ++q) {
    const double* bi = B + (int64_t)clist[q] * k;
    for (int32_t e = R_rp[q]; e < R_rp[q + 1]; ++e) {
      const int32_t j = R_ci[e];
      if (cf[j]) continue;
      cov[j] = 1;
      for (int a = 0; a < k; ++a) {
        r[(int64_t)j * k + a] += R_va[e] * bi[a];
        for (int b = 0; b < k; ++b) G[(int64_t)j * k * k + a * k + b] += bi[a] * bi[b];
      }
    }
  }
  int64_t unc = 0;
  double a[64], w[8], v[64], lam[8];
  for (int32_t j = 0; j < n; ++j) {
    if (cf[j]) continue;
    if (!cov[j]) { ++unc; continue; }
    double* rj = r + (int64_t)j * k;
    for (int t = 0; t < k; ++t) rj[t] -= B[(int64_t)j * k + t];
    memcpy(a, G + (int64_t)j * k * k, sizeof(double) * k * k);
    sym_eig(k, a, w, v);
    double wmax = 0.0;
    for (int t = 0; t < k; ++t) wmax = fmax(wmax, fabs(w[t]));
    for (int t = 0; t < k; ++t) lam[t] = 0.0;
    for (int m = 0; m < k; ++m) {
      if (!(fabs(w[m]) > rcond * wmax)) continue;
      double proj = 0.0;
      for (int t = 0; t < k; ++t) proj += v[t * k + m] * rj[t];
      for (int t = 0; t < k; ++t) lam[t] += v[t * k + m] * proj / w[m];
    }
    memcpy(rj, lam, sizeof(double) * k); /* r_j now holds lambda_j */
  }
  for (int32_t q = 0; q < n_c; ++q) {
    const double* bi = B + (int64_t)clist[q] * k;
    for (int32_t e = R_rp[q]; e < R_rp[q + 1]; ++e) {
      const int32_t j = R_ci[e];
      if (cf[j]) continue;
      double dz = 0.0;
      for (int t = 0; t < k; ++t) dz += bi[t] * r[(int64_t)j * k + t];
      R_va[e] -= dz;
    }
  }
  if (n_uncovered) *n_uncovered = unc;
  free(clist); free(G); free(r); free(cov);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Approximate block inverses (Section 3.1.2: a block-diagonal approximate     */
/* inverse of A_ff^{(*)}, one block per C-point, e.g. diagonal or ILU; the    */
/* footnote of the comparison with root-node names the local diagonal         */
/* inverse).  Algorithm 1 with such inverses, on the pattern of an R built    */
/* beforehand:                                                                 */
/*   tentative weights -a_ij on the pattern;                                   */
/*   with B: each F-column j is replaced by the minimum-norm solution of its  */
/*     constraint, z_ij = B_i B_j / d_j, d_j = sum_{i in I_j} B_i^2;          */
/*   `iterations` times:                                                       */
/*     residual of row i on its pattern: rho_ij = -(R A)_ij, j in N(i)        */
/*       (R's row holds z on N(i) and 1 at i, so (R A)_ij = a_ij +            */
/*       sum_{l in N(i)} z_il a_lj: the residual -a_i - A[N,N]^T z_i);        */
/*     u_i = Khat_i^{-1} rho_i with K_i = A[N,N]^T: inverse = 1 takes the     */
/*       diagonal (u_ij = rho_ij / a_jj), inverse = 2 the incomplete LU       */
/*       factorisation of K_i without fill (ILU(0): the factors keep K_i's    */
/*       nonzero pattern; row-oriented elimination, unit lower factor),       */
/*       inverse = 3 `krylov` steps of GMRES on K_i u = rho_i from u = 0      */
/*       (the minimal residual over the Krylov space; Arnoldi with modified   */
/*       Gram-Schmidt, Givens rotations; it stops early when the new basis    */
/*       vector's norm is at most 1e-12 of the vector it came from);          */
/*     with B: u_ij -= B_i (sum_i u_ij B_i) / d_j (the projection; Q Q^T is  */
/*       diagonal);                                                            */
/*     z += u.                                                                 */
/* The residual is formed row by row: row i of R times the rows of A.         */
/* Returns ORC_ERR_SINGULAR (bad_row = the smallest C-point concerned) when a */
/* pattern column has no nonzero diagonal entry (diagonal) or a pivot of the  */
/* incomplete factorisation is zero (ILU(0)).                                 */
/* ------------------------------------------------------------------------ */
/* ILU(0) of the s x s matrix K (row-major) in place: multipliers below the
   diagonal (unit lower factor), U on and above; only positions where K is
   nonzero on entry are updated.  Returns 1 on a zero pivot. */
static int ilu0(double* K, int32_t s, unsigned char* mask) {
  for (int64_t t = 0; t < (int64_t)s * s; ++t) mask[t] = K[t] != 0.0;
  for (int32_t a = 0; a < s; ++a) {
    for (int32_t b = 0; b < a; ++b) {
      if (!mask[(int64_t)a * s + b]) continue;
      K[(int64_t)a * s + b] /= K[(int64_t)b * s + b];
      const double m = K[(int64_t)a * s + b];
      for (int32_t c = b + 1; c < s; ++c)
        if (mask[(int64_t)a * s + c]) K[(int64_t)a * s + c] -= m * K[(int64_t)b * s + c];
    }
    if (K[(int64_t)a * s + a] == 0.0) return 1;
  }
  return 0;
}

/* x = (L U)^{-1} x with the factors of ilu0 */
static void ilu0_solve(const double* K, int32_t s, double* x) {
  for (int32_t a = 0; a < s; ++a)
    for (int32_t b = 0; b < a; ++b) x[a] -= K[(int64_t)a * s + b] * x[b];
  for (int32_t a = s - 1; a >= 0; --a) {
    for (int32_t c = a + 1; c < s; ++c) x[a] -= K[(int64_t)a * s + c] * x[c];
    x[a] /= K[(int64_t)a * s + a];
  }
}

/* x = the GMRES(m) approximation of K^{-1} b from x = 0 (K s x s row-major);
   work: (m + 1) * s + (m + 1) * m + 3 * (m + 1) doubles */
static void gmres_apply(const double* K, int32_t s, int32_t m, const double* b, double* x, double* work) {
  double* V = work;                      /* (m + 1) x s, rows are basis vectors */
  double* H = V + (int64_t)(m + 1) * s;  /* (m + 1) x m, column j = step j */
  double* cs = H + (int64_t)(m + 1) * m;
  double* sn = cs + (m + 1);
  double* g = sn + (m + 1);
  for (int32_t a = 0; a < s; ++a) x[a] = 0.0;
  double beta = 0.0;
  for (int32_t a = 0; a < s; ++a) beta += b[a] * b[a];
  beta = sqrt(beta);
  if (beta == 0.0 || m == 0) return;
  for (int32_t a = 0; a < s; ++a) V[a] = b[a] / beta;
  for (int32_t t = 0; t <= m; ++t) g[t] = 0.0;
  g[0] = beta;
  int32_t k = 0;
  for (int32_t j = 0; j < m; ++j) {
    double* w = V + (int64_t)(j + 1) * s;
    for (int32_t a = 0; a < s; ++a) {
      double acc = 0.0;
      for (int32_t c = 0; c < s; ++c) acc += K[(int64_t)a * s + c] * V[(int64_t)j * s + c];
      w[a] = acc;
    }
    double w0 = 0.0;
    for (int32_t a = 0; a < s; ++a) w0 += w[a] * w[a];
    w0 = sqrt(w0);
    for (int32_t i = 0; i <= j; ++i) {
      double h = 0.0;
      for (int32_t a = 0; a < s; ++a) h += w[a] * V[(int64_t)i * s + a];
      H[(int64_t)i * m + j] = h;
      for (int32_t a = 0; a < s; ++a) w[a] -= h * V[(int64_t)i * s + a];
    }
    double hn = 0.0;
    for (int32_t a = 0; a < s; ++a) hn += w[a] * w[a];
    hn = sqrt(hn);
    /* earlier rotations on column j, then the one that zeroes H[j+1][j] */
    for (int32_t i = 0; i < j; ++i) {
      const double h0 = H[(int64_t)i * m + j], h1 = H[(int64_t)(i + 1) * m + j];
      H[(int64_t)i * m + j] = cs[i] * h0 + sn[i] * h1;
      H[(int64_t)(i + 1) * m + j] = -sn[i] * h0 + cs[i] * h1;
    }
    const double hjj = H[(int64_t)j * m + j];
    const double rr = sqrt(hjj * hjj + hn * hn);
    cs[j] = rr > 0.0 ? hjj / rr : 1.0;
    sn[j] = rr > 0.0 ? hn / rr : 0.0;
    H[(int64_t)j * m + j] = rr;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    k = j + 1;
    if (!(hn > 1e-12 * w0)) break; /* the Krylov space is invariant: exact */
    for (int32_t a = 0; a < s; ++a) w[a] /= hn;
  }
  /* H[0..k)[0..k) y = g[0..k), then x = V y */
  double* y = g; /* solved in place */
  for (int32_t i = k - 1; i >= 0; --i) {
    double v = y[i];
    for (int32_t c = i + 1; c < k; ++c) v -= H[(int64_t)i * m + c] * y[c];
    y[i] = H[(int64_t)i * m + i] != 0.0 ? v / H[(int64_t)i * m + i] : 0.0;
  }
  for (int32_t i = 0; i < k; ++i)
    for (int32_t a = 0; a < s; ++a) x[a] += y[i] * V[(int64_t)i * s + a];
}

int orc_iterate_approx(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, const int8_t* cf,
                       const double* B, int32_t n_c, const int32_t* R_rp, const int32_t* R_ci, double* R_va,
                       int32_t inverse, int32_t krylov, int32_t iterations, int32_t* bad_row) {
  if (iterations < 0 || inverse < 1 || inverse > 3 || (inverse == 3 && (krylov < 1 || krylov > 64)) ||
      check_csr(n, rp, ci))
    return ORC_ERR_INVALID;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const int64_t nnz = R_rp[n_c];
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_c > 0 ? n_c : 1));
  double* diag = (double*)calloc(nn, sizeof(double));
  double* d = (double*)calloc(nn, sizeof(double));
  double* sj = (double*)calloc(nn, sizeof(double));
  double* u = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  if (!clist || !diag || !d || !sj || !u) {
    free(clist); free(diag); free(d); free(sj); free(u);
    return ORC_ERR_NOMEM;
  }
  int32_t nc_seen = 0;
  for (int32_t j = 0; j < n; ++j)
    if (cf[j]) {
      if (nc_seen < n_c) clist[nc_seen] = j;
      ++nc_seen;
    }
  if (nc_seen != n_c) {
    free(clist); free(diag); free(d); free(sj); free(u);
    return ORC_ERR_INVALID;
  }
  for (int32_t j = 0; j < n; ++j)
    for (int32_t e = rp[j]; e < rp[j + 1]; ++e)
      if (ci[e] == j) diag[j] += va[e];
  int32_t first_bad = -1;
  if (inverse == 1)
    for (int32_t r = 0; r < n_c && first_bad < 0; ++r)
      for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e)
        if (R_ci[e] != clist[r] && diag[R_ci[e]] == 0.0) { first_bad = clist[r]; break; }
  /* ILU(0) factors of every block K_i = A[N,N]^T (N = the row's F-columns) */
  double* fac = NULL;
  int64_t* foff = NULL;
  if (inverse >= 2 && first_bad < 0) {
    foff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_c + 1));
    if (!foff) { free(clist); free(diag); free(d); free(sj); free(u); return ORC_ERR_NOMEM; }
    foff[0] = 0;
    int32_t smax = 0;
    for (int32_t r = 0; r < n_c; ++r) {
      const int32_t sr = R_rp[r + 1] - R_rp[r] - 1;
      foff[r + 1] = foff[r] + (int64_t)sr * sr;
      if (sr > smax) smax = sr;
    }
    fac = (double*)calloc((size_t)(foff[n_c] > 0 ? foff[n_c] : 1), sizeof(double));
    int32_t* N = (int32_t*)malloc(sizeof(int32_t) * (size_t)(smax > 0 ? smax : 1));
    unsigned char* mask = (unsigned char*)malloc((size_t)smax * smax + 1);
    if (!fac || !N || !mask) {
      free(fac); free(foff); free(N); free(mask); free(clist); free(diag); free(d); free(sj); free(u);
      return ORC_ERR_NOMEM;
    }
    for (int32_t r = 0; r < n_c && first_bad < 0; ++r) {
      const int32_t i = clist[r];
      int32_t sr = 0;
      for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e)
        if (R_ci[e] != i) N[sr++] = R_ci[e];
      double* K = fac + foff[r];
      /* K[q][p] = a_{N_p, N_q} */
      for (int32_t p2 = 0; p2 < sr; ++p2) {
        const int32_t row = N[p2];
        for (int32_t e = rp[row]; e < rp[row + 1]; ++e) {
          const int32_t q = find_sorted(N, sr, ci[e]);
          if (q >= 0) K[(int64_t)q * sr + p2] += va[e];
        }
      }
      if (inverse == 2 && sr > 0 && ilu0(K, sr, mask)) first_bad = i;
    }
    free(N);
    free(mask);
  }
  if (first_bad >= 0) {
    if (bad_row) *bad_row = first_bad;
    free(fac); free(foff); free(clist); free(diag); free(d); free(sj); free(u);
    return ORC_ERR_SINGULAR;
  }
  int32_t maxlen = 1;
  for (int32_t r = 0; r < n_c; ++r)
    if (R_rp[r + 1] - R_rp[r] > maxlen) maxlen = R_rp[r + 1] - R_rp[r];
  double* xs = (double*)malloc(sizeof(double) * (size_t)maxlen * 2);
  const int32_t km = inverse == 3 ? krylov : 0;
  const size_t gsize = (size_t)(km + 1) * (size_t)maxlen + (size_t)(km + 1) * km + 3 * (size_t)(km + 1);
  double* gw = (double*)malloc(sizeof(double) * gsize);
  if (!xs || !gw) {
    free(xs); free(gw); free(fac); free(foff); free(clist); free(diag); free(d); free(sj); free(u);
    return ORC_ERR_NOMEM;
  }
  /* tentative weights, then the constraint fit */
  for (int32_t r = 0; r < n_c; ++r) {
    const int32_t i = clist[r];
    for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) {
      const int32_t j = R_ci[e];
      if (j == i) { R_va[e] = 1.0; continue; }
      double a = 0.0;
      for (int32_t t = rp[i]; t < rp[i + 1]; ++t)
        if (ci[t] == j) a += va[t];
      R_va[e] = -a;
      if (B) d[j] += B[i] * B[i];
    }
  }
  if (B)
    for (int32_t r = 0; r < n_c; ++r) {
      const int32_t i = clist[r];
      for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) {
        const int32_t j = R_ci[e];
        if (j == i) continue;
        R_va[e] = d[j] > 0.0 ? B[i] * B[j] / d[j] : 0.0;
      }
    }
  for (int32_t it = 0; it < iterations; ++it) {
    /* u = D^{-1} (-(R A)) on the pattern, every row from the same R */
    for (int32_t r = 0; r < n_c; ++r) {
      const int32_t i = clist[r];
      const int32_t e0 = R_rp[r], len = R_rp[r + 1] - e0;
      for (int32_t e = e0; e < e0 + len; ++e) u[e] = 0.0;
      for (int32_t e = e0; e < e0 + len; ++e) {
        const int32_t l = R_ci[e];
        const double zl = R_va[e];
        for (int32_t t = rp[l]; t < rp[l + 1]; ++t) {
          const int32_t p = find_sorted(R_ci + e0, len, ci[t]);
          if (p >= 0) u[e0 + p] += zl * va[t];
        }
      }
      if (inverse == 1) {
        for (int32_t e = e0; e < e0 + len; ++e) {
          const int32_t j = R_ci[e];
          u[e] = (j == i) ? 0.0 : -u[e] / diag[j];
        }
      } else {
        /* the row's F-entries in order, then (L U)^{-1} */
        int32_t sr = 0;
        for (int32_t e = e0; e < e0 + len; ++e)
          if (R_ci[e] != i) xs[sr++] = -u[e];
        if (inverse == 2) {
          ilu0_solve(fac + foff[r], sr, xs);
        } else {
          memcpy(xs + maxlen, xs, sizeof(double) * (size_t)sr);
          gmres_apply(fac + foff[r], sr, km, xs + maxlen, xs, gw);
        }
        sr = 0;
        for (int32_t e = e0; e < e0 + len; ++e) u[e] = (R_ci[e] == i) ? 0.0 : xs[sr++];
      }
    }
    if (B) {
      memset(sj, 0, sizeof(double) * nn);
      for (int32_t r = 0; r < n_c; ++r)
        for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) sj[R_ci[e]] += u[e] * B[clist[r]];
      for (int32_t r = 0; r < n_c; ++r) {
        const int32_t i = clist[r];
        for (int32_t e = R_rp[r]; e < R_rp[r + 1]; ++e) {
          const int32_t j = R_ci[e];
          if (j != i && d[j] > 0.0) u[e] -= B[i] * sj[j] / d[j];
        }
      }
    }
    for (int64_t e = 0; e < nnz; ++e) R_va[e] += u[e];
  }
  free(xs); free(gw); free(fac); free(foff); free(clist); free(diag); free(d); free(sj); free(u);
  return ORC_OK;
}

int orc_max_threads(void) { return set_threads(0); }
