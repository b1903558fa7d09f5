// clair_device.h -- device-side types and building blocks of libclair.
//
// Layout of one setup pass over `nmat` matrices (all device memory):
//   MatDesc[nmat]     caller pointers + per-matrix geometry
//   MatStatus[nmat]   results and error state, reset by the host upload
//   chunk arrays      the fine points of every matrix are cut into chunks of
//                     `chunk` consecutive indices; the symbolic pass counts
//                     C-rows and nnz(R) per chunk
//   clocal / lnz      per chunk, the C-points of the chunk in ascending order
//                     and the exclusive prefix of (|N(i)|+1) inside the chunk,
//                     stored at the chunk's own fine offsets
//   chead / clink     the projection's column lists: per fine point the last R
//                     entry of its column, per R entry the previous one and
//                     the C-point of its row (a list per F-column, in no order)
//   slots A / B       sorted neighbourhoods of rows small enough for the
//                     lane-group solvers, per fine point
//   bin C             rows queued for the workgroup-per-row solver
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clair {

constexpr int kMaxBlock = 1024;  // largest |N(i)| accepted (CLAIR_MAX_BLOCK)

struct MatDesc {
  const int32_t* rp;
  const int32_t* ci;
  const double* va;
  const int8_t* cf;
  const double* B;  // may be null
  int32_t* Rrp;
  int32_t* Rci;
  double* Rva;
  int64_t nnz_cap;
  int32_t row_cap;
  int32_t n;
  int32_t ell;
  int32_t chunk0;   // first global chunk of this matrix
  int32_t nchunks;
  int32_t nnz;      // nnz(A)
  int64_t fine0;    // offset of this matrix in fine-indexed workspaces
  const double* cmax;  // largest off-diagonal |a_wv| of column v (filled when theta > 0)
  double theta;        // strength threshold of the search (0: every stored nonzero)
  // aggregation-based base pattern (null: classical, T = S_fc): the caller's
  // root of every point's aggregate, and the member lists built from it
  // (root c's F-members at agg_list[agg_rp[c] .. agg_rp[c+1]), agg_rp
  // offset to the matrix)
  const int32_t* agg;
  const int32_t* agg_rp;
  const int32_t* agg_list;
  // the graph of the neighbourhood search: A itself, or a strength matrix
  // the caller gives (n x n CSR; its stored entries u -> v are the edges,
  // theta filters them against its own column maxima)
  const int32_t* grp;
  const int32_t* gci;
  const double* gva;
  int64_t link_base;   // first entry of this matrix in the projection's column lists (capacities summed)
  // the compact adjacency of the search graph (null: the search reads the
  // graph's rows): adj_w slots per point, matrix-local indices
  const int32_t* fadj;
  int32_t literal;  // 1: the pattern of S^{ell-1} T taken literally (C-points may be interior vertices)
  int32_t pad;
};

// Pointers into device (global) memory.  Pointers that kernels load from a
// descriptor in memory are generic to the compiler, and generic (flat) loads
// count against the LDS/scalar wait counter too, so every LDS or scalar wait
// would also wait for them.  Kernels read the matrix descriptor through GDesc,
// whose loads and stores compile to global_* instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}

struct GDesc {
  gptr<const int32_t> rp;
  gptr<const int32_t> ci;
  gptr<const double> va;
  gptr<const int8_t> cf;
  gptr<const double> B;  // may be null
  gptr<int32_t> Rrp;
  gptr<int32_t> Rci;
  gptr<double> Rva;
  int64_t nnz_cap;
  int32_t row_cap;
  int32_t n;
  int32_t ell;
  int32_t chunk0;
  int32_t nchunks;
  int32_t nnz;
  int64_t fine0;
  gptr<const double> cmax;
  double theta;
  gptr<const int32_t> agg;
  gptr<const int32_t> agg_rp;
  gptr<const int32_t> agg_list;
  gptr<const int32_t> grp;
  gptr<const int32_t> gci;
  gptr<const double> gva;
  int64_t link_base;
  gptr<const int32_t> fadj;
  int32_t literal;
};

__device__ __forceinline__ GDesc gview(const MatDesc& m) {
  GDesc g;
  g.rp = to_global(m.rp);
  g.ci = to_global(m.ci);
  g.va = to_global(m.va);
  g.cf = to_global(m.cf);
  g.B = to_global(m.B);
  g.Rrp = to_global(m.Rrp);
  g.Rci = to_global(m.Rci);
  g.Rva = to_global(m.Rva);
  g.nnz_cap = m.nnz_cap;
  g.row_cap = m.row_cap;
  g.n = m.n;
  g.ell = m.ell;
  g.chunk0 = m.chunk0;
  g.nchunks = m.nchunks;
  g.nnz = m.nnz;
  g.fine0 = m.fine0;
  g.cmax = to_global(m.cmax);
  g.theta = m.theta;
  g.agg = to_global(m.agg);
  g.agg_rp = to_global(m.agg_rp);
  g.grp = to_global(m.grp);
  g.gci = to_global(m.gci);
  g.gva = to_global(m.gva);
  g.agg_list = to_global(m.agg_list);
  g.link_base = m.link_base;
  g.fadj = to_global(m.fadj);
  g.literal = m.literal;
  return g;
}

// The search's edge test beyond "stored, nonzero, off-diagonal": the pattern
// comes from the classical strength matrix of A^T (the matrix the algorithm
// runs on for R), in which v depends strongly on u when |a_uv| is at least
// theta times the largest off-diagonal magnitude of column v of A.
__device__ __forceinline__ bool strong_edge(double a_uv, int v, double theta, gptr<const double> cmax) {
  return theta == 0.0 || fabs(a_uv) >= theta * cmax[v];
}

struct MatStatus {
  int32_t status;      // clair_status code (0 = ok)
  int32_t first_bad;   // smallest fine index of a failing row (INT32_MAX = none)
  int32_t n_c;
  int32_t max_block;
  int64_t nnz;
  int64_t n_uncovered;
  int32_t refine_max;
  int32_t n_fp64;
  int32_t row_base;    // first global row of this matrix
  int32_t n_retry;     // rows whose BF16-update factorisation was redone with FP32 updates
  int64_t nz_base;     // first global R entry of this matrix (batch-wide numbering)
};

struct Counters {
  int32_t total_rows;  // sum of n_c over all matrices
  int32_t nA;          // rows for the small lane-group solver (|N| <= GA)
  int32_t nB;          // rows for the 32-lane solver (GA < |N| <= 32)
  int32_t nC;          // rows queued for the workgroup solver (larger, or FP32 not trusted)
  int32_t nbig;        // rows with more than 32 points queued for k_count_big
  int32_t nmid;        // chunks k_count left to k_count_mid (queued in midq)
  int32_t pad1, pad2;
};

// Row t of chunk c: fine offset base = fine0 + (c - chunk0) * chunk of its
// matrix; its sorted neighbourhood sits at slotA[(base + t) * GA] when
// |N| <= GA, else at slotB[(base + t) * 32] when |N| <= 32.  Rows for the
// workgroup solver are queued as c * chunk + t.
struct Work {
  MatDesc* desc;
  MatStatus* st;
  Counters* cnt;
  int32_t* chunk_nc;      // [nchunks]
  int32_t* chunk_nnz;     // [nchunks]
  int32_t* chunk_rbase;   // [nchunks+1] first global row of each chunk
  int64_t* chunk_nzglob;  // [nchunks] first R entry of each chunk, batch-wide
  int32_t* chunk_mat;     // [nchunks]
  int2* chunk_bins;       // [nchunks] rows of the chunk in bin A (x) and bin B (y)
  int32_t* row_block_chunk;  // [n_total / 256 + 2] chunk holding global row 256 b
  int32_t* clocal;        // [n_total] chunk-local C-points (negative while unsized)
  int32_t* lnz;           // [n_total] chunk-local prefix of |N(i)|+1
  int32_t* chead;         // [n_total] projection lists: the last R entry (batch-wide number) of each F-column, -1 = none
  int2* clink;            // [link_cap] per R entry (matrix m's entry p at desc[m].link_base + p): the column's
                          // previous entry and the row's C-point
  int32_t* slotA;         // [n_total * GA]
  int32_t* slotB;         // [n_total * 32]
  int32_t* binC;          // [capC] rows for the workgroup solver
  int32_t* chunk_unsized;  // [nchunks] rows of the chunk not yet sized (more than 32 points)
  int32_t* bigq;           // [capC] those rows, c * chunk + t
  int32_t* big_size;       // [n_total] their sizes, until the chunk's prefix is redone
  double* cmax;            // [n_total] column maxima for the strength test (theta > 0)
  int32_t* agg_cnt;        // [n_total] aggregate sizes, then fill cursors (aggregates given)
  int32_t* agg_rp;         // [n_total + 1] member-list offsets, batch-wide
  int32_t* agg_list;       // [n_total] members (matrix-local indices), sorted per root
  int32_t* agg_sums;       // scan scratch
  double* scratch;        // FP64 blocks for oversized rows: scratch_slots slots of scratch_stride doubles (may be null)
  int64_t scratch_slots;
  int64_t scratch_stride; // doubles per slot: the square of the largest block the host sized it for
  int64_t link_cap;       // entries of clink (the R capacities summed over the batch when any B is given)
  int32_t nmat;
  int32_t nchunks;
  int32_t chunk;
  int32_t GA;             // lane-group size of the small solver (8, 16 or 32)
  int32_t capC;
  int32_t adj_w;          // slots per point of the compact adjacency (0: none built)
  int32_t* fadj;          // [n_total * adj_w]
  int32_t bf16;           // 1: the workgroup solver's trailing updates take bfloat16 inputs
  int32_t pad1;
  int32_t* midq;          // [nchunks] chunks k_count left unfinished
};

// status codes (mirror clair_status)
enum : int32_t { ST_OK = 0, ST_INVALID = 1, ST_CAPACITY = 2, ST_SINGULAR = 3, ST_HIP = 4, ST_UNSUPPORTED = 5 };

// wavefront-local fence and barrier: lanes of one wavefront exchange data
// through LDS
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive prefix sum of v over the workgroup (blockDim.x a multiple of 64)
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  // sh: at least blockDim.x / 64 ints.  Inclusive scan inside each wavefront
  // (six shuffle steps), then the wavefront totals through LDS: two barriers.
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    const int t = sh[k];
    base += (k < wid) ? t : 0;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return base + x - v;
}

// index of the first element >= key in sorted a[0..len)
__device__ __forceinline__ int lower_bound_i32(const int* a, int len, int key) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int find_sorted(const int* a, int len, int key) {
  int p = lower_bound_i32(a, len, key);
  return (p < len && a[p] == key) ? p : -1;
}

// Sorting network over P (a power of two) registers, ascending; compile-time
// indices only.
template <int P>
__device__ __forceinline__ void bitonic_sort(int (&v)[P]) {
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int l = q ^ j;
        if (l > q) {
          const int a = v[q], b = v[l];
          const bool up = (q & k) == 0;
          v[q] = up ? min(a, b) : max(a, b);
          v[l] = up ? max(a, b) : min(a, b);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Compact adjacency of the search graph.  Expanding a point u adds the points
// v of its row that pass the search's edge test (stored nonzero, v != u,
// strong_edge, v an F-point).  A prepass writes that list once per point, in
// W int32 slots (ascending, padded with -1; kAdjOverflow in slot 0 when u has
// more than W), so that a search takes a whole level's frontier in one round
// of loads instead of reading row bounds, entries and C/F markers point by
// point.  Points that overflow are expanded from the graph's rows.
// ---------------------------------------------------------------------------
constexpr int kAdjOverflow = -2;
typedef int adj_v4 __attribute__((ext_vector_type(4)));

template <int W>
__device__ __forceinline__ void adj_load(gptr<const int32_t> __restrict__ adj, int u, int* o) {
  static_assert(W % 4 == 0, "adjacency rows are read as int4");
  const gptr<const adj_v4> p = (gptr<const adj_v4>)(adj + (int64_t)u * W);
#pragma unroll
  for (int q = 0; q < W / 4; ++q) {
    const adj_v4 t = p[q];
    o[4 * q] = t.x;
    o[4 * q + 1] = t.y;
    o[4 * q + 2] = t.z;
    o[4 * q + 3] = t.w;
  }
}

// Register-resident neighbourhood search of one thread, for neighbourhoods of
// at most SM <= 32 points.  N(i) = the F-points reachable from C-point i by a
// walk of at most ell edges (u -> v with u != v, a stored nonzero a_uv and
// strong_edge) whose interior vertices are F-points.  Points are appended in
// the order found, so the points first reached at one distance form a run
// [lo, hi) that the next level expands; an insert is a membership test and
// one slot write, and the set is sorted once at the end.
template <int SM>
struct RegSetA {
  static_assert(SM <= 32 && (SM & (SM - 1)) == 0, "a power of two up to 32");
  int v[SM];  // points in the order found, INT32_MAX beyond s
  int s;
  bool ovf;

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int j = 0; j < SM; ++j) v[j] = 0x7fffffff;
    s = 0;
    ovf = false;
  }
  __device__ __forceinline__ void insert(int k) {
    bool present = false;
#pragma unroll
    for (int j = 0; j < SM; ++j) present |= (v[j] == k);
    if (present) return;
    if (s == SM) { ovf = true; return; }
#pragma unroll
    for (int j = 0; j < SM; ++j)
      if (j == s) v[j] = k;
    ++s;
  }
  __device__ __forceinline__ int get(int p) const {
    int x = 0;
#pragma unroll
    for (int j = 0; j < SM; ++j)
      if (j == p) x = v[j];
    return x;
  }
};

// the F-neighbours of u from row u of the graph, eight entries per batch
template <int SM>
__device__ __forceinline__ void rowa_expand(RegSetA<SM>& S, int n, int u, gptr<const int32_t> __restrict__ rp,
                                            gptr<const int32_t> __restrict__ ci, gptr<const double> __restrict__ va,
                                            gptr<const int8_t> __restrict__ cf, double theta,
                                            gptr<const double> __restrict__ cmax) {
  const int e1 = rp[u + 1];
  for (int e = rp[u]; e < e1 && !S.ovf; e += 8) {
    int k[8];
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      k[j] = u;
      x[j] = 0.0;
      if (e + j < e1) { k[j] = ci[e + j]; x[j] = va[e + j]; }
    }
    int8_t c8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) c8[j] = ((unsigned)k[j] < (unsigned)n) ? cf[k[j]] : (int8_t)1;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k[j] != u && x[j] != 0.0 && c8[j] == 0 && strong_edge(x[j], k[j], theta, cmax)) S.insert(k[j]);
  }
}

// The search.  W = 4 or 8: expansions read the compact adjacency adj (the
// rows of points that overflow it are read instead), 32 / W frontier points
// at a time; W = 0: every expansion reads the graph's rows.  mrp/mem (may be
// null): the aggregate members that replace the first step.  Returns |N(i)|
// with S.v[0..s) ascending, or -1 when more than SM points are found.
template <int SM, int W>
__device__ __forceinline__ int rega_bfs(RegSetA<SM>& S, int n, int i, int ell, gptr<const int32_t> __restrict__ adj,
                                        gptr<const int32_t> __restrict__ rp, gptr<const int32_t> __restrict__ ci,
                                        gptr<const double> __restrict__ va, gptr<const int8_t> __restrict__ cf,
                                        double theta, gptr<const double> __restrict__ cmax,
                                        gptr<const int32_t> __restrict__ mrp, gptr<const int32_t> __restrict__ mem) {
  S.clear();
  if (mrp) {
    for (int e = mrp[i]; e < mrp[i + 1] && !S.ovf; ++e) S.insert(mem[e]);
  } else if constexpr (W > 0) {
    int a[W];
    adj_load<W>(adj, i, a);
    if (a[0] == kAdjOverflow) {
      rowa_expand(S, n, i, rp, ci, va, cf, theta, cmax);
    } else {
#pragma unroll
      for (int q = 0; q < W; ++q)
        if (a[q] >= 0) S.insert(a[q]);
    }
  } else {
    rowa_expand(S, n, i, rp, ci, va, cf, theta, cmax);
  }
  int lo = 0;
  for (int L = 2; L <= ell && !S.ovf; ++L) {
    const int hi = S.s;
    if (lo == hi) break;
    if constexpr (W > 0) {
      constexpr int FG = 32 / W;
      for (int p = lo; p < hi && !S.ovf; p += FG) {
        int u[FG];
        int a[FG][W];
#pragma unroll
        for (int g = 0; g < FG; ++g) u[g] = (p + g < hi) ? S.get(p + g) : -1;
#pragma unroll
        for (int g = 0; g < FG; ++g) {
          if (u[g] >= 0) {
            adj_load<W>(adj, u[g], a[g]);
          } else {
#pragma unroll
            for (int q = 0; q < W; ++q) a[g][q] = -1;
          }
        }
#pragma unroll
        for (int g = 0; g < FG; ++g) {
          if (u[g] < 0) continue;
          if (a[g][0] == kAdjOverflow) {
            rowa_expand(S, n, u[g], rp, ci, va, cf, theta, cmax);
          } else {
#pragma unroll
            for (int q = 0; q < W; ++q)
              if (a[g][q] >= 0) S.insert(a[g][q]);
          }
        }
      }
    } else {
      for (int p = lo; p < hi && !S.ovf; ++p) rowa_expand(S, n, S.get(p), rp, ci, va, cf, theta, cmax);
    }
    lo = hi;
  }
  if (S.ovf) return -1;
  bitonic_sort<SM>(S.v);
  return S.s;
}

// The literal reading of Algorithm 1's pattern S^{ell-1} T, T = [S_fc, I]:
// the first step reaches i's F-neighbours; the second step expands i itself
// (T's identity part) and those points; from the second step on, C-points
// may be interior vertices of a walk (they stay in the set until the last
// step and are dropped at the end); i never enters.  The graph's rows only
// (the compact adjacency lists F-points alone).  Returns |N(i)| with
// S.v[0..s) ascending, or -1 when more than SM points (C-points included)
// are met.
template <int SM>
__device__ __forceinline__ void rowa_expand_literal(RegSetA<SM>& S, int n, int u, int i, bool allow_c,
                                                    gptr<const int32_t> __restrict__ rp,
                                                    gptr<const int32_t> __restrict__ ci,
                                                    gptr<const double> __restrict__ va,
                                                    gptr<const int8_t> __restrict__ cf, double theta,
                                                    gptr<const double> __restrict__ cmax) {
  const int e1 = rp[u + 1];
  for (int e = rp[u]; e < e1 && !S.ovf; e += 8) {
    int k[8];
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      k[j] = u;
      x[j] = 0.0;
      if (e + j < e1) { k[j] = ci[e + j]; x[j] = va[e + j]; }
    }
    bool in[8];
    int8_t c8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      in[j] = (unsigned)k[j] < (unsigned)n;
      c8[j] = in[j] ? cf[k[j]] : (int8_t)0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (in[j] && k[j] != u && k[j] != i && x[j] != 0.0 && (c8[j] == 0 || allow_c) &&
          strong_edge(x[j], k[j], theta, cmax))
        S.insert(k[j]);
  }
}

template <int SM>
__device__ __forceinline__ int rega_bfs_literal(RegSetA<SM>& S, int n, int i, int ell,
                                                gptr<const int32_t> __restrict__ rp,
                                                gptr<const int32_t> __restrict__ ci,
                                                gptr<const double> __restrict__ va,
                                                gptr<const int8_t> __restrict__ cf, double theta,
                                                gptr<const double> __restrict__ cmax) {
  S.clear();
  rowa_expand_literal(S, n, i, i, false, rp, ci, va, cf, theta, cmax);
  int lo = 0;
  for (int L = 2; L <= ell && !S.ovf; ++L) {
    const int hi = S.s;
    const bool allow_c = L < ell;
    if (L == 2) rowa_expand_literal(S, n, i, i, allow_c, rp, ci, va, cf, theta, cmax);
    else if (lo == hi) break;
    for (int p = lo; p < hi && !S.ovf; ++p)
      rowa_expand_literal(S, n, S.get(p), i, allow_c, rp, ci, va, cf, theta, cmax);
    lo = hi;
  }
  if (S.ovf) return -1;
  // the C-points were interior vertices only
  int8_t c8[SM];
#pragma unroll
  for (int j = 0; j < SM; ++j) c8[j] = (S.v[j] != 0x7fffffff) ? cf[S.v[j]] : (int8_t)0;
  int f = 0;
#pragma unroll
  for (int j = 0; j < SM; ++j) {
    if (c8[j] != 0) S.v[j] = 0x7fffffff;
    f += S.v[j] != 0x7fffffff ? 1 : 0;
  }
  bitonic_sort<SM>(S.v);
  S.s = f;
  return f;
}

// matrix owning global chunk c (desc[].chunk0 ascending): the last matrix
// whose first chunk is at or before c.  For a wavefront whose 64 lanes all
// ask for the same c, with every lane active: lane l reads the first chunk
// of matrix b + l for blocks of 64 matrices and a ballot counts them, one
// round of loads per 64 matrices instead of a dependent binary search.
__device__ __forceinline__ int chunk_matrix(const MatDesc* desc, int nmat, int c) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int b = 0; b < nmat; b += 64) {
    const int k = b + lane;
    const uint64_t bal = __ballot(k < nmat && desc[k].chunk0 <= c);
    cnt += __popcll(bal);
    if (bal != ~0ull) break;  // ascending: no later matrix starts at or before c
  }
  return cnt > 0 ? cnt - 1 : 0;
}

__device__ __forceinline__ void flag_row(MatStatus* st, int32_t code, int fine_row) {
  atomicCAS(&st->status, 0, code);
  atomicMin(&st->first_bad, fine_row);
}

}  // namespace clair
