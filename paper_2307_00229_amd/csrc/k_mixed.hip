// k_mixed.hip -- the batched, mixed-precision restriction setup.
//
// Stages (one launch each, over all matrices of a batch):
//   k_adj        the compact adjacency of the search graph (ell >= 2, sparse
//                graphs): for every point, the F-points one step reaches.
//   k_count      symbolic pass per chunk of fine points: the C-points of the
//                chunk; rows at ell = 1 (up to 8 entries) and at ell = 2 over
//                a width-4 adjacency sized by one thread each from a sorted
//                candidate list and written to their slot; a chunk with every
//                row sized gets its chunk-local prefix of |N(i)|+1 here;
//                clears the projection's column lists of the chunk.
//   k_count_mid  the other rows of unfinished chunks: one thread per row, up
//                to 32 points in registers (over the adjacency when built),
//                then the chunk's prefix.  Rows of more than 32 points are
//                queued, unsized.
//   k_count_big  one workgroup per queued row: a workgroup-wide search sizes
//                it (queued for the workgroup solver); the last row of a chunk
//                to be sized redoes the chunk's prefix.
//   k_scan       one workgroup: chunk bases -> global row numbers, R offsets,
//                n_c and nnz(R) per matrix, bin sizes, capacity check,
//                R.row_ptr[n_c].
//   k_numeric    persistent over the rows in grid order (each XCD a contiguous
//                slice), G lanes per row with |N| <= G (bin A, G = GA), or with
//                GA < |N| <= 32 (bin B, G = 16 or 32): gather of the local
//                block into LDS, FP32 inverse (Gauss-Jordan) and FP64
//                iterative refinement of (A[N,N])^T z = -A[i,N]^T, R row
//                write, projection sums.  Rows whose FP32 factorisation is not
//                trusted are queued for k_rows_wg.
//                k_quad8 (4 lanes per row) and k_rows8 (one thread per row)
//                are the other bin-A solvers.
//   k_rows_wg    persistent, one workgroup per queued row: for 33..128 points
//                an FP32 blocked LU with matrix-core trailing updates and FP64
//                refinement; otherwise, or when that does not converge, FP64 LU
//                with partial pivoting (block in LDS, or in global scratch when
//                large).
//   k_project    persistent, one thread per row:
//                z_ij -= B_i (sum_k z_kj B_k - B_j) / sum_k B_k^2 per F-entry;
//                counts F-points no row reaches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>

#include "clair_device.h"
#include "clair_launch.h"

namespace clair {

namespace {

constexpr int kNT = 256;  // threads per workgroup of the symbolic pass
// workgroup-wide search caps
constexpr int kWN = kMaxBlock;
constexpr int kWC = 4096;

// Workgroup-wide neighbourhood search for rows of any size up to kWN points:
// the same set as rega_bfs (F-points reachable from C-point i by at most ell
// edges with F-points inside the walk).  The entries of a level's frontier
// rows are taken in windows of kWC: each window is sorted (bitonic, in LDS),
// reduced to points that are new (first of their run, not yet in N, not yet
// in this level) and merged into the level.  No bound on the number of
// candidates, so dense coarse-level rows work too.
struct WideBuf {
  int nb0[kWN], nb1[kWN];  // neighbourhood, double buffered, sorted
  int fr[kWN];             // frontier: the previous level's new points, sorted
  int nl[kWN];             // this level's new points so far, sorted
  int dp[kWN + 1];         // prefix of the frontier's row lengths
  int cand[kWC];           // window candidates (sorted in place)
  int kb[kWC];             // kept candidates of the window, sorted
  int sh[kNT];             // scan scratch
};

// Returns |N(i)| with the sorted list in *out, or -1 when it exceeds kWN
// (block-uniform).  Must be called by all kNT threads of the workgroup.
__device__ int block_bfs(int n, int i, int ell, gptr<const int32_t> __restrict__ rp, gptr<const int32_t> __restrict__ ci,
                         gptr<const double> __restrict__ va, gptr<const int8_t> __restrict__ cf, double theta,
                         gptr<const double> __restrict__ cmax, gptr<const int32_t> __restrict__ mrp,
                         gptr<const int32_t> __restrict__ mem, WideBuf& b, int** out, bool literal = false) {
  const int tid = threadIdx.x;
  constexpr int nt = kNT;
  int* cur = b.nb0;
  int* nxt = b.nb1;
  int s = 0;
  int fsz = 1;  // level-0 frontier is {i}
  int d0 = 1;
  if (mrp) {
    // aggregation-based: level 1 is the aggregate's F-points (sorted)
    const int a0 = mrp[i], na = mrp[i + 1] - a0;
    if (na > kWN) return -1;
    for (int t = tid; t < na; t += nt) {
      cur[t] = mem[a0 + t];
      b.fr[t] = mem[a0 + t];
    }
    __syncthreads();
    s = na;
    fsz = na;
    d0 = 2;
  }
  // literal reading (S^{ell-1} T taken as written): the second step also
  // expands i itself, C-points may be interior vertices until the last step
  // (and are dropped at the end), and i never enters
  for (int depth = d0; depth <= ell && (fsz > 0 || (literal && depth == 2)); ++depth) {
    const bool with_i = literal && depth == 2;  // frontier slot fsz is i
    const int fn = fsz + (with_i ? 1 : 0);
    const bool allow_c = literal && depth >= 2 && depth < ell;
    auto fu = [&](int t) { return (depth == 1 || (with_i && t == fsz)) ? i : b.fr[t]; };
    // row lengths of the frontier, prefix
    const int per = (fn + nt - 1) / nt;
    const int t0 = tid * per, t1 = min(t0 + per, fn);
    int sum = 0;
    for (int t = t0; t < t1; ++t) {
      const int u = fu(t);
      sum += rp[u + 1] - rp[u];
    }
    int E;
    int pre = block_exclusive_scan(sum, b.sh, &E);
    for (int t = t0; t < t1; ++t) {
      const int u = fu(t);
      b.dp[t] = pre;
      pre += rp[u + 1] - rp[u];
    }
    if (tid == 0) b.dp[fn] = E;
    __syncthreads();
    int nnl = 0;
    for (int w0 = 0; w0 < E; w0 += kWC) {
      const int wn = min(kWC, E - w0);
      int P = 1;
      while (P < wn) P <<= 1;
      for (int t = tid; t < P; t += nt) {
        int k = INT32_MAX;
        if (t < wn) {
          const int ef = w0 + t;
          int lo = 0, hi = fn - 1;  // last frontier vertex with dp <= ef
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.dp[mid] <= ef) lo = mid; else hi = mid - 1;
          }
          const int u = fu(lo);
          const int e = rp[u] + (ef - b.dp[lo]);
          const int kk = ci[e];
          if (kk != u && kk != i && (unsigned)kk < (unsigned)n && va[e] != 0.0 && (cf[kk] == 0 || allow_c) &&
              strong_edge(va[e], kk, theta, cmax))
            k = kk;
        }
        b.cand[t] = k;
      }
      __syncthreads();
      for (int kk = 2; kk <= P; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
          for (int t = tid; t < P; t += nt) {
            const int x = t ^ j;
            if (x > t) {
              const int a = b.cand[t], c2 = b.cand[x];
              if ((a > c2) == ((t & kk) == 0)) { b.cand[t] = c2; b.cand[x] = a; }
            }
          }
          __syncthreads();
        }
      }
      const int per2 = (P + nt - 1) / nt;
      const int q0 = tid * per2, q1 = min(q0 + per2, P);
      int kept = 0;
      for (int t = q0; t < q1; ++t) {
        const int x = b.cand[t];
        kept += (x != INT32_MAX && (t == 0 || b.cand[t - 1] != x) && find_sorted(cur, s, x) < 0 &&
                 find_sorted(b.nl, nnl, x) < 0) ? 1 : 0;
      }
      int kn;
      int kp = block_exclusive_scan(kept, b.sh, &kn);
      for (int t = q0; t < q1; ++t) {
        const int x = b.cand[t];
        if (x != INT32_MAX && (t == 0 || b.cand[t - 1] != x) && find_sorted(cur, s, x) < 0 &&
            find_sorted(b.nl, nnl, x) < 0)
          b.kb[kp++] = x;
      }
      __syncthreads();
      if (s + nnl + kn > kWN) return -1;
      for (int t = tid; t < nnl; t += nt) nxt[t + lower_bound_i32(b.kb, kn, b.nl[t])] = b.nl[t];
      for (int t = tid; t < kn; t += nt) nxt[t + lower_bound_i32(b.nl, nnl, b.kb[t])] = b.kb[t];
      __syncthreads();
      nnl += kn;
      for (int t = tid; t < nnl; t += nt) b.nl[t] = nxt[t];
      __syncthreads();
    }
    for (int t = tid; t < s; t += nt) nxt[t + lower_bound_i32(b.nl, nnl, cur[t])] = cur[t];
    for (int t = tid; t < nnl; t += nt) {
      nxt[t + lower_bound_i32(cur, s, b.nl[t])] = b.nl[t];
      b.fr[t] = b.nl[t];
    }
    __syncthreads();
    int* tmp = cur;
    cur = nxt;
    nxt = tmp;
    s += nnl;
    fsz = nnl;
  }
  if (literal) {  // the C-points were interior vertices only: keep the F-points, in order
    const int per = (s + nt - 1) / nt;
    const int t0 = tid * per, t1 = min(t0 + per, s);
    int kf = 0;
    for (int t = t0; t < t1; ++t) kf += cf[cur[t]] == 0 ? 1 : 0;
    int f;
    int pos = block_exclusive_scan(kf, b.sh, &f);
    for (int t = t0; t < t1; ++t)
      if (cf[cur[t]] == 0) nxt[pos++] = cur[t];
    __syncthreads();
    *out = nxt;
    return f;
  }
  *out = cur;
  return s;
}

// chunk index of global row g: binary search in chunk_rbase[0..nch]
__device__ __forceinline__ int row_chunk(const int32_t* rbase, int nch, int g) {
  int lo = 0, hi = nch - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rbase[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// chunk index of global row g (0 <= g < total rows): the chunk holding the
// first row of g's block of kRowBlock rows, then a short forward walk
constexpr int kRowBlockLog = 8;
__device__ __forceinline__ int row_chunk_fast(const Work& w, int g) {
  int c = w.row_block_chunk[g >> kRowBlockLog];
  while (w.chunk_rbase[c + 1] <= g) ++c;
  return c;
}

struct RowInfo {
  int m;     // matrix
  int i;     // fine index of the C-point
  int r;     // matrix-local row of R
  int off;   // first R entry of the row
  int s;     // |N(i)|
  int64_t fine0;
};

// row t of chunk c
__device__ __forceinline__ RowInfo row_info(const Work& w, int c, int t) {
  RowInfo ri;
  ri.m = w.chunk_mat[c];
  const GDesc d = gview(w.desc[ri.m]);
  const int64_t base = d.fine0 + (int64_t)(c - d.chunk0) * w.chunk;
  ri.i = w.clocal[base + t];
  const int l0 = w.lnz[base + t];
  const int l1 = (t + 1 < w.chunk_nc[c]) ? w.lnz[base + t + 1] : w.chunk_nnz[c];
  ri.off = (int)(w.chunk_nzglob[c] - w.st[ri.m].nz_base) + l0;
  ri.s = l1 - l0 - 1;
  ri.r = w.chunk_rbase[c] + t - w.st[ri.m].row_base;
  ri.fine0 = d.fine0;
  return ri;
}

__device__ __forceinline__ bool matrix_live(const MatStatus& st) {
  return st.status != ST_CAPACITY && st.status != ST_INVALID;
}

// F-entry (i, j) of R at position pos of its matrix: the value, and with a
// constraint vector the entry joins the list of column j for the projection
// (list entry link_base + pos, below the matrix's R capacity; one atomic
// exchange on the list head; the projection orders each list itself, so the
// exchange order does not matter)
__device__ __forceinline__ void put_f_entry(const Work& w, const GDesc& d, int64_t fine0, int pos, int j, int i,
                                            double z) {
  d.Rci[pos] = j;
  d.Rva[pos] = z;
  if (d.B) {
    const int64_t eg = d.link_base + pos;
    const int prev = atomicExch(&w.chead[fine0 + j], (int32_t)eg);
    w.clink[eg] = make_int2(prev, i);
  }
}

// Per-lane cache of the chunk a run of consecutive rows lies in: reloaded only
// when the row index crosses into another chunk, so a row costs one level of
// (coalesced) per-row loads instead of the chunk -> matrix -> descriptor chain.
struct ChunkCursor {
  int c = -1;
  int rb = 0, re = 0;   // global rows [rb, re) of chunk c
  int m = 0;
  int nc = 0;           // C-rows in the chunk
  int tot = 0;          // nnz(R) of the chunk
  int zoff = 0;         // R offset of the chunk inside its matrix
  int rbase_m = 0;      // first global row of the matrix
  int64_t fbase = 0;    // fine offset of the chunk's first point (batch-wide)
  int64_t fine0 = 0;    // fine offset of the matrix (batch-wide)
  bool live = false;
  GDesc md;             // the matrix's pointers and geometry

  __device__ __forceinline__ void seek(const Work& w, int g) {
    if (c >= 0 && g >= rb && g < re) return;
    c = row_chunk_fast(w, g);
    rb = w.chunk_rbase[c];
    re = w.chunk_rbase[c + 1];
    m = w.chunk_mat[c];
    md = gview(w.desc[m]);
    const MatStatus& st = w.st[m];
    nc = w.chunk_nc[c];
    tot = w.chunk_nnz[c];
    zoff = (int)(w.chunk_nzglob[c] - st.nz_base);
    rbase_m = st.row_base;
    fine0 = md.fine0;
    fbase = md.fine0 + (int64_t)(c - md.chunk0) * w.chunk;
    live = matrix_live(st);
  }
  // row g (inside the chunk): fine index, R offset and |N|
  __device__ __forceinline__ void row(const Work& w, int g, int* t, int* i, int* off, int* sz) const {
    const int tt = g - rb;
    *t = tt;
    *i = w.clocal[fbase + tt];
    const int l0 = w.lnz[fbase + tt];
    const int l1 = (tt + 1 < nc) ? w.lnz[fbase + tt + 1] : tot;
    *off = zoff + l0;
    *sz = l1 - l0 - 1;
  }
};


// Logical workgroup index: the hardware deals workgroups to the 8 XCDs
// round-robin (block b runs on XCD b % 8).  Give each XCD a contiguous range
// of logical indices, so the rows one XCD works on are neighbours in the grid
// and share its L2.
__device__ __forceinline__ int xcd_logical_block(int nb) {
  const int b = blockIdx.x;
  const int x = b % 8, q = nb / 8, r = nb % 8;
  return x * q + min(x, r) + b / 8;
}
__device__ __forceinline__ int xcd_logical_block() { return xcd_logical_block(gridDim.x); }
// The same ranges, each walked from its end: the first workgroups of an XCD
// take the last blocks of its range.
__device__ __forceinline__ int xcd_logical_block_reversed() {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int x = b % 8, q = nb / 8, r = nb % 8;
  return x * q + min(x, r) + (q + (x < r ? 1 : 0)) - 1 - b / 8;
}

// Rows of the persistent numeric kernels: XCD x (= blockIdx.x % 8, the
// hardware deals workgroups round-robin) owns a contiguous eighth of all
// rows, and its workgroups take blocks of nb rows from it in turn.  The rows
// in flight on one XCD at any time are then neighbours, whose blocks share A
// rows in that XCD's L2 (with a contiguous range per workgroup they would be
// as many separate streams through A as there are workgroups).
struct RowBlocks {
  int xb, xe, k, nx, nb;
  __device__ __forceinline__ RowBlocks(int total, int nb_) {
    const int x = blockIdx.x % 8;
    const int per = (total + 7) / 8;
    xb = min(total, x * per);
    xe = min(total, xb + per);
    nx = (int)gridDim.x / 8 + ((int)(gridDim.x % 8) > x ? 1 : 0);
    k = blockIdx.x / 8;
    nb = nb_;
  }
  // the j-th block of this workgroup: rows [*b, *e); false past the end
  __device__ __forceinline__ bool block(int j, int* b, int* e) const {
    const int64_t s0 = xb + ((int64_t)k + (int64_t)j * nx) * nb;
    if (s0 >= xe) return false;
    *b = (int)s0;
    *e = min(xe, (int)s0 + nb);
    return true;
  }
};

// Most refinement steps of the rows a thread (lane 0 of a group) finished,
// per matrix: gathered in registers and sent with one global atomic when the
// thread moves on to another matrix or ends (one atomic per row would meet
// at a handful of addresses in a batch of many matrices).
struct RefineMax {
  int m = -1, v = 0;
  __device__ __forceinline__ void flush(const Work& w) {
    if (m >= 0 && v > __hip_atomic_load(&w.st[m].refine_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&w.st[m].refine_max, v);
  }
  __device__ __forceinline__ void add(const Work& w, int mm, int it) {
    if (mm != m) {
      flush(w);
      m = mm;
      v = 0;
    }
    v = max(v, it);
  }
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// wave-aggregated queue append: every lane with `want` gets a distinct slot
// (or -1 once the queue is full); one atomic per wave
__device__ __forceinline__ int wave_append(bool want, int32_t* counter, int cap) {
  const uint64_t mask = __ballot(want);
  if (!mask) return -1;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader, 64);
  const int rank = __popcll(mask & ((1ull << lane_id()) - 1ull));
  const int slot = base + rank;
  return (want && slot < cap) ? slot : -1;
}

// ---------------------------------------------------------------------------
// validation: CSR sorted, in range; cf is not checked (any nonzero is C)
// ---------------------------------------------------------------------------
__global__ void k_validate(Work w) {
  for (int m = 0; m < w.nmat; ++m) {
    const GDesc d = gview(w.desc[m]);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
      const int e0 = d.rp[r], e1 = d.rp[r + 1];
      bool bad = (e1 < e0) || e0 < 0 || e1 > d.nnz || (r == 0 && e0 != 0) || (r == d.n - 1 && e1 != d.nnz);
      for (int e = e0; e < e1 && !bad; ++e) {
        const int k = d.ci[e];
        bad = (k < 0 || k >= d.n || (e > e0 && k <= d.ci[e - 1]));
      }
      if (d.grp != d.rp) {  // a strength matrix: sorted rows, indices in range
        const int g0 = d.grp[r], g1 = d.grp[r + 1];
        bad = bad || g1 < g0 || g0 < 0 || (r == 0 && g0 != 0);
        for (int e = g0; e < g1 && !bad; ++e) {
          const int k = d.gci[e];
          bad = (k < 0 || k >= d.n || (e > g0 && k <= d.gci[e - 1]));
        }
      }
      if (bad) flag_row(&w.st[m], ST_INVALID, r);
    }
  }
}

// ---------------------------------------------------------------------------
// symbolic pass
// ---------------------------------------------------------------------------

// rows the small solvers take: |N| <= 8 for the thread-per-row solver
// (GA == 1), |N| <= GA for the lane-group solver
__device__ __forceinline__ int small_limit(int GA) { return GA <= 4 ? 8 : GA; }
// stride of a row's slot in slotA
__device__ __forceinline__ int slot_stride(int GA) { return GA <= 4 ? 8 : GA; }

// The compact adjacency of the matrices whose descriptor carries one: the
// workgroup of logical block b takes 256 * kAdjPP points of chunk
// b / ceil(chunk / (256 * kAdjPP)) (the chunk's XCD is the one k_count gives
// it), kAdjPP points per thread with their loads in flight together (two per
// thread were slower than one: 98 VGPRs instead of 44 halve the wavefronts).
constexpr int kAdjPP = 1;

template <int W>
__global__ __launch_bounds__(256) void k_adj(Work w) {
  const int per = (w.chunk + 256 * kAdjPP - 1) / (256 * kAdjPP);
  const int b = xcd_logical_block();
  const int c = b / per;
  const int m = chunk_matrix(w.desc, w.nmat, c);
  const GDesc d = gview(w.desc[m]);
  if (!d.fadj) return;
  const int f0 = (c - d.chunk0) * w.chunk;
  const int f1 = min(f0 + w.chunk, d.n);
  const int ub = f0 + (b - c * per) * 256 * kAdjPP + (int)threadIdx.x;
  int u[kAdjPP], e0[kAdjPP], e1[kAdjPP], cnt[kAdjPP];
  int o[kAdjPP][W];
#pragma unroll
  for (int p = 0; p < kAdjPP; ++p) {
    u[p] = ub + 256 * p;
    e0[p] = 0;
    e1[p] = 0;
    cnt[p] = 0;
    if (u[p] < f1) { e0[p] = d.grp[u[p]]; e1[p] = d.grp[u[p] + 1]; }
#pragma unroll
    for (int q = 0; q < W; ++q) o[p][q] = -1;
  }
  for (int e = 0;; e += 8) {
    bool any = false;
#pragma unroll
    for (int p = 0; p < kAdjPP; ++p) any |= e0[p] + e < e1[p] && cnt[p] <= W;
    if (!any) break;
    int k[kAdjPP][8];
    double x[kAdjPP][8];
#pragma unroll
    for (int p = 0; p < kAdjPP; ++p) {
      const bool go = cnt[p] <= W;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        k[p][j] = u[p];
        x[p][j] = 0.0;
        if (go && e0[p] + e + j < e1[p]) { k[p][j] = d.gci[e0[p] + e + j]; x[p][j] = d.gva[e0[p] + e + j]; }
      }
    }
    int8_t c8[kAdjPP][8];
#pragma unroll
    for (int p = 0; p < kAdjPP; ++p)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        c8[p][j] = ((unsigned)k[p][j] < (unsigned)d.n) ? d.cf[k[p][j]] : (int8_t)1;
#pragma unroll
    for (int p = 0; p < kAdjPP; ++p) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (k[p][j] != u[p] && x[p][j] != 0.0 && c8[p][j] == 0 && strong_edge(x[p][j], k[p][j], d.theta, d.cmax)) {
#pragma unroll
          for (int q = 0; q < W; ++q)
            if (q == cnt[p]) o[p][q] = k[p][j];
          ++cnt[p];
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kAdjPP; ++p) {
    if (u[p] >= f1) continue;
    if (cnt[p] > W) o[p][0] = kAdjOverflow;
    gptr<adj_v4> dst = (gptr<adj_v4>)(to_global(w.fadj) + (d.fine0 + u[p]) * W);
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
      adj_v4 t;
      t.x = o[p][4 * q];
      t.y = o[p][4 * q + 1];
      t.z = o[p][4 * q + 2];
      t.w = o[p][4 * q + 3];
      dst[q] = t;
    }
  }
}

// The distinct values of v (sorted, INT32_MAX = none) into the row's slot:
// bin A's (stride SA) when there are at most lim of them, else bin B's.
// Returns their number (at most P <= 32).
template <int P>
__device__ __forceinline__ int emit_distinct(const int (&v)[P], const Work& w, int64_t row, int SA, int lim) {
  static_assert(P <= 32, "bin B slots hold 32 points");
  int sz = 0;
#pragma unroll
  for (int q = 0; q < P; ++q) sz += (v[q] != 0x7fffffff && (q == 0 || v[q] != v[q - 1])) ? 1 : 0;
  gptr<int32_t> dst = sz <= lim ? to_global(w.slotA) + row * SA : to_global(w.slotB) + row * 32;
  int pos = 0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const bool u = v[q] != 0x7fffffff && (q == 0 || v[q] != v[q - 1]);
    if (u) dst[pos] = v[q];
    pos += u ? 1 : 0;
  }
  return sz;
}

// N(i) at ell = 2 from the compact adjacency of width 4: the four slots of
// i and the four of each of them, sorted, duplicates dropped.  -1 when a
// point overflows its slots (the row is left to k_count_mid).
__device__ __forceinline__ int count_adj4_ell2(const Work& w, const GDesc& d, int i, int64_t row, int SA, int lim) {
  int a[4];
  adj_load<4>(d.fadj, i, a);
  if (a[0] == kAdjOverflow) return -1;
  int b[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (a[q] >= 0) {
      adj_load<4>(d.fadj, a[q], b[q]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) b[q][r] = -1;
    }
  }
  int v[32];
  bool ovf = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ovf |= b[q][0] == kAdjOverflow;
    v[q] = a[q] >= 0 ? a[q] : 0x7fffffff;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[4 + 4 * q + r] = b[q][r] >= 0 ? b[q][r] : 0x7fffffff;
  }
  if (ovf) return -1;
#pragma unroll
  for (int q = 20; q < 32; ++q) v[q] = 0x7fffffff;
  bitonic_sort<32>(v);
  return emit_distinct<32>(v, w, row, SA, lim);
}

// N(i) at ell = 1 from row i of the search graph (at most 8 stored entries;
// -1 otherwise, the row is left to k_count_mid)
__device__ __forceinline__ int count_row_ell1(const Work& w, const GDesc& d, int i, int64_t row, int SA, int lim) {
  const int e0 = d.grp[i], e1 = d.grp[i + 1];
  if (e1 - e0 > 8) return -1;
  int k[8];
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    k[j] = i;
    x[j] = 0.0;
    if (e0 + j < e1) { k[j] = d.gci[e0 + j]; x[j] = d.gva[e0 + j]; }
  }
  int v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int8_t c8 = ((unsigned)k[j] < (unsigned)d.n) ? d.cf[k[j]] : (int8_t)1;
    v[j] = (k[j] != i && x[j] != 0.0 && c8 == 0 && strong_edge(x[j], k[j], d.theta, d.cmax)) ? k[j] : 0x7fffffff;
  }
  bitonic_sort<8>(v);
  return emit_distinct<8>(v, w, row, SA, lim);
}

// The chunk's bookkeeping once every row is sized (s_size; the rows left to
// k_count_big have size 0, a negative s_rows entry and their index in
// s_unres[0..nunres)): bin counts, the queue of k_count_big, the chunk-local
// exclusive prefix of |N(i)|+1, the chunk totals.
__device__ __forceinline__ void finish_chunk(const Work& w, int c, int m, MatStatus* st, int64_t base, int nc,
                                             const int* s_rows, const int16_t* s_size, const int16_t* s_unres,
                                             int nunres, int* s_scan, int* s_flag, int* s_qbase) {
  const int tid = threadIdx.x;
  const int lim = small_limit(w.GA);
  if (nunres) {
    if (tid == 0) *s_qbase = atomicAdd(&w.cnt->nbig, nunres);
    __syncthreads();
    for (int k = tid; k < nunres; k += kNT) {
      const int q = *s_qbase + k;
      if (q < w.capC) w.bigq[q] = c * w.chunk + s_unres[k];
      else flag_row(st, ST_UNSUPPORTED, -s_rows[s_unres[k]] - 1);
    }
  }
  const int per2 = (nc + kNT - 1) / kNT;
  const int t0 = tid * per2;
  int mysum = 0, mymax = 0, inA = 0, inB = 0;
  for (int t = t0; t < min(t0 + per2, nc); ++t) {
    const int sz = s_size[t];
    mysum += sz + 1;
    mymax = max(mymax, sz);
    if (s_rows[t] >= 0) {
      inA += sz <= lim ? 1 : 0;
      inB += sz > lim ? 1 : 0;
    }
  }
  int tot;
  int pre = block_exclusive_scan(mysum, s_scan, &tot);
  for (int t = t0; t < min(t0 + per2, nc); ++t) { w.lnz[base + t] = pre; pre += s_size[t] + 1; }
  if (mymax) atomicMax(&s_flag[0], mymax);
  if (inA) atomicAdd(&s_flag[2], inA);
  if (inB) atomicAdd(&s_flag[3], inB);
  __syncthreads();
  if (tid == 0) {
    w.chunk_nc[c] = nc;
    w.chunk_nnz[c] = tot;
    w.chunk_mat[c] = m;
    // bin sizes per chunk (summed by k_scan); the largest block only when it
    // grows, so that few workgroups meet at one address
    w.chunk_bins[c] = make_int2(s_flag[2], s_flag[3]);
    if (s_flag[0] > __hip_atomic_load(&st->max_block, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&st->max_block, s_flag[0]);
    w.chunk_unsized[c] = nunres;
  }
}

// Symbolic pass, first part: one workgroup per chunk of fine points.  The
// chunk's C-points are compacted; rows at ell = 1 with at most 8 stored
// entries, and rows at ell = 2 of matrices with a width-4 compact adjacency,
// are sized by one thread each from a sorted candidate list (no search
// state); a chunk whose rows are all sized is finished here.  Other rows
// (larger stencils, ell >= 3, aggregates, overflowing points) are marked -1
// in lnz and left, with the chunk's bookkeeping, to k_count_mid.
template <int W>
__global__ __launch_bounds__(kNT) void k_count(Work w) {
  __shared__ int s_rows[kMaxChunk];
  __shared__ int16_t s_size[kMaxChunk];
  __shared__ int s_scan[kNT];
  __shared__ int s_flag[4];  // max |N|, -, rows in bin A, rows in bin B
  __shared__ int s_ndef, s_qbase;

  // each XCD's chunks newest first: k_adj wrote them in ascending order, so
  // the last ones' adjacency is the part most likely still cached (and the
  // numeric kernels, walking rows in ascending order, then first read the
  // slots written last here)
  const int c = xcd_logical_block_reversed();
  const int tid = threadIdx.x;
  const int m = chunk_matrix(w.desc, w.nmat, c);
  const GDesc d = gview(w.desc[m]);
  MatStatus* st = &w.st[m];
  const int f0 = (c - d.chunk0) * w.chunk;
  const int f1 = min(f0 + w.chunk, d.n);
  const int64_t base = d.fine0 + f0;

  if (st->status == ST_INVALID) {  // validation failed: contribute nothing
    if (tid == 0) { w.chunk_nc[c] = 0; w.chunk_nnz[c] = 0; w.chunk_mat[c] = m; w.chunk_bins[c] = make_int2(0, 0); w.chunk_unsized[c] = 0; }
    return;
  }

  // empty the projection's column lists of this chunk's fine points
  if (d.B) {
    for (int j = f0 + tid; j < f1; j += kNT) w.chead[d.fine0 + j] = -1;
  }

  // compaction of the chunk's C-points, ascending: each thread's run of up
  // to 8 markers is read once, all loads in flight together
  static_assert(kMaxChunk <= 8 * kNT, "a thread's run of markers fits one byte mask");
  const int per = (w.chunk + kNT - 1) / kNT;
  const int j0 = f0 + tid * per;
  const int j1 = min(j0 + per, f1);
  uint32_t cbits = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (j0 + k < j1 && d.cf[j0 + k] != 0) cbits |= 1u << k;
  int nc;
  int rank = block_exclusive_scan(__popc(cbits), s_scan, &nc);
  for (uint32_t b = cbits; b; b &= b - 1) {
    const int j = j0 + __ffs(b) - 1;
    s_rows[rank] = j;
    w.clocal[base + rank] = j;
    ++rank;
  }
  if (tid == 0) { s_flag[0] = 0; s_flag[1] = 0; s_flag[2] = 0; s_flag[3] = 0; s_ndef = 0; }
  __syncthreads();

  const int SA = slot_stride(w.GA);
  const int lim = small_limit(w.GA);
  int ndef = 0;
  for (int t = tid; t < nc; t += kNT) {
    int sz = -1;
    if (!d.agg_rp) {
      if constexpr (W == 4) {
        if (d.fadj && d.ell == 2) sz = count_adj4_ell2(w, d, s_rows[t], base + t, SA, lim);
      }
      if (d.ell == 1) sz = count_row_ell1(w, d, s_rows[t], base + t, SA, lim);
    }
    s_size[t] = (int16_t)sz;
    ndef += sz < 0 ? 1 : 0;
  }
  if (ndef) atomicAdd(&s_ndef, ndef);
  __syncthreads();
  if (s_ndef == 0) {
    finish_chunk(w, c, m, st, base, nc, s_rows, s_size, nullptr, 0, s_scan, s_flag, &s_qbase);
    return;
  }
  // left to k_count_mid: the sizes so far (-1 = not sized), the chunk queued
  for (int t = tid; t < nc; t += kNT) w.lnz[base + t] = s_size[t];
  if (tid == 0) {
    w.chunk_nc[c] = nc;
    w.chunk_mat[c] = m;
    w.chunk_nnz[c] = -1;
    w.midq[atomicAdd(&w.cnt->nmid, 1)] = c;
  }
}

// Symbolic pass, second part: the chunks k_count left unfinished (queued by
// it; the workgroups take them in turn, so an empty queue costs one load per
// workgroup).  One thread per row not
// yet sized searches up to 32 points in registers (over the compact
// adjacency when the matrix has one); larger rows are left unsized for
// k_count_big.  Then the chunk's bookkeeping.
template <int W>
__global__ __launch_bounds__(kNT) void k_count_mid(Work w) {
  __shared__ int s_rows[kMaxChunk];
  __shared__ int16_t s_size[kMaxChunk];
  __shared__ int s_scan[kNT];
  __shared__ int s_flag[4];  // max |N|, rows left unsized, rows in bin A, rows in bin B
  __shared__ int16_t s_list[kMaxChunk];   // rows to size here
  __shared__ int16_t s_unres[kMaxChunk];  // rows with more than 32 points
  __shared__ int s_nlist, s_qbase;

  const int tid = threadIdx.x;
  const int nq = w.cnt->nmid;
  for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
  const int c = w.midq[qi];
  __syncthreads();  // the previous chunk's LDS is free
  const int m = w.chunk_mat[c];
  const GDesc d = gview(w.desc[m]);
  MatStatus* st = &w.st[m];
  const int64_t base = d.fine0 + (int64_t)(c - d.chunk0) * w.chunk;
  const int nc = w.chunk_nc[c];
  if (tid == 0) { s_flag[0] = 0; s_flag[1] = 0; s_flag[2] = 0; s_flag[3] = 0; s_nlist = 0; }
  __syncthreads();
  for (int t = tid; t < nc; t += kNT) {
    s_rows[t] = w.clocal[base + t];
    const int sz = w.lnz[base + t];
    s_size[t] = (int16_t)sz;
    if (sz < 0) s_list[atomicAdd(&s_nlist, 1)] = (int16_t)t;
  }
  __syncthreads();
  const int SA = slot_stride(w.GA);
  const int lim = small_limit(w.GA);
  const int nl = s_nlist;
  for (int k = tid; k < nl; k += kNT) {
    const int t = s_list[k];
    const int i = s_rows[t];
    RegSetA<32> S;
    int sz;
    if (d.literal && d.ell >= 3) {
      sz = rega_bfs_literal<32>(S, d.n, i, d.ell, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax);
    } else if constexpr (W > 0) {
      if (d.fadj)
        sz = rega_bfs<32, W>(S, d.n, i, d.ell, d.fadj, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax, nullptr, nullptr);
      else
        sz = rega_bfs<32, 0>(S, d.n, i, d.ell, nullptr, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax, d.agg_rp,
                             d.agg_list);
    } else {
      sz = rega_bfs<32, 0>(S, d.n, i, d.ell, nullptr, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax, d.agg_rp,
                           d.agg_list);
    }
    if (sz < 0) {
      s_size[t] = 0;
      s_rows[t] = -(i + 1);
      w.clocal[base + t] = -(i + 1);
      s_unres[atomicAdd(&s_flag[1], 1)] = (int16_t)t;
    } else if (sz <= lim) {
      s_size[t] = (int16_t)sz;
#pragma unroll
      for (int p = 0; p < 32; ++p)
        if (p < sz) w.slotA[(base + t) * SA + p] = S.v[p];
    } else {
      s_size[t] = (int16_t)sz;
#pragma unroll
      for (int p = 0; p < 32; ++p)
        if (p < sz) w.slotB[(base + t) * 32 + p] = S.v[p];
    }
  }
  __syncthreads();
  finish_chunk(w, c, m, st, base, nc, s_rows, s_size, s_unres, s_flag[1], s_scan, s_flag, &s_qbase);
  }
}

// Rows with more than 32 points, one workgroup per row (grid-stride over the
// queue): the workgroup search sizes the row, which is queued for the
// workgroup solver.  The workgroup that sizes the last such row of a chunk
// then redoes the chunk's prefix.
__global__ __launch_bounds__(kNT) void k_count_big(Work w) {
  __shared__ WideBuf bb;
  __shared__ int s_size[kMaxChunk];
  __shared__ int s_scan[kNT];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int nq = min(w.cnt->nbig, w.capC);
  for (int qi = blockIdx.x; qi < nq; qi += gridDim.x) {
    const int e = w.bigq[qi];
    const int c = e / w.chunk, t = e - c * w.chunk;
    const int m = w.chunk_mat[c];
    const GDesc d = gview(w.desc[m]);
    MatStatus* st = &w.st[m];
    const int64_t base = d.fine0 + (int64_t)(c - d.chunk0) * w.chunk;
    const int i = -w.clocal[base + t] - 1;
    int* nl;
    const int s = block_bfs(d.n, i, d.ell, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax, d.agg_rp, d.agg_list, bb, &nl,
                            d.literal != 0);
    __syncthreads();
    // A row the register search gave up on may still hold at most 32 points
    // (the literal reading counts the C-points a walk passes through): it
    // then joins its size bin, whose solvers take every row of that size,
    // and not the workgroup solver as well.
    const int lim = small_limit(w.GA);
    const bool toA = s >= 0 && s <= lim, toB = s > lim && s <= 32;
    if (toA) {
      const int SA = slot_stride(w.GA);
      for (int p = tid; p < s; p += kNT) w.slotA[(base + t) * SA + p] = nl[p];
    } else if (toB) {
      for (int p = tid; p < s; p += kNT) w.slotB[(base + t) * 32 + p] = nl[p];
    }
    if (tid == 0) {
      w.big_size[base + t] = s < 0 ? 0 : s;
      if (s < 0) {
        flag_row(st, ST_UNSUPPORTED, i);
      } else {
        if (s > __hip_atomic_load(&st->max_block, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          atomicMax(&st->max_block, s);
        if (toA || toB) {
          atomicAdd(reinterpret_cast<int*>(&w.chunk_bins[c]) + (toA ? 0 : 1), 1);
        } else {
          const int q = atomicAdd(&w.cnt->nC, 1);
          if (q < w.capC) w.binC[q] = e;
          else flag_row(st, ST_UNSUPPORTED, i);
        }
      }
      __threadfence();  // the size is visible before the count drops
      s_last = atomicSub(&w.chunk_unsized[c], 1) == 1;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();  // every size of the chunk is visible here
      // sizes: k_count's prefix (0 for the unsized rows) and the unsized
      // rows' own sizes; their C-point index is restored
      const int nc = w.chunk_nc[c];
      for (int tt = tid; tt < nc; tt += kNT) {
        const int l1 = (tt + 1 < nc) ? w.lnz[base + tt + 1] : w.chunk_nnz[c];
        int sz = l1 - w.lnz[base + tt] - 1;
        const int ci = w.clocal[base + tt];
        if (ci < 0) sz = w.big_size[base + tt];
        s_size[tt] = sz;
      }
      __syncthreads();
      for (int tt = tid; tt < nc; tt += kNT) {
        const int ci = w.clocal[base + tt];
        if (ci < 0) w.clocal[base + tt] = -ci - 1;
      }
      const int per2 = (nc + kNT - 1) / kNT;
      const int t0 = tid * per2;
      int mysum = 0;
      for (int tt = t0; tt < min(t0 + per2, nc); ++tt) mysum += s_size[tt] + 1;
      int tot;
      int pre = block_exclusive_scan(mysum, s_scan, &tot);
      for (int tt = t0; tt < min(t0 + per2, nc); ++tt) { w.lnz[base + tt] = pre; pre += s_size[tt] + 1; }
      if (tid == 0) w.chunk_nnz[c] = tot;
    }
    __syncthreads();
  }
}

// One workgroup: global row base and global R offset of every chunk (all
// matrices in order).  Each thread sums a contiguous run of chunks, one block
// scan joins the runs; then one thread per matrix sizes R, checks capacity and
// writes R.row_ptr[n_c].  Per-matrix R offsets are the global ones minus the
// matrix's base.
__global__ __launch_bounds__(1024) void k_scan(Work w) {
  __shared__ long long s_wr[17], s_wz[17];
  __shared__ int s_wa[17], s_wb[17];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int nch = w.nchunks;
  // tiles of 4096 consecutive chunks, four per thread (their loads in flight
  // together), scanned in order with the running totals carried over (four
  // per thread were faster than one and than sixteen: 42, 30 and 44 us on
  // 13,400 chunks)
  constexpr int CPT = 4;
  long long carry_r = 0, carry_z = 0;
  int na = 0, nb = 0;
  for (int t0 = 0; t0 < nch; t0 += 1024 * CPT) {
    const int cb = t0 + tid * CPT;
    int ncs[CPT];
    long long nzs[CPT];
    int nc = 0, a = 0, bbin = 0;
    long long nz = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      ncs[k] = 0;
      nzs[k] = 0;
      if (cb + k < nch) {
        ncs[k] = w.chunk_nc[cb + k];
        nzs[k] = w.chunk_nnz[cb + k];
        const int2 bn = w.chunk_bins[cb + k];
        a += bn.x;
        bbin += bn.y;
      }
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) { nc += ncs[k]; nz += nzs[k]; }
    // inclusive scans inside each wavefront, then across the 16 wavefronts
    long long xr = nc, xz = nz;
    int xa = a, xb = bbin;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const long long yr = __shfl_up(xr, o, 64);
      const long long yz = __shfl_up(xz, o, 64);
      const int ya = __shfl_up(xa, o, 64);
      const int yb = __shfl_up(xb, o, 64);
      if (lane >= o) { xr += yr; xz += yz; xa += ya; xb += yb; }
    }
    if (lane == 63) { s_wr[wid] = xr; s_wz[wid] = xz; s_wa[wid] = xa; s_wb[wid] = xb; }
    __syncthreads();
    // the first wavefront scans the 16 wavefront totals: exclusive prefixes
    // in place, the tile's totals in slot 16
    if (wid == 0) {
      const long long r0 = lane < 16 ? s_wr[lane] : 0, z0 = lane < 16 ? s_wz[lane] : 0;
      const int a0 = lane < 16 ? s_wa[lane] : 0, b0 = lane < 16 ? s_wb[lane] : 0;
      long long r = r0, z = z0;
      int a1 = a0, b1 = b0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const long long yr = __shfl_up(r, o, 64);
        const long long yz = __shfl_up(z, o, 64);
        const int ya = __shfl_up(a1, o, 64);
        const int yb = __shfl_up(b1, o, 64);
        if (lane >= o) { r += yr; z += yz; a1 += ya; b1 += yb; }
      }
      if (lane < 16) { s_wr[lane] = r - r0; s_wz[lane] = z - z0; }
      if (lane == 15) { s_wr[16] = r; s_wz[16] = z; s_wa[16] = a1; s_wb[16] = b1; }
    }
    __syncthreads();
    const long long br = s_wr[wid], bz = s_wz[wid], tr = s_wr[16], tz = s_wz[16];
    const int ta = s_wa[16], tb = s_wb[16];
    __syncthreads();  // read before the next tile writes them
    long long rr = carry_r + br + xr - nc;
    long long zz = carry_z + bz + xz - nz;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int c = cb + k;
      if (c < nch) {
        w.chunk_rbase[c] = (int32_t)rr;
        w.chunk_nzglob[c] = zz;
        // row blocks whose first row lies in this chunk
        for (long long b = (rr + (1 << kRowBlockLog) - 1) >> kRowBlockLog; (b << kRowBlockLog) < rr + ncs[k]; ++b)
          w.row_block_chunk[b] = c;
      }
      rr += ncs[k];
      zz += nzs[k];
    }
    carry_r += tr;
    carry_z += tz;
    na += ta;
    nb += tb;
  }
  const long long rows_total = carry_r, nnz_total = carry_z;
  __syncthreads();
  for (int m = tid; m < w.nmat; m += 1024) {
    const GDesc d = gview(w.desc[m]);
    MatStatus* st = &w.st[m];
    const int cb = d.chunk0, ce = d.chunk0 + d.nchunks;
    const long long rb = cb < nch ? w.chunk_rbase[cb] : rows_total;
    const long long re = ce < nch ? w.chunk_rbase[ce] : rows_total;
    const long long zb = cb < nch ? w.chunk_nzglob[cb] : nnz_total;
    const long long ze = ce < nch ? w.chunk_nzglob[ce] : nnz_total;
    const int n_c = (int)(re - rb);
    const long long nnz = ze - zb;
    st->row_base = (int32_t)rb;
    st->nz_base = zb;
    st->n_c = n_c;
    st->nnz = nnz;
    if (st->status != ST_INVALID) {
      const bool fits = d.Rrp && d.Rci && d.Rva && (int64_t)n_c + 1 <= d.row_cap && nnz <= d.nnz_cap &&
                        nnz <= 0x7fffffffLL;
      if (!fits) {
        st->status = ST_CAPACITY;
      } else {
        d.Rrp[n_c] = (int32_t)nnz;
      }
    }
  }
  if (tid == 0) {
    w.chunk_rbase[nch] = (int32_t)rows_total;
    w.cnt->total_rows = (int32_t)rows_total;
    w.cnt->nA = na;
    w.cnt->nB = nb;
  }
}

// ---------------------------------------------------------------------------
// numeric pass: G lanes per queued row
// ---------------------------------------------------------------------------
// LDS of one lane group: blocks of up to SM points (SM <= G)
template <int G, int SM>
struct NumGroupBuf {
  double K[SM * (SM + 1)];  // FP64 block, row q = row q of (A[N,N])^T, stride SM+1
  // -A[i,N] (written by the gather, read once after the factorisation), the
  // refinement broadcast z and a correction's FP32 right-hand side y are
  // never live together, so they share one buffer: every store to it comes
  // after the group's last load of the previous contents in program order,
  // and a wavefront's LDS instructions execute in order.  (At 24 points
  // this holds a group to 5,120 bytes, eight workgroups of four per CU.)
  union {
    double f[SM];
    double z[SM];
    float y[SM];
  };
  int nb[G];  // sorted N(i), INT32_MAX beyond |N|
};

// Communication inside a group of G lanes (G = 8, 16 or 32; groups are
// aligned runs of G lanes of a wavefront).
//
// gbi: lane k of the group to all its lanes.  ds_swizzle in bit mode keeps
// the lane bits above the group (and-mask 32 - G) and sets the rest to k; the
// pattern is an immediate, so k must fold to a constant (unrolled loops).
template <int G>
__device__ __forceinline__ int gbi(int v, int k) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group size");
#define CLAIR_SWZ(K) \
  case K: return __builtin_amdgcn_ds_swizzle(v, (32 - G) | ((K) << 5));
  switch (k) {
    CLAIR_SWZ(0) CLAIR_SWZ(1) CLAIR_SWZ(2) CLAIR_SWZ(3) CLAIR_SWZ(4) CLAIR_SWZ(5) CLAIR_SWZ(6) CLAIR_SWZ(7)
    CLAIR_SWZ(8) CLAIR_SWZ(9) CLAIR_SWZ(10) CLAIR_SWZ(11) CLAIR_SWZ(12) CLAIR_SWZ(13) CLAIR_SWZ(14) CLAIR_SWZ(15)
    CLAIR_SWZ(16) CLAIR_SWZ(17) CLAIR_SWZ(18) CLAIR_SWZ(19) CLAIR_SWZ(20) CLAIR_SWZ(21) CLAIR_SWZ(22) CLAIR_SWZ(23)
    CLAIR_SWZ(24) CLAIR_SWZ(25) CLAIR_SWZ(26) CLAIR_SWZ(27) CLAIR_SWZ(28) CLAIR_SWZ(29) CLAIR_SWZ(30)
    default: return __builtin_amdgcn_ds_swizzle(v, (32 - G) | (31 << 5));
  }
#undef CLAIR_SWZ
}
template <int G>
__device__ __forceinline__ float gbf(float v, int k) { return __int_as_float(gbi<G>(__float_as_int(v), k)); }

// gpart: the value of a partner lane for a butterfly-like reduction.  Steps 1
// and 2 pair lanes inside a quad (DPP quad_perm [1,0,3,2] and [2,3,0,1]), step
// 4 mirrors the halves of 8 lanes (DPP row_half_mirror), step 8 mirrors the
// halves of 16 (DPP row_mirror), step 16 swaps the halves of 32 (ds_swizzle
// xor 16).  After the steps up to G/2 every lane holds the group's reduction.
template <int STEP>
__device__ __forceinline__ int gpart(int v) {
  if constexpr (STEP == 1) return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
  else if constexpr (STEP == 2) return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);
  else if constexpr (STEP == 4) return __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);
  else if constexpr (STEP == 8) return __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);
  else return __builtin_amdgcn_ds_swizzle(v, 0x1f | (0x10 << 10));
}
template <int STEP>
__device__ __forceinline__ double gpartd(double v) {
  return __hiloint2double(gpart<STEP>(__double2hiint(v)), gpart<STEP>(__double2loint(v)));
}

template <int G>
__device__ __forceinline__ float group_maxf(float v) {
  v = fmaxf(v, __int_as_float(gpart<1>(__float_as_int(v))));
  if constexpr (G >= 4) v = fmaxf(v, __int_as_float(gpart<2>(__float_as_int(v))));
  if constexpr (G >= 8) v = fmaxf(v, __int_as_float(gpart<4>(__float_as_int(v))));
  if constexpr (G >= 16) v = fmaxf(v, __int_as_float(gpart<8>(__float_as_int(v))));
  if constexpr (G >= 32) v = fmaxf(v, __int_as_float(gpart<16>(__float_as_int(v))));
  return v;
}
template <int G>
__device__ __forceinline__ double group_maxd(double v) {
  v = fmax(v, gpartd<1>(v));
  if constexpr (G >= 4) v = fmax(v, gpartd<2>(v));
  if constexpr (G >= 8) v = fmax(v, gpartd<4>(v));
  if constexpr (G >= 16) v = fmax(v, gpartd<8>(v));
  if constexpr (G >= 32) v = fmax(v, gpartd<16>(v));
  return v;
}
template <int G>
__device__ __forceinline__ int group_ori(int v) {
  v |= gpart<1>(v);
  if constexpr (G >= 4) v |= gpart<2>(v);
  if constexpr (G >= 8) v |= gpart<4>(v);
  if constexpr (G >= 16) v |= gpart<8>(v);
  if constexpr (G >= 32) v |= gpart<16>(v);
  return v;
}

// y_lane = sum_p Kinv[lane][p] v_p: the group's right-hand side goes through
// LDS once (v_p from lane p), then every lane reads all of it (broadcast
// reads, no dependence between the steps).  kf holds this lane's row of the
// FP32 inverse; lanes at or beyond SM hold no row.
template <int SM>
__device__ __forceinline__ float inv_apply(const float (&kf)[SM], float* ybuf, bool rowl, int lane, float v) {
  if (rowl) ybuf[lane] = v;
  wave_sync();
  float y = 0.f;
#pragma unroll
  for (int p = 0; p < SM; ++p) y = fmaf(kf[p], ybuf[p], y);
  wave_sync();  // the buffer is reused by the next call
  return y;
}

// Position of key in the G sorted entries nb[0..G) (padded with INT32_MAX),
// or -1: a branch-free lower bound of fixed depth log2(G).  Several searches
// in a row have no loop between them, so their LDS reads overlap.
template <int G>
__device__ __forceinline__ int find_pos(const int* nb, int key) {
  int pos = 0;
#pragma unroll
  for (int step = G / 2; step >= 1; step >>= 1) pos += (nb[pos + step - 1] < key) ? step : 0;
  return (pos < G && nb[pos] == key) ? pos : -1;
}

constexpr int kRefineMax = 5;

// G lanes per row, blocks of up to SM <= G points.  which = 0: bin A
// (|N| <= G = GA); which = 1: bin B (GA < |N| <= 32), rows with |N| > SM are
// handed to the workgroup solver.
// (at SM = 20 the registers fit four wavefronts per SIMD without spilling;
// the other shapes are held to fewer by their LDS or would spill)
template <int G, int NT, int SM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((SM == 18 || SM == 20 || SM == 24) ? 4 : 1))) void k_numeric(Work w, int which) {
  static_assert(SM <= G, "block bound");
  constexpr int NG = NT / G;
  constexpr int LD = SM + 1;
  __shared__ NumGroupBuf<G, SM> sb[NG];

  const int tid = threadIdx.x;
  const int grp = tid / G;
  const int lane = tid % G;
  const bool rowl = lane < SM;  // this lane can hold a row of the block
  NumGroupBuf<G, SM>& gb = sb[grp];

  // rows of this solver
  if ((which ? w.cnt->nB : w.cnt->nA) == 0) return;
  const int smin = which ? small_limit(w.GA) + 1 : 0;
  const int32_t* slots = which ? w.slotB : w.slotA;
  const int sstride = which ? 32 : w.GA;
  const int total = w.cnt->total_rows;
  const RowBlocks rbk(total, 4 * NG);
  int r0, r1;
  if (!rbk.block(0, &r0, &r1)) return;
  RefineMax rmx;
  ChunkCursor cc;
  // The group works one row ahead: while row g is solved, the chunk-local
  // data, the slot entry and the A-row bounds of row g + NG (same chunk) are
  // already on their way, so a row starts with only its A entries to load.
  int nx_t = 0, nx_i = 0, nx_off = 0, nx_s = -1, nx_N = 0, nx_e0 = 0, nx_e1 = 0, nx_f0 = 0, nx_f1 = 0;
  bool ahead = false;

  for (int jb = 0; rbk.block(jb, &r0, &r1); ++jb) {
  ahead = false;
  for (int gbase = r0; gbase < r1; gbase += NG) {
    const int g = gbase + grp;
    if (g >= r1) break;  // group-uniform
    int t, i, off, s, myN0, ae0, ae1, fe0, fe1;
    if (ahead) {
      t = nx_t; i = nx_i; off = nx_off; s = nx_s; myN0 = nx_N;
      ae0 = nx_e0; ae1 = nx_e1; fe0 = nx_f0; fe1 = nx_f1;
    } else {
      cc.seek(w, g);
      cc.row(w, g, &t, &i, &off, &s);
      myN0 = slots[(cc.fbase + t) * sstride + min(lane, sstride - 1)];
      ae0 = 0; ae1 = 0; fe0 = 0; fe1 = 0;
      if (s >= smin && s <= SM && cc.live) {
        if (lane < s) { ae0 = cc.md.rp[myN0]; ae1 = cc.md.rp[myN0 + 1]; }
        fe0 = cc.md.rp[i];
        fe1 = cc.md.rp[i + 1];
      }
    }
    // the next row of this group, if it lies in the same chunk: its
    // chunk-local data and slot entry now, its A-row bounds after the gather
    const int gn = g + NG;
    ahead = gn < r1 && gn < cc.re;
    if (ahead) {
      cc.row(w, gn, &nx_t, &nx_i, &nx_off, &nx_s);
      nx_N = slots[(cc.fbase + nx_t) * sstride + min(lane, sstride - 1)];
    }
    const bool mine = s >= smin && s <= SM && cc.live;  // group-uniform
    const bool nx_mine = ahead && nx_s >= smin && nx_s <= SM && cc.live;
    if (!mine) {
      if (which && s > SM && s <= 32 && cc.live && lane == 0) {
        // a bin-B row larger than this kernel's blocks: the workgroup solver
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = cc.c * w.chunk + t;
        else flag_row(&w.st[cc.m], ST_UNSUPPORTED, i);
      }
      if (nx_mine) {
        nx_e0 = 0; nx_e1 = 0;
        if (lane < nx_s) { nx_e0 = cc.md.rp[nx_N]; nx_e1 = cc.md.rp[nx_N + 1]; }
        nx_f0 = cc.md.rp[nx_i];
        nx_f1 = cc.md.rp[nx_i + 1];
      }
      continue;  // another solver's row
    }
    const int c = cc.c;
    const int entry = c * w.chunk + t;
    const GDesc& d = cc.md;
    MatStatus* st = &w.st[cc.m];
    RowInfo ri;
    ri.m = cc.m;
    ri.i = i;
    ri.r = g - cc.rbase_m;
    ri.off = off;
    ri.s = s;
    ri.fine0 = cc.fine0;
    if (lane == 0) d.Rrp[ri.r] = ri.off;
    const int myN = (lane < s) ? myN0 : 0x7fffffff;
    gb.nb[lane] = myN;
    const uint64_t below = __ballot(lane < s && myN < i);
    const int dpos = __popcll((below >> ((threadIdx.x & 63) - lane)) & ((G >= 64) ? ~0ull : ((1ull << G) - 1)));

    // ---- gather: K = (A[N,N])^T (padded with identity), f = -A[i,N] ----
    if (rowl) {
#pragma unroll
      for (int tt = 0; tt < SM; ++tt) gb.K[tt * LD + lane] = (tt == lane && tt >= s) ? 1.0 : 0.0;
      gb.f[lane] = 0.0;
    }
    wave_sync();
    for (int e = ae0; e < ae1; e += 4) {
      int k[4];
      double v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        k[j] = -1;
        v[j] = 0.0;
        if (e + j < ae1) { k[j] = d.ci[e + j]; v[j] = d.va[e + j]; }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int qq = find_pos<G>(gb.nb, k[j]);
        if (qq >= 0) gb.K[qq * LD + lane] = v[j];
      }
    }
    for (int e = fe0 + lane; e < fe1; e += G) {
      const int qq = find_pos<G>(gb.nb, d.ci[e]);
      if (qq >= 0) gb.f[qq] = -d.va[e];
    }
    wave_sync();
    if (nx_mine) {
      nx_e0 = 0; nx_e1 = 0;
      if (lane < nx_s) { nx_e0 = d.rp[nx_N]; nx_e1 = d.rp[nx_N + 1]; }
      nx_f0 = d.rp[nx_i];
      nx_f1 = d.rp[nx_i + 1];
    }

    // ---- FP32 inverse of the row-scaled block ----
    float amax = 0.f;
    double knorm = 0.0;
#pragma unroll
    for (int p = 0; p < SM; ++p) {
      const double v = rowl ? gb.K[lane * LD + p] : 0.0;
      amax = fmaxf(amax, (float)fabs(v));
      knorm += fabs(v);
    }
    amax = group_maxf<G>(amax);
    knorm = group_maxd<G>(knorm);
    int ex = 0;
    frexpf(amax, &ex);
    const double scale = ldexp(1.0, -ex);
    float kf[SM];
#pragma unroll
    for (int p = 0; p < SM; ++p) kf[p] = rowl ? (float)(gb.K[lane * LD + p] * scale) : 0.f;
    int bad = !(amax > 0.f) || !(amax < 3.0e38f);
    // Gauss-Jordan in place, no pivoting: step k scales pivot row k and
    // clears column k in every other row; column k then holds the inverse's
    // column k.  The pivots are those of the LU factorisation, so the same
    // tiny-pivot test applies.  Each lane holds one row; the pivot row reaches
    // the group by ds_swizzle.  One update serves every lane: the pivot lane
    // subtracts (1 - 1/pivot) times its own row, which scales it by 1/pivot.
#pragma unroll
    for (int k = 0; k < SM; ++k) {
      float u[SM];
#pragma unroll
      for (int p = 0; p < SM; ++p) u[p] = gbf<G>(kf[p], k);
      // FP32 factors only precondition the FP64 refinement: the hardware
      // reciprocal (1 ulp) is accurate enough
      const float pinv = __builtin_amdgcn_rcpf(u[k]);
      bad |= !(fabsf(u[k]) >= 0x1p-24f);
      const bool pl = lane == k;
      const float lk = kf[k] * pinv;
      const float l = pl ? 1.f - pinv : lk;
#pragma unroll
      for (int p = 0; p < SM; ++p)
        if (p != k) kf[p] = fmaf(-l, u[p], kf[p]);
      kf[k] = pl ? pinv : -lk;
    }
    bad = group_ori<G>(bad);

    // ---- solve and refine in FP64 ----
    const double fq = rowl ? gb.f[lane] : 0.0;
    const double fnorm = group_maxd<G>(fabs(fq));
    double z = 0.0;
    int it = 0;
    bool conv = false;
    if (!bad) {
      z = (double)inv_apply<SM>(kf, gb.y, rowl, lane, (float)(fq * scale));
      for (it = 1; it <= kRefineMax; ++it) {
        if (rowl) gb.z[lane] = z;
        wave_sync();
        double r = fq;
        if (rowl) {
#pragma unroll
          for (int p = 0; p < SM; ++p) r = fma(-gb.K[lane * LD + p], gb.z[p], r);
        }
        // the FP32 solution itself is never accurate to FP64 rounding: the
        // first correction is applied unchecked
        if (it > 1) {
          const double rn = group_maxd<G>(fabs(r));
          const double zn = group_maxd<G>(fabs(z));
          if (rn <= 0x1p-47 * (knorm * zn + fnorm)) { conv = true; break; }
        }
        const float dz = inv_apply<SM>(kf, gb.y, rowl, lane, (float)(r * scale));
        z += (double)dz;
        wave_sync();
      }
      if (!(z == z)) conv = false;
      conv = group_ori<G>(conv ? 0 : 1) == 0;
    }
    if (!conv) {
      // FP32 factorisation not trusted: the workgroup solver redoes the row in FP64
      if (lane == 0) {
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = entry;
        else flag_row(st, ST_UNSUPPORTED, i);
      }
      continue;
    }
    if (lane == 0) rmx.add(w, ri.m, it);

    // ---- R row: F-entries of N(i) around the injected C-point ----
    if (lane < s) put_f_entry(w, d, ri.fine0, ri.off + lane + (lane >= dpos ? 1 : 0), myN, i, z);
    if (lane == 0) {
      d.Rci[ri.off + dpos] = i;
      d.Rva[ri.off + dpos] = 1.0;
    }
  }
  }
  if (lane == 0) rmx.flush(w);
}

// ---------------------------------------------------------------------------
// numeric pass, G lanes per row with R block rows per lane: block row q lives
// in lane q % G, register slot q / G.  Every lane works on R rows of the
// block, so a wavefront solves 64 / G rows at a time with no lane idle when
// G R = |N|, and each Gauss-Jordan step broadcasts the pivot row once for
// the R rows of a lane (the lane-per-row kernel above broadcasts it once per
// block row and leaves G - |N| lanes idle).
// ---------------------------------------------------------------------------
constexpr int pow2_at_least(int x) { return x <= 1 ? 1 : 2 * pow2_at_least((x + 1) / 2); }

// LDS of one row of k_lanes: blocks of up to SM points
// (f, zb and nb hold a slot for every lane row, dummies included, so that
// no store or load on them depends on the lane)
template <int SM, int RS>
struct LaneRowsBuf {
  double K[SM * SM];                 // FP64 block, row q = row q of (A[N,N])^T
  double f[RS];                      // -A[i,N], 0 beyond |N|
  double zb[RS];                     // broadcast buffer: z (FP64), or a correction's right-hand side (FP32)
  int nb[pow2_at_least(SM)];         // sorted N(i), INT32_MAX beyond |N|
};

// y_q = sum_p Kinv[q][p] v_p for the R rows q of a lane (v = scale * x in
// FP32): v goes through LDS once, then every lane reads all of it
template <int G, int R, int SM>
__device__ __forceinline__ void lanes_apply_inv(const float (&kf)[R][SM], float* yb, int lane, const double (&x)[R],
                                                double scale, float (&y)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) yb[lane + G * r] = (float)(x[r] * scale);  // dummy rows write past SM, unread
  wave_sync();
  float vs[SM];
#pragma unroll
  for (int p = 0; p < SM; ++p) vs[p] = yb[p];
  wave_sync();  // the buffer is reused next
#pragma unroll
  for (int r = 0; r < R; ++r) {
    float acc = 0.f;
#pragma unroll
    for (int p = 0; p < SM; ++p) acc = fmaf(kf[r][p], vs[p], acc);
    y[r] = acc;
  }
}

// One Gauss-Jordan step of k_lanes, K a compile-time constant (the swizzle
// pattern is an immediate; a loop over K is not always unrolled in full).
template <int G, int R, int SM, int K>
__device__ __forceinline__ void lanes_gj_step(float (&kf)[R][SM], int lane, int& bad) {
  constexpr int src = K % G, slot = K / G;
  float u[SM];
#pragma unroll
  for (int p = 0; p < SM; ++p)
    u[p] = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(kf[slot][p]), (32 - G) | (src << 5)));
  // FP32 factors only precondition the FP64 refinement: the hardware
  // reciprocal (1 ulp) is accurate enough
  const float pinv = __builtin_amdgcn_rcpf(u[K]);
  bad |= !(fabsf(u[K]) >= 0x1p-24f);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool pl = (r == slot) && (lane == src);
    const float lk = kf[r][K] * pinv;
    const float l = pl ? 1.f - pinv : lk;
#pragma unroll
    for (int p = 0; p < SM; ++p)
      if (p != K) kf[r][p] = fmaf(-l, u[p], kf[r][p]);
    kf[r][K] = pl ? pinv : -lk;
  }
  // keep the scheduler from interleaving steps (that multiplies live rows)
  __builtin_amdgcn_sched_barrier(0);
}

template <int G, int R, int SM, int... Ks>
__device__ __forceinline__ void lanes_gj(float (&kf)[R][SM], int lane, int& bad, std::integer_sequence<int, Ks...>) {
  (lanes_gj_step<G, R, SM, Ks>(kf, lane, bad), ...);
}

template <int G, int R, int SM, int NT>
__global__ __launch_bounds__(NT) void k_lanes(Work w, int which) {
  static_assert(SM <= G * R && SM > G * (R - 1), "block bound");
  static_assert(NT % 64 == 0 && 64 % G == 0, "shape");
  constexpr int NG = NT / G;
  constexpr int NBP = pow2_at_least(SM);
  __shared__ LaneRowsBuf<SM, G * R> sb[NG];

  const int tid = threadIdx.x;
  const int grp = tid / G;
  const int lane = tid % G;
  LaneRowsBuf<SM, G * R>& gb = sb[grp];
  const uint64_t gmask = (G >= 64) ? ~0ull : (((1ull << G) - 1ull) << ((threadIdx.x & 63) - lane));
  // block rows of this lane: q_r = lane + G r; rows at or beyond SM are dummies
  bool rowl[R];
#pragma unroll
  for (int r = 0; r < R; ++r) rowl[r] = lane + G * r < SM;

  if ((which ? w.cnt->nB : w.cnt->nA) == 0) return;
  const int smin = which ? small_limit(w.GA) + 1 : 0;
  const int32_t* slots = which ? w.slotB : w.slotA;
  const int sstride = which ? 32 : slot_stride(w.GA);
  const int total = w.cnt->total_rows;
  const RowBlocks rbk(total, 4 * NG);
  int r0, r1;
  if (!rbk.block(0, &r0, &r1)) return;
  RefineMax rmx;
  ChunkCursor cc;
  // one row ahead, as in k_numeric: chunk data, slot entries and A-row bounds
  // of row g + NG are loaded while row g is solved
  int nx_t = 0, nx_i = 0, nx_off = 0, nx_s = -1, nx_f0 = 0, nx_f1 = 0;
  int nx_N[R], nx_e0[R], nx_e1[R];
  bool ahead = false;

  for (int jb = 0; rbk.block(jb, &r0, &r1); ++jb) {
  ahead = false;
  for (int gbase = r0; gbase < r1; gbase += NG) {
    const int g = gbase + grp;
    if (g >= r1) break;  // group-uniform
    int t, i, off, s, fe0, fe1;
    int myN0[R], ae0[R], ae1[R];
    if (ahead) {
      t = nx_t; i = nx_i; off = nx_off; s = nx_s; fe0 = nx_f0; fe1 = nx_f1;
#pragma unroll
      for (int r = 0; r < R; ++r) { myN0[r] = nx_N[r]; ae0[r] = nx_e0[r]; ae1[r] = nx_e1[r]; }
    } else {
      cc.seek(w, g);
      cc.row(w, g, &t, &i, &off, &s);
      fe0 = 0; fe1 = 0;
      const bool ok = s >= smin && s <= SM && cc.live;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = lane + G * r;
        myN0[r] = slots[(cc.fbase + t) * sstride + min(q, sstride - 1)];
        ae0[r] = 0; ae1[r] = 0;
        if (ok && q < s) { ae0[r] = cc.md.rp[myN0[r]]; ae1[r] = cc.md.rp[myN0[r] + 1]; }
      }
      if (ok) { fe0 = cc.md.rp[i]; fe1 = cc.md.rp[i + 1]; }
    }
    const int gn = g + NG;
    ahead = gn < r1 && gn < cc.re;
    if (ahead) {
      cc.row(w, gn, &nx_t, &nx_i, &nx_off, &nx_s);
#pragma unroll
      for (int r = 0; r < R; ++r) nx_N[r] = slots[(cc.fbase + nx_t) * sstride + min(lane + G * r, sstride - 1)];
    }
    const bool mine = s >= smin && s <= SM && cc.live;  // group-uniform
    const bool nx_mine = ahead && nx_s >= smin && nx_s <= SM && cc.live;
    if (!mine) {
      if (which && s > SM && s <= 32 && cc.live && lane == 0) {
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = cc.c * w.chunk + t;
        else flag_row(&w.st[cc.m], ST_UNSUPPORTED, i);
      }
      if (nx_mine) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          nx_e0[r] = 0; nx_e1[r] = 0;
          if (lane + G * r < nx_s) { nx_e0[r] = cc.md.rp[nx_N[r]]; nx_e1[r] = cc.md.rp[nx_N[r] + 1]; }
        }
        nx_f0 = cc.md.rp[nx_i];
        nx_f1 = cc.md.rp[nx_i + 1];
      }
      continue;
    }
    const int entry = cc.c * w.chunk + t;
    const GDesc& d = cc.md;
    MatStatus* st = &w.st[cc.m];
    const int rr = g - cc.rbase_m;
    if (lane == 0) d.Rrp[rr] = off;
    int myN[R];
    int below = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = lane + G * r;
      myN[r] = (q < s) ? myN0[r] : 0x7fffffff;
      gb.nb[q] = myN[r];
      gb.f[q] = 0.0;
      below += __popcll(__ballot(q < s && myN[r] < i) & gmask);
    }
    if constexpr (G * R < NBP) {
      for (int q = G * R + lane; q < NBP; q += G) gb.nb[q] = 0x7fffffff;
    }
    const int dpos = below;

    // ---- gather: K = (A[N,N])^T (identity on the padding), f = -A[i,N] ----
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = lane + G * r;
      if (q < SM) {
#pragma unroll
        for (int p = 0; p < SM; ++p) gb.K[q * SM + p] = (p == q && q >= s) ? 1.0 : 0.0;
      }
    }
    wave_sync();
    {
      int len = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) len = max(len, ae1[r] - ae0[r]);
      for (int o = 0; o < len; o += 4) {
        int k[R][4];
        double v[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            k[r][j] = -1;
            v[r][j] = 0.0;
            if (ae0[r] + o + j < ae1[r]) { k[r][j] = d.ci[ae0[r] + o + j]; v[r][j] = d.va[ae0[r] + o + j]; }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int qq = find_pos<NBP>(gb.nb, k[r][j]);
            if (qq >= 0) gb.K[qq * SM + lane + G * r] = v[r][j];
          }
        }
      }
    }
    for (int e = fe0 + lane; e < fe1; e += G) {
      const int qq = find_pos<NBP>(gb.nb, d.ci[e]);
      if (qq >= 0) gb.f[qq] = -d.va[e];
    }
    wave_sync();
    if (nx_mine) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        nx_e0[r] = 0; nx_e1[r] = 0;
        if (lane + G * r < nx_s) { nx_e0[r] = d.rp[nx_N[r]]; nx_e1[r] = d.rp[nx_N[r] + 1]; }
      }
      nx_f0 = d.rp[nx_i];
      nx_f1 = d.rp[nx_i + 1];
    }

    // ---- FP32 inverse of the scaled block ----
    // (loops over columns that index no register array stay rolled, so the
    // compiler does not hoist every LDS load of the block at once)
    float amax = 0.f;
    double knorm = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // a dummy row (beyond SM) reads the last row and is ignored
      const double* kr = gb.K + min(lane + G * r, SM - 1) * SM;
      double rs = 0.0;
#pragma unroll 4
      for (int p = 0; p < SM; ++p) {
        const double v = (lane + G * r < s) ? fabs(kr[p]) : 0.0;  // the identity padding does not count
        amax = fmaxf(amax, (float)v);
        rs += v;
      }
      knorm = fmax(knorm, rs);
    }
    amax = group_maxf<G>(amax);
    knorm = group_maxd<G>(knorm);
    int ex = 0;
    frexpf(amax, &ex);
    const double scale = ldexp(1.0, -ex);
    float kf[R][SM];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int p = 0; p < SM; ++p) {
        const float x = (float)(gb.K[min(lane + G * r, SM - 1) * SM + p] * scale);
        // padding rows keep a unit pivot whatever the scale (they are
        // decoupled from the block, and their z stays 0)
        kf[r][p] = !rowl[r] ? 0.f : (lane + G * r >= s) ? (p == lane + G * r ? 1.f : 0.f) : x;
        if ((p & 7) == 7) __builtin_amdgcn_sched_barrier(0);
      }
    }
    int bad = !(amax > 0.f) || !(amax < 3.0e38f);
    // Gauss-Jordan in place without pivoting (as in k_numeric): step k
    // broadcasts pivot row k from lane k % G, slot k / G, once for all R rows
    // of every lane
    lanes_gj<G, R, SM>(kf, lane, bad, std::make_integer_sequence<int, SM>{});
    bad = group_ori<G>(bad);

    // ---- solve and refine in FP64 ----
    double fq[R], z[R];
    double fmaxv = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      fq[r] = gb.f[lane + G * r];  // 0 on padding and dummy rows
      fmaxv = fmax(fmaxv, fabs(fq[r]));
      z[r] = 0.0;
    }
    const double fnorm = group_maxd<G>(fmaxv);
    int it = 0;
    bool conv = false;
    // Every group runs the solve, also one whose factorisation is not
    // trusted (its result is then discarded): a branch on `bad` here lets the
    // compiler sink the last elimination steps into it, which keeps the
    // broadcasts of many steps alive at once and spills.
    {
      {
        float y[R];
        lanes_apply_inv<G, R, SM>(kf, reinterpret_cast<float*>(gb.zb), lane, fq, scale, y);
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] = (double)y[r];
      }
      for (it = 1; it <= kRefineMax; ++it) {
#pragma unroll
        for (int r = 0; r < R; ++r) gb.zb[lane + G * r] = z[r];  // dummy rows write past SM, unread
        wave_sync();
        double res[R];
        double rmax = 0.0, zmax = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) res[r] = fq[r];
        // (a dummy row, beyond SM, reads the last row and is ignored: no
        // branch on the lane inside the loop)
#pragma unroll 2
        for (int p = 0; p < SM; ++p) {
          const double zp = gb.zb[p];
#pragma unroll
          for (int r = 0; r < R; ++r) res[r] = fma(-gb.K[min(lane + G * r, SM - 1) * SM + p], zp, res[r]);
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          rmax = fmax(rmax, rowl[r] ? fabs(res[r]) : 0.0);
          zmax = fmax(zmax, rowl[r] ? fabs(z[r]) : 0.0);
        }
        // the FP32 solution is never accurate to FP64 rounding: the first
        // correction is applied unchecked
        if (bad) break;  // group-uniform: the FP64 solver takes the row
        if (it > 1) {
          const double rn = group_maxd<G>(rmax);
          const double zn = group_maxd<G>(zmax);
          if (rn <= 0x1p-47 * (knorm * zn + fnorm)) { conv = true; break; }
        }
        float y[R];
        lanes_apply_inv<G, R, SM>(kf, reinterpret_cast<float*>(gb.zb), lane, res, scale, y);
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] += (double)y[r];
      }
      bool nan = false;
#pragma unroll
      for (int r = 0; r < R; ++r) nan |= !(z[r] == z[r]);
      if (nan || bad) conv = false;
      conv = group_ori<G>(conv ? 0 : 1) == 0;
    }
    if (!conv) {
      // FP32 factorisation not trusted: the workgroup solver redoes the row in FP64
      if (lane == 0) {
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = entry;
        else flag_row(st, ST_UNSUPPORTED, i);
      }
      continue;
    }
    if (lane == 0) rmx.add(w, cc.m, it);

    // ---- R row: F-entries of N(i) around the injected C-point ----
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = lane + G * r;
      if (q < s) put_f_entry(w, d, cc.fine0, off + q + (q >= dpos ? 1 : 0), myN[r], i, z[r]);
    }
    if (lane == 0) {
      d.Rci[off + dpos] = i;
      d.Rva[off + dpos] = 1.0;
    }
  }
  }
  if (lane == 0) rmx.flush(w);
}

// ---------------------------------------------------------------------------
// numeric pass, four lanes (a quad) per row with |N| <= 8.  Lane l of the quad
// owns rows 2l and 2l+1 of K = (A[N,N])^T.  The block is transposed once
// through LDS after the gather; the LU, both triangular solves and the FP64
// residual then broadcast within the quad with DPP quad permutations
// (register moves, no LDS round trip).  A row of at most four points takes
// the 4 x 4 corner only, one block row per lane.  The kernel runs at three
// wavefronts per SIMD: at four the compiler spills the two paths' registers.
// ---------------------------------------------------------------------------
// lane src of the quad, to all four (src is a constant once the calling loops
// are unrolled, so the switch folds to one DPP move)
__device__ __forceinline__ int qbi(int v, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0xAA, 0xF, 0xF, false);
    default: return __builtin_amdgcn_mov_dpp(v, 0xFF, 0xF, 0xF, false);
  }
}
__device__ __forceinline__ float qb(float v, int src) { return __int_as_float(qbi(__float_as_int(v), src)); }
__device__ __forceinline__ double qbd(double v, int src) {
  return __hiloint2double(qbi(__double2hiint(v), src), qbi(__double2loint(v), src));
}
// quad reductions: partners lane^1 and lane^2 (quad_perm [1,0,3,2] and [2,3,0,1])
__device__ __forceinline__ float qmaxf(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false)));
  return v;
}
__device__ __forceinline__ double qxd(double v, int ctrl_is_b1) {
  const int lo = ctrl_is_b1 ? __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false)
                            : __builtin_amdgcn_mov_dpp(__double2loint(v), 0x4E, 0xF, 0xF, false);
  const int hi = ctrl_is_b1 ? __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false)
                            : __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x4E, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double qmaxd(double v) {
  v = fmax(v, qxd(v, 1));
  v = fmax(v, qxd(v, 0));
  return v;
}
__device__ __forceinline__ int qori(int v) {
  v |= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  v |= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  return v;
}

constexpr int kQG = 5;  // entries per gather round of k_quad8

struct QuadBuf {
  double K[8 * 8];  // gathered block, row q of K at stride 8
  double f[8];
  int nb[8];
};

// value of register slot S (0/1) of lane SRC = row 2*SRC+S, broadcast in the quad
#define QB_ROW(arr0, arr1, k, p) ((k) & 1 ? qb(arr1[p], (k) / 2) : qb(arr0[p], (k) / 2))

template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_quad8(Work w) {
  constexpr int NQ = NT / 4;
  __shared__ QuadBuf qbuf[NQ];
  const int tid = threadIdx.x;
  const int qd = tid >> 2;
  const int ql = tid & 3;
  QuadBuf& B = qbuf[qd];
  if (w.cnt->nA == 0) return;
  const int total = w.cnt->total_rows;
  const RowBlocks rbk(total, 4 * NQ);
  int r0, r1;
  if (!rbk.block(0, &r0, &r1)) return;
  RefineMax rmx;
  const int q0 = 2 * ql, q1 = 2 * ql + 1;  // this lane's rows of K
  ChunkCursor cc;

  for (int jb = 0; rbk.block(jb, &r0, &r1); ++jb) {
  for (int g = r0 + qd; g < r1; g += NQ) {  // quad-uniform
    cc.seek(w, g);
    int t, i, off, s;
    cc.row(w, g, &t, &i, &off, &s);
    if (s > 8 || !cc.live) continue;
    const int c = cc.c;
    MatStatus* st = &w.st[cc.m];
    const GDesc& d = cc.md;
    RowInfo ri;
    ri.m = cc.m;
    ri.i = i;
    ri.r = g - cc.rbase_m;
    ri.off = off;
    ri.s = s;
    ri.fine0 = cc.fine0;
    const int64_t fbase = cc.fbase;
    const int2 nn = *reinterpret_cast<const int2*>(w.slotA + (fbase + t) * 8 + q0);
    const int n0 = q0 < s ? nn.x : 0x7fffffff;
    const int n1 = q1 < s ? nn.y : 0x7fffffff;
    if (ql == 0) d.Rrp[ri.r] = ri.off;
    B.nb[q0] = n0;
    B.nb[q1] = n1;
#pragma unroll
    for (int u = 0; u < 16; ++u) {  // zero the block, identity on the padding
      const int idx = ql * 16 + u;
      const int rq = idx / 8, cp = idx % 8;
      B.K[idx] = (rq == cp && rq >= s) ? 1.0 : 0.0;
    }
    B.f[q0] = 0.0;
    B.f[q1] = 0.0;
    wave_sync();
    // gather: lane l walks rows N_{2l}, N_{2l+1} of A (columns 2l, 2l+1 of
    // K) side by side, kQG entries of each at a time (a five-point row in
    // one round)
    {
      int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
      if (q0 < s) { a0 = d.rp[n0]; a1 = d.rp[n0 + 1]; }
      if (q1 < s) { b0 = d.rp[n1]; b1 = d.rp[n1 + 1]; }
      // row i's bounds and its first eight entries (two per lane) go out with
      // the block rows' loads
      const int i0 = d.rp[i], i1 = d.rp[i + 1];
      int kf[2];
      double vf[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = i0 + ql + 4 * h;
        kf[h] = -1;
        vf[h] = 0.0;
        if (e < i1) { kf[h] = d.ci[e]; vf[h] = d.va[e]; }
      }
      for (int o = 0; a0 + o < a1 || b0 + o < b1; o += kQG) {
        int ka[kQG], kb[kQG];
        double va_[kQG], vb_[kQG];
#pragma unroll
        for (int j = 0; j < kQG; ++j) {
          ka[j] = -1;
          kb[j] = -1;
          va_[j] = 0.0;
          vb_[j] = 0.0;
          if (a0 + o + j < a1) { ka[j] = d.ci[a0 + o + j]; va_[j] = d.va[a0 + o + j]; }
          if (b0 + o + j < b1) { kb[j] = d.ci[b0 + o + j]; vb_[j] = d.va[b0 + o + j]; }
        }
#pragma unroll
        for (int j = 0; j < kQG; ++j) {
          const int qa = find_pos<8>(B.nb, ka[j]);
          const int qb_ = find_pos<8>(B.nb, kb[j]);
          if (qa >= 0) B.K[qa * 8 + q0] = va_[j];
          if (qb_ >= 0) B.K[qb_ * 8 + q1] = vb_[j];
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int qq = find_pos<8>(B.nb, kf[h]);
        if (qq >= 0) B.f[qq] = -vf[h];
      }
      for (int e = i0 + ql + 8; e < i1; e += 4) {  // rows of more than eight entries
        const int qq = find_pos<8>(B.nb, d.ci[e]);
        if (qq >= 0) B.f[qq] = -d.va[e];
      }
    }
    wave_sync();
    if (s <= 4) {
      // Blocks of at most four points (every row at distance 1 on a
      // five-point graph): lane l owns row l of the 4 x 4 corner of K (the
      // padding rows are identity there as in the full block), so the LU, the
      // substitutions and the residual take four steps instead of eight.
      const int q = ql;
      double kq[4];
      float amax = 0.f;
      double rs = 0.0;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        kq[p] = B.K[q * 8 + p];
        amax = fmaxf(amax, (float)fabs(kq[p]));
        rs += fabs(kq[p]);
      }
      const double fq = B.f[q];
      const int nq = B.nb[q];  // INT32_MAX on padding rows
      amax = qmaxf(amax);
      const double knorm = qmaxd(rs);
      const double fnorm = qmaxd(fabs(fq));
      int ex = 0;
      frexpf(amax, &ex);
      const double scale = ldexp(1.0, -ex);
      float a[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) a[p] = (float)(kq[p] * scale);
      int bad = !(amax > 0.f) || !(amax < 3.0e38f);
      float ui = 1.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float pr[4];
#pragma unroll
        for (int p = k; p < 4; ++p) pr[p] = qb(a[p], k);
        bad |= !(fabsf(pr[k]) >= 0x1p-24f);
        const float pinv = __builtin_amdgcn_rcpf(pr[k]);
        if (q == k) ui = pinv;
        if (q > k) {
          const float l = a[k] * pinv;
          a[k] = l;
#pragma unroll
          for (int p = k + 1; p < 4; ++p) a[p] = fmaf(-l, pr[p], a[p]);
        }
      }
      bad = qori(bad);
      double z = 0.0;
      int it = 0;
      bool conv = false;
      if (!bad) {
        // K y = rhs for this lane's entry of y
        auto solve4 = [&](float y) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {  // forward, unit lower
            const float yk = qb(y, k);
            if (q > k) y = fmaf(-a[k], yk, y);
          }
#pragma unroll
          for (int k = 3; k >= 0; --k) {  // backward, upper
            if (q == k) y *= ui;
            const float zk = qb(y, k);
            if (q < k) y = fmaf(-a[k], zk, y);
          }
          return y;
        };
        z = solve4((float)(fq * scale));
        for (it = 1; it <= kRefineMax; ++it) {
          double r = fq;
#pragma unroll
          for (int p = 0; p < 4; ++p) r = fma(-kq[p], qbd(z, p), r);
          const double rn = qmaxd(fabs(r));
          const double zn = qmaxd(fabs(z));
          if (rn <= 0x1p-47 * (knorm * zn + fnorm)) { conv = true; break; }
          z += (double)solve4((float)(r * scale));
        }
        conv = conv && (z == z);
        conv = qori(conv ? 0 : 1) == 0;
      }
      if (!conv) {
        if (ql == 0) {
          const int qc = atomicAdd(&w.cnt->nC, 1);
          if (qc < w.capC) w.binC[qc] = c * w.chunk + t;
          else flag_row(st, ST_UNSUPPORTED, i);
        }
        continue;
      }
      if (ql == 0) rmx.add(w, ri.m, it);
      const int below = nq < i ? 1 : 0;
      const int b2 = below + __builtin_amdgcn_mov_dpp(below, 0xB1, 0xF, 0xF, false);
      const int dpos4 = b2 + __builtin_amdgcn_mov_dpp(b2, 0x4E, 0xF, 0xF, false);
      if (q < s) put_f_entry(w, d, ri.fine0, ri.off + q + (q >= dpos4 ? 1 : 0), nq, i, z);
      if (ql == 0) {
        d.Rci[ri.off + dpos4] = i;
        d.Rva[ri.off + dpos4] = 1.0;
      }
      continue;
    }
    // rows q0, q1 of K (FP64), scaled FP32 copies
    double k0[8], k1[8];
    float amax = 0.f;
    double rs0 = 0.0, rs1 = 0.0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      k0[p] = B.K[q0 * 8 + p];
      k1[p] = B.K[q1 * 8 + p];
      amax = fmaxf(amax, fmaxf((float)fabs(k0[p]), (float)fabs(k1[p])));
      rs0 += fabs(k0[p]);
      rs1 += fabs(k1[p]);
    }
    const double f0 = B.f[q0], f1 = B.f[q1];
    amax = qmaxf(amax);
    const double knorm = qmaxd(fmax(rs0, rs1));
    const double fnorm = qmaxd(fmax(fabs(f0), fabs(f1)));
    int ex = 0;
    frexpf(amax, &ex);
    const double scale = ldexp(1.0, -ex);
    float a0[8], a1[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      a0[p] = (float)(k0[p] * scale);
      a1[p] = (float)(k1[p] * scale);
    }
    // LU without pivoting: lane-local rows, pivot rows broadcast in the quad
    int bad = !(amax > 0.f) || !(amax < 3.0e38f);
    float ui0 = 1.f, ui1 = 1.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float pr[8];
#pragma unroll
      for (int p = k; p < 8; ++p) pr[p] = QB_ROW(a0, a1, k, p);
      const float piv = pr[k];
      bad |= !(fabsf(piv) >= 0x1p-24f);
      const float pinv = __builtin_amdgcn_rcpf(piv);
      if (q0 == k) ui0 = pinv;
      if (q1 == k) ui1 = pinv;
      if (q0 > k) {
        const float l = a0[k] * pinv;
        a0[k] = l;
#pragma unroll
        for (int p = k + 1; p < 8; ++p) a0[p] = fmaf(-l, pr[p], a0[p]);
      }
      if (q1 > k) {
        const float l = a1[k] * pinv;
        a1[k] = l;
#pragma unroll
        for (int p = k + 1; p < 8; ++p) a1[p] = fmaf(-l, pr[p], a1[p]);
      }
    }
    bad = qori(bad);

    double z0 = 0.0, z1 = 0.0;
    int it = 0;
    bool conv = false;
    if (!bad) {
      // solve K y = rhs for this lane's two entries y0, y1
      auto solve = [&](float y0, float y1, float* o0, float* o1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {  // forward, unit lower
          const float yk = (k & 1) ? qb(y1, k / 2) : qb(y0, k / 2);
          if (q0 > k) y0 = fmaf(-a0[k], yk, y0);
          if (q1 > k) y1 = fmaf(-a1[k], yk, y1);
        }
#pragma unroll
        for (int k = 7; k >= 0; --k) {  // backward, upper
          if (q0 == k) y0 *= ui0;
          if (q1 == k) y1 *= ui1;
          const float zk = (k & 1) ? qb(y1, k / 2) : qb(y0, k / 2);
          if (q0 < k) y0 = fmaf(-a0[k], zk, y0);
          if (q1 < k) y1 = fmaf(-a1[k], zk, y1);
        }
        *o0 = y0;
        *o1 = y1;
      };
      float y0, y1;
      solve((float)(f0 * scale), (float)(f1 * scale), &y0, &y1);
      z0 = y0;
      z1 = y1;
      for (it = 1; it <= kRefineMax; ++it) {
        // r = f - K z in FP64: all of z broadcast in the quad
        // (the FP64 rows are read from LDS again rather than kept live)
        double r0 = f0, r1 = f1;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const double zp = (p & 1) ? qbd(z1, p / 2) : qbd(z0, p / 2);
          r0 = fma(-B.K[q0 * 8 + p], zp, r0);
          r1 = fma(-B.K[q1 * 8 + p], zp, r1);
        }
        const double rn = qmaxd(fmax(fabs(r0), fabs(r1)));
        const double zn = qmaxd(fmax(fabs(z0), fabs(z1)));
        if (rn <= 0x1p-47 * (knorm * zn + fnorm)) { conv = true; break; }
        float d0, d1;
        solve((float)(r0 * scale), (float)(r1 * scale), &d0, &d1);
        z0 += (double)d0;
        z1 += (double)d1;
      }
      conv = conv && (z0 == z0) && (z1 == z1);
      conv = qori(conv ? 0 : 1) == 0;
    }
    if (!conv) {
      // FP32 factorisation not trusted: the workgroup solver redoes the row in FP64
      if (ql == 0) {
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = c * w.chunk + t;
        else flag_row(st, ST_UNSUPPORTED, i);
      }
      continue;
    }
    if (ql == 0) rmx.add(w, ri.m, it);
    // R row
    const int dpos_l = (n0 < i ? 1 : 0) + (n1 < i ? 1 : 0);
    const int dpos = dpos_l + __builtin_amdgcn_mov_dpp(dpos_l, 0xB1, 0xF, 0xF, false);
    const int dposq = dpos + __builtin_amdgcn_mov_dpp(dpos, 0x4E, 0xF, 0xF, false);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = q0 + h;
      if (p < s) put_f_entry(w, d, ri.fine0, ri.off + p + (p >= dposq ? 1 : 0), h ? n1 : n0, i, h ? z1 : z0);
    }
    if (ql == 0) {
      d.Rci[ri.off + dposq] = i;
      d.Rva[ri.off + dposq] = 1.0;
    }
  }
  }
  if (ql == 0) rmx.flush(w);
}

// ---------------------------------------------------------------------------
// numeric pass, one thread per row with |N| <= 8.  The neighbourhood comes
// from the row's slot; the FP64 block, its FP32 LU and the right-hand side
// stay in the thread's registers, so the solve needs no communication.  A
// wavefront takes 64 consecutive rows (neighbouring C-points: their A rows
// share cache lines), and the rows of A are read eight entries at a time, two
// rows side by side.
// ---------------------------------------------------------------------------
constexpr int kS8 = 8;

// position of column k in the sorted neighbourhood N (and whether it is there)
__device__ __forceinline__ int pos8(const int (&N)[kS8], int k, bool* hit) {
  int q = 0;
  bool h = false;
#pragma unroll
  for (int j = 0; j < kS8; ++j) {
    q += (N[j] < k) ? 1 : 0;
    h |= (N[j] == k);
  }
  *hit = h;
  return q;
}

// y <- K^{-1} y with the packed no-pivot LU of K (unit lower L, upper U)
__device__ __forceinline__ void lu8_solve(const float (&K)[kS8][kS8], const float (&inv)[kS8], float (&y)[kS8]) {
#pragma unroll
  for (int q = 1; q < kS8; ++q)
#pragma unroll
    for (int k = 0; k < q; ++k) y[q] = fmaf(-K[q][k], y[k], y[q]);
#pragma unroll
  for (int q = kS8 - 1; q >= 0; --q) {
#pragma unroll
    for (int k = q + 1; k < kS8; ++k) y[q] = fmaf(-K[q][k], y[k], y[q]);
    y[q] *= inv[q];
  }
}

// K[q][p] = A[N_p][N_q] for the entries of rows N_pa and N_pb (columns pa, pb
// of K), eight entries of each row per batch
template <int PA>
__device__ __forceinline__ void gather8_pair(gptr<const int32_t> __restrict__ ci, gptr<const double> __restrict__ va,
                                             const int (&N)[kS8], const int (&e0)[kS8], const int (&e1)[kS8],
                                             double (&K)[kS8][kS8]) {
  constexpr int PB = PA + 1;
  for (int o = 0; e0[PA] + o < e1[PA] || e0[PB] + o < e1[PB]; o += 8) {
    int ka[8], kb[8];
    double xa[8], xb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ka[j] = -1;
      kb[j] = -1;
      xa[j] = 0.0;
      xb[j] = 0.0;
      if (e0[PA] + o + j < e1[PA]) { ka[j] = ci[e0[PA] + o + j]; xa[j] = va[e0[PA] + o + j]; }
      if (e0[PB] + o + j < e1[PB]) { kb[j] = ci[e0[PB] + o + j]; xb[j] = va[e0[PB] + o + j]; }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (ka[j] >= 0) {
        bool hit;
        const int q = pos8(N, ka[j], &hit);
#pragma unroll
        for (int qq = 0; qq < kS8; ++qq)
          if (hit && q == qq) K[qq][PA] = xa[j];
      }
      if (kb[j] >= 0) {
        bool hit;
        const int q = pos8(N, kb[j], &hit);
#pragma unroll
        for (int qq = 0; qq < kS8; ++qq)
          if (hit && q == qq) K[qq][PB] = xb[j];
      }
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_rows8(Work w) {
  if (w.cnt->nA == 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int total = w.cnt->total_rows;
  const RowBlocks rbk(total, 4 * NT);
  int r0, r1;
  if (!rbk.block(0, &r0, &r1)) return;
  RefineMax rmx;
  ChunkCursor cc;

  for (int jb = 0; rbk.block(jb, &r0, &r1); ++jb) {
  for (int gw = r0 + (tid & ~63); gw < r1; gw += NT) {
    const int g = gw + lane;
    const int gend = min(gw + 64, r1);
    for (int gc = gw; gc < gend;) {  // wavefront-uniform: one chunk at a time
      cc.seek(w, __builtin_amdgcn_readfirstlane(gc));
      const int cend = min(gend, cc.re);
      int t = 0, i = 0, off = 0, s = kS8 + 1;
      if (g >= gc && g < cend && cc.live) cc.row(w, g, &t, &i, &off, &s);
      gc = cend;
      if (s > kS8) continue;  // not this thread's row, or another solver's
      const GDesc& d = cc.md;
      MatStatus* st = &w.st[cc.m];
      const gptr<const int32_t> __restrict__ rp = d.rp;
      const gptr<const int32_t> __restrict__ ci = d.ci;
      const gptr<const double> __restrict__ va = d.va;
      d.Rrp[g - cc.rbase_m] = off;

      // N(i) from the slot; unused entries INT32_MAX
      const int4* sp = reinterpret_cast<const int4*>(w.slotA + (cc.fbase + t) * kS8);
      const int4 sa = sp[0], sb = sp[1];
      int N[kS8] = {sa.x, sa.y, sa.z, sa.w, sb.x, sb.y, sb.z, sb.w};
      int e0[kS8], e1[kS8];
#pragma unroll
      for (int p = 0; p < kS8; ++p) {
        if (p >= s) N[p] = 0x7fffffff;
        e0[p] = 0;
        e1[p] = 0;
        if (p < s) { e0[p] = rp[N[p]]; e1[p] = rp[N[p] + 1]; }
      }
      const int fi0 = rp[i], fi1 = rp[i + 1];

      // f = -A[i,N]
      double f[kS8];
#pragma unroll
      for (int q = 0; q < kS8; ++q) f[q] = 0.0;
      for (int e = fi0; e < fi1; e += 8) {
        int kk[8];
        double xx[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          kk[j] = -1;
          xx[j] = 0.0;
          if (e + j < fi1) { kk[j] = ci[e + j]; xx[j] = va[e + j]; }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (kk[j] >= 0) {
            bool hit;
            const int q = pos8(N, kk[j], &hit);
#pragma unroll
            for (int qq = 0; qq < kS8; ++qq)
              if (hit && q == qq) f[qq] = -xx[j];
          }
        }
      }

      // K = (A[N,N])^T in FP64, identity on the padding
      double K[kS8][kS8];
#pragma unroll
      for (int q = 0; q < kS8; ++q)
#pragma unroll
        for (int p = 0; p < kS8; ++p) K[q][p] = (q == p && q >= s) ? 1.0 : 0.0;
      gather8_pair<0>(ci, va, N, e0, e1, K);
      gather8_pair<2>(ci, va, N, e0, e1, K);
      gather8_pair<4>(ci, va, N, e0, e1, K);
      gather8_pair<6>(ci, va, N, e0, e1, K);

      // scale by a power of two, FP32 LU without pivoting; a small or
      // non-finite pivot hands the row to the FP64 solver with pivoting
      double amax = 0.0, knorm = 0.0, fnorm = 0.0;
#pragma unroll
      for (int q = 0; q < kS8; ++q) {
        double rs = 0.0;
#pragma unroll
        for (int p = 0; p < kS8; ++p) {
          amax = fmax(amax, fabs(K[q][p]));
          rs += fabs(K[q][p]);
        }
        knorm = fmax(knorm, rs);
        fnorm = fmax(fnorm, fabs(f[q]));
      }
      int ex = 0;
      frexp(amax > 0.0 ? amax : 1.0, &ex);
      const double scale = ldexp(1.0, -ex);
      float L[kS8][kS8];
#pragma unroll
      for (int q = 0; q < kS8; ++q)
#pragma unroll
        for (int p = 0; p < kS8; ++p) L[q][p] = (float)(K[q][p] * scale);
      float inv[kS8];
      bool bad = !(amax > 0.0) || !(amax * scale < 1e30);
#pragma unroll
      for (int k = 0; k < kS8; ++k) {
        const float piv = L[k][k];
        bad |= !(fabsf(piv) >= 0x1p-24f);
        inv[k] = __builtin_amdgcn_rcpf(piv);
#pragma unroll
        for (int q = k + 1; q < kS8; ++q) {
          const float l = L[q][k] * inv[k];
          L[q][k] = l;
#pragma unroll
          for (int p = k + 1; p < kS8; ++p) L[q][p] = fmaf(-l, L[k][p], L[q][p]);
        }
      }

      double z[kS8];
      int it = 0;
      bool conv = false;
      if (!bad) {
        float y[kS8];
#pragma unroll
        for (int q = 0; q < kS8; ++q) y[q] = (float)(f[q] * scale);
        lu8_solve(L, inv, y);
#pragma unroll
        for (int q = 0; q < kS8; ++q) z[q] = (double)y[q];
        for (it = 1; it <= kRefineMax; ++it) {
          double rn = 0.0, zn = 0.0;
#pragma unroll
          for (int q = 0; q < kS8; ++q) {
            double r = f[q];
#pragma unroll
            for (int p = 0; p < kS8; ++p) r = fma(-K[q][p], z[p], r);
            y[q] = (float)(r * scale);
            rn = fmax(rn, fabs(r));
            zn = fmax(zn, fabs(z[q]));
          }
          if (rn <= 0x1p-47 * (knorm * zn + fnorm)) { conv = true; break; }
          lu8_solve(L, inv, y);
#pragma unroll
          for (int q = 0; q < kS8; ++q) z[q] += (double)y[q];
        }
#pragma unroll
        for (int q = 0; q < kS8; ++q) conv &= (z[q] == z[q]);
      }
      if (!conv) {
        // FP32 factorisation not trusted: the workgroup solver redoes the row in FP64
        const int qc = atomicAdd(&w.cnt->nC, 1);
        if (qc < w.capC) w.binC[qc] = cc.c * w.chunk + t;
        else flag_row(st, ST_UNSUPPORTED, i);
        continue;
      }
      rmx.add(w, cc.m, it);

      // R row: the F-entries of N(i) around the injected C-point
      int dpos = 0;
#pragma unroll
      for (int p = 0; p < kS8; ++p) dpos += (N[p] < i) ? 1 : 0;
#pragma unroll
      for (int p = 0; p < kS8; ++p)
        if (p < s) put_f_entry(w, d, cc.fine0, off + p + (p >= dpos ? 1 : 0), N[p], i, z[p]);
      d.Rci[off + dpos] = i;
      d.Rva[off + dpos] = 1.0;
    }
  }
  }
  rmx.flush(w);
}

// ---------------------------------------------------------------------------
// workgroup-per-row FP64 solver (bin C)
// ---------------------------------------------------------------------------
constexpr int kWT = 256;
static_assert(kWT == kNT, "block_bfs runs on kNT threads");

__device__ __forceinline__ void block_argmax(double v, int idx, double* shv, int* shi, double* outv, int* outi) {
  const int tid = threadIdx.x;
  shv[tid] = v;
  shi[tid] = idx;
  __syncthreads();
  for (int o = kWT / 2; o > 0; o >>= 1) {
    if (tid < o) {
      const double a = shv[tid], b = shv[tid + o];
      const int ia = shi[tid], ib = shi[tid + o];
      if (b > a || (b == a && ib < ia)) { shv[tid] = b; shi[tid] = ib; }
    }
    __syncthreads();
  }
  *outv = shv[0];
  *outi = shi[0];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// blocks of 32 < |N| <= 128 in the workgroup solver: FP32 LU of the scaled
// block in LDS, blocked by panels of 32 columns, the trailing updates on the
// matrix cores (v_mfma_f32_32x32x2f32, one 32x32 tile per wavefront and
// step), FP32 triangular solves, FP64 residuals from A's CSR rows and
// iterative refinement.  No pivoting: a tiny pivot or no convergence hands
// the row to the FP64 solver with partial pivoting.
// ---------------------------------------------------------------------------
constexpr int kMfmaMax = 128;
constexpr int kRefineMaxBf16 = 10;  // refinement steps of the BF16-update factorisation
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// x rounded to bfloat16 (nearest, ties to even), as its 16 bits; x finite
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// max of v over the workgroup (all threads call; result to all)
__device__ __forceinline__ double block_maxd(double v, double* shv) {
  const int tid = threadIdx.x;
  shv[tid] = v;
  __syncthreads();
  for (int o = kWT / 2; o > 0; o >>= 1) {
    if (tid < o) shv[tid] = fmax(shv[tid], shv[tid + o]);
    __syncthreads();
  }
  const double r = shv[0];
  __syncthreads();
  return r;
}

// y <- K^{-1} y for the packed LU (unit lower L below the diagonal, U on and
// above it) of the S x S block in LDS (stride lda, S a multiple of 32); y in
// LDS.  All threads call.  Blocked by 32: wavefront 0 solves a diagonal block
// (unrolled, the solved entry of each step to all lanes by v_readlane), then
// every thread updates the remaining entries with that block's column strip,
// one mat-vec row per thread.
__device__ __forceinline__ void mf_lu_solve(const float* K, int lda, int S, float* y) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int o = 0; o < S; o += 32) {  // forward, unit lower
    if (tid < 64) {
      float v = (lane < 32) ? y[o + lane] : 0.f;
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const float yk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
        if (lane > k && lane < 32) v = fmaf(-K[(o + lane) * lda + o + k], yk, v);
      }
      if (lane < 32) y[o + lane] = v;
    }
    __syncthreads();
    for (int q = o + 32 + tid; q < S; q += kWT) {
      float acc = y[q];
#pragma unroll 8
      for (int k = 0; k < 32; ++k) acc = fmaf(-K[q * lda + o + k], y[o + k], acc);
      y[q] = acc;
    }
    __syncthreads();
  }
  for (int o = S - 32; o >= 0; o -= 32) {  // backward, upper
    if (tid < 64) {
      float v = (lane < 32) ? y[o + lane] : 0.f;
#pragma unroll
      for (int k = 31; k >= 0; --k) {
        if (lane == k) v = v / K[(o + k) * lda + o + k];
        const float yk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
        if (lane < k) v = fmaf(-K[(o + lane) * lda + o + k], yk, v);
      }
      if (lane < 32) y[o + lane] = v;
    }
    __syncthreads();
    for (int q = tid; q < o; q += kWT) {
      float acc = y[q];
#pragma unroll 8
      for (int k = 0; k < 32; ++k) acc = fmaf(-K[q * lda + o + k], y[o + k], acc);
      y[q] = acc;
    }
    __syncthreads();
  }
}

// Returns true with the solution in z[0..s) when the row converged.
// N: sorted neighbourhood (LDS); K: LDS buffer of (kMfmaMax+1)*kMfmaMax
// floats; f, z, r: LDS FP64 vectors of kMfmaMax; y: LDS FP32 vector of
// kMfmaMax.  bf16: the trailing updates take their L21 and U12 tiles
// rounded to bfloat16 (v_mfma_f32_32x32x8bf16_1k, FP32 accumulation), and
// the refinement may take up to kRefineMaxBf16 steps.
// LDS scratch of the residual's column lists (see below)
struct ResidLists {
  int* cnt;  // [kMfmaMax + 1]
  int* off;  // [kMfmaMax + 1]
  int* pp;   // [cap] block row p of each entry
  int* pe;   // [cap] its entry in A
  int* bnd;  // [2 kMfmaMax] row bounds, for rows whose lists exceed cap
  int cap;
};

__device__ __forceinline__ bool mixed_big_row(const GDesc& d, int i, const int* N, int s, float* K, double* f, double* z,
                              double* r, float* y, double* shv, int* s_flag, int* it_out, const ResidLists& rl,
                              bool bf16) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int S = (s + 31) & ~31;
  const int lda = S + 1;
  // scale: a power of two from the largest entry of the rows of N; norms
  double amax = 0.0, rsum = 0.0;
  for (int p = tid; p < s; p += kWT) {
    const int u = N[p];
    double rs = 0.0;
    for (int ee = d.rp[u]; ee < d.rp[u + 1]; ++ee) {
      const double v = fabs(d.va[ee]);
      amax = fmax(amax, v);
      rs += v;
    }
    rsum = fmax(rsum, rs);
  }
  amax = block_maxd(amax, shv);
  const double knorm = block_maxd(rsum, shv);
  if (!(amax > 0.0) || !(amax < 1e300)) return false;
  int ex = 0;
  frexp(amax, &ex);
  const double scale = ldexp(1.0, -ex);
  // the scaled block in FP32, identity on the padding; f = -A[i,N] in FP64
  for (int t = tid; t < S * lda; t += kWT) {
    const int q = t / lda, p = t - q * lda;
    K[t] = (q == p && q >= s) ? 1.f : 0.f;
  }
  for (int t = tid; t < kMfmaMax; t += kWT) { f[t] = 0.0; z[t] = 0.0; }
  __syncthreads();
  for (int p = tid; p < s; p += kWT) {
    const int u = N[p];
    for (int ee = d.rp[u]; ee < d.rp[u + 1]; ++ee) {
      const int q = find_sorted(N, s, d.ci[ee]);
      if (q >= 0) K[q * lda + p] = (float)(d.va[ee] * scale);
    }
  }
  for (int ee = d.rp[i] + tid; ee < d.rp[i + 1]; ee += kWT) {
    const int q = find_sorted(N, s, d.ci[ee]);
    if (q >= 0) f[q] = -d.va[ee];
  }
  if (tid == 0) s_flag[0] = 0;
  __syncthreads();

  // ---- blocked LU, panels of 32 columns ----
  for (int P0 = 0; P0 < S; P0 += 32) {
    const int Pe = P0 + 32;
    for (int k = P0; k < Pe; ++k) {
      const float piv = K[k * lda + k];
      if (tid == 0 && !(fabsf(piv) >= 0x1p-24f)) s_flag[0] = 1;
      const float pinv = __builtin_amdgcn_rcpf(piv);
      for (int q = k + 1 + tid; q < S; q += kWT) K[q * lda + k] *= pinv;
      __syncthreads();
      // rows of this block row: every column to the right (they become U);
      // rows below: the panel's columns only
      const int nr1 = Pe - k - 1, nc1 = S - k - 1;  // block-row part
      const int nr2 = S - Pe, nc2 = Pe - k - 1;     // panel part below
      const int n1 = nr1 * nc1, n2 = nr2 * nc2;
      for (int t = tid; t < n1 + n2; t += kWT) {
        int q, c;
        if (t < n1) { q = k + 1 + t / nc1; c = k + 1 + t % nc1; }
        else { const int u = t - n1; q = Pe + u / nc2; c = k + 1 + u % nc2; }
        K[q * lda + c] = fmaf(-K[q * lda + k], K[k * lda + c], K[q * lda + c]);
      }
      __syncthreads();
    }
    // trailing update K22 -= L21 U12 on the matrix cores
    const int T = (S - Pe) / 32;
    for (int tile = wv; tile < T * T; tile += kWT / 64) {
      const int i0 = Pe + 32 * (tile / T), j0 = Pe + 32 * (tile % T);
      floatx16 acc;
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int row = i0 + 8 * (rr / 4) + 4 * (lane / 32) + (rr % 4);
        acc[rr] = K[row * lda + j0 + (lane % 32)];
      }
      if (bf16) {
        // lane l supplies A[l % 32][4 (l / 32) + j] and B[4 (l / 32) + j][l % 32], j < 4
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int kc = P0 + 8 * kk + 4 * (lane / 32);
          bf16x4 a, b;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            a[j] = to_bf16(-K[(i0 + lane % 32) * lda + kc + j]);
            b[j] = to_bf16(K[(kc + j) * lda + j0 + lane % 32]);
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          const int kc = P0 + 2 * kk + lane / 32;
          const float a = -K[(i0 + lane % 32) * lda + kc];
          const float b = K[kc * lda + j0 + lane % 32];
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int row = i0 + 8 * (rr / 4) + 4 * (lane / 32) + (rr % 4);
        K[row * lda + j0 + (lane % 32)] = acc[rr];
      }
    }
    __syncthreads();
  }
  if (s_flag[0]) return false;

  // ---- solve and refine ----
  const double fnorm = [&] {
    double m = 0.0;
    for (int t = tid; t < s; t += kWT) m = fmax(m, fabs(f[t]));
    return block_maxd(m, shv);
  }();
  for (int t = tid; t < S; t += kWT) y[t] = (t < s) ? (float)(f[t] * scale) : 0.f;
  __syncthreads();
  mf_lu_solve(K, lda, S, y);
  for (int t = tid; t < s; t += kWT) z[t] = y[t];
  __syncthreads();
  // The residual r_q = f_q - sum_p a_{N_p, N_q} z_p reads, for each q, the
  // entries of column N_q in the rows N_p: lists built once per row (counted,
  // placed, then each ordered by p), so every residual sums in ascending p
  // (the same bits on every run) with independent loads.  Rows whose lists
  // exceed the scratch search each row N_p by bisection instead.
  int* cnt = rl.cnt;
  int* off = rl.off;
  for (int q = tid; q <= s; q += kWT) cnt[q] = 0;
  __syncthreads();
  for (int p = tid; p < s; p += kWT) {
    const int u = N[p];
    const int e1 = d.rp[u + 1];
    for (int e = d.rp[u]; e < e1; ++e) {
      const int q = find_sorted(N, s, d.ci[e]);
      if (q >= 0) atomicAdd(&cnt[q], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int o = 0;
    for (int q = 0; q < s; ++q) {
      off[q] = o;
      o += cnt[q];
      cnt[q] = 0;
    }
    off[s] = o;
  }
  __syncthreads();
  const bool lists = off[s] <= rl.cap;  // workgroup-uniform
  if (lists) {
    for (int p = tid; p < s; p += kWT) {
      const int u = N[p];
      const int e1 = d.rp[u + 1];
      for (int e = d.rp[u]; e < e1; ++e) {
        const int q = find_sorted(N, s, d.ci[e]);
        if (q >= 0) {
          const int k = off[q] + atomicAdd(&cnt[q], 1);
          rl.pp[k] = p;
          rl.pe[k] = e;
        }
      }
    }
    __syncthreads();
    for (int q = tid; q < s; q += kWT) {  // insertion sort of list q by p
      for (int k = off[q] + 1; k < off[q + 1]; ++k) {
        const int kp = rl.pp[k], ke = rl.pe[k];
        int m = k - 1;
        while (m >= off[q] && rl.pp[m] > kp) {
          rl.pp[m + 1] = rl.pp[m];
          rl.pe[m + 1] = rl.pe[m];
          --m;
        }
        rl.pp[m + 1] = kp;
        rl.pe[m + 1] = ke;
      }
    }
  } else {
    for (int p = tid; p < s; p += kWT) { rl.bnd[2 * p] = d.rp[N[p]]; rl.bnd[2 * p + 1] = d.rp[N[p] + 1]; }
  }
  __syncthreads();
  const int itmax = bf16 ? kRefineMaxBf16 : kRefineMax;
  for (int it = 1; it <= itmax; ++it) {
    // r = f - K z with the FP64 entries of A, summed in ascending p
    for (int q = tid; q < s; q += kWT) {
      double acc = f[q];
      if (lists) {
        const int k1 = off[q + 1];
        for (int k = off[q]; k < k1; ++k) acc = fma(-d.va[rl.pe[k]], z[rl.pp[k]], acc);
      } else {
        const int col = N[q];
        for (int p = 0; p < s; ++p) {
          int lo = rl.bnd[2 * p];
          const int e1 = rl.bnd[2 * p + 1];
          int hi = e1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (d.ci[mid] < col) lo = mid + 1; else hi = mid;
          }
          if (lo < e1 && d.ci[lo] == col) acc = fma(-d.va[lo], z[p], acc);
        }
      }
      r[q] = acc;
    }
    __syncthreads();
    if (it > 1) {
      double rn = 0.0, zn = 0.0;
      for (int t = tid; t < s; t += kWT) { rn = fmax(rn, fabs(r[t])); zn = fmax(zn, fabs(z[t])); }
      rn = block_maxd(rn, shv);
      zn = block_maxd(zn, shv);
      if (rn <= 0x1p-47 * (knorm * zn + fnorm)) {
        *it_out = it;
        bool finite = true;
        for (int t = 0; t < s; ++t) finite &= (z[t] == z[t]);
        return finite;
      }
    }
    for (int t = tid; t < S; t += kWT) y[t] = (t < s) ? (float)(r[t] * scale) : 0.f;
    __syncthreads();
    mf_lu_solve(K, lda, S, y);
    for (int t = tid; t < s; t += kWT) z[t] += (double)y[t];
    __syncthreads();
  }
  return false;
}

__global__ __launch_bounds__(kWT) void k_rows_wg(Work w) {
  __shared__ WideBuf bb;
  // the FP64 block of the pivoting solver and the FP32 block of the mixed
  // solver share this buffer (one row at a time)
  constexpr int kBlkBytes = (int)std::max(sizeof(double) * kLdsBlockMax * (kLdsBlockMax + 1),
                                          sizeof(float) * kMfmaMax * (kMfmaMax + 1));
  __shared__ __align__(16) char s_blk[kBlkBytes];
  double* sK = reinterpret_cast<double*>(s_blk);
  float* sK32 = reinterpret_cast<float*>(s_blk);
  __shared__ double sf[kMaxBlock];
  __shared__ double s_z[kMfmaMax], s_r[kMfmaMax];
  __shared__ float s_y[kMfmaMax];
  __shared__ double shv[kWT];
  __shared__ int shi[kWT];
  __shared__ int s_bad, s_mflag;

  const int tid = threadIdx.x;
  const int qlen = min(w.cnt->nC, w.capC);
  // FP64 rows solved by this workgroup, per run of rows of one matrix
  int run_m = -1, run_n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    // pass 0: blocks that fit in LDS, all workgroups; pass 1: larger blocks,
    // one global scratch slot per workgroup
    if (pass == 1 && (int64_t)blockIdx.x >= w.scratch_slots) {
      if (w.scratch_slots == 0) {
        // no scratch: report oversized rows instead of solving them
        for (int qi = blockIdx.x; qi < qlen; qi += gridDim.x) {
          const int e = w.binC[qi];
          const int c = e / w.chunk;
          const RowInfo ri = row_info(w, c, e - c * w.chunk);
          if (ri.s > kLdsBlockMax && tid == 0) flag_row(&w.st[ri.m], ST_UNSUPPORTED, ri.i);
        }
      }
      continue;
    }
    const int stride = (pass == 0) ? gridDim.x : (int)min<int64_t>(gridDim.x, w.scratch_slots);
    for (int qi = blockIdx.x; qi < qlen; qi += stride) {
      const int e = w.binC[qi];
      const int c = e / w.chunk;
      const RowInfo ri = row_info(w, c, e - c * w.chunk);
      const bool big = ri.s > kLdsBlockMax;
      if (big != (pass == 1)) continue;
      MatStatus* st = &w.st[ri.m];
      if (!matrix_live(*st)) continue;
      const GDesc d = gview(w.desc[ri.m]);
      const int i = ri.i;
      if (tid == 0) d.Rrp[ri.r] = ri.off;
      int* N;
      const int s = block_bfs(d.n, i, d.ell, d.grp, d.gci, d.gva, d.cf, d.theta, d.cmax, d.agg_rp, d.agg_list, bb,
                              &N, d.literal != 0);
      __syncthreads();
      if (s != ri.s) {
        if (tid == 0) flag_row(st, s < 0 ? ST_UNSUPPORTED : ST_INVALID, i);
        __syncthreads();
        continue;
      }
      // blocks above 32 points: the mixed solver first
      int itm = 0;
      bool mixed_ok = false;
      if (s > 32 && s <= kMfmaMax) {
        static_assert(kWN >= kMfmaMax + 1 && kWN + 1 >= 2 * kMfmaMax, "the residual's lists fit the search's buffers");
        const ResidLists rl{bb.fr, bb.nl, bb.cand, bb.kb, bb.dp, kWC};
        mixed_ok = mixed_big_row(d, i, N, s, sK32, sf, s_z, s_r, s_y, shv, &s_mflag, &itm, rl, w.bf16 != 0);
        if (!mixed_ok && w.bf16) {
          // the BF16-update factorisation did not converge: FP32 updates next
          if (tid == 0) atomicAdd(&st->n_retry, 1);
          mixed_ok = mixed_big_row(d, i, N, s, sK32, sf, s_z, s_r, s_y, shv, &s_mflag, &itm, rl, false);
        }
      }
      if (mixed_ok) {
        for (int t = tid; t < s; t += kWT) sf[t] = s_z[t];
        if (tid == 0 && itm > __hip_atomic_load(&st->refine_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          atomicMax(&st->refine_max, itm);
        __syncthreads();
      } else {
      if (big && (int64_t)s * s > w.scratch_stride) {
        // the scratch was sized for smaller blocks (an asynchronous call
        // after a smaller batch): report the row instead of solving it
        if (tid == 0) flag_row(st, ST_UNSUPPORTED, i);
        __syncthreads();
        continue;
      }
      const int ld = big ? s : (kLdsBlockMax + 1);
      double* K = big ? (w.scratch + (int64_t)blockIdx.x * w.scratch_stride) : sK;
      for (int t = tid; t < s * ld; t += kWT) K[t] = 0.0;
      for (int t = tid; t < s; t += kWT) sf[t] = 0.0;
      __syncthreads();
      // K[q][p] = a_{N_p, N_q}: thread p walks row N_p
      for (int p = tid; p < s; p += kWT) {
        const int u = N[p];
        const int e1 = d.rp[u + 1];
        for (int ee = d.rp[u]; ee < e1; ++ee) {
          const int q = find_sorted(N, s, d.ci[ee]);
          if (q >= 0) K[(int64_t)q * ld + p] = d.va[ee];
        }
      }
      for (int ee = d.rp[i] + tid; ee < d.rp[i + 1]; ee += kWT) {
        const int q = find_sorted(N, s, d.ci[ee]);
        if (q >= 0) sf[q] = -d.va[ee];
      }
      __syncthreads();
      // max |K| for the singularity threshold
      double amax = 0.0;
      for (int t = tid; t < s * s; t += kWT) amax = fmax(amax, fabs(K[(int64_t)(t / s) * ld + (t % s)]));
      int dummy;
      block_argmax(amax, 0, shv, shi, &amax, &dummy);
      const double tiny = 1e-14 * amax;
      if (tid == 0) s_bad = 0;
      __syncthreads();
      for (int k = 0; k < s; ++k) {
        double best = -1.0;
        int bi = k;
        for (int q = k + tid; q < s; q += kWT) {
          const double v = fabs(K[(int64_t)q * ld + k]);
          if (v > best) { best = v; bi = q; }
        }
        int p;
        block_argmax(best, bi, shv, shi, &best, &p);
        if (!(best > tiny)) { if (tid == 0) s_bad = 1; __syncthreads(); break; }
        if (p != k) {
          for (int cc = tid; cc < s; cc += kWT) {
            const double t0 = K[(int64_t)k * ld + cc];
            K[(int64_t)k * ld + cc] = K[(int64_t)p * ld + cc];
            K[(int64_t)p * ld + cc] = t0;
          }
          if (tid == 0) { const double t0 = sf[k]; sf[k] = sf[p]; sf[p] = t0; }
          __syncthreads();
        }
        const double piv = K[(int64_t)k * ld + k];
        const int rem = s - k - 1;
        for (int t = tid; t < rem * (rem + 1); t += kWT) {
          const int q = k + 1 + t / (rem + 1);
          const int cc = k + t % (rem + 1);  // cc == k handles the right-hand side
          const double l = K[(int64_t)q * ld + k] / piv;
          if (cc == k) sf[q] -= l * sf[k];
          else K[(int64_t)q * ld + cc] -= l * K[(int64_t)k * ld + cc];
        }
        __syncthreads();
      }
      if (s_bad) {
        if (tid == 0) flag_row(st, ST_SINGULAR, i);
        for (int t = tid; t < s; t += kWT) sf[t] = 0.0;
        __syncthreads();
      } else {
        for (int k = s - 1; k >= 0; --k) {
          if (tid == 0) sf[k] /= K[(int64_t)k * ld + k];
          __syncthreads();
          for (int q = tid; q < k; q += kWT) sf[q] -= K[(int64_t)q * ld + k] * sf[k];
          __syncthreads();
        }
      }
      if (tid == 0) {
        if (ri.m != run_m) {
          if (run_n) atomicAdd(&w.st[run_m].n_fp64, run_n);
          run_m = ri.m;
          run_n = 0;
        }
        ++run_n;
      }
      }  // FP64 solver
      // R row
      int dpos = 0;
      {
        int cntb = 0;
        for (int p = tid; p < s; p += kWT) cntb += N[p] < i;
        shi[tid] = cntb;
        __syncthreads();
        for (int o = kWT / 2; o > 0; o >>= 1) { if (tid < o) shi[tid] += shi[tid + o]; __syncthreads(); }
        dpos = shi[0];
        __syncthreads();
      }
      for (int p = tid; p < s; p += kWT) put_f_entry(w, d, ri.fine0, ri.off + p + (p >= dpos ? 1 : 0), N[p], i, sf[p]);
      if (tid == 0) {
        d.Rci[ri.off + dpos] = i;
        d.Rva[ri.off + dpos] = 1.0;
      }
      __syncthreads();
    }
  }
  if (tid == 0 && run_n) atomicAdd(&w.st[run_m].n_fp64, run_n);
}

// ---------------------------------------------------------------------------
// projection
// ---------------------------------------------------------------------------
// LPR = 1: one thread per row (short rows: a wavefront covers 64
// consecutive rows, a contiguous run of R).  LPR = 8: eight lanes per row,
// entry by entry (long rows).  Workgroups [0, nproj) project (nproj a
// multiple of 8); the rest count the uncovered F-points at the same time.
// Constraint projection, one workgroup per chunk of fine points, one thread
// per F-point j (the survey's exchange step: Algorithm 1's projection applied
// per F-column, QQ^T being diagonal): the entries of column j are those
// linked into its list by the solvers; the thread orders them by R position
// (ascending row, so the sums are the same on every run), forms
// d_j = sum B_i^2 and r_j = sum z_ij B_i - B_j in that order and sets
// z_ij -= B_i r_j / d_j.  A column with d_j = 0 is left alone and counted as
// uncovered.  Lists of up to kPL entries are ordered in registers; a longer
// list is taken kPL entries at a time, each pass keeping the smallest
// positions above the last one summed.
constexpr int kPL = 4;

struct ColEntry {
  int e[kPL];     // batch-wide R entry, INT32_MAX when empty
  int ci[kPL];    // the row's C-point
  double z[kPL];  // the entry's value before the projection
  int n;

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int k = 0; k < kPL; ++k) { e[k] = INT32_MAX; ci[k] = 0; z[k] = 0.0; }
    n = 0;
  }
  // keep the kPL smallest positions (sorted); returns false when an entry
  // had to be dropped
  __device__ __forceinline__ bool insert(int ee, int ii, double zz) {
    int pos = 0;
#pragma unroll
    for (int k = 0; k < kPL; ++k) pos += (e[k] < ee) ? 1 : 0;
    const bool full = n == kPL;
    if (pos >= kPL) return false;
#pragma unroll
    for (int k = kPL - 1; k > 0; --k)
      if (k > pos) { e[k] = e[k - 1]; ci[k] = ci[k - 1]; z[k] = z[k - 1]; }
#pragma unroll
    for (int k = 0; k < kPL; ++k)
      if (k == pos) { e[k] = ee; ci[k] = ii; z[k] = zz; }
    n = full ? kPL : n + 1;
    return !full;
  }
};

// One F-column of any length (the general path of k_colproj): returns true
// when the column is uncovered (d_j = 0)
__device__ bool project_column(const Work& w, const GDesc& d, int64_t nzb, int j, int head) {
  // A list holds at most one record per row, so a walk of more than n steps
  // means a record linked twice (a cycle): the column is then left as
  // written and counted as uncovered rather than walked for ever.
  // first pass: the kPL smallest positions of the list
  ColEntry L;
  L.clear();
  bool more = false;
  int steps = 0;
  for (int e = head; e >= 0;) {
    const int2 lk = w.clink[e];
    const double zv = d.Rva[e - nzb];
    more |= !L.insert(e, lk.y, zv);
    e = lk.x;
    if (++steps > d.n) return true;
  }
  double dsum = 0.0, rsum = 0.0;
#pragma unroll
  for (int k = 0; k < kPL; ++k) {
    if (k < L.n) {
      const double bi = d.B[L.ci[k]];
      dsum = fma(bi, bi, dsum);
      rsum = fma(L.z[k], bi, rsum);
    }
  }
  // longer lists: further passes, each over the positions above the last
  // one taken
  int last = L.e[kPL - 1];
  while (more) {
    ColEntry M;
    M.clear();
    more = false;
    for (int e = head; e >= 0;) {
      const int2 lk = w.clink[e];
      if (e > last) more |= !M.insert(e, lk.y, d.Rva[e - nzb]);
      e = lk.x;
    }  // (the first walk ended, so this one does)
#pragma unroll
    for (int k = 0; k < kPL; ++k) {
      if (k < M.n) {
        const double bi = d.B[M.ci[k]];
        dsum = fma(bi, bi, dsum);
        rsum = fma(M.z[k], bi, rsum);
      }
    }
    last = M.e[kPL - 1];
  }
  if (!(dsum > 0.0)) return true;
  const double q = (rsum - d.B[j]) / dsum;
  if (L.n < kPL || L.e[kPL - 1] == last) {
    // the whole list is in registers
#pragma unroll
    for (int k = 0; k < kPL; ++k)
      if (k < L.n) d.Rva[L.e[k] - nzb] = L.z[k] - d.B[L.ci[k]] * q;
  } else {
    for (int e = head; e >= 0;) {  // the walk ended above, so no cycle here
      const int2 lk = w.clink[e];
      d.Rva[e - nzb] -= d.B[lk.y] * q;
      e = lk.x;
    }
  }
  return false;
}

// Constraint projection kernel: IC F-points per thread walked together (their
// list loads in flight at once), each list of up to kPI records in
// registers; a longer list takes the general path.
constexpr int kIC = 4, kPI = 4;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_colproj(Work w) {
  __shared__ int s_unc;
  // chunks newest first: the numeric kernels walked each XCD's rows in
  // ascending order, so the last chunks' records and values are the ones
  // most likely still in the caches
  const int c = xcd_logical_block_reversed();
  const int tid = threadIdx.x;
  const int m = w.chunk_mat[c];
  const GDesc d = gview(w.desc[m]);
  if (!d.B || !matrix_live(w.st[m])) return;
  const int64_t nzb = d.link_base;  // list entry of R position p: nzb + p
  const int f0 = (c - d.chunk0) * w.chunk;
  const int f1 = min(f0 + w.chunk, d.n);
  if (tid == 0) s_unc = 0;
  __syncthreads();
  int unc = 0;
  for (int jb = f0 + tid; jb < f1; jb += blockDim.x * kIC) {
    int j[kIC], e[kIC], head[kIC], n[kIC];
    int re[kIC][kPI], ri[kIC][kPI];
    double rz[kIC][kPI];
#pragma unroll
    for (int q = 0; q < kIC; ++q) {
      j[q] = jb + q * (int)blockDim.x;
      head[q] = -1;
      n[q] = 0;
      if (j[q] < f1) {
        const int8_t cj = d.cf[j[q]];
        const int h = w.chead[d.fine0 + j[q]];
        if (cj == 0) {
          head[q] = h;
          if (h < 0) ++unc;
        }
      }
      e[q] = head[q];
    }
    // walk the lists together, kPI steps
#pragma unroll
    for (int k = 0; k < kPI; ++k) {
#pragma unroll
      for (int q = 0; q < kIC; ++q) {
        re[q][k] = INT32_MAX;
        ri[q][k] = 0;
        rz[q][k] = 0.0;
        if (e[q] >= 0) {
          const int2 lk = w.clink[e[q]];
          re[q][k] = e[q];
          ri[q][k] = lk.y;
          rz[q][k] = d.Rva[e[q] - nzb];
          e[q] = lk.x;
          ++n[q];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kIC; ++q) {
      if (head[q] < 0) continue;
      if (e[q] >= 0) {  // more than kPI records
        unc += project_column(w, d, nzb, j[q], head[q]) ? 1 : 0;
        continue;
      }
      // order the records by R position (a sorting network on kPI = 4)
#define CLAIR_CS(A, B)                                                   \
  if (re[q][B] < re[q][A]) {                                            \
    const int te = re[q][A]; re[q][A] = re[q][B]; re[q][B] = te;         \
    const int ti = ri[q][A]; ri[q][A] = ri[q][B]; ri[q][B] = ti;         \
    const double tz = rz[q][A]; rz[q][A] = rz[q][B]; rz[q][B] = tz;      \
  }
      CLAIR_CS(0, 1) CLAIR_CS(2, 3) CLAIR_CS(0, 2) CLAIR_CS(1, 3) CLAIR_CS(1, 2)
#undef CLAIR_CS
      double bi[kPI];
#pragma unroll
      for (int k = 0; k < kPI; ++k) bi[k] = (k < n[q]) ? d.B[ri[q][k]] : 0.0;
      const double bj = d.B[j[q]];
      double dsum = 0.0, rsum = 0.0;
#pragma unroll
      for (int k = 0; k < kPI; ++k) {
        if (k < n[q]) {
          dsum = fma(bi[k], bi[k], dsum);
          rsum = fma(rz[q][k], bi[k], rsum);
        }
      }
      if (!(dsum > 0.0)) { ++unc; continue; }
      const double qq = (rsum - bj) / dsum;
#pragma unroll
      for (int k = 0; k < kPI; ++k)
        if (k < n[q]) d.Rva[re[q][k] - nzb] = rz[q][k] - bi[k] * qq;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) unc += __shfl_xor(unc, o, 64);
  if ((tid & 63) == 0 && unc) atomicAdd(&s_unc, unc);
  __syncthreads();
  if (tid == 0 && s_unc) atomicAdd((unsigned long long*)&w.st[m].n_uncovered, (unsigned long long)s_unc);
}

// a numeric pass without the symbolic pass before it: projection sums of all
// fine points to zero, and R.row_ptr[n_c] of every matrix
// Column maxima for the strength test: cmax[v] = max over w != v of |a_wv|,
// for every matrix of the batch (batch-wide fine numbering).  Non-negative
// doubles order like their bit patterns, so an unsigned 64-bit atomic max
// takes the maximum.
__global__ void k_colmax_clear(Work w, int64_t n_total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total; g += (int64_t)gridDim.x * blockDim.x)
    w.cmax[g] = 0.0;
}

__global__ void k_colmax(Work w, int64_t n_total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total; g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = w.nmat - 1;  // the matrix holding fine point g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (w.desc[mid].fine0 <= g) lo = mid; else hi = mid - 1;
    }
    const GDesc d = gview(w.desc[lo]);
    if (d.theta == 0.0 || !matrix_live(w.st[lo])) continue;
    const int u = (int)(g - d.fine0);
    for (int e = d.grp[u]; e < d.grp[u + 1]; ++e) {  // column maxima of the search graph
      const int v = d.gci[e];
      if (v == u || (unsigned)v >= (unsigned)d.n) continue;
      atomicMax(reinterpret_cast<unsigned long long*>(w.cmax + d.fine0 + v),
                (unsigned long long)__double_as_longlong(fabs(d.gva[e])));
    }
  }
}

// Member lists of the aggregates (matrices given with aggregates only):
// count per root, scan (host), scatter through cursors, sort per root.  An
// F-point j joins root r = agg[j] when r is a C-point index in range.
__device__ __forceinline__ int fine_matrix(const Work& w, int64_t g) {
  int lo = 0, hi = w.nmat - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w.desc[mid].fine0 <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int agg_root(const GDesc& d, int j) {
  if (!d.agg || d.cf[j] != 0) return -1;
  const int r = d.agg[j];
  return ((unsigned)r < (unsigned)d.n && d.cf[r] != 0) ? r : -1;
}

__global__ void k_agg_count(Work w, int64_t n_total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total; g += (int64_t)gridDim.x * blockDim.x) {
    const int m = fine_matrix(w, g);
    const GDesc d = gview(w.desc[m]);
    const int r = agg_root(d, (int)(g - d.fine0));
    if (r >= 0) atomicAdd(&w.agg_cnt[d.fine0 + r], 1);
  }
}

__global__ void k_agg_fill(Work w, int64_t n_total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total; g += (int64_t)gridDim.x * blockDim.x) {
    const int m = fine_matrix(w, g);
    const GDesc d = gview(w.desc[m]);
    const int j = (int)(g - d.fine0);
    const int r = agg_root(d, j);
    if (r >= 0) w.agg_list[w.agg_rp[d.fine0 + r] + atomicAdd(&w.agg_cnt[d.fine0 + r], 1)] = j;
  }
}

__global__ void k_agg_sort(Work w, int64_t n_total) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_total; g += (int64_t)gridDim.x * blockDim.x) {
    const int e0 = w.agg_rp[g], e1 = w.agg_rp[g + 1];
    for (int a = e0 + 1; a < e1; ++a) {
      const int k = w.agg_list[a];
      int b = a - 1;
      while (b >= e0 && w.agg_list[b] > k) {
        w.agg_list[b + 1] = w.agg_list[b];
        --b;
      }
      w.agg_list[b + 1] = k;
    }
  }
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) a[g] = v;
}

__global__ void k_clear_sums(Work w, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    w.chead[j] = -1;
  if (blockIdx.x == 0) {
    for (int m = threadIdx.x; m < w.nmat; m += blockDim.x) {
      const MatStatus& st = w.st[m];
      if (matrix_live(st) && w.desc[m].Rrp) w.desc[m].Rrp[st.n_c] = (int32_t)st.nnz;
    }
  }
}

}  // namespace

// a kernel, not a memset: the call may be captured into a graph
hipError_t launch_clear_sums(const Work& w, int64_t n_total, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_sums, dim3(blocks), dim3(256), 0, s, w, n_total);
  return hipGetLastError();
}

hipError_t launch_colmax(const Work& w, int64_t n_total, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_colmax_clear, dim3(blocks), dim3(256), 0, s, w, n_total);
  hipLaunchKernelGGL(k_colmax, dim3(blocks), dim3(256), 0, s, w, n_total);
  return hipGetLastError();
}

hipError_t launch_agg_lists(const Work& w, int64_t n_total, int blocks, int cus, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, w.agg_cnt, n_total, 0);
  hipLaunchKernelGGL(k_agg_count, dim3(blocks), dim3(256), 0, s, w, n_total);
  hipError_t e = launch_exclusive_scan(w.agg_cnt, (int)n_total, w.agg_rp, w.agg_sums, cus, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, w.agg_cnt, n_total, 0);
  hipLaunchKernelGGL(k_agg_fill, dim3(blocks), dim3(256), 0, s, w, n_total);
  hipLaunchKernelGGL(k_agg_sort, dim3(blocks), dim3(256), 0, s, w, n_total);
  return hipGetLastError();
}

hipError_t launch_validate(const Work& w, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_adj(const Work& w, hipStream_t s) {
  if (w.nchunks == 0 || w.adj_w == 0) return hipSuccess;
  const int per = (w.chunk + 256 * kAdjPP - 1) / (256 * kAdjPP);
  const dim3 grid((unsigned)w.nchunks * (unsigned)per);
  if (w.adj_w == 4) hipLaunchKernelGGL(k_adj<4>, grid, dim3(256), 0, s, w);
  else if (w.adj_w == 8) hipLaunchKernelGGL(k_adj<8>, grid, dim3(256), 0, s, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_count(const Work& w, hipStream_t s) {
  if (w.nchunks == 0) return hipSuccess;
  const dim3 grid(w.nchunks), block(kNT);
  if (w.adj_w == 4) hipLaunchKernelGGL(k_count<4>, grid, block, 0, s, w);
  else if (w.adj_w == 0 || w.adj_w == 8) hipLaunchKernelGGL(k_count<0>, grid, block, 0, s, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_count_mid(const Work& w, int blocks, hipStream_t s) {
  if (w.nchunks == 0) return hipSuccess;
  const dim3 grid(std::min(w.nchunks, std::max(1, blocks))), block(kNT);
  if (w.adj_w == 0) hipLaunchKernelGGL(k_count_mid<0>, grid, block, 0, s, w);
  else if (w.adj_w == 4) hipLaunchKernelGGL(k_count_mid<4>, grid, block, 0, s, w);
  else if (w.adj_w == 8) hipLaunchKernelGGL(k_count_mid<8>, grid, block, 0, s, w);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_count_big(const Work& w, int blocks, hipStream_t s) {
  if (w.nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_big, dim3(blocks), dim3(kNT), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_scan(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, w);
  return hipGetLastError();
}

// persistent grid: as many workgroups as fit on the device at once.
// which = 0: bin A with `group` lanes per row; which = 1: bin B with blocks of
// up to sm points (16: 16 lanes per row; 18, 20, 24 or 32: 32 lanes per row).
hipError_t launch_numeric(const Work& w, int which, int group, int sm, int wg_threads, int cus, hipStream_t s) {
#define CLAIR_NUM(GG, NTT, SMM)                                                                         \
  if (group == GG && wg_threads == NTT && sm == SMM) {                                                  \
    int per = 0;                                                                                        \
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_numeric<GG, NTT, SMM>, NTT, 0); \
    if (e != hipSuccess) return e;                                                                      \
    const int blocks = (std::max(1, per) * cus + 7) / 8 * 8;                                           \
    hipLaunchKernelGGL((k_numeric<GG, NTT, SMM>), dim3(blocks), dim3(NTT), 0, s, w, which);             \
    return hipGetLastError();                                                                           \
  }
  CLAIR_NUM(8, 256, 8)
  CLAIR_NUM(8, 128, 8)
  CLAIR_NUM(8, 64, 8)
  CLAIR_NUM(16, 256, 16)
  CLAIR_NUM(16, 128, 16)
  CLAIR_NUM(16, 64, 16)
  CLAIR_NUM(32, 256, 32)
  CLAIR_NUM(32, 128, 32)
  CLAIR_NUM(32, 64, 32)
  CLAIR_NUM(32, 128, 18)
  CLAIR_NUM(32, 128, 20)
  CLAIR_NUM(32, 128, 24)
#undef CLAIR_NUM
  return hipErrorInvalidValue;
}

// G lanes per row, R block rows per lane, blocks of up to SM points, one
// wavefront per workgroup; persistent grid as for k_numeric
hipError_t launch_lanes(const Work& w, int which, int group, int rows_per_lane, int sm, int wg_threads, int cus,
                        hipStream_t s) {
#define CLAIR_LR(GG, RR, SMM, NTT)                                                                          \
  if (group == GG && rows_per_lane == RR && sm == SMM && wg_threads == NTT) {                               \
    int per = 0;                                                                                            \
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_lanes<GG, RR, SMM, NTT>, NTT, 0);   \
    if (e != hipSuccess) return e;                                                                          \
    const int blocks = (std::max(1, per) * cus + 7) / 8 * 8;                                               \
    hipLaunchKernelGGL((k_lanes<GG, RR, SMM, NTT>), dim3(blocks), dim3(NTT), 0, s, w, which);               \
    return hipGetLastError();                                                                               \
  }
  CLAIR_LR(8, 2, 16, 64)
  CLAIR_LR(8, 3, 20, 64)
  CLAIR_LR(8, 3, 24, 64)
  CLAIR_LR(16, 1, 16, 64)
  CLAIR_LR(16, 2, 20, 64)
  CLAIR_LR(16, 2, 24, 64)
  CLAIR_LR(16, 2, 32, 64)
  CLAIR_LR(32, 1, 20, 64)
  CLAIR_LR(32, 1, 24, 64)
  CLAIR_LR(32, 1, 32, 64)
  CLAIR_LR(4, 2, 8, 64)
  CLAIR_LR(4, 2, 8, 128)
  CLAIR_LR(2, 4, 8, 64)
  CLAIR_LR(2, 4, 8, 128)
#undef CLAIR_LR
  return hipErrorInvalidValue;
}

hipError_t launch_rows8(const Work& w, int wg_threads, int cus, hipStream_t s) {
#define CLAIR_R8(NTT)                                                                       \
  if (wg_threads == NTT) {                                                                  \
    int per = 0;                                                                            \
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rows8<NTT>, NTT, 0); \
    if (e != hipSuccess) return e;                                                          \
    const int blocks = (std::max(1, per) * cus + 7) / 8 * 8;                               \
    hipLaunchKernelGGL((k_rows8<NTT>), dim3(blocks), dim3(NTT), 0, s, w);                   \
    return hipGetLastError();                                                               \
  }
  CLAIR_R8(256)
  CLAIR_R8(128)
  CLAIR_R8(64)
#undef CLAIR_R8
  return hipErrorInvalidValue;
}

hipError_t launch_quad8(const Work& w, int wg_threads, int cus, hipStream_t s) {
#define CLAIR_Q8(NTT)                                                                       \
  if (wg_threads == NTT) {                                                                  \
    int per = 0;                                                                            \
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_quad8<NTT>, NTT, 0); \
    if (e != hipSuccess) return e;                                                          \
    const int blocks = (std::max(1, per) * cus + 7) / 8 * 8;                               \
    hipLaunchKernelGGL((k_quad8<NTT>), dim3(blocks), dim3(NTT), 0, s, w);                   \
    return hipGetLastError();                                                               \
  }
  CLAIR_Q8(256)
  CLAIR_Q8(128)
  CLAIR_Q8(64)
#undef CLAIR_Q8
  return hipErrorInvalidValue;
}

hipError_t launch_rows_wg(const Work& w, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_wg, dim3(blocks), dim3(kWT), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_project(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_colproj, dim3(w.nchunks), dim3(256), 0, s, w);
  return hipGetLastError();
}

}  // namespace clair
