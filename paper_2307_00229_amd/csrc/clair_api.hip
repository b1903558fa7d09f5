// clair_api.hip -- the C ABI of libclair (declared in include/clair.h).
//
// Host side only: argument checks, the per-context device workspace, the
// descriptor upload, kernel sequencing, status read-back, per-stage timing,
// the autotuner and hipGraph capture.  Every arithmetic step of the setup runs
// in the kernels of k_mixed.hip / k_plain.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "clair.h"
#include "clair_device.h"
#include "clair_launch.h"

using namespace clair;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t size = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    size = 0;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= size) return hipSuccess;
    release();
    size_t want = std::max<size_t>(bytes, 4096);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    size = want;
    return hipSuccess;
  }
};

struct HostPinned {
  void* p = nullptr;
  size_t size = 0;
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    size = 0;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= size) return hipSuccess;
    release();
    size_t want = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    size = want;
    return hipSuccess;
  }
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t desc, st, cnt, chunk_nc, chunk_nnz, chunk_rbase, chunk_nzbase, chunk_mat, chunk_bins, row_block_chunk, clocal, lnz, chead,
      slotA, slotB, binC, bigq, big_size, ovf, cmax, agg_cnt, agg_rp, agg_list, agg_sums, fadj, midq, total;
  size_t head_bytes;  // desc + st + counters (the uploaded head)
  int64_t capC;
};

Layout make_layout(int nmat, int nchunks, int64_t n_total, int GA, bool any_agg, int adj_w) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.desc = take(sizeof(MatDesc) * nmat);
  L.st = o;
  o += sizeof(MatStatus) * nmat;
  L.cnt = o;
  o += sizeof(Counters);
  L.head_bytes = o - L.desc;
  o = align_up(o, 256);
  L.capC = n_total + 1;
  L.chunk_nc = take(sizeof(int32_t) * (nchunks + 1));
  L.chunk_nnz = take(sizeof(int32_t) * (nchunks + 1));
  L.chunk_rbase = take(sizeof(int32_t) * (nchunks + 2));
  L.chunk_nzbase = take(sizeof(int64_t) * (nchunks + 1));
  L.chunk_mat = take(sizeof(int32_t) * (nchunks + 1));
  L.chunk_bins = take(sizeof(int2) * (nchunks + 1));
  L.row_block_chunk = take(sizeof(int32_t) * (n_total / 256 + 2));
  L.clocal = take(sizeof(int32_t) * (n_total + 1));
  L.lnz = take(sizeof(int32_t) * (n_total + 1));
  L.chead = take(sizeof(int32_t) * (n_total + 1));
  const int SA = GA <= 4 ? 8 : GA;  // slot stride of bin A
  L.slotA = take(sizeof(int32_t) * (SA ? (n_total + 1) * SA : 1));
  L.slotB = take(sizeof(int32_t) * (n_total + 1) * (GA < 32 ? 32 : 1));
  L.binC = take(sizeof(int32_t) * L.capC);
  L.bigq = take(sizeof(int32_t) * L.capC);
  L.big_size = take(sizeof(int32_t) * (n_total + 1));
  L.ovf = take(sizeof(int32_t) * (nchunks + 1));
  L.cmax = take(sizeof(double) * (n_total + 1));
  const int64_t na = any_agg ? n_total : 0;
  L.agg_cnt = take(sizeof(int32_t) * (na + 1));
  L.agg_rp = take(sizeof(int32_t) * (na + 2));
  L.agg_list = take(sizeof(int32_t) * (na + 1));
  L.agg_sums = take(sizeof(int32_t) * (na / 1024 + 4));
  L.fadj = take(sizeof(int32_t) * (adj_w ? n_total * adj_w : 1));
  L.midq = take(sizeof(int32_t) * (nchunks + 1));
  L.total = o;
  return L;
}

constexpr int kMaxStages = 16;
constexpr int kNoAllocDevices = 64;      // devices the fixed-memory entry point serves
constexpr int kNoAllocHostBytes = 8192;  // its host staging per device (descriptor upload + status read-back)

struct StageEvents {
  hipEvent_t ev[kMaxStages + 1];
  const char* name[kMaxStages];
  int n = 0;
};

}  // namespace

struct clair_ctx {
  int device = 0;
  int cus = 256;
  // tuning
  int group = 8;  // lanes per row of the small solver: 1, 4 or 8 (|N| <= 8), 16/32 (|N| <= group)
  double theta = 0.0;  // strength threshold of the neighbourhood search
  int adj_mode = -1;   // the search's compact adjacency: -1 automatic width, 0 off, 4 or 8 forced width
  std::vector<clair_csr_t> graph;  // strength matrices of the search, one per matrix (empty: A's graph)
  int literal = 0;  // the literal S^{ell-1} T pattern (both forms; the same pattern as the default at ell <= 2)
  int binB_max = 32;  // largest block of the last batch whose sizes were read back (9..32)
  int binB_lanes = 32;  // lanes per row of the bin-B solver (8, 16 or 32)
  int tune_timed = 0;   // timing runs of the last clair_autotune (0: the cache held the histogram)
  int last_maxb = 0;  // the same, unclamped (0: none read back yet)
  int wg_threads = 256;
  int chunk = 1024;
  // memory
  DevBuf ws;
  // fixed memory (clair_build_R_noalloc): the workspace and the column lists
  // in the library's static device array, host staging in a static host
  // array; nothing is allocated or grown
  bool fixed = false;
  char* fixed_dev = nullptr;
  size_t fixed_dev_bytes = 0;
  char* fixed_host = nullptr;
  size_t fixed_host_bytes = 0;
  DevBuf links;    // the projection's column lists: one int2 per R entry of a batch
  int64_t link_cap = 0;
  DevBuf scratch;  // FP64 blocks of oversized rows
  int64_t scratch_slots = 0;
  int64_t scratch_stride = 0;  // doubles per slot (the largest block sized for, squared)
  HostPinned stage;     // descriptor/status upload
  HostPinned readback;  // status download
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  bool capturing = false;  // inside hipStreamBeginCapture: no event records
  // last call
  int last_nmat = 0;
  hipStream_t last_stream = nullptr;
  Layout last_layout{};
  Work last_work{};
  bool last_plain = false;
  std::vector<clair_info_t> plain_info;  // results of the last plain-form call
  std::vector<int64_t> plain_nnz;
  // timing
  std::vector<StageEvents> timing;
  size_t timing_used = 0;
  // plain-form scratch
  DevBuf plain_ws;
  DevBuf plain_k;
  // transpose and P-side buffers: A^T, the restriction built on it, scratch
  DevBuf t_rp, t_ci, t_va, q_rp, q_ci, q_va, t_scratch;
  // sparse products: row pointers of a product, the intermediate A P
  DevBuf g_rp, g_cnt, ap_rp, ap_ci, ap_va;
  // smoothing of B: two vectors and a flag
  DevBuf sm_x, sm_y, sm_flag;
  // k constraint vectors: R^T, the row -> C-point map, lambda, counters
  DevBuf pk_scratch;
  // diagonal block inverse: diagonal, column sums, updates, row of each entry
  DevBuf ap_ws;
  // normal-equations minimiser: blocks, Cholesky factors, CG vectors
  DevBuf kkt_ws;
};

namespace {

std::mutex g_default_mu;
std::vector<clair_ctx*> g_default;  // one per device

thread_local char g_last_error[512] = "";

void set_last_error(const char* what, hipError_t e, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s failed: %s (%d) at clair_api.hip:%d", what,
           hipGetErrorString(e), (int)e, line);
}

// While capturing, name the first operation after which the capture is no
// longer active (the runtime only reports the failure at hipStreamEndCapture).
int capture_check(bool capturing, hipStream_t s, const char* what, int line) {
  if (!capturing) return 0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess || cs != hipStreamCaptureStatusActive) {
    snprintf(g_last_error, sizeof(g_last_error), "stream capture not active after %s (status %d, err %d) at clair_api.hip:%d",
             what, (int)cs, (int)e, line);
    return 1;
  }
  return 0;
}

#define HIPCHK(expr)                                \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) {                         \
      set_last_error(#expr, e_, __LINE__);          \
      return CLAIR_ERR_HIP;                         \
    }                                               \
  } while (0)

// Per-stage events: c->timing[0..timing_used) are the sets recorded since the
// last clair_ctx_stage_times; each set brackets the stages of one call.
int timing_begin(clair_ctx* c, bool on) {
  if (!on) return CLAIR_OK;
  if (c->timing_used == c->timing.size()) {
    StageEvents se;
    for (int k = 0; k <= kMaxStages; ++k) HIPCHK(hipEventCreate(&se.ev[k]));
    c->timing.push_back(se);
  }
  c->timing[c->timing_used].n = 0;
  c->timing_used += 1;
  return CLAIR_OK;
}

void timing_mark(clair_ctx* c, bool on, hipStream_t s, const char* name) {
  if (!on || c->timing_used == 0) return;
  StageEvents& se = c->timing[c->timing_used - 1];
  if (se.n >= kMaxStages) return;
  if (se.n == 0) (void)hipEventRecord(se.ev[0], s);
  se.name[se.n] = name;
  se.n += 1;
  (void)hipEventRecord(se.ev[se.n], s);
}

// ---------------------------------------------------------------------------
// batch preparation
// ---------------------------------------------------------------------------
struct Batch {
  int nmat;
  int nchunks;
  int64_t n_total;
  int64_t cap_sum = 0;  // R capacities summed over the batch (bounds the R entries of an asynchronous call)
  bool any_B;
  bool any_agg = false;
  int adj_w = 0;  // slots per point of the search's compact adjacency (0: not built)
  Layout L;
  Work w;
};

// device workspace, host staging (upload) and host read-back area
char* ws_base(clair_ctx* c) { return c->fixed ? c->fixed_dev : static_cast<char*>(c->ws.p); }
char* stage_base(clair_ctx* c) { return c->fixed ? c->fixed_host : static_cast<char*>(c->stage.p); }
char* readback_base(clair_ctx* c) {
  return c->fixed ? c->fixed_host + c->fixed_host_bytes / 2 : static_cast<char*>(c->readback.p);
}

int check_args(int32_t nmat, const clair_csr_t* A, const int8_t* const* cf, const int32_t* ell,
               clair_csr_out_t* R) {
  if (nmat < 0 || (nmat > 0 && (!A || !cf || !ell || !R))) return CLAIR_ERR_INVALID;
  for (int m = 0; m < nmat; ++m) {
    if (A[m].n < 0 || A[m].nnz < 0 || ell[m] < 1 || ell[m] > 64) return CLAIR_ERR_INVALID;
    if (A[m].n > 0 && (!A[m].row_ptr || !cf[m])) return CLAIR_ERR_INVALID;
    if (A[m].nnz > 0 && (!A[m].col_idx || !A[m].val)) return CLAIR_ERR_INVALID;
    if (R[m].row_capacity < 0 || R[m].nnz_capacity < 0) return CLAIR_ERR_INVALID;
  }
  return CLAIR_OK;
}

int prepare(clair_ctx* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
            const double* const* B, const int32_t* ell, const clair_csr_out_t* R, Batch* b,
            const int32_t* const* agg = nullptr) {
  if (!c->graph.empty()) {  // the context's strength matrices must match the batch
    if ((int32_t)c->graph.size() != nmat) return CLAIR_ERR_INVALID;
    for (int m = 0; m < nmat; ++m)
      if (c->graph[m].n != A[m].n) return CLAIR_ERR_INVALID;
  }
  b->nmat = nmat;
  b->nchunks = 0;
  b->n_total = 0;
  b->any_B = false;
  b->any_agg = false;
  b->cap_sum = 0;
  for (int m = 0; m < nmat; ++m) {
    b->nchunks += (A[m].n + c->chunk - 1) / c->chunk;
    b->n_total += A[m].n;
    b->cap_sum += std::max<int64_t>(0, R[m].nnz_capacity);
    b->any_B |= (B && B[m]);
    b->any_agg |= (agg && agg[m]);
  }
  // the compact adjacency serves the searches of distance 2 and more on
  // sparse graphs: width 4 when every such graph has at most five stored
  // entries per row on average, else 8 (points beyond it are searched from
  // the rows); denser graphs, aggregates and the fixed-memory entry point go
  // without
  std::vector<char> use_adj(nmat, 0);
  b->adj_w = 0;
  if (!c->fixed && c->adj_mode != 0) {
    int w_need = 0;
    for (int m = 0; m < nmat; ++m) {
      const int64_t gnnz = c->graph.empty() ? A[m].nnz : c->graph[m].nnz;
      // (the literal reading from distance 3 on walks through C-points, which
      // the adjacency leaves out)
      if (ell[m] < 2 || A[m].n <= 0 || (agg && agg[m]) || gnnz > 9 * (int64_t)A[m].n ||
          (c->literal && ell[m] >= 3))
        continue;
      use_adj[m] = 1;
      w_need = std::max(w_need, gnnz <= 5 * (int64_t)A[m].n ? 4 : 8);
    }
    b->adj_w = c->adj_mode > 0 ? (w_need ? c->adj_mode : 0) : w_need;
  }
  b->L = make_layout(nmat, b->nchunks, b->n_total, c->group, b->any_agg, b->adj_w);
  if (c->fixed) {
    if (b->L.total > c->fixed_dev_bytes || b->L.head_bytes > c->fixed_host_bytes / 2) {
      snprintf(g_last_error, sizeof(g_last_error),
               "clair_build_R_noalloc: the workspace of %lld fine points needs %zu bytes, above the %zu-byte "
               "static scratch", (long long)b->n_total, b->L.total, c->fixed_dev_bytes);
      return CLAIR_ERR_UNSUPPORTED;
    }
  } else {
    HIPCHK(c->ws.ensure(b->L.total));
    HIPCHK(c->stage.ensure(b->L.head_bytes));
    HIPCHK(c->readback.ensure(b->L.head_bytes));
  }
  // the previous upload must have left the staging buffer before it is rewritten
  if (c->upload_pending) {
    HIPCHK(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  char* base = ws_base(c);
  Work& w = b->w;
  w.desc = reinterpret_cast<MatDesc*>(base + b->L.desc);
  w.st = reinterpret_cast<MatStatus*>(base + b->L.st);
  w.cnt = reinterpret_cast<Counters*>(base + b->L.cnt);
  w.chunk_nc = reinterpret_cast<int32_t*>(base + b->L.chunk_nc);
  w.chunk_nnz = reinterpret_cast<int32_t*>(base + b->L.chunk_nnz);
  w.chunk_rbase = reinterpret_cast<int32_t*>(base + b->L.chunk_rbase);
  w.chunk_nzglob = reinterpret_cast<int64_t*>(base + b->L.chunk_nzbase);
  w.chunk_mat = reinterpret_cast<int32_t*>(base + b->L.chunk_mat);
  w.chunk_bins = reinterpret_cast<int2*>(base + b->L.chunk_bins);
  w.row_block_chunk = reinterpret_cast<int32_t*>(base + b->L.row_block_chunk);
  w.clocal = reinterpret_cast<int32_t*>(base + b->L.clocal);
  w.lnz = reinterpret_cast<int32_t*>(base + b->L.lnz);
  w.chead = reinterpret_cast<int32_t*>(base + b->L.chead);
  w.clink = static_cast<int2*>(c->links.p);
  w.link_cap = c->link_cap;
  w.slotA = reinterpret_cast<int32_t*>(base + b->L.slotA);
  w.slotB = reinterpret_cast<int32_t*>(base + b->L.slotB);
  w.binC = reinterpret_cast<int32_t*>(base + b->L.binC);
  w.chunk_unsized = reinterpret_cast<int32_t*>(base + b->L.ovf);
  w.bigq = reinterpret_cast<int32_t*>(base + b->L.bigq);
  w.big_size = reinterpret_cast<int32_t*>(base + b->L.big_size);
  w.cmax = reinterpret_cast<double*>(base + b->L.cmax);
  w.agg_cnt = reinterpret_cast<int32_t*>(base + b->L.agg_cnt);
  w.agg_rp = reinterpret_cast<int32_t*>(base + b->L.agg_rp);
  w.agg_list = reinterpret_cast<int32_t*>(base + b->L.agg_list);
  w.agg_sums = reinterpret_cast<int32_t*>(base + b->L.agg_sums);
  w.scratch = static_cast<double*>(c->scratch.p);
  w.scratch_slots = c->scratch_slots;
  w.scratch_stride = c->scratch_stride;
  w.nmat = nmat;
  w.nchunks = b->nchunks;
  w.chunk = c->chunk;
  w.GA = c->group;
  w.capC = (int32_t)std::min<int64_t>(b->L.capC, INT32_MAX);
  w.adj_w = b->adj_w;
  w.fadj = reinterpret_cast<int32_t*>(base + b->L.fadj);
  w.bf16 = 0;
  w.pad1 = 0;
  w.midq = reinterpret_cast<int32_t*>(base + b->L.midq);

  char* h = stage_base(c);
  MatDesc* hd = reinterpret_cast<MatDesc*>(h);
  MatStatus* hs = reinterpret_cast<MatStatus*>(h + (b->L.st - b->L.desc));
  Counters* hc = reinterpret_cast<Counters*>(h + (b->L.cnt - b->L.desc));
  int chunk0 = 0;
  int64_t fine0 = 0;
  int64_t link0 = 0;
  for (int m = 0; m < nmat; ++m) {
    MatDesc d{};
    d.link_base = link0;
    link0 += std::max<int64_t>(0, R[m].nnz_capacity);
    d.rp = A[m].row_ptr;
    d.ci = A[m].col_idx;
    d.va = A[m].val;
    d.grp = c->graph.empty() ? A[m].row_ptr : c->graph[m].row_ptr;
    d.gci = c->graph.empty() ? A[m].col_idx : c->graph[m].col_idx;
    d.gva = c->graph.empty() ? A[m].val : c->graph[m].val;
    d.cf = cf[m];
    d.B = B ? B[m] : nullptr;
    d.Rrp = R[m].row_ptr;
    d.Rci = R[m].col_idx;
    d.Rva = R[m].val;
    d.nnz_cap = R[m].nnz_capacity;
    d.row_cap = R[m].row_capacity;
    d.n = A[m].n;
    d.ell = ell[m];
    d.chunk0 = chunk0;
    d.nnz = A[m].nnz;
    d.nchunks = (A[m].n + c->chunk - 1) / c->chunk;
    d.fine0 = fine0;
    d.cmax = w.cmax + fine0;
    d.theta = c->theta;
    d.agg = (agg && agg[m]) ? agg[m] : nullptr;
    d.agg_rp = d.agg ? w.agg_rp + fine0 : nullptr;
    d.agg_list = d.agg ? w.agg_list : nullptr;
    d.fadj = (b->adj_w && use_adj[m]) ? w.fadj + fine0 * b->adj_w : nullptr;
    d.literal = (c->literal && !d.agg) ? 1 : 0;
    d.pad = 0;
    hd[m] = d;
    chunk0 += d.nchunks;
    fine0 += A[m].n;
    MatStatus s{};
    s.first_bad = INT32_MAX;
    hs[m] = s;
  }
  *hc = Counters{};
  return CLAIR_OK;
}

int upload(clair_ctx* c, const Batch& b, hipStream_t s) {
  if (c->fixed) {
    // the calls of the fixed-memory entry point end with a stream
    // synchronisation, so the staging area is free again at the next call
    HIPCHK(hipMemcpyAsync(b.w.desc, stage_base(c), b.L.head_bytes, hipMemcpyHostToDevice, s));
    return CLAIR_OK;
  }
  if (!c->upload_done) HIPCHK(hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming));
  HIPCHK(hipMemcpyAsync(b.w.desc, c->stage.p, b.L.head_bytes, hipMemcpyHostToDevice, s));
  if (capture_check(c->capturing, s, "descriptor upload", __LINE__)) return CLAIR_ERR_HIP;
  if (!c->capturing) {
    HIPCHK(hipEventRecord(c->upload_done, s));
    c->upload_pending = true;
  }
  return CLAIR_OK;
}

int read_status(clair_ctx* c, const Batch& b, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(readback_base(c), b.w.desc, b.L.head_bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return CLAIR_OK;
}

const MatStatus* host_status(clair_ctx* c, const Batch& b) {
  return reinterpret_cast<const MatStatus*>(readback_base(c) + (b.L.st - b.L.desc));
}

int occupancy_blocks(clair_ctx* c, int per_cu) { return std::max(8, c->cus * per_cu); }

// one slot per workgroup of the FP64 solver, each holding a block of the
// largest size read back (rounded up to a multiple of 8 points)
int ensure_scratch(clair_ctx* c, int slots, int maxb) {
  if (c->fixed) return CLAIR_OK;  // no FP64 scratch: the solver reports rows above 64 points
  const int64_t side = std::min<int64_t>(kMaxBlock, ((int64_t)std::max(maxb, 1) + 7) / 8 * 8);
  const int64_t stride = side * side;
  if (c->scratch_slots >= slots && c->scratch_stride >= stride) return CLAIR_OK;
  const int64_t want_slots = std::max<int64_t>(slots, c->scratch_slots);
  const int64_t want_stride = std::max(stride, c->scratch_stride);
  const size_t bytes = (size_t)want_slots * (size_t)want_stride * sizeof(double);
  if (c->scratch.ensure(bytes) != hipSuccess) {
    c->scratch_slots = 0;  // the old buffer is gone too
    c->scratch_stride = 0;
    return CLAIR_ERR_NOMEM;
  }
  c->scratch_slots = want_slots;
  c->scratch_stride = want_stride;
  return CLAIR_OK;
}

// Column lists of the projection: one int2 per R entry the caller's
// capacities allow, numbered through the batch (int32 numbers).
int ensure_links(clair_ctx* c, Batch& b) {
  if (!b.any_B) return CLAIR_OK;
  const int64_t entries = b.cap_sum;
  if (entries > INT32_MAX) return CLAIR_ERR_UNSUPPORTED;
  if (c->fixed) {  // after the workspace in the static scratch
    const size_t at = align_up(b.L.total, 256);
    const int64_t room = at < c->fixed_dev_bytes ? (int64_t)((c->fixed_dev_bytes - at) / sizeof(int2)) : 0;
    if (entries > room) {
      snprintf(g_last_error, sizeof(g_last_error),
               "clair_build_R_noalloc: %lld R entries of capacity need %lld bytes of column lists beyond the "
               "workspace; the %zu-byte static scratch leaves %lld", (long long)entries,
               (long long)(entries * (int64_t)sizeof(int2)), c->fixed_dev_bytes, (long long)(room * sizeof(int2)));
      return CLAIR_ERR_UNSUPPORTED;
    }
    b.w.clink = reinterpret_cast<int2*>(c->fixed_dev + at);
    b.w.link_cap = entries;
    return CLAIR_OK;
  }
  if (c->link_cap < entries) {
    if (c->links.ensure(sizeof(int2) * (size_t)std::max<int64_t>(entries, 1)) != hipSuccess) {
      c->link_cap = 0;
      return CLAIR_ERR_NOMEM;
    }
    c->link_cap = entries;
  }
  b.w.clink = static_cast<int2*>(c->links.p);
  b.w.link_cap = c->link_cap;
  return CLAIR_OK;
}

const Counters* host_counters(clair_ctx* c, const Batch& b) {
  return reinterpret_cast<const Counters*>(readback_base(c) + (b.L.cnt - b.L.desc));
}

// enqueue the numeric half (after the symbolic pass).  `known` holds the queue
// lengths when the host has read them back (synchronous calls): empty queues
// then launch nothing.
int enqueue_numeric(clair_ctx* c, Batch& b, hipStream_t s, bool timing, const Counters* known) {
  b.w.scratch = static_cast<double*>(c->scratch.p);
  b.w.scratch_slots = c->scratch_slots;
  b.w.scratch_stride = c->scratch_stride;
  if (!known || known->nA > 0) {
    if (c->group == 1) {
      HIPCHK(launch_rows8(b.w, c->wg_threads, c->cus, s));
    } else if (c->group == 4) {
      HIPCHK(launch_quad8(b.w, c->wg_threads, c->cus, s));
    } else {
      HIPCHK(launch_numeric(b.w, 0, c->group, c->group, c->wg_threads, c->cus, s));
    }
    if (capture_check(c->capturing, s, "k_numeric", __LINE__)) return CLAIR_ERR_HIP;
  }
  timing_mark(c, timing, s, "numeric");
  if (c->group < 32 && (!known || known->nB > 0)) {
    // bin B: the smallest block bound that holds the largest block seen (rows
    // beyond it go to the workgroup solver, so any bound is correct)
    // block bound 16, 18, 20, 24 or 32 (the smallest that holds the largest
    // block read back).  binB_lanes = 32: one lane per block row (16 lanes at
    // the bound 16); 8 or 16: ceil(bound / lanes) block rows per lane (8
    // lanes at 32 points would need more LDS than a workgroup has: 16 then)
    const int bsm = c->binB_max <= 16 ? 16 : c->binB_max <= 20 ? 20 : c->binB_max <= 24 ? 24 : 32;
    if (c->binB_lanes == 32) {
      // (17 and 18 points, the 128^3 seven-point rows, have a bound of their own)
      const int b32 = (c->binB_max > 16 && c->binB_max <= 18) ? 18 : bsm;
      HIPCHK(launch_numeric(b.w, 1, b32 == 16 ? 16 : 32, b32, 128, c->cus, s));
    } else {
      const int bg = (bsm == 32 && c->binB_lanes == 8) ? 16 : c->binB_lanes;
      const int br = (bsm + bg - 1) / bg;
      HIPCHK(launch_lanes(b.w, 1, bg, br, bsm, 64, c->cus, s));
    }
    if (capture_check(c->capturing, s, "k_numeric32", __LINE__)) return CLAIR_ERR_HIP;
    timing_mark(c, timing, s, "numeric32");
  }
  HIPCHK(launch_rows_wg(b.w, occupancy_blocks(c, 1), s));
  if (capture_check(c->capturing, s, "k_rows_wg", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "rows_wg");
  if (b.any_B) {
    // rows of up to 8 points: one thread per row; longer rows: eight lanes each
    HIPCHK(launch_project(b.w, s));
    if (capture_check(c->capturing, s, "k_project", __LINE__)) return CLAIR_ERR_HIP;
    timing_mark(c, timing, s, "project");
  }
  return CLAIR_OK;
}

int enqueue_symbolic(clair_ctx* c, Batch& b, hipStream_t s, bool validate, bool timing) {
  int rc = upload(c, b, s);
  if (rc) return rc;
  timing_mark(c, timing, s, "upload");
  if (validate) {
    HIPCHK(launch_validate(b.w, occupancy_blocks(c, 4), s));
    timing_mark(c, timing, s, "validate");
  }
  if (b.any_agg) {
    HIPCHK(launch_agg_lists(b.w, b.n_total, occupancy_blocks(c, 4), c->cus, s));
    if (capture_check(c->capturing, s, "aggregate lists", __LINE__)) return CLAIR_ERR_HIP;
    timing_mark(c, timing, s, "aggregates");
  }
  if (c->theta > 0.0) {
    HIPCHK(launch_colmax(b.w, b.n_total, occupancy_blocks(c, 4), s));
    if (capture_check(c->capturing, s, "k_colmax", __LINE__)) return CLAIR_ERR_HIP;
    timing_mark(c, timing, s, "colmax");
  }
  if (b.adj_w) {
    HIPCHK(launch_adj(b.w, s));
    if (capture_check(c->capturing, s, "k_adj", __LINE__)) return CLAIR_ERR_HIP;
    timing_mark(c, timing, s, "adj");
  }
  HIPCHK(launch_count(b.w, s));
  if (capture_check(c->capturing, s, "k_count", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "count");
  HIPCHK(launch_count_mid(b.w, occupancy_blocks(c, 4), s));
  if (capture_check(c->capturing, s, "k_count_mid", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "count_mid");
  HIPCHK(launch_count_big(b.w, std::max(8, c->cus * 2), s));
  if (capture_check(c->capturing, s, "k_count_big", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "count_big");
  HIPCHK(launch_scan(b.w, s));
  if (capture_check(c->capturing, s, "k_scan", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "scan");
  return CLAIR_OK;
}

void fill_results(const MatStatus* hs, int nmat, clair_csr_out_t* R, clair_info_t* info, const clair_csr_t* A) {
  for (int m = 0; m < nmat; ++m) {
    if (R) {
      R[m].n_rows = hs[m].n_c;
      R[m].n_cols = A ? A[m].n : R[m].n_cols;
      R[m].nnz = hs[m].nnz;
    }
    if (info) {
      clair_info_t& in = info[m];
      in.status = hs[m].status;
      in.first_bad_row = hs[m].first_bad == INT32_MAX ? -1 : hs[m].first_bad;
      in.n_c = hs[m].n_c;
      in.max_block = hs[m].max_block;
      in.nnz = hs[m].nnz;
      in.n_uncovered = hs[m].n_uncovered;
      in.refine_iters_max = hs[m].refine_max;
      in.n_fp64_rows = hs[m].n_fp64;
      in.n_bf16_retries = hs[m].n_retry;
      in.reserved = 0;
    }
  }
}

int first_error(const MatStatus* hs, int nmat) {
  for (int m = 0; m < nmat; ++m)
    if (hs[m].status != 0) return hs[m].status;
  return CLAIR_OK;
}

int run_mixed(clair_ctx* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf, const double* const* B,
              const int32_t* ell, clair_csr_out_t* R, const clair_opts_t* o, clair_info_t* info,
              const int32_t* const* agg = nullptr) {
  const hipStream_t s = static_cast<hipStream_t>(o ? o->stream : nullptr);
  const bool async = o && o->async;
  const bool timing = o && o->timing;
  const bool validate = o && o->validate;
  Batch b;
  int rc = prepare(c, nmat, A, cf, B, ell, R, &b, agg);
  if (rc) return rc;
  b.w.bf16 = (o && o->precision == CLAIR_PREC_MIXED_BF16) ? 1 : 0;
  c->last_nmat = nmat;
  c->last_stream = s;
  c->last_layout = b.L;
  c->last_work = b.w;
  c->last_plain = false;
  if (timing) {
    rc = timing_begin(c, true);
    if (rc) return rc;
  }
  rc = enqueue_symbolic(c, b, s, validate, timing);
  if (rc) return rc;
  if (!async) {
    rc = read_status(c, b, s);
    if (rc) return rc;
    const MatStatus* hs = host_status(c, b);
    int maxb = 0;
    bool any_live = false;
    for (int m = 0; m < nmat; ++m) {
      maxb = std::max(maxb, hs[m].max_block);
      any_live |= (hs[m].status == 0);
    }
    if (!any_live) {
      fill_results(hs, nmat, R, info, A);
      return first_error(hs, nmat);
    }
    c->binB_max = std::max(9, std::min(32, maxb));
    c->last_maxb = maxb;
    if (maxb > kLdsBlockMax) {
      rc = ensure_scratch(c, std::max(1, c->cus), maxb);
      if (rc) return rc;
    }
  }
  rc = ensure_links(c, b);
  if (rc) return rc;
  Counters known{};
  if (!async) known = *host_counters(c, b);
  rc = enqueue_numeric(c, b, s, timing, async ? nullptr : &known);
  if (rc) return rc;
  c->last_work = b.w;
  if (async) return CLAIR_OK;
  rc = read_status(c, b, s);
  if (rc) return rc;
  const MatStatus* hs = host_status(c, b);
  fill_results(hs, nmat, R, info, A);
  return first_error(hs, nmat);
}

// ---------------------------------------------------------------------------
// plain FP64 per-row form
// ---------------------------------------------------------------------------
// pattern_only: stop after R's row_ptr and col_idx; *clist_out then points to
// the C-point list in the workspace (valid until the next plain-form call)
int run_plain_one(clair_ctx* c, const clair_csr_t& A, const int8_t* cf, const double* B, int ell,
                  clair_csr_out_t* R, hipStream_t s, clair_info_t* info, bool pattern_only = false,
                  const int32_t** clist_out = nullptr, const clair_csr_t* graph = nullptr) {
  const int n = A.n;
  const int nb = (n + 255) / 256;
  // workspace: blk_cnt[nb+1] clist[n] sizes[n+1] scan_tmp[nb+2] dsum[n] rsum[n] flags[8]
  const size_t o_blk = 0;
  const size_t o_clist = align_up(o_blk + sizeof(int32_t) * (nb + 2), 256);
  const size_t o_sizes = align_up(o_clist + sizeof(int32_t) * (n + 1), 256);
  const size_t o_tmp = align_up(o_sizes + sizeof(int32_t) * (n + 2), 256);
  const size_t o_dsum = align_up(o_tmp + sizeof(int32_t) * (nb + 4), 256);
  const size_t o_rsum = align_up(o_dsum + sizeof(double) * (n + 1), 256);
  const size_t o_cmax = align_up(o_rsum + sizeof(double) * (n + 1), 256);
  const size_t o_flags = align_up(o_cmax + sizeof(double) * (n + 1), 256);
  const size_t total = o_flags + 64;
  if (c->plain_ws.ensure(total) != hipSuccess) return CLAIR_ERR_NOMEM;
  HIPCHK(c->readback.ensure(64));
  char* base = static_cast<char*>(c->plain_ws.p);
  PlainWork p{};
  p.rp = A.row_ptr;
  p.ci = A.col_idx;
  p.va = A.val;
  p.literal = c->literal;
  p.grp = graph ? graph->row_ptr : A.row_ptr;
  p.gci = graph ? graph->col_idx : A.col_idx;
  p.gva = graph ? graph->val : A.val;
  p.cf = cf;
  p.B = B;
  p.n = n;
  p.ell = ell;
  p.theta = c->theta;
  p.cmax = reinterpret_cast<double*>(base + o_cmax);
  p.blk_cnt = reinterpret_cast<int32_t*>(base + o_blk);
  p.clist = reinterpret_cast<int32_t*>(base + o_clist);
  p.sizes = reinterpret_cast<int32_t*>(base + o_sizes);
  p.scan_tmp = reinterpret_cast<int32_t*>(base + o_tmp);
  p.dsum = reinterpret_cast<double*>(base + o_dsum);
  p.rsum = reinterpret_cast<double*>(base + o_rsum);
  p.flags = reinterpret_cast<int32_t*>(base + o_flags);
  p.Rrp = R->row_ptr;
  p.Rci = R->col_idx;
  p.Rva = R->val;
  int32_t hflags[8] = {0, INT32_MAX, 0, 0, 0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(p.flags, hflags, sizeof(hflags), hipMemcpyHostToDevice, s));
  HIPCHK(plain_colmax(p, s));
  HIPCHK(plain_count_c(p, s));
  HIPCHK(plain_scan_blocks(p.blk_cnt, nb, s));
  HIPCHK(plain_clist(p, s));
  int32_t n_c = 0;
  HIPCHK(hipMemcpyAsync(&n_c, p.blk_cnt + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  clair_info_t in{};
  in.first_bad_row = -1;
  in.n_c = n_c;
  if (n_c + 1 > R->row_capacity || !R->row_ptr) {
    in.status = CLAIR_ERR_CAPACITY;
  }
  HIPCHK(plain_sizes(p, n_c, s));
  // scan writes R.row_ptr; without row capacity scan into the workspace instead
  PlainWork q = p;
  if (in.status) q.Rrp = p.clist;  // clist is dead after sizes; it holds n+1 >= n_c+1 entries
  HIPCHK(plain_scan(q, n_c, s));
  int32_t nnz = 0;
  HIPCHK(hipMemcpyAsync(&nnz, q.Rrp + n_c, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hflags, p.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  in.nnz = nnz;
  in.max_block = hflags[2];
  R->n_rows = n_c;
  R->n_cols = n;
  R->nnz = nnz;
  if (in.status == 0 && (nnz > R->nnz_capacity || !R->col_idx || !R->val)) in.status = CLAIR_ERR_CAPACITY;
  if (in.status == 0 && hflags[0]) {
    in.status = hflags[0];
    in.first_bad_row = hflags[1];
  }
  if (in.status) {
    if (info) *info = in;
    return in.status;
  }
  HIPCHK(plain_fill(p, n_c, s));
  if (pattern_only) {
    if (clist_out) *clist_out = p.clist;
    if (info) *info = in;
    return CLAIR_OK;
  }
  const int smax = std::max(1, hflags[2]);
  const size_t kb = (size_t)n_c * ((size_t)smax * smax + smax) * sizeof(double);
  if (c->plain_k.ensure(std::max<size_t>(kb, 64)) != hipSuccess) return CLAIR_ERR_NOMEM;
  p.kbuf = static_cast<double*>(c->plain_k.p);
  HIPCHK(plain_solve(p, n_c, smax, s));
  if (B) {
    HIPCHK(hipMemsetAsync(p.dsum, 0, sizeof(double) * (n + 1), s));
    HIPCHK(hipMemsetAsync(p.rsum, 0, sizeof(double) * (n + 1), s));
    HIPCHK(plain_colsum(p, n_c, s));
    HIPCHK(plain_project(p, n_c, s));
  }
  HIPCHK(hipMemcpyAsync(hflags, p.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  in.status = hflags[0];
  in.first_bad_row = hflags[0] ? hflags[1] : -1;
  in.n_uncovered = B ? hflags[3] : 0;
  in.n_fp64_rows = n_c;
  if (info) *info = in;
  return in.status;
}

int run_plain(clair_ctx* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf, const double* const* B,
              const int32_t* ell, clair_csr_out_t* R, const clair_opts_t* o, clair_info_t* info) {
  const hipStream_t s = static_cast<hipStream_t>(o ? o->stream : nullptr);
  const bool timing = o && o->timing;
  int first = CLAIR_OK;
  c->last_plain = true;
  c->last_nmat = nmat;
  c->plain_info.assign(nmat, clair_info_t{});
  if (timing) {
    int rc = timing_begin(c, true);
    if (rc) return rc;
    timing_mark(c, true, s, "start");
  }
  for (int m = 0; m < nmat; ++m) {
    clair_info_t in{};
    if (!c->graph.empty() && ((int32_t)c->graph.size() != nmat || c->graph[m].n != A[m].n)) return CLAIR_ERR_INVALID;
    int rc = run_plain_one(c, A[m], cf[m], B ? B[m] : nullptr, ell[m], &R[m], s, &in, false, nullptr,
                           c->graph.empty() ? nullptr : &c->graph[m]);
    if (rc == CLAIR_ERR_HIP || rc == CLAIR_ERR_NOMEM) return rc;
    in.status = rc;
    c->plain_info[m] = in;
    if (info) info[m] = in;
    if (rc && !first) first = rc;
  }
  if (timing) timing_mark(c, true, s, "plain");
  return first;
}

clair_ctx* default_ctx() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_default_mu);
  if ((int)g_default.size() <= dev) g_default.resize(dev + 1, nullptr);
  if (!g_default[dev]) {
    clair_ctx* c = nullptr;
    if (clair_ctx_create(&c) != CLAIR_OK) return nullptr;
    g_default[dev] = c;
  }
  return g_default[dev];
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int clair_ctx_create(clair_ctx_t** out) {
  if (!out) return CLAIR_ERR_INVALID;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CLAIR_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CLAIR_ERR_HIP;
  clair_ctx* c = new (std::nothrow) clair_ctx();
  if (!c) return CLAIR_ERR_NOMEM;
  c->device = dev;
  c->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = c;
  return CLAIR_OK;
}

void clair_ctx_destroy(clair_ctx_t* c) {
  if (!c) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->ws.release();
  c->scratch.release();
  c->links.release();
  c->plain_ws.release();
  c->plain_k.release();
  c->stage.release();
  c->readback.release();
  if (c->upload_done) (void)hipEventDestroy(c->upload_done);
  for (auto& se : c->timing)
    for (int k = 0; k <= kMaxStages; ++k) (void)hipEventDestroy(se.ev[k]);
  delete c;
  (void)hipSetDevice(prev);
}

int clair_build_R_batched(clair_ctx_t* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
                          const double* const* B, const int32_t* ell, clair_csr_out_t* R,
                          const clair_opts_t* o, clair_info_t* info) {
  if (!c) return CLAIR_ERR_INVALID;
  int rc = check_args(nmat, A, cf, ell, R);
  if (rc) return rc;
  if (nmat == 0) return CLAIR_OK;
  if (o && o->precision == CLAIR_PREC_FP64) return run_plain(c, nmat, A, cf, B, ell, R, o, info);
  if (o && o->precision != CLAIR_PREC_MIXED && o->precision != CLAIR_PREC_MIXED_BF16) return CLAIR_ERR_INVALID;
  try {
    return run_mixed(c, nmat, A, cf, B, ell, R, o, info);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_build_R_agg(clair_ctx_t* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
                      const int32_t* const* agg, const double* const* B, const int32_t* ell, clair_csr_out_t* R,
                      const clair_opts_t* o, clair_info_t* info) {
  if (!c) return CLAIR_ERR_INVALID;
  int rc = check_args(nmat, A, cf, ell, R);
  if (rc) return rc;
  if (nmat > 0 && !agg) return CLAIR_ERR_INVALID;
  if (nmat == 0) return CLAIR_OK;
  if (o && o->precision == CLAIR_PREC_FP64) return CLAIR_ERR_UNSUPPORTED;
  if (o && o->precision != CLAIR_PREC_MIXED && o->precision != CLAIR_PREC_MIXED_BF16) return CLAIR_ERR_INVALID;
  try {
    return run_mixed(c, nmat, A, cf, B, ell, R, o, info, agg);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_build_R_ex(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell,
                     clair_csr_out_t* R, const clair_opts_t* o, clair_info_t* info) {
  const double* Bs[1] = {B};
  const int8_t* cfs[1] = {cf};
  int32_t ells[1] = {ell};
  return clair_build_R_batched(c, 1, A, cfs, Bs, ells, R, o, info);
}

int clair_build_R(const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell, clair_csr_out_t* R) {
  clair_ctx* c = default_ctx();
  if (!c) return CLAIR_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_default_mu);
  return clair_build_R_ex(c, A, cf, B, ell, R, nullptr, nullptr);
}

namespace {

// B = A^T (A: m x ncol) into device arrays of sufficient size; synchronous
// row_ptr[0] == 0 and row_ptr[m] == nnz on the device (the buffers that
// follow are sized from nnz, the kernels follow row_ptr); synchronous
int check_row_ptr_ends(const int32_t* rp, int32_t m, int64_t nnz, hipStream_t s) {
  if (m <= 0) return nnz == 0 ? CLAIR_OK : CLAIR_ERR_INVALID;
  int32_t ends[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&ends[0], rp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&ends[1], rp + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return (ends[0] == 0 && (int64_t)ends[1] == nnz) ? CLAIR_OK : CLAIR_ERR_INVALID;
}

int transpose_into(clair_ctx* c, const clair_csr_t& A, int32_t ncol, int32_t* trp, int32_t* tci, double* tva,
                   hipStream_t s) {
  if (int rc = check_row_ptr_ends(A.row_ptr, A.n, A.nnz, s)) return rc;
  const size_t ints = transpose_scratch_ints(ncol);
  HIPCHK(c->t_scratch.ensure(sizeof(int32_t) * ints));
  int32_t* scr = static_cast<int32_t*>(c->t_scratch.p);
  HIPCHK(launch_transpose(A.n, ncol, A.row_ptr, A.col_idx, A.val, trp, tci, tva, scr, c->cus, s));
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, scr + ncol, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return bad ? CLAIR_ERR_INVALID : CLAIR_OK;
}

int check_csr_args(const clair_csr_t* A) {
  if (!A || A->n < 0 || A->nnz < 0) return CLAIR_ERR_INVALID;
  if (A->n > 0 && !A->row_ptr) return CLAIR_ERR_INVALID;
  if (A->nnz > 0 && (!A->col_idx || !A->val)) return CLAIR_ERR_INVALID;
  return CLAIR_OK;
}

}  // namespace

int clair_transpose(clair_ctx_t* c, const clair_csr_t* A, int32_t ncol, clair_csr_out_t* AT, void* stream) {
  if (!c || !AT || ncol < 0 || check_csr_args(A)) return CLAIR_ERR_INVALID;
  AT->n_rows = ncol;
  AT->n_cols = A->n;
  AT->nnz = A->nnz;
  if (AT->row_capacity < ncol + 1 || AT->nnz_capacity < A->nnz || !AT->row_ptr ||
      (A->nnz > 0 && (!AT->col_idx || !AT->val)))
    return CLAIR_ERR_CAPACITY;
  try {
    return transpose_into(c, *A, ncol, AT->row_ptr, AT->col_idx, AT->val, static_cast<hipStream_t>(stream));
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_build_P(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell,
                  clair_csr_out_t* P, const clair_opts_t* o, clair_info_t* info) {
  if (!c || !P || !cf || ell < 1 || ell > 64 || check_csr_args(A)) return CLAIR_ERR_INVALID;
  if (!c->graph.empty()) return CLAIR_ERR_UNSUPPORTED;  // a strength matrix of A^T would be needed
  if (o && o->precision != CLAIR_PREC_MIXED && o->precision != CLAIR_PREC_FP64) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(o ? o->stream : nullptr);
  const int32_t n = A->n;
  try {
    // A^T
    HIPCHK(c->t_rp.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIPCHK(c->t_ci.ensure(sizeof(int32_t) * std::max<size_t>(1, (size_t)A->nnz)));
    HIPCHK(c->t_va.ensure(sizeof(double) * std::max<size_t>(1, (size_t)A->nnz)));
    clair_csr_t At{n, A->nnz, static_cast<int32_t*>(c->t_rp.p), static_cast<int32_t*>(c->t_ci.p),
                   static_cast<double*>(c->t_va.p)};
    int rc = transpose_into(c, *A, n, static_cast<int32_t*>(c->t_rp.p), static_cast<int32_t*>(c->t_ci.p),
                            static_cast<double*>(c->t_va.p), s);
    if (rc) return rc;
    // the restriction of A^T, Q = (W(A))^T, in library buffers
    int32_t n_c = 0;
    int64_t nnz = 0;
    rc = clair_size_R(c, 1, &At, &cf, &ell, &n_c, &nnz, s);
    if (rc && rc != CLAIR_ERR_CAPACITY) return rc;
    if (nnz > INT32_MAX) return CLAIR_ERR_UNSUPPORTED;
    HIPCHK(c->q_rp.ensure(sizeof(int32_t) * ((size_t)n_c + 1)));
    HIPCHK(c->q_ci.ensure(sizeof(int32_t) * std::max<int64_t>(1, nnz)));
    HIPCHK(c->q_va.ensure(sizeof(double) * std::max<int64_t>(1, nnz)));
    clair_csr_out_t Q{};
    Q.row_capacity = n_c + 1;
    Q.nnz_capacity = nnz;
    Q.row_ptr = static_cast<int32_t*>(c->q_rp.p);
    Q.col_idx = static_cast<int32_t*>(c->q_ci.p);
    Q.val = static_cast<double*>(c->q_va.p);
    clair_opts_t so = o ? *o : clair_opts_t{};
    so.async = 0;
    so.timing = 0;
    clair_info_t qi{};
    rc = clair_build_R_ex(c, &At, cf, B, ell, &Q, &so, &qi);
    if (info) *info = qi;
    P->n_rows = n;
    P->n_cols = n_c;
    P->nnz = nnz;
    if (rc) return rc;
    // P = Q^T: n x n_c
    if (P->row_capacity < n + 1 || P->nnz_capacity < nnz || !P->row_ptr || (nnz > 0 && (!P->col_idx || !P->val)))
      return CLAIR_ERR_CAPACITY;
    clair_csr_t Qin{n_c, (int32_t)nnz, Q.row_ptr, Q.col_idx, Q.val};
    return transpose_into(c, Qin, n, P->row_ptr, P->col_idx, P->val, s);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

namespace {

// Symbolic phase of C = X Y (X: X.n rows, k columns; Y: k rows, ny columns):
// row pointers into c->g_rp (X.n + 1 entries), nnz(C) and the hash-table size
// the numeric phase takes.  Synchronous.
int spgemm_symbolic(clair_ctx* c, const clair_csr_t& X, int32_t k, const clair_csr_t& Y, int32_t ny, int64_t* nnz,
                    int* lg, hipStream_t s) {
  const int m = X.n;
  HIPCHK(c->g_rp.ensure(sizeof(int32_t) * ((size_t)m + 1)));
  HIPCHK(c->g_cnt.ensure(sizeof(int32_t) * ((size_t)m + 4 + scan_scratch_ints(m))));
  int32_t* cnt = static_cast<int32_t*>(c->g_cnt.p);
  int32_t* flags = cnt + m;
  int32_t* sums = flags + 4;
  int32_t* crp = static_cast<int32_t*>(c->g_rp.p);
  HIPCHK(hipMemsetAsync(flags, 0, sizeof(int32_t) * 4, s));
  HIPCHK(launch_spgemm_count(m, X.row_ptr, X.col_idx, k, Y.row_ptr, Y.col_idx, ny, cnt, flags, lg, c->cus, s));
  HIPCHK(launch_exclusive_scan(cnt, m, crp, sums, c->cus, s));
  int32_t hf[2] = {0, 0};
  int32_t total = 0;
  HIPCHK(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&total, crp + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hf[1]) return CLAIR_ERR_INVALID;
  if (hf[0]) return CLAIR_ERR_UNSUPPORTED;
  *nnz = total;
  return CLAIR_OK;
}

int check_product_args(const clair_csr_t* X, int32_t x_cols, const clair_csr_t* Y, int32_t y_cols) {
  if (check_csr_args(X) || check_csr_args(Y) || x_cols < 0 || y_cols < 0 || x_cols != Y->n) return CLAIR_ERR_INVALID;
  return CLAIR_OK;
}

// C = X Y into C (capacities already checked); symbolic phase done (g_rp)
int spgemm_numeric(clair_ctx* c, const clair_csr_t& X, const clair_csr_t& Y, int lg, int32_t* crp, int32_t* cci,
                   double* cva, hipStream_t s) {
  const int m = X.n;
  if (crp != c->g_rp.p)
    HIPCHK(hipMemcpyAsync(crp, c->g_rp.p, sizeof(int32_t) * ((size_t)m + 1), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_spgemm_fill(m, X.row_ptr, X.col_idx, X.val, Y.row_ptr, Y.col_idx, Y.val, crp, cci, cva, lg, c->cus,
                            s));
  HIPCHK(hipStreamSynchronize(s));
  return CLAIR_OK;
}

bool fits(const clair_csr_out_t* C, int32_t rows, int64_t nnz) {
  return C->row_capacity >= rows + 1 && C->nnz_capacity >= nnz && C->row_ptr && (nnz == 0 || (C->col_idx && C->val));
}

}  // namespace

int clair_spgemm(clair_ctx_t* c, const clair_csr_t* X, int32_t x_cols, const clair_csr_t* Y, int32_t y_cols,
                 clair_csr_out_t* C, void* stream) {
  if (!c || !C || check_product_args(X, x_cols, Y, y_cols)) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    int64_t nnz = 0;
    int lg = 6;
    int rc = spgemm_symbolic(c, *X, x_cols, *Y, y_cols, &nnz, &lg, s);
    C->n_rows = X->n;
    C->n_cols = y_cols;
    C->nnz = nnz;
    if (rc) return rc;
    if (!fits(C, X->n, nnz)) return CLAIR_ERR_CAPACITY;
    return spgemm_numeric(c, *X, *Y, lg, C->row_ptr, C->col_idx, C->val, s);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_galerkin(clair_ctx_t* c, const clair_csr_t* R, const clair_csr_t* A, const clair_csr_t* P, int32_t n_c,
                   clair_csr_out_t* Ac, void* stream) {
  if (!c || !Ac || !A || !R || !P || R->n != n_c || P->n != A->n) return CLAIR_ERR_INVALID;
  if (check_product_args(A, A->n, P, n_c) || check_product_args(R, A->n, A, A->n)) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    // A P (n x n_c) in library buffers
    int64_t nnz_ap = 0;
    int lg = 6;
    int rc = spgemm_symbolic(c, *A, A->n, *P, n_c, &nnz_ap, &lg, s);
    if (rc) return rc;
    if (nnz_ap > INT32_MAX) return CLAIR_ERR_UNSUPPORTED;
    HIPCHK(c->ap_rp.ensure(sizeof(int32_t) * ((size_t)A->n + 1)));
    HIPCHK(c->ap_ci.ensure(sizeof(int32_t) * std::max<int64_t>(1, nnz_ap)));
    HIPCHK(c->ap_va.ensure(sizeof(double) * std::max<int64_t>(1, nnz_ap)));
    rc = spgemm_numeric(c, *A, *P, lg, static_cast<int32_t*>(c->ap_rp.p), static_cast<int32_t*>(c->ap_ci.p),
                        static_cast<double*>(c->ap_va.p), s);
    if (rc) return rc;
    const clair_csr_t AP{A->n, (int32_t)nnz_ap, static_cast<int32_t*>(c->ap_rp.p), static_cast<int32_t*>(c->ap_ci.p),
                         static_cast<double*>(c->ap_va.p)};
    // R (A P)
    int64_t nnz = 0;
    rc = spgemm_symbolic(c, *R, A->n, AP, n_c, &nnz, &lg, s);
    Ac->n_rows = n_c;
    Ac->n_cols = n_c;
    Ac->nnz = nnz;
    if (rc) return rc;
    if (!fits(Ac, n_c, nnz)) return CLAIR_ERR_CAPACITY;
    return spgemm_numeric(c, *R, AP, lg, Ac->row_ptr, Ac->col_idx, Ac->val, s);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_smooth_B(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B_in, double* B_out,
                   int32_t iterations, double omega, int32_t transpose, void* stream) {
  if (!c || check_csr_args(A) || iterations < 0 || !(omega == omega) || (A->n > 0 && (!cf || !B_in || !B_out)))
    return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = A->n;
  if (n == 0) return CLAIR_OK;
  try {
    clair_csr_t M = *A;
    if (transpose) {
      HIPCHK(c->t_rp.ensure(sizeof(int32_t) * ((size_t)n + 1)));
      HIPCHK(c->t_ci.ensure(sizeof(int32_t) * std::max<size_t>(1, (size_t)A->nnz)));
      HIPCHK(c->t_va.ensure(sizeof(double) * std::max<size_t>(1, (size_t)A->nnz)));
      int rc = transpose_into(c, *A, n, static_cast<int32_t*>(c->t_rp.p), static_cast<int32_t*>(c->t_ci.p),
                              static_cast<double*>(c->t_va.p), s);
      if (rc) return rc;
      M = clair_csr_t{n, A->nnz, static_cast<int32_t*>(c->t_rp.p), static_cast<int32_t*>(c->t_ci.p),
                      static_cast<double*>(c->t_va.p)};
    }
    HIPCHK(c->sm_x.ensure(sizeof(double) * n));
    HIPCHK(c->sm_y.ensure(sizeof(double) * n));
    HIPCHK(c->sm_flag.ensure(sizeof(int32_t)));
    double* x = static_cast<double*>(c->sm_x.p);
    double* y = static_cast<double*>(c->sm_y.p);
    int32_t* flag = static_cast<int32_t*>(c->sm_flag.p);
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    HIPCHK(hipMemcpyAsync(x, B_in, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    for (int it = 0; it < iterations; ++it) {
      const int which[3] = {1, 0, 0};  // C, then F twice
      for (int w = 0; w < 3; ++w) {
        HIPCHK(launch_jacobi_sweep(n, M.row_ptr, M.col_idx, M.val, cf, which[w], omega, x, y, flag, c->cus, s));
        std::swap(x, y);
      }
    }
    HIPCHK(hipMemcpyAsync(B_out, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    int32_t hf = 0;
    HIPCHK(hipMemcpyAsync(&hf, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hf == 2) return CLAIR_ERR_INVALID;
    if (hf == 1) return CLAIR_ERR_SINGULAR;
    return CLAIR_OK;
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_project_constraints(clair_ctx_t* c, clair_csr_out_t* R, int32_t n, const int8_t* cf, const double* B,
                              int32_t k, double rcond, int64_t* n_uncovered, void* stream) {
  if (!c || !R || n < 0 || k < 1 || k > 8 || !(rcond >= 0.0) || R->n_rows < 0 || R->nnz < 0) return CLAIR_ERR_INVALID;
  if (R->nnz > INT32_MAX) return CLAIR_ERR_UNSUPPORTED;
  if (n > 0 && (!cf || !B)) return CLAIR_ERR_INVALID;
  if (R->n_rows > 0 && (!R->row_ptr || (R->nnz > 0 && (!R->col_idx || !R->val)))) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (int rc = check_row_ptr_ends(R->row_ptr, R->n_rows, R->nnz, s)) return rc;
  const size_t nn = (size_t)n, nr = (size_t)R->n_rows, nz = (size_t)std::max<int64_t>(1, R->nnz);
  try {
    // one allocation, 256-byte aligned pieces
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~size_t(255);
      return o;
    };
    const size_t o_trp = take(sizeof(int32_t) * (nn + 1)), o_tci = take(sizeof(int32_t) * nz),
                 o_tva = take(sizeof(double) * nz), o_ts = take(sizeof(int32_t) * transpose_scratch_ints(n)),
                 o_flag = take(sizeof(int32_t) * std::max<size_t>(1, nn)), o_pos = take(sizeof(int32_t) * (nn + 1)),
                 o_sums = take(sizeof(int32_t) * scan_scratch_ints(n)),
                 o_rowc = take(sizeof(int32_t) * std::max<size_t>(1, nr)),
                 o_lam = take(sizeof(double) * std::max<size_t>(1, nn * k)), o_cnt = take(sizeof(unsigned long long));
    HIPCHK(c->pk_scratch.ensure(off));
    char* base = static_cast<char*>(c->pk_scratch.p);
    ProjectScratch w{reinterpret_cast<int32_t*>(base + o_trp),  reinterpret_cast<int32_t*>(base + o_tci),
                     reinterpret_cast<double*>(base + o_tva),   reinterpret_cast<int32_t*>(base + o_ts),
                     reinterpret_cast<int32_t*>(base + o_flag), reinterpret_cast<int32_t*>(base + o_pos),
                     reinterpret_cast<int32_t*>(base + o_sums), reinterpret_cast<int32_t*>(base + o_rowc),
                     reinterpret_cast<double*>(base + o_lam)};
    unsigned long long* unc = reinterpret_cast<unsigned long long*>(base + o_cnt);
    HIPCHK(hipMemsetAsync(unc, 0, sizeof(unsigned long long), s));
    HIPCHK(launch_project_k(n, R->n_rows, R->row_ptr, R->col_idx, R->val, cf, B, k, rcond, w, unc, c->cus, s));
    unsigned long long h_unc = 0;
    int32_t h_bad = 0, h_nc = 0;
    HIPCHK(hipMemcpyAsync(&h_unc, unc, sizeof(h_unc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&h_bad, w.t_scratch + n, sizeof(h_bad), hipMemcpyDeviceToHost, s));
    if (n > 0) HIPCHK(hipMemcpyAsync(&h_nc, w.pos + n, sizeof(h_nc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h_bad || h_nc != R->n_rows) return CLAIR_ERR_INVALID;
    if (n_uncovered) *n_uncovered = (int64_t)h_unc;
    return CLAIR_OK;
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_build_R_diag(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell,
                       int32_t iterations, clair_csr_out_t* R, clair_info_t* info, void* stream) {
  return clair_build_R_approx(c, A, cf, B, ell, CLAIR_INVERSE_DIAG, 0, iterations, R, info, stream);
}

int clair_build_R_approx(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell,
                         int32_t inverse, int32_t krylov, int32_t iterations, clair_csr_out_t* R, clair_info_t* info,
                         void* stream) {
  if (!c || !R || ell < 1 || ell > 64 || iterations < 0 || check_csr_args(A)) return CLAIR_ERR_INVALID;
  if (inverse != CLAIR_INVERSE_DIAG && inverse != CLAIR_INVERSE_ILU0 && inverse != CLAIR_INVERSE_GMRES)
    return CLAIR_ERR_INVALID;
  if (inverse == CLAIR_INVERSE_GMRES && (krylov < 1 || krylov > 32)) return CLAIR_ERR_INVALID;
  if (!cf && A->n > 0) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t n = A->n;
  try {
    // the pattern (strength threshold of the context), no local solves
    clair_info_t in{};
    const int32_t* clist = nullptr;
    if (!c->graph.empty() && (c->graph.size() != 1 || c->graph[0].n != A->n)) return CLAIR_ERR_INVALID;
    int rc = run_plain_one(c, *A, cf, B, ell, R, s, &in, true, &clist, c->graph.empty() ? nullptr : &c->graph[0]);
    if (info) *info = in;
    if (rc) return rc;
    const int32_t n_c = R->n_rows;
    const int64_t nnz = R->nnz;
    // A^T for the column gathers of the residual
    HIPCHK(c->t_rp.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIPCHK(c->t_ci.ensure(sizeof(int32_t) * std::max<size_t>(1, (size_t)A->nnz)));
    HIPCHK(c->t_va.ensure(sizeof(double) * std::max<size_t>(1, (size_t)A->nnz)));
    rc = transpose_into(c, *A, n, static_cast<int32_t*>(c->t_rp.p), static_cast<int32_t*>(c->t_ci.p),
                        static_cast<double*>(c->t_va.p), s);
    if (rc) return rc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~size_t(255);
      return o;
    };
    const size_t nn = std::max<size_t>(1, (size_t)n), nz = std::max<size_t>(1, (size_t)nnz);
    const bool ilu = inverse == CLAIR_INVERSE_ILU0, gmres = inverse == CLAIR_INVERSE_GMRES;
    const int km = gmres ? krylov : 0;
    const int smax = std::max(1, in.max_block);
    const int64_t fstride = (int64_t)smax * smax;  // per row: K
    const size_t o_diag = take(sizeof(double) * nn), o_d = take(sizeof(double) * nn), o_sj = take(sizeof(double) * nn),
                 o_u = take(sizeof(double) * nz), o_cnt = take(sizeof(int32_t) * nn),
                 o_erow = take(sizeof(int32_t) * nz), o_flags = take(64),
                 o_fac = take((ilu || gmres) ? sizeof(double) * (size_t)fstride * std::max<size_t>(1, (size_t)n_c) : 8),
                 o_gw = take(gmres ? sizeof(double) * (size_t)(km + 1) * (size_t)(smax + km + 3) *
                                         std::max<size_t>(1, (size_t)n_c)
                                   : 8);
    HIPCHK(c->ap_ws.ensure(off));
    char* base = static_cast<char*>(c->ap_ws.p);
    DiagWork w{};
    w.ilu = ilu ? 1 : 0;
    w.gmres = gmres ? 1 : 0;
    w.krylov = km;
    w.gw = reinterpret_cast<double*>(base + o_gw);
    w.fac = reinterpret_cast<double*>(base + o_fac);
    w.smax = smax;
    w.n = n;
    w.n_c = n_c;
    w.nnz = nnz;
    w.cus = c->cus;
    w.rp = A->row_ptr;
    w.ci = A->col_idx;
    w.va = A->val;
    w.trp = static_cast<const int32_t*>(c->t_rp.p);
    w.tci = static_cast<const int32_t*>(c->t_ci.p);
    w.tva = static_cast<const double*>(c->t_va.p);
    w.cf = cf;
    w.B = B;
    w.Rrp = R->row_ptr;
    w.Rci = R->col_idx;
    w.Rva = R->val;
    w.clist = clist;
    w.diag = reinterpret_cast<double*>(base + o_diag);
    w.d = reinterpret_cast<double*>(base + o_d);
    w.sj = reinterpret_cast<double*>(base + o_sj);
    w.u = reinterpret_cast<double*>(base + o_u);
    w.cnt = reinterpret_cast<int32_t*>(base + o_cnt);
    w.erow = reinterpret_cast<int32_t*>(base + o_erow);
    w.bad_row = reinterpret_cast<int32_t*>(base + o_flags);
    w.uncovered = reinterpret_cast<unsigned long long*>(base + o_flags + 8);
    HIPCHK(hipMemsetAsync(w.d, 0, sizeof(double) * nn, s));
    HIPCHK(hipMemsetAsync(w.cnt, 0, sizeof(int32_t) * nn, s));
    const int32_t hinit[4] = {INT32_MAX, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(w.bad_row, hinit, sizeof(hinit), hipMemcpyHostToDevice, s));
    HIPCHK(launch_diag_start(w, s));
    int32_t hbad[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hbad, w.bad_row, sizeof(hbad), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad[0] != INT32_MAX) {
      in.status = CLAIR_ERR_SINGULAR;
      in.first_bad_row = hbad[0];
      if (info) *info = in;
      return CLAIR_ERR_SINGULAR;
    }
    for (int32_t it = 0; it < iterations; ++it) HIPCHK(launch_diag_iteration(w, s));
    unsigned long long unc = 0;
    HIPCHK(hipMemcpyAsync(&unc, w.uncovered, sizeof(unc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    in.n_uncovered = B ? (int64_t)unc : 0;
    in.first_bad_row = -1;
    if (info) *info = in;
    return CLAIR_OK;
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_build_R_kkt(clair_ctx_t* c, const clair_csr_t* A, const int8_t* cf, const double* B, int32_t ell,
                      clair_csr_out_t* R, clair_info_t* info, void* stream) {
  if (!c || !R || ell < 1 || ell > 64 || check_csr_args(A)) return CLAIR_ERR_INVALID;
  if (!cf && A->n > 0) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    // the unconstrained minimiser: the exact l-AIR rows
    clair_opts_t o{};
    o.stream = stream;
    o.precision = CLAIR_PREC_MIXED;
    clair_info_t in{};
    int rc = clair_build_R_ex(c, A, cf, nullptr, ell, R, &o, &in);
    if (info) *info = in;
    if (rc || !B) return rc;
    const int32_t n = A->n, n_rows = R->n_rows;
    const int smax = std::max(1, in.max_block);
    if (smax > 64) return CLAIR_ERR_UNSUPPORTED;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      const size_t o2 = off;
      off += (bytes + 255) & ~size_t(255);
      return o2;
    };
    const size_t nn = std::max<size_t>(1, (size_t)n), nr = std::max<size_t>(1, (size_t)n_rows);
    const size_t o_flag = take(sizeof(int32_t) * nn), o_pos = take(sizeof(int32_t) * (nn + 1)),
                 o_sums = take(sizeof(int32_t) * scan_scratch_ints(n)), o_rowc = take(sizeof(int32_t) * nr),
                 o_cnt = take(sizeof(int32_t) * nn), o_bad = take(64),
                 o_K = take(sizeof(double) * (size_t)smax * smax * nr), o_L = take(sizeof(double) * (size_t)smax * smax * nr),
                 o_T = take(sizeof(double) * (size_t)smax * nr), o_rhs = take(sizeof(double) * nn),
                 o_res = take(sizeof(double) * nn), o_p = take(sizeof(double) * nn), o_x = take(sizeof(double) * nn),
                 o_Ap = take(sizeof(double) * nn), o_dot = take(64);
    HIPCHK(c->kkt_ws.ensure(off));
    char* base = static_cast<char*>(c->kkt_ws.p);
    KktWork w{};
    w.n = n;
    w.n_rows = n_rows;
    w.smax = smax;
    w.cus = c->cus;
    w.rp = A->row_ptr;
    w.ci = A->col_idx;
    w.va = A->val;
    w.cf = cf;
    w.B = B;
    w.Rrp = R->row_ptr;
    w.Rci = R->col_idx;
    w.Rva = R->val;
    w.flag = reinterpret_cast<int32_t*>(base + o_flag);
    w.pos = reinterpret_cast<int32_t*>(base + o_pos);
    w.scan_sums = reinterpret_cast<int32_t*>(base + o_sums);
    w.rowc = reinterpret_cast<int32_t*>(base + o_rowc);
    w.cnt = reinterpret_cast<int32_t*>(base + o_cnt);
    w.bad = reinterpret_cast<int32_t*>(base + o_bad);
    w.K = reinterpret_cast<double*>(base + o_K);
    w.L = reinterpret_cast<double*>(base + o_L);
    w.T = reinterpret_cast<double*>(base + o_T);
    w.rhs = reinterpret_cast<double*>(base + o_rhs);
    w.res = reinterpret_cast<double*>(base + o_res);
    w.p = reinterpret_cast<double*>(base + o_p);
    w.x = reinterpret_cast<double*>(base + o_x);
    w.Ap = reinterpret_cast<double*>(base + o_Ap);
    double* dot = reinterpret_cast<double*>(base + o_dot);
    HIPCHK(hipMemsetAsync(w.cnt, 0, sizeof(int32_t) * nn, s));
    HIPCHK(hipMemsetAsync(w.rhs, 0, sizeof(double) * nn, s));
    const int32_t hbad0[2] = {0, INT32_MAX};
    HIPCHK(hipMemcpyAsync(w.bad, hbad0, sizeof(hbad0), hipMemcpyHostToDevice, s));
    HIPCHK(launch_kkt_setup(w, s));
    int32_t hbad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hbad, w.bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad[0]) return CLAIR_ERR_INVALID;
    if (hbad[1] != INT32_MAX) {
      in.status = CLAIR_ERR_SINGULAR;
      in.first_bad_row = hbad[1];
      if (info) *info = in;
      return CLAIR_ERR_SINGULAR;
    }
    // conjugate gradients on M lambda = Q z0 - B_F (M SPD), from lambda = 0;
    // the scalars stay on the device, the host reads the flag every 8 steps
    w.sc = dot;
    w.done = reinterpret_cast<int32_t*>(dot + 6);
    w.steps = w.done + 1;
    HIPCHK(hipMemsetAsync(dot, 0, 64, s));
    HIPCHK(launch_kkt_dot(w, w.res, w.res, w.sc, s));
    double rr0 = 0.0;
    HIPCHK(hipMemcpyAsync(&rr0, w.sc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double stop = rr0 * 1e-28;  // |res| <= 1e-14 |rhs|
    HIPCHK(hipMemcpyAsync(w.sc + 3, &stop, sizeof(double), hipMemcpyHostToDevice, s));
    int32_t hs[2] = {rr0 > 0.0 ? 0 : 1, 0};
    HIPCHK(hipMemcpyAsync(w.done, hs, sizeof(int32_t), hipMemcpyHostToDevice, s));
    int queued = 0;
    while (!hs[0] && queued < 10000) {
      for (int k = 0; k < 8; ++k) HIPCHK(launch_kkt_step(w, s));
      queued += 8;
      HIPCHK(hipMemcpyAsync(hs, w.done, sizeof(hs), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    const int it = hs[1];
    HIPCHK(launch_kkt_apply(w, s));
    HIPCHK(hipStreamSynchronize(s));
    in.refine_iters_max = it;
    if (info) *info = in;
    return CLAIR_OK;
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
}

int clair_ctx_info(clair_ctx_t* c, int32_t nmat, clair_csr_out_t* R, clair_info_t* info) {
  if (!c || nmat < 0) return CLAIR_ERR_INVALID;
  if (c->last_plain) {
    if (nmat > (int)c->plain_info.size()) return CLAIR_ERR_INVALID;
    int first = 0;
    for (int m = 0; m < nmat; ++m) {
      if (info) info[m] = c->plain_info[m];
      if (R) {
        R[m].n_rows = c->plain_info[m].n_c;
        R[m].nnz = c->plain_info[m].nnz;
      }
      if (!first && c->plain_info[m].status) first = c->plain_info[m].status;
    }
    return first;
  }
  if (nmat > c->last_nmat) return CLAIR_ERR_INVALID;
  Batch b;
  b.L = c->last_layout;
  b.w = c->last_work;
  int rc = read_status(c, b, c->last_stream);
  if (rc) return rc;
  const MatStatus* hs = host_status(c, b);
  fill_results(hs, nmat, R, info, nullptr);
  return first_error(hs, nmat);
}

int clair_size_R(clair_ctx_t* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf, const int32_t* ell,
                 int32_t* n_c, int64_t* nnz, void* stream) {
  if (!c || !n_c || !nnz) return CLAIR_ERR_INVALID;
  std::vector<clair_csr_out_t> R(nmat > 0 ? nmat : 1);
  for (auto& r : R) r = clair_csr_out_t{};
  int rc = check_args(nmat, A, cf, ell, R.data());
  if (rc) return rc;
  if (nmat == 0) return CLAIR_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  Batch b;
  rc = prepare(c, nmat, A, cf, nullptr, ell, R.data(), &b);
  if (rc) return rc;
  c->last_nmat = nmat;
  c->last_stream = s;
  c->last_layout = b.L;
  c->last_work = b.w;
  c->last_plain = false;
  rc = enqueue_symbolic(c, b, s, false, false);
  if (rc) return rc;
  rc = read_status(c, b, s);
  if (rc) return rc;
  const MatStatus* hs = host_status(c, b);
  int first = 0, maxb = 0;
  for (int m = 0; m < nmat; ++m) {
    n_c[m] = hs[m].n_c;
    nnz[m] = hs[m].nnz;
    maxb = std::max(maxb, hs[m].max_block);
    if (hs[m].status != 0 && hs[m].status != CLAIR_ERR_CAPACITY && !first) first = hs[m].status;
  }
  c->binB_max = std::max(9, std::min(32, maxb));
  c->last_maxb = maxb;
  return first;
}

int clair_ctx_stage_times(clair_ctx_t* c, const char** names, float* ms, int32_t cap) {
  if (!c) return 0;
  int nst = 0;
  std::vector<std::string> keys;
  std::vector<float> acc;
  for (size_t t = 0; t < c->timing_used; ++t) {
    StageEvents& se = c->timing[t];
    if (se.n == 0) continue;
    if (hipEventSynchronize(se.ev[se.n]) != hipSuccess) return 0;
    for (int k = 0; k < se.n; ++k) {
      float v = 0.f;
      (void)hipEventElapsedTime(&v, se.ev[k], se.ev[k + 1]);
      std::string key = se.name[k];
      auto it = std::find(keys.begin(), keys.end(), key);
      if (it == keys.end()) {
        keys.push_back(key);
        acc.push_back(v);
      } else {
        acc[it - keys.begin()] += v;
      }
    }
  }
  for (size_t k = 0; k < keys.size() && (int)k < cap; ++k) {
    if (names) {
      // stage names are string literals with static storage
      for (size_t t = 0; t < c->timing_used; ++t) {
        StageEvents& se = c->timing[t];
        for (int q = 0; q < se.n; ++q)
          if (keys[k] == se.name[q]) names[k] = se.name[q];
      }
    }
    if (ms) ms[k] = acc[k];
    ++nst;
  }
  c->timing_used = 0;
  return nst;
}

int clair_ctx_set_tuning(clair_ctx_t* c, int32_t group, int32_t wg_threads, int32_t chunk) {
  if (!c) return CLAIR_ERR_INVALID;
  if (group && group != 1 && group != 4 && group != 8 && group != 16 && group != 32) return CLAIR_ERR_INVALID;
  if (wg_threads && wg_threads != 64 && wg_threads != 128 && wg_threads != 256) return CLAIR_ERR_INVALID;
  if (chunk && (chunk < 256 || chunk > kMaxChunk || (chunk % 256))) return CLAIR_ERR_INVALID;
  if (group) c->group = group;
  if (wg_threads) c->wg_threads = wg_threads;
  if (chunk) c->chunk = chunk;
  return CLAIR_OK;
}

int clair_ctx_set_literal_pattern(clair_ctx_t* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return CLAIR_ERR_INVALID;
  c->literal = on;
  return CLAIR_OK;
}

int clair_ctx_set_graph(clair_ctx_t* c, int32_t nmat, const clair_csr_t* S) {
  if (!c || nmat < 0) return CLAIR_ERR_INVALID;
  if (nmat == 0 || !S) {
    c->graph.clear();
    return CLAIR_OK;
  }
  for (int m = 0; m < nmat; ++m)
    if (check_csr_args(&S[m])) return CLAIR_ERR_INVALID;
  try {
    c->graph.assign(S, S + nmat);
  } catch (...) {
    return CLAIR_ERR_NOMEM;
  }
  return CLAIR_OK;
}

int clair_ctx_set_strength(clair_ctx_t* c, double theta) {
  if (!c || !(theta >= 0.0 && theta <= 1.0)) return CLAIR_ERR_INVALID;
  c->theta = theta;
  return CLAIR_OK;
}

int clair_ctx_set_search_adjacency(clair_ctx_t* c, int32_t mode) {
  if (!c || !(mode == -1 || mode == 0 || mode == 4 || mode == 8)) return CLAIR_ERR_INVALID;
  c->adj_mode = mode;
  return CLAIR_OK;
}

int clair_ctx_get_strength(clair_ctx_t* c, double* theta) {
  if (!c || !theta) return CLAIR_ERR_INVALID;
  *theta = c->theta;
  return CLAIR_OK;
}

// clair_build_R_noalloc: the whole workspace of one setup (descriptors,
// chunk arrays, neighbourhood slots, queues, column lists) lives in this
// static device array, one copy per device the library runs on, kept until
// the process ends.  Kernels get its device address (hipGetSymbolAddress,
// once per device), never the name, which in host code is only a stand-in.
static __device__ __align__(256) char scratch[CLAIR_NOALLOC_SCRATCH_BYTES];

int clair_build_R_noalloc(const clair_csr_t* A, const int8_t* cf_marker, const double* B, int32_t ell,
                          clair_csr_out_t* R_out, void* stream, clair_info_t* info) {
  static std::mutex mu;
  static char* dev_ptr[kNoAllocDevices];
  static clair_ctx ctx_of[kNoAllocDevices];
  alignas(256) static char host_stage[kNoAllocDevices][kNoAllocHostBytes];
  if (!A || !R_out) return CLAIR_ERR_INVALID;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return CLAIR_ERR_UNSUPPORTED;
  clair_ctx* c = &ctx_of[dev];
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!dev_ptr[dev]) {
      // set-up on this device's first call, with the device current
      char* p = nullptr;
      HIPCHK(hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch)));
      int cus = 0;
      HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      c->device = dev;
      c->cus = cus > 0 ? cus : 256;
      c->fixed = true;
      c->fixed_dev = p;
      c->fixed_dev_bytes = CLAIR_NOALLOC_SCRATCH_BYTES;
      c->fixed_host = host_stage[dev];
      c->fixed_host_bytes = kNoAllocHostBytes;
      dev_ptr[dev] = p;
    }
  }
  clair_opts_t o{};
  o.stream = stream;
  const int8_t* cfs[1] = {cf_marker};
  const double* Bs[1] = {B};
  const int32_t ells[1] = {ell};
  return run_mixed(c, 1, A, cfs, Bs, ells, R_out, &o, info);
}

int clair_ctx_set_bin_shape(clair_ctx_t* c, int32_t binB_lanes) {
  if (!c || !(binB_lanes == 0 || binB_lanes == 8 || binB_lanes == 16 || binB_lanes == 32)) return CLAIR_ERR_INVALID;
  if (binB_lanes) c->binB_lanes = binB_lanes;
  return CLAIR_OK;
}

int clair_ctx_get_bin_shape(clair_ctx_t* c, int32_t* binB_lanes) {
  if (!c || !binB_lanes) return CLAIR_ERR_INVALID;
  *binB_lanes = c->binB_lanes;
  return CLAIR_OK;
}

int clair_ctx_scratch_bytes(clair_ctx_t* c, int64_t* bytes) {
  if (!c || !bytes) return CLAIR_ERR_INVALID;
  *bytes = c->scratch.p ? c->scratch_slots * c->scratch_stride * (int64_t)sizeof(double) : 0;
  return CLAIR_OK;
}

int clair_ctx_get_tuning(clair_ctx_t* c, int32_t* group, int32_t* wg_threads, int32_t* chunk) {
  if (!c) return CLAIR_ERR_INVALID;
  if (group) *group = c->group;
  if (wg_threads) *wg_threads = c->wg_threads;
  if (chunk) *chunk = c->chunk;
  return CLAIR_OK;
}

// The autotuner's cache: the tuning picked for a block-size histogram, per
// device and search setting.  The histogram counts the rows of each block
// size 0..32 and above 32 over the whole batch; its signature keeps, per size,
// the binary order of magnitude of the count (so batches of the same shape
// and similar size share an entry).
struct TuneKey {
  int device;
  int nmat_class;  // 1, 2..7, 8..63, 64+ matrices
  double theta;
  int literal, graph, agg;
  uint8_t hist[34];
  bool operator<(const TuneKey& o) const {
    if (device != o.device) return device < o.device;
    if (nmat_class != o.nmat_class) return nmat_class < o.nmat_class;
    if (theta != o.theta) return theta < o.theta;
    if (literal != o.literal) return literal < o.literal;
    if (graph != o.graph) return graph < o.graph;
    if (agg != o.agg) return agg < o.agg;
    return std::memcmp(hist, o.hist, sizeof(hist)) < 0;
  }
};
struct TuneVal {
  int group, wg_threads, chunk, binB_lanes;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

int clair_autotune(clair_ctx_t* c, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
                   const double* const* B, const int32_t* ell, clair_csr_out_t* R, void* stream, int32_t reps) {
  if (!c || reps < 1) return CLAIR_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // one synchronous setup: sizes, validity, and R's row pointers for the
  // histogram of block sizes
  std::vector<clair_info_t> info(nmat);
  clair_opts_t o{};
  o.stream = stream;
  int rc = clair_build_R_batched(c, nmat, A, cf, B, ell, R, &o, info.data());
  if (rc) return rc;
  int64_t hist[34] = {0};
  for (int m = 0; m < nmat; ++m) {
    const int nc = info[m].n_c;
    if (nc <= 0) continue;
    std::vector<int32_t> rp((size_t)nc + 1);
    HIPCHK(hipMemcpy(rp.data(), R[m].row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
    for (int r = 0; r < nc; ++r) {
      const int sz = rp[r + 1] - rp[r] - 1;
      hist[sz < 0 ? 0 : sz > 32 ? 33 : sz] += 1;
    }
  }
  TuneKey key{};
  key.device = c->device;
  key.nmat_class = nmat <= 1 ? 0 : nmat < 8 ? 1 : nmat < 64 ? 2 : 3;
  key.theta = c->theta;
  key.literal = c->literal;
  key.graph = c->graph.empty() ? 0 : 1;
  key.agg = 0;
  for (int k = 0; k < 34; ++k) {
    int mag = 0;
    for (int64_t v = hist[k]; v > 0; v >>= 1) ++mag;
    key.hist[k] = (uint8_t)mag;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c->group = it->second.group;
      c->wg_threads = it->second.wg_threads;
      c->chunk = it->second.chunk;
      c->binB_lanes = it->second.binB_lanes;
      c->tune_timed = 0;
      o.async = 0;
      return clair_build_R_batched(c, nmat, A, cf, B, ell, R, &o, nullptr);
    }
  }
  int maxs = 0;
  int64_t above8 = 0, above16 = 0, binB_rows = 0;
  for (int k = 0; k < 34; ++k) {
    if (hist[k]) maxs = k;
    if (k > 8) above8 += hist[k];
    if (k > 16) above16 += hist[k];
  }
  // candidates for the bin-A bound, from the histogram: 16 and 32 lanes per
  // row only when rows above 8 (16) points exist
  std::vector<int> groups = {1, 4, 8};
  if (above8) groups.push_back(16);
  if (above16) groups.push_back(32);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int timed = 0;
  auto time_one = [&](float* ms) -> int {
    int r2 = clair_build_R_batched(c, nmat, A, cf, B, ell, R, &o, nullptr);  // warm-up
    if (r2) return r2;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !r2; ++r) r2 = clair_build_R_batched(c, nmat, A, cf, B, ell, R, &o, nullptr);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
    ++timed;
    return r2;
  };
  TuneVal best{c->group, c->wg_threads, c->chunk, c->binB_lanes};
  float best_ms = 1e30f;
  o.async = 1;
  // stage 1: bin-A lanes and workgroup size (chunk 1024)
  for (int g : groups) {
    for (int t : {64, 128, 256}) {
      if (g == 32 && t == 256) continue;
      c->group = g;
      c->wg_threads = t;
      c->chunk = 1024;
      float ms = 0.f;
      if (!time_one(&ms) && ms < best_ms) { best_ms = ms; best = {g, t, 1024, c->binB_lanes}; }
    }
  }
  // stage 2: the symbolic pass's chunk
  for (int ch : {512, 2048}) {
    c->group = best.group;
    c->wg_threads = best.wg_threads;
    c->chunk = ch;
    float ms = 0.f;
    if (!time_one(&ms) && ms < best_ms) { best_ms = ms; best.chunk = ch; }
  }
  // stage 3: the bin-B layout, when rows fall between the bin-A bound and 32
  const int abound = best.group <= 8 ? 8 : best.group;
  for (int k = abound + 1; k <= 32; ++k) binB_rows += hist[k];
  if (binB_rows) {
    for (int lanes : {8, 16, 32}) {
      if (lanes == best.binB_lanes) continue;
      c->group = best.group;
      c->wg_threads = best.wg_threads;
      c->chunk = best.chunk;
      c->binB_lanes = lanes;
      float ms = 0.f;
      if (!time_one(&ms) && ms < best_ms) { best_ms = ms; best.binB_lanes = lanes; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)maxs;
  c->group = best.group;
  c->wg_threads = best.wg_threads;
  c->chunk = best.chunk;
  c->binB_lanes = best.binB_lanes;
  c->tune_timed = timed;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  // leave R consistent with the chosen shape
  o.async = 0;
  return clair_build_R_batched(c, nmat, A, cf, B, ell, R, &o, nullptr);
}

int clair_ctx_autotune_runs(clair_ctx_t* c, int32_t* timed) {
  if (!c || !timed) return CLAIR_ERR_INVALID;
  *timed = c->tune_timed;
  return CLAIR_OK;
}

struct clair_graph {
  clair_ctx* ctx = nullptr;  // private context: its buffers are baked into the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int clair_graph_create(clair_ctx_t* parent, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
                       const double* const* B, const int32_t* ell, clair_csr_out_t* R, void* stream,
                       clair_graph_t** out) {
  if (!parent || !out) return CLAIR_ERR_INVALID;
  *out = nullptr;
  clair_graph* g = new (std::nothrow) clair_graph();
  if (!g) return CLAIR_ERR_NOMEM;
  int rc = clair_ctx_create(&g->ctx);
  if (rc) {
    delete g;
    return rc;
  }
  g->ctx->group = parent->group;
  g->ctx->wg_threads = parent->wg_threads;
  g->ctx->chunk = parent->chunk;
  g->ctx->theta = parent->theta;
  g->ctx->graph = parent->graph;
  g->ctx->literal = parent->literal;
  g->ctx->binB_lanes = parent->binB_lanes;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  clair_opts_t o{};
  o.stream = stream;
  // one synchronous run sizes every buffer (including scratch) and checks the inputs
  rc = clair_build_R_batched(g->ctx, nmat, A, cf, B, ell, R, &o, nullptr);
  if (rc) {
    clair_graph_destroy(g);
    return rc;
  }
  o.async = 1;
  // the staging buffer must not be waited on during capture (no synchronising
  // call may run inside it); it keeps the captured descriptors for every replay
  hipError_t es = hipEventSynchronize(g->ctx->upload_done);
  if (es != hipSuccess) {
    set_last_error("hipEventSynchronize", es, __LINE__);
    clair_graph_destroy(g);
    return CLAIR_ERR_HIP;
  }
  g->ctx->upload_pending = false;
  hipError_t eb = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    set_last_error("hipStreamBeginCapture", eb, __LINE__);
    clair_graph_destroy(g);
    return CLAIR_ERR_HIP;
  }
  g->ctx->capturing = true;
  rc = capture_check(true, s, "hipStreamBeginCapture", __LINE__) ? CLAIR_ERR_HIP
                                                                 : clair_build_R_batched(g->ctx, nmat, A, cf, B, ell, R, &o, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  g->ctx->capturing = false;
  if (rc || e != hipSuccess) {
    if (e != hipSuccess && !rc) set_last_error("hipStreamEndCapture", e, __LINE__);
    if (graph) (void)hipGraphDestroy(graph);
    clair_graph_destroy(g);
    return rc ? rc : CLAIR_ERR_HIP;
  }
  g->graph = graph;
  hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    set_last_error("hipGraphInstantiate", ei, __LINE__);
    clair_graph_destroy(g);
    return CLAIR_ERR_HIP;
  }
  *out = g;
  return CLAIR_OK;
}

int clair_graph_launch(clair_graph_t* g, void* stream) {
  if (!g || !g->exec) return CLAIR_ERR_INVALID;
  g->ctx->last_stream = static_cast<hipStream_t>(stream);
  HIPCHK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return CLAIR_OK;
}

struct clair_plan {
  clair_ctx* ctx = nullptr;  // private context: holds the symbolic state
  Batch b;                   // layout and device pointers of the planned batch
  std::vector<char> head;    // descriptors, status and counters after the symbolic phase
  std::vector<int32_t> n, n_c;
  std::vector<int64_t> nnz, nnzA;
};

int clair_plan_create(clair_ctx_t* parent, int32_t nmat, const clair_csr_t* A, const int8_t* const* cf,
                      const int32_t* ell, clair_csr_out_t* R, void* stream, clair_plan_t** out) {
  if (!parent || !out) return CLAIR_ERR_INVALID;
  *out = nullptr;
  int rc = check_args(nmat, A, cf, ell, R);
  if (rc) return rc;
  if (nmat == 0) return CLAIR_ERR_INVALID;
  clair_plan* pl = new (std::nothrow) clair_plan();
  if (!pl) return CLAIR_ERR_NOMEM;
  try {
    rc = clair_ctx_create(&pl->ctx);
    if (rc) {
      delete pl;
      return rc;
    }
    clair_ctx* c = pl->ctx;
    c->group = parent->group;
    c->wg_threads = parent->wg_threads;
    c->chunk = parent->chunk;
    c->theta = parent->theta;
    c->graph = parent->graph;
    c->literal = parent->literal;
    c->binB_lanes = parent->binB_lanes;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    Batch& b = pl->b;
    rc = prepare(c, nmat, A, cf, nullptr, ell, R, &b);
    if (!rc) rc = enqueue_symbolic(c, b, s, false, false);
    if (!rc) rc = read_status(c, b, s);
    if (rc) {
      clair_plan_destroy(pl);
      return rc;
    }
    const MatStatus* hs = host_status(c, b);
    fill_results(hs, nmat, R, nullptr, A);
    const int first = first_error(hs, nmat);
    if (first) {
      clair_plan_destroy(pl);
      return first;
    }
    int maxb = 0;
    for (int m = 0; m < nmat; ++m) maxb = std::max(maxb, hs[m].max_block);
    c->binB_max = std::max(9, std::min(32, maxb));
    c->last_maxb = maxb;
    if (maxb > kLdsBlockMax) {
      rc = ensure_scratch(c, std::max(1, c->cus), maxb);
      if (rc) {
        clair_plan_destroy(pl);
        return rc;
      }
    }
    const char* rb = static_cast<const char*>(c->readback.p);
    pl->head.assign(rb, rb + b.L.head_bytes);
    for (int m = 0; m < nmat; ++m) {
      pl->n.push_back(A[m].n);
      pl->nnzA.push_back(A[m].nnz);
      pl->n_c.push_back(hs[m].n_c);
      pl->nnz.push_back(hs[m].nnz);
    }
  } catch (...) {
    clair_plan_destroy(pl);
    return CLAIR_ERR_NOMEM;
  }
  *out = pl;
  return CLAIR_OK;
}

int clair_plan_execute(clair_plan_t* pl, int32_t nmat, const clair_csr_t* A, const double* const* B,
                       clair_csr_out_t* R, const clair_opts_t* o, clair_info_t* info) {
  if (!pl || !A || !R || nmat != pl->b.nmat) return CLAIR_ERR_INVALID;
  if (o && o->precision != CLAIR_PREC_MIXED) return CLAIR_ERR_INVALID;
  for (int m = 0; m < nmat; ++m) {
    if (A[m].n != pl->n[m] || A[m].nnz != pl->nnzA[m]) return CLAIR_ERR_INVALID;
    if (A[m].n > 0 && !A[m].row_ptr) return CLAIR_ERR_INVALID;
    if (A[m].nnz > 0 && (!A[m].col_idx || !A[m].val)) return CLAIR_ERR_INVALID;
    if (R[m].row_capacity < (int64_t)pl->n_c[m] + 1 || R[m].nnz_capacity < pl->nnz[m] || !R[m].row_ptr ||
        (pl->nnz[m] > 0 && (!R[m].col_idx || !R[m].val)))
      return CLAIR_ERR_CAPACITY;
  }
  clair_ctx* c = pl->ctx;
  const hipStream_t s = static_cast<hipStream_t>(o ? o->stream : nullptr);
  const bool async = o && o->async;
  const bool timing = o && o->timing;
  Batch b = pl->b;
  // the previous upload must have left the staging buffer before it is rewritten
  if (c->upload_pending) {
    HIPCHK(hipEventSynchronize(c->upload_done));
    c->upload_pending = false;
  }
  // descriptors with the new values, B and R; status and counters as the
  // symbolic phase left them
  char* h = static_cast<char*>(c->stage.p);
  std::memcpy(h, pl->head.data(), pl->head.size());
  MatDesc* hd = reinterpret_cast<MatDesc*>(h);
  b.any_B = false;
  b.cap_sum = 0;
  for (int m = 0; m < nmat; ++m) {
    hd[m].link_base = b.cap_sum;
    b.cap_sum += R[m].nnz_capacity;
    hd[m].rp = A[m].row_ptr;
    hd[m].ci = A[m].col_idx;
    hd[m].va = A[m].val;
    if (pl->ctx->graph.empty()) {  // the search (workgroup rows re-run it) follows the new A
      hd[m].grp = A[m].row_ptr;
      hd[m].gci = A[m].col_idx;
      hd[m].gva = A[m].val;
    }
    hd[m].B = B ? B[m] : nullptr;
    hd[m].Rrp = R[m].row_ptr;
    hd[m].Rci = R[m].col_idx;
    hd[m].Rva = R[m].val;
    hd[m].nnz_cap = R[m].nnz_capacity;
    hd[m].row_cap = R[m].row_capacity;
    b.any_B |= (B && B[m]);
  }
  c->last_nmat = nmat;
  c->last_stream = s;
  c->last_layout = b.L;
  c->last_work = b.w;
  c->last_plain = false;
  int rc = 0;
  if (timing) {
    rc = timing_begin(c, true);
    if (rc) return rc;
  }
  rc = upload(c, b, s);
  if (rc) return rc;
  timing_mark(c, timing, s, "upload");
  // empty the projection's column lists (k_count does that in a full call)
  // and write R.row_ptr[n_c] of the (possibly new) R buffers
  HIPCHK(launch_clear_sums(b.w, b.n_total, occupancy_blocks(c, 4), s));
  if (capture_check(c->capturing, s, "k_clear_sums", __LINE__)) return CLAIR_ERR_HIP;
  timing_mark(c, timing, s, "clear");
  rc = ensure_links(c, b);
  if (rc) return rc;
  const Counters* known = async ? nullptr : reinterpret_cast<const Counters*>(pl->head.data() + (b.L.cnt - b.L.desc));
  rc = enqueue_numeric(c, b, s, timing, known);
  if (rc) return rc;
  if (async) return CLAIR_OK;
  rc = read_status(c, b, s);
  if (rc) return rc;
  const MatStatus* hs = host_status(c, b);
  fill_results(hs, nmat, R, info, A);
  return first_error(hs, nmat);
}

int clair_plan_info(clair_plan_t* pl, int32_t nmat, clair_csr_out_t* R, clair_info_t* info) {
  if (!pl) return CLAIR_ERR_INVALID;
  return clair_ctx_info(pl->ctx, nmat, R, info);
}

void clair_plan_destroy(clair_plan_t* pl) {
  if (!pl) return;
  clair_ctx_destroy(pl->ctx);
  delete pl;
}

const char* clair_last_error(void) { return g_last_error; }

void clair_graph_destroy(clair_graph_t* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  clair_ctx_destroy(g->ctx);
  delete g;
}

// results of the last graph launch
int clair_graph_info(clair_graph_t* g, int32_t nmat, clair_csr_out_t* R, clair_info_t* info) {
  if (!g) return CLAIR_ERR_INVALID;
  return clair_ctx_info(g->ctx, nmat, R, info);
}

const char* clair_strerror(int st) {
  switch (st) {
    case CLAIR_OK: return "ok";
    case CLAIR_ERR_INVALID: return "invalid argument or malformed CSR input";
    case CLAIR_ERR_CAPACITY: return "output capacity too small (required sizes reported)";
    case CLAIR_ERR_SINGULAR: return "singular local block";
    case CLAIR_ERR_HIP: return "HIP runtime error";
    case CLAIR_ERR_UNSUPPORTED: return "unsupported: a neighbourhood larger than CLAIR_MAX_BLOCK, or an input or option this entry point does not take";
    case CLAIR_ERR_NOMEM: return "workspace allocation failed";
    default: return "unknown status";
  }
}

}  // extern "C"
