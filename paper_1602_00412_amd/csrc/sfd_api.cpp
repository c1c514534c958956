// Host orchestrator and C ABI of the Sparse Frequent Directions library (declarations and
// conventions in include/sfd.h).
//
// Device state of a handle: per stream (one for sfd_t, nstreams for sfd_batch_t) the sketch B
// stored transposed as a d x L panel (row-major, L = 32, 64, 128 or 256 >= ell, zero-padded) and the
// pending buffer A' as CSR; and up to kLanes "lanes" shared by the streams.
// A lane is the workspace of one buffer step with its own HIP stream: a CSR view of the buffer,
// its CSC copy and chunk schedules, the SimultaneousIteration panels X (d x L) and Y (m x L),
// P^T (d x L) and the small FP64 work.  The buffer step (Alg 2's flush) is:
//   CSC build -> G (Philox) -> q x { Y = A' X T_x; X = A'^T Y T_y } -> Y = A' X T_x
//   -> P^T = A'^T Y T_y   (T_* = inverse Cholesky factor of the previous panel's Gram)
//   -> eig(P P^T) -> M = H D (so B'^T = P^T M)                     [SparseShrink, Alg 3]
//   -> VerifySpectral on the lane (Alg 6), retry with the next attempt's G on reject [Alg 4]
//   -> DenseShrink (Alg 5) of [B; B'] through the Gram of [B^T | P^T] -> B^T = [B^T | P^T] T2.
// SparseShrink never reads B, so the lanes run the SimultaneousIteration of successive full
// buffers concurrently; VerifySpectral and DenseShrink are issued in buffer order, so the
// persistent VerifySpectral counter and the random draws follow the stream order exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "sfd.h"
#include "sfd_internal.h"

using namespace sfd;

namespace {

constexpr double kAlpha = 6.0 / 41.0;                 // alpha of Alg 4 / Theorem 3.1
constexpr double kUnitRoundoff32 = 1.0 / 16777216.0;  // 2^-24: the panels' arithmetic
constexpr double kCholDropTol = 1e-5;                 // relative residual^2 below which a column is dependent
constexpr int kPurposeSI = 0, kPurposeVS = 1, kPurposeQuerySI = 2, kPurposeQueryVS = 3;
constexpr int kLanes = 16;        // lanes of a batch handle; a single-stream handle uses 4
constexpr int kLanesSingle = 4;
constexpr int kLanesWide = 8;  // a single-stream handle with ell > 128

// State of one stream (Alg 2): the sketch B (stored transposed, d x L), the pending buffer A'
// (CSR), the flush index b, the persistent VerifySpectral counter i and the structural count
// of live rows of B.
struct StreamState {
  uint64_t stream_id = 0;
  int live = 0;
  int64_t flushes = 0, vs_calls = 0;
  sfd_stats_t stats{};
  float* B = nullptr;
  int* prow = nullptr;
  int* pcol = nullptr;
  float* pval = nullptr;
  int pm = 0, pnnz = 0;
  hipEvent_t ev_dsh = nullptr;  // the stream's last DenseShrink (B is current after it)
};

struct Lane {
  hipStream_t st = nullptr;
  // the buffer: CSR view (rowptr may be the lane's own array or the handle's pending buffer)
  int* own_rowptr = nullptr;
  const int* rowptr = nullptr;
  const int* colidx = nullptr;
  const float* val = nullptr;
  int m = 0, nnz = 0;
  int64_t buffer = 0;
  int pg = 0, px = 0;  // purposes of the start block and of the VerifySpectral vector
  int q = 0;
  // CSC and schedules
  int *cscptr = nullptr, *cscrow = nullptr;
  float* cscval = nullptr;
  CscWork csc{};
  int* scan_tmp = nullptr;
  Schedule sr{}, scs{};
  float* partial = nullptr;
  // panels and small work
  float *X = nullptr, *Y = nullptr, *Pt = nullptr;
  uint16_t *Xb = nullptr, *Yb = nullptr;  // BF16 panels of the precision form
  uint16_t *valb = nullptr, *cscvalb = nullptr;  // BF16 copies of the buffer's CSR / CSC values
  float* gram_part = nullptr;
  double *W = nullptr, *W2 = nullptr;
  double *evals = nullptr, *evecs = nullptr, *SS = nullptr, *M64 = nullptr;
  char* eig_work = nullptr;  // workspace of the larger eigensolves (ell or 2 ell > 112)
  double* cholw = nullptr;   // the Cholesky factor between its two passes (ell > 128)
  float *M32 = nullptr, *T = nullptr, *T2 = nullptr;
  float *vs_w = nullptr, *vs_wraw = nullptr, *vs_z = nullptr, *vs_c2 = nullptr, *vs_gpart = nullptr;
  double* vs_npart = nullptr;
  DevScalars* sc = nullptr;
  DevScalars* sc_host = nullptr;  // pinned
  StreamState* ss = nullptr;      // the stream whose buffer the lane holds
  float* Bq = nullptr;            // d x L: a query's copy of B with the pending rows folded in
};

// Workspace of a lockstep group: up to kmax buffers of different streams stacked into one
// block-diagonal buffer (rows one after another, buffer k's columns moved to k d ..), so each
// step of their SimultaneousIteration and VerifySpectral is one launch for all of them.
struct GroupWork {
  int kmax = 0;
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  int *rowptr = nullptr, *colidx = nullptr;
  float* val = nullptr;
  int *cscptr = nullptr, *cscrow = nullptr;
  float* cscval = nullptr;
  CscWork csc{};
  int* scan_tmp = nullptr;
  Schedule sr{}, scs{};
  float* partial = nullptr;
  float *X = nullptr, *Y = nullptr, *Pt = nullptr;
  float* gram_part = nullptr;
  double *W = nullptr, *Wp = nullptr;
  float* T = nullptr;
  double *evals = nullptr, *evecs = nullptr, *M64 = nullptr;
  float* M32 = nullptr;
  char* eig_work = nullptr;  // per buffer: workspace of the ell x ell eigensolve (ell > 112)
  double* cholw = nullptr;   // per buffer: the Cholesky factor between its passes (ell > 128)
  DevScalars* sc = nullptr;
  DevScalars* sc_host = nullptr;  // pinned
  GroupSeg *segs_x = nullptr, *segs_y = nullptr;
  int64_t* seg_rows = nullptr;
  int* tsteps = nullptr;
  int* qdev = nullptr;  // q of each buffer, then the iteration counter (kmax + 1)
  GroupSeg* segs_host = nullptr;  // pinned: 2 kmax segments, kmax + 1 row offsets, kmax steps, kmax q
  float *vs_w = nullptr, *vs_wraw = nullptr, *vs_z = nullptr, *vs_c2 = nullptr, *vs_gpart = nullptr;
  double *vs_npart = nullptr, *fro_part = nullptr;
  int64_t cap_rows = 0, cap_nnz = 0;
};

}  // namespace

struct sfd_s {
  int device = 0;
  hipStream_t user_stream = nullptr;  // the caller's stream (inputs are ordered on it), or null
  int64_t d = 0;
  int ell = 0;
  int L = 0;
  double eps = 0.25;
  uint64_t seed = 0;
  double delta = 0.01;
  int q_override = 0;
  int max_attempts = 16;
  int verify = 1;
  int bands_opt = 0;      // SFD_OPT_CSC_BANDS: 0 automatic, 1 off, kXcdBands on
  int hot_min = kHotMinDefault;  // SFD_OPT_CSC_HOT_MIN
  int64_t hot_cap = 0;           // hot columns a schedule with XCD-local pieces holds: min(d, kHotCap)
  int lanes_alloc = kLanesSingle;  // lanes with workspaces
  int nlanes = kLanesSingle;       // SFD_OPT_LANES: lanes used for successive buffers
  int precision = SFD_PRECISION_FP32;  // SFD_OPT_PRECISION
  int cqr2 = SFD_CQR2_FINAL;           // SFD_OPT_CQR2 (precision form)
  int autotune = 0;                    // SFD_OPT_AUTOTUNE
  int launch = 0;                      // SFD_OPT_PRODUCT_LAUNCH
  int graphs = 1;                      // SFD_OPT_GRAPHS (lockstep groups of a batch handle)
  int algorithm = SFD_ALGO_SFD;        // SFD_OPT_ALGORITHM
  int test_zero_row = -1;              // SFD_OPT_TEST_ZERO_ROW
  int test_zero_attempts = 1;          // SFD_OPT_TEST_ZERO_ATTEMPTS
  // streams (one for an sfd_t handle, nstreams for a batch handle)
  std::vector<StreamState> streams;
  GroupWork grp;  // batch handles: lockstep groups of buffers (grp.kmax = 0: none)
  int error = 0;
  int64_t cap = 0;
  Lane lanes[kLanes];
  // single-stream handles: the sketch and (when a host block could overwrite it) the pending
  // buffer as they were before an append, restored when a BoostedSparseShrink loop is exhausted
  float* Bsave = nullptr;
  int* psave_row = nullptr;
  int* psave_col = nullptr;
  float* psave_val = nullptr;
  int* err_dev = nullptr;
  int64_t* cut_dev = nullptr;
  int64_t cut_cap = 0;
  int64_t* i64_host = nullptr;  // pinned small readbacks
  hipEvent_t ev_in = nullptr;   // caller's stream -> lanes
  std::vector<void*> allocs;
  // per-class profile (SFD_OPT_PROFILE)
  int prof = 0;
  sfd_profile_t profile{};
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
    int launches;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename T>
bool dalloc(sfd_t* h, T** p, int64_t count) {
  void* q = nullptr;
  size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
  if (hipMalloc(&q, bytes) != hipSuccess) return false;
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return true;
}

void free_all(sfd_t* h) {
  for (auto& p : h->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  h->pending.clear();
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  h->ev_pool.clear();
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (Lane& ln : h->lanes) {
    if (ln.sc_host) (void)hipHostFree(ln.sc_host);
    ln.sc_host = nullptr;
    if (ln.st) (void)hipStreamDestroy(ln.st);
    ln.st = nullptr;
  }
  for (StreamState& ss : h->streams) {
    if (ss.ev_dsh) (void)hipEventDestroy(ss.ev_dsh);
    ss.ev_dsh = nullptr;
  }
  if (h->grp.sc_host) (void)hipHostFree(h->grp.sc_host);
  if (h->grp.segs_host) (void)hipHostFree(h->grp.segs_host);
  if (h->grp.st) (void)hipStreamDestroy(h->grp.st);
  if (h->grp.done) (void)hipEventDestroy(h->grp.done);
  h->grp.sc_host = nullptr;
  h->grp.segs_host = nullptr;
  h->grp.st = nullptr;
  h->grp.done = nullptr;
  if (h->i64_host) (void)hipHostFree(h->i64_host);
  h->i64_host = nullptr;
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  h->ev_in = nullptr;
}

int fail(sfd_t* h, int code) {
  if (code == SFD_E_DEVICE) h->error = code;
  return code;
}

#define CK(expr)                                        \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return fail(h, SFD_E_DEVICE); \
  } while (0)

// HIP events bracketing the launches of one kernel class on a lane's stream.
struct ProfScope {
  sfd_t* h;
  hipStream_t st;
  int cls;
  double bytes, flops;
  int launches;
  hipEvent_t a = nullptr;
  static hipEvent_t take(sfd_t* h) {
    if (!h->ev_pool.empty()) {
      hipEvent_t e = h->ev_pool.back();
      h->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ProfScope(sfd_t* h_, hipStream_t st_, int cls_, double bytes_, double flops_ = 0.0, int launches_ = 1)
      : h(h_), st(st_), cls(cls_), bytes(bytes_), flops(flops_), launches(launches_) {
    if (h->prof) {
      a = take(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (!h->prof || !a) return;
    hipEvent_t b = take(h);
    if (!b) {
      h->ev_pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, st);
    h->pending.push_back({cls, a, b, bytes, flops, launches});
  }
};

void prof_resolve(sfd_t* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->profile.ms[p.cls] += ms;
      h->profile.launches[p.cls] += p.launches;
      h->profile.calls[p.cls] += 1;
      h->profile.bytes[p.cls] += p.bytes;
      h->profile.flops[p.cls] += p.flops;
    }
    h->ev_pool.push_back(p.a);
    h->ev_pool.push_back(p.b);
  }
  h->pending.clear();
}

int sync_lane(sfd_t* h, Lane& ln) {
  CK(hipStreamSynchronize(ln.st));
  return SFD_OK;
}

int sync_all(sfd_t* h) {
  for (int i = 0; i < h->lanes_alloc; ++i) CK(hipStreamSynchronize(h->lanes[i].st));
  if (h->grp.st) CK(hipStreamSynchronize(h->grp.st));
  if (!h->pending.empty()) prof_resolve(h);
  return SFD_OK;
}

// the caller's stream must have produced its inputs before any lane reads them
int order_after_caller(sfd_t* h) {
  if (!h->user_stream) return SFD_OK;
  CK(hipEventRecord(h->ev_in, h->user_stream));
  for (int i = 0; i < h->lanes_alloc; ++i) CK(hipStreamWaitEvent(h->lanes[i].st, h->ev_in, 0));
  return SFD_OK;
}

int read_scalars(sfd_t* h, Lane& ln) {
  CK(hipMemcpyAsync(ln.sc_host, ln.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ln.st));
  return sync_lane(h, ln);
}

// Workspaces and stream of one lane (a buffer step in flight).
int alloc_lane(sfd_t* h, Lane& ln) {
  const int64_t d = h->d, L = h->L, cap = h->cap;
  const int64_t tiles = (cap + 2047) / 2048;
  // chunk capacity: one per row (empty rows included) plus the extra chunks of long rows, and
  // for the CSC with XCD-local pieces up to kXcdBands pieces of each of at most hot_cap hot
  // columns; partial slots likewise
  const int64_t max_chunks = d + 2 * cap / kSpmmChunk + kXcdBands * h->hot_cap + 2;
  const int64_t slots = 2 * cap / kSpmmChunk + 16 + kXcdBands * h->hot_cap;
  const int64_t vrows = (int64_t)(kXcdBands + 1) * d + 1;  // chunk-count rows of the hot schedule
  bool ok = true;
  ok = ok && dalloc(h, &ln.own_rowptr, d + 1) && dalloc(h, &ln.Bq, d * L);
  ok = ok && dalloc(h, &ln.cscptr, d + 1) && dalloc(h, &ln.cscrow, cap) && dalloc(h, &ln.cscval, cap);
  ok = ok && dalloc(h, &ln.csc.counts, 1) && dalloc(h, &ln.csc.rowid, cap);
  ok = ok && dalloc(h, &ln.csc.keys0, cap) && dalloc(h, &ln.csc.keys1, cap);
  ok = ok && dalloc(h, &ln.csc.vals0, cap) && dalloc(h, &ln.csc.vals1, cap);
  ok = ok && dalloc(h, &ln.csc.hist, 256 * tiles + 1) && dalloc(h, &ln.csc.part, fro2_part_doubles(1));
  ok = ok && dalloc(h, &ln.scan_tmp, scan_tmp_ints(std::max<int64_t>(256 * tiles + 1, vrows)) + 16);
  ln.csc.scan_tmp = ln.scan_tmp;
  for (Schedule* s : {&ln.sr, &ln.scs}) {
    const int64_t rows = (s == &ln.scs) ? vrows : d + 1;
    ok = ok && dalloc(h, &s->nch, rows) && dalloc(h, &s->pslot, d + 1) && dalloc(h, &s->desc, max_chunks) &&
         dalloc(h, &s->long_rows, d + 1) && dalloc(h, &s->counters, 4) && dalloc(h, &s->regions, kXcdBands + 2) &&
         dalloc(h, &s->queue, kXcdBands + 2);
    s->max_chunks = max_chunks;
  }
  ok = ok && dalloc(h, &ln.sr.stage_idx, cap) && dalloc(h, &ln.sr.hot_cols, 512) && dalloc(h, &ln.sr.hot_n, 34) &&
       dalloc(h, &ln.sr.slot_of, d);
  ok = ok && dalloc(h, &ln.partial, slots * L);
  ln.scs.transposed = true;
  ok = ok && dalloc(h, &ln.X, d * L) && dalloc(h, &ln.Y, d * L) && dalloc(h, &ln.Pt, d * L);
  ok = ok && dalloc(h, &ln.Xb, d * L) && dalloc(h, &ln.Yb, d * L);
  ok = ok && dalloc(h, &ln.valb, cap) && dalloc(h, &ln.cscvalb, cap);
  ok = ok && dalloc(h, &ln.gram_part, (int64_t)gram_max_blocks() * 4 * L * L) && dalloc(h, &ln.W, L * L) &&
       dalloc(h, &ln.W2, 4 * L * L);
  ok = ok && dalloc(h, &ln.evals, 2 * L) && dalloc(h, &ln.evecs, 4 * L * L) && dalloc(h, &ln.SS, 4 * L * L);
  ok = ok && dalloc(h, &ln.eig_work, std::max(eig_work_bytes(h->ell), eig_work_bytes(2 * h->ell)));
  ok = ok && dalloc(h, &ln.cholw, chol_work_doubles(h->L));
  ok = ok && dalloc(h, &ln.M64, L * L) && dalloc(h, &ln.M32, L * L) && dalloc(h, &ln.T, L * L) &&
       dalloc(h, &ln.T2, 2 * L * L);
  ok = ok && dalloc(h, &ln.vs_w, d) && dalloc(h, &ln.vs_wraw, d) && dalloc(h, &ln.vs_z, d) &&
       dalloc(h, &ln.vs_c2, 2 * L) && dalloc(h, &ln.vs_gpart, (int64_t)gemv_blocks(d) * L) &&
       dalloc(h, &ln.vs_npart, 2048);
  ok = ok && dalloc(h, &ln.sc, 1);
  if (!ok) return SFD_E_NOMEM;
  if (hipHostMalloc((void**)&ln.sc_host, sizeof(DevScalars)) != hipSuccess) return SFD_E_NOMEM;
  if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess) return SFD_E_DEVICE;
  return SFD_OK;
}

int alloc_state(sfd_t* h) {
  const int64_t d = h->d, L = h->L;
  const int64_t cap = h->ell * d + d;
  h->cap = cap;
  h->hot_cap = std::min<int64_t>(d, kHotCap);
  bool ok = true;
  for (StreamState& ss : h->streams) {
    ok = ok && dalloc(h, &ss.B, d * L);
    ok = ok && dalloc(h, &ss.prow, d + 1) && dalloc(h, &ss.pcol, cap) && dalloc(h, &ss.pval, cap);
    if (!ok) return SFD_E_NOMEM;
    if (hipEventCreateWithFlags(&ss.ev_dsh, hipEventDisableTiming) != hipSuccess) return SFD_E_DEVICE;
  }
  if (h->streams.size() == 1) ok = ok && dalloc(h, &h->Bsave, d * L);
  ok = ok && dalloc(h, &h->err_dev, 4);
  if (!ok) return SFD_E_NOMEM;
  for (int li = 0; li < h->lanes_alloc; ++li) {
    int rc = alloc_lane(h, h->lanes[li]);
    if (rc) return rc;
  }
  if (hipHostMalloc((void**)&h->i64_host, sizeof(int64_t) * 16) != hipSuccess) return SFD_E_NOMEM;
  if (hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess) return SFD_E_DEVICE;
  return SFD_OK;
}

int reset_state(sfd_t* h) {
  h->error = 0;
  Lane& l0 = h->lanes[0];
  int rc = sync_all(h);
  if (rc) return rc;
  for (StreamState& ss : h->streams) {
    ss.live = 0;
    ss.flushes = 0;
    ss.vs_calls = 0;
    ss.pm = 0;
    ss.pnnz = 0;
    std::memset(&ss.stats, 0, sizeof(ss.stats));
    CK(fill_f32(ss.B, h->d * h->L, 0.f, l0.st));
    CK(fill_i32(ss.prow, 1, 0, l0.st));
    CK(hipEventRecord(ss.ev_dsh, l0.st));
  }
  return sync_all(h);
}

int si_iterations(const sfd_t* h, int m) {
  if (h->q_override > 0) return h->q_override;
  return (int)std::ceil(std::log((double)m / h->eps) / h->eps);
}

// Alg 2's flush rule: rows(A') = d or nnz(A') >= ell*d; FrequentDirections (Sec. 2.1) in
// batches of ell rows: rows(A') = ell, each buffer folded exactly by DenseShrink.
int64_t flush_rows(const sfd_t* h) { return h->algorithm == SFD_ALGO_FD ? (int64_t)h->ell : h->d; }
int64_t flush_nnz(const sfd_t* h) {
  return h->algorithm == SFD_ALGO_FD ? ((int64_t)1 << 62) : (int64_t)h->ell * h->d;
}

int vs_steps(const sfd_t* h, int64_t i) {
  double di = h->delta / (2.0 * (double)i * (double)i);
  return (int)std::ceil(std::log2((double)h->d / di));
}

// algorithmic bytes of one sparse product over the buffer: the stored entries (id + value)
// and row pointers once, the input panel read once, the output panel written once (bx, by:
// bytes per panel element; bv: bytes per stored value)
double spmm_bytes(const sfd_t* h, const Lane& ln, bool transposed, double bx, double by, double bv) {
  const double N = ln.nnz, m = ln.m, d = (double)h->d, ell = h->ell;
  const double in_rows = transposed ? m : d, out_rows = transposed ? d : m;
  return (4.0 + bv) * N + 4.0 * (out_rows + 1) + ell * (bx * in_rows + by * out_rows);
}

inline double pbytes(PanelType t) { return t == PanelType::BF16 ? 2.0 : 4.0; }

// ---- Autotuner of the sparse products' launch configuration (SFD_OPT_AUTOTUNE).  A product is
// keyed by its panel width, direction, element types, XCD-local pieces and the binary orders of
// magnitude of its stored entries and of its input and output rows.  The first product with a
// new key runs every candidate configuration three times on its real operands, alone on the
// device (all give the same bits, so the extra runs change nothing but the time), with HIP events
// around each, and the fastest (by its best run) is kept for the process, and appended to the file named by the environment variable
// SFD_TUNE_CACHE when it is set (read back at the first use, so a later process starts tuned).
using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int>;

struct Tuner {
  std::mutex mu;
  std::map<TuneKey, SpmmConfig> best;
  bool loaded = false;
  void load() {
    if (loaded) return;
    loaded = true;
    const char* path = std::getenv("SFD_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    int k[9], u, qu, oc, sg;
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6],
                       &k[7], &k[8], &u, &qu, &oc, &sg) == 13) {
      SpmmConfig c;
      c.unroll = u;
      c.queue = qu != 0;
      c.occupancy = oc;
      c.stage = sg != 0;
      best[TuneKey{k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8]}] = c;
    }
    std::fclose(f);
  }
  void store(const TuneKey& key, const SpmmConfig& c) {
    best[key] = c;
    const char* path = std::getenv("SFD_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(key), std::get<1>(key), std::get<2>(key),
                 std::get<3>(key), std::get<4>(key), std::get<5>(key), std::get<6>(key), std::get<7>(key),
                 std::get<8>(key), c.unroll, c.queue ? 1 : 0, c.occupancy, c.stage ? 1 : 0);
    std::fclose(f);
  }
};
Tuner g_tuner;

inline int log2_bucket(int64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

// The launch of a product (s, idx, val, X -> Y) on stream st: the one SFD_OPT_PRODUCT_LAUNCH forces,
// else the tuned one with SFD_OPT_AUTOTUNE (tuning first when the key is new), else the static
// grid.  Not during stream capture (tuning synchronises).
int product_config_tuned(sfd_t* h, hipStream_t st, const Schedule& s, const int* idx, const void* val, bool vb,
                         const void* X, PanelType xt, void* Y, PanelType yt, float* partial, int64_t in_rows,
                         int64_t nnz, SpmmConfig* out) {
  *out = SpmmConfig{};
  if (h->launch > 0) {
    // a fixed launch: static grid, work-queue grid, or work-queue grid staging (where possible)
    out->queue = h->launch >= 2;
    out->stage = h->launch == 3 && !s.transposed && s.stage_idx != nullptr;
    return SFD_OK;
  }
  if (!h->autotune) return SFD_OK;
  const bool can_stage = !s.transposed && s.stage_idx != nullptr;
  const TuneKey key{h->L, s.transposed ? 1 : 0, (int)xt, (int)yt, vb ? 1 : 0, (s.nlocal > 0 ? 1 : 0) + (can_stage ? 2 : 0),
                    log2_bucket(nnz), log2_bucket(in_rows), log2_bucket(s.rows)};
  std::lock_guard<std::mutex> lock(g_tuner.mu);
  g_tuner.load();
  auto it = g_tuner.best.find(key);
  if (it != g_tuner.best.end()) {
    *out = it->second;
    return SFD_OK;
  }
  std::vector<SpmmConfig> cand;
  for (int q = 0; q < 3; ++q) {
    if (q == 2 && !can_stage) continue;
    for (int u : {8, 4}) {
      if (xt == PanelType::BF16 && u != 4) continue;  // BF16 panels gather in batches of 4 only
      SpmmConfig c;
      c.unroll = xt == PanelType::BF16 ? 0 : u;
      c.queue = q != 0;    // 1: work-queue grid
      c.stage = q == 2;    // 2: work-queue grid with the popular rows of X staged in LDS
      cand.push_back(c);
    }
  }
  // measured alone: the work of the other lanes and streams finishes first, so the candidates'
  // times are not mixed with theirs (once per key, in a warm-up)
  CK(hipDeviceSynchronize());
  hipEvent_t a = nullptr, b = nullptr;
  CK(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return SFD_E_DEVICE;
  }
  std::vector<float> best_ms(cand.size(), 1e30f);
  hipError_t e = hipSuccess;
  for (int round = 0; round < 3 && e == hipSuccess; ++round) {
    for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
      if ((e = spmm_queue_reset(s, st)) != hipSuccess) break;
      if ((e = hipEventRecord(a, st)) != hipSuccess) break;
      if ((e = spmm(s, idx, val, vb, X, xt, h->L, Y, yt, h->L, h->L, partial, cand[i], st)) != hipSuccess) break;
      if ((e = hipEventRecord(b, st)) != hipSuccess) break;
      if ((e = hipEventSynchronize(b)) != hipSuccess) break;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
      best_ms[i] = std::min(best_ms[i], ms);
    }
  }
  if (e == hipSuccess) e = spmm_queue_reset(s, st);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return SFD_E_DEVICE;
  size_t bi = 0;
  for (size_t i = 1; i < cand.size(); ++i)
    if (best_ms[i] < best_ms[bi]) bi = i;
  g_tuner.store(key, cand[bi]);
  *out = cand[bi];
  return SFD_OK;
}

// The configuration of a product: its launch (above), gathering only the 16-byte segments of a
// panel row that reach the 64-byte sector holding column ell - 1 (the columns past ell are zero in
// every panel, so the results are the same bits).
int product_config(sfd_t* h, hipStream_t st, const Schedule& s, const int* idx, const void* val, bool vb,
                   const void* X, PanelType xt, void* Y, PanelType yt, float* partial, int64_t in_rows, int64_t nnz,
                   SpmmConfig* out) {
  const int rc = product_config_tuned(h, st, s, idx, val, vb, X, xt, Y, yt, partial, in_rows, nnz, out);
  out->live = live_segments(h->ell, (int)pbytes(xt));
  return rc;
}

// `body` (launches on st only, no host synchronisation) run n times: captured once as a HIP graph
// and launched n times when SFD_OPT_GRAPHS is on, else issued n times (also while the per-class
// profile is on: its events bracket each launch).
template <class F>
int replay(sfd_t* h, hipStream_t st, int n, F&& body) {
  if (n <= 0) return SFD_OK;
  if (!h->graphs || h->prof || n == 1) {
    for (int i = 0; i < n; ++i) {
      int rc = body();
      if (rc) return rc;
    }
    return SFD_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = body();
  const hipError_t ce = hipStreamEndCapture(st, &graph);
  if (rc || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : SFD_E_DEVICE;
  }
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  for (int i = 0; i < n && e == hipSuccess; ++i) e = hipGraphLaunch(exec, st);
  if (exec) (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  return e == hipSuccess ? SFD_OK : SFD_E_DEVICE;
}

// The output of a product whose input panel had transform T (the lane's current one):
// panel <- panel T (so the product becomes A' (X T), resp. A'^T (Y T)), then the new T from
// the transformed panel's Gram.
int orth_out(sfd_t* h, Lane& ln, void* panel, PanelType pt, int64_t rows) {
  const int L = h->L;
  const double ell = h->ell;
  {
    // flops the method needs: panel x triangular T and the symmetric Gram, rows ell (ell + 1) each
    ProfScope ps(h, ln.st, SFD_PROF_GRAM, 2.0 * pbytes(pt) * rows * ell, 2.0 * rows * ell * (ell + 1), 2);
    CK(xform_gram(panel, pt, L, rows, L, ln.T, ln.gram_part, ln.W, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_CHOL, 8.0 * ell * ell, ell * ell * ell, 1);
    CK(chol_inv(ln.W, L, h->ell, L, kCholDropTol, ln.T, ln.sc, ln.cholw, ln.st));
  }
  return SFD_OK;
}

// Y = A' X (the input's transform is applied to Y by orth_out); vb: BF16 values
int spmm_csr(sfd_t* h, Lane& ln, const void* X, PanelType xt, void* Y, PanelType yt, bool vb = false) {
  const void* val = vb ? static_cast<const void*>(ln.valb) : static_cast<const void*>(ln.val);
  SpmmConfig cfg;
  int rc = product_config(h, ln.st, ln.sr, ln.colidx, val, vb, X, xt, Y, yt, ln.partial, h->d, ln.nnz, &cfg);
  if (rc) return rc;
  {
    ProfScope ps(h, ln.st, SFD_PROF_SPMM_CSR, spmm_bytes(h, ln, false, pbytes(xt), pbytes(yt), vb ? 2.0 : 4.0),
                 2.0 * ln.nnz * h->ell + 2.0 * ln.m * h->ell * h->ell, 1);
    CK(spmm(ln.sr, ln.colidx, val, vb, X, xt, h->L, Y, yt, h->L, h->L, ln.partial, cfg, ln.st));
  }
  ProfScope ps(h, ln.st, SFD_PROF_FIXUP, 0.0, 0.0, 1);
  CK(spmm_finish(ln.sr, ln.partial, Y, yt, h->L, h->L, ln.st));
  return SFD_OK;
}

// X = A'^T Y; vb: BF16 values
int spmm_csc(sfd_t* h, Lane& ln, const void* Y, PanelType yt, void* X, PanelType xt, bool vb = false) {
  const void* val = vb ? static_cast<const void*>(ln.cscvalb) : static_cast<const void*>(ln.cscval);
  SpmmConfig cfg;
  int rc = product_config(h, ln.st, ln.scs, ln.cscrow, val, vb, Y, yt, X, xt, ln.partial, ln.m, ln.nnz, &cfg);
  if (rc) return rc;
  {
    ProfScope ps(h, ln.st, SFD_PROF_SPMM_CSC, spmm_bytes(h, ln, true, pbytes(yt), pbytes(xt), vb ? 2.0 : 4.0),
                 2.0 * ln.nnz * h->ell + 2.0 * h->d * h->ell * h->ell, 1);
    CK(spmm(ln.scs, ln.cscrow, val, vb, Y, yt, h->L, X, xt, h->L, h->L, ln.partial, cfg, ln.st));
  }
  ProfScope ps(h, ln.st, SFD_PROF_FIXUP, 0.0, 0.0, 1);
  CK(spmm_finish(ln.scs, ln.partial, X, xt, h->L, h->L, ln.st));
  return SFD_OK;
}

// XCD-local pieces of the hot columns for the transposed products of a buffer of m rows
// (SFD_OPT_CSC_BANDS): automatic when the gathered panel (m rows of the panel width) is larger
// than one XCD's L2 (4 MB) and one band of it (an eighth) still fits in twice that; the lockstep
// groups of a batch handle build plain schedules, so such buffers take the lanes there.
bool csc_hot(const sfd_t* h, int64_t m, int64_t nnz) {
  if (m <= h->ell || nnz == 0 || h->bands_opt == 1) return false;
  if (h->bands_opt == kXcdBands) return true;
  const int64_t bytes = m * h->L * (h->precision == SFD_PRECISION_BF16 ? 2 : 4);
  return bytes > ((int64_t)4 << 20) && bytes <= ((int64_t)64 << 20);
}

// Buffer set-up on the lane: CSC (with ||A'||_F^2) and, for m > ell, the chunk schedules.
int prepare(sfd_t* h, Lane& ln) {
  const int64_t d = h->d;
  {
    ProfScope ps(h, ln.st, SFD_PROF_CSC_BUILD, 16.0 * ln.nnz + 4.0 * (ln.m + d), 0.0, 1);
    const int* keys = nullptr;
    CK(build_csc(ln.rowptr, ln.colidx, ln.val, ln.m, ln.nnz, d, ln.cscptr, ln.cscrow, ln.cscval, ln.csc, &keys,
                 ln.st));
    CK(fro2_segments(ln.cscptr, keys, ln.cscrow, ln.cscval, d, 1, ln.csc.part, ln.sc, ln.st));
  }
  if (ln.m > h->ell) {
    ProfScope ps(h, ln.st, SFD_PROF_OTHER, 0.0, 0.0, 2);
    if (h->precision == SFD_PRECISION_BF16) {
      // the precision form's products 1 .. 2q+1 read BF16 copies of the values
      CK(to_bf16(ln.val, ln.nnz, ln.valb, ln.st));
      CK(to_bf16(ln.cscval, ln.nnz, ln.cscvalb, ln.st));
    }
    ln.sr.max_chunks = (int64_t)ln.m + (int64_t)ln.nnz / kSpmmChunk + 2;
    CK(schedule_build(ln.rowptr, ln.m, ln.sr, ln.scan_tmp, ln.st));
    // the rows a product Y = A' X may stage in LDS (a launch candidate of the autotuner)
    if (h->autotune || h->launch == 3)
      CK(stage_build(ln.cscptr, (int)d, ln.colidx, ln.nnz, h->L, h->precision == SFD_PRECISION_BF16, ln.sr, ln.st));
    if (csc_hot(h, ln.m, ln.nnz)) {
      // at most nnz / hot columns reach `hot`, so at most hot_cap
      const int64_t hot = std::max<int64_t>(h->hot_min, (ln.nnz + h->hot_cap - 1) / h->hot_cap);
      ln.scs.max_chunks = d + 2 * (int64_t)ln.nnz / kSpmmChunk + kXcdBands * std::min<int64_t>(d, ln.nnz / hot) + 2;
      CK(schedule_build_hot(ln.cscptr, ln.cscrow, (int)d, ln.rowptr, ln.m, ln.nnz, (int)hot, ln.scs, ln.scan_tmp,
                            ln.st));
    } else {
      ln.scs.max_chunks = d + (int64_t)ln.nnz / kSpmmChunk + 2;
      CK(schedule_build(ln.cscptr, (int)d, ln.scs, ln.scan_tmp, ln.st));
    }
  }
  return SFD_OK;
}

// SparseShrink (Alg 3) of the lane's buffer with the start block of `attempt`: leaves P^T in
// ln.Pt, M = H D and the scalars of Alg 4 (S, Delta/2) on the device.  Asynchronous.
int sparse_shrink(sfd_t* h, Lane& ln, int attempt) {
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  const int m = ln.m;
  int rc;
  {
    ProfScope ps(h, ln.st, SFD_PROF_OTHER, 4.0 * d * ell, 0.0, 2);
    CK(fill_f32(ln.X, d * L, 0.f, ln.st));
    CK(start_block(h->seed, ln.ss->stream_id, (uint64_t)ln.buffer, (uint64_t)attempt, (uint64_t)ln.pg, d, ell, ln.X,
                   L, ln.st));
    if (h->test_zero_row >= 0 && h->test_zero_row < d && attempt < h->test_zero_attempts)
      CK(fill_f32(ln.X + (int64_t)h->test_zero_row * L, L, 0.f, ln.st));
  }
  // panels of the iteration: FP32, or BF16 in the precision form, where the products 1 .. 2q+1
  // read BF16 values and BF16 panels and write BF16 panels (FP32 accumulation; transforms and
  // Grams on BF16 MFMA), and the last one, P^T = A'^T Y T_y, reads the FP32 values and the stored
  // BF16 Y with T_y from that Y's own Gram and writes FP32: P P^T is then the compression of
  // A'^T A' onto span(Y), so B'^T B' <= A'^T A' still holds for the FP32 values.  CholeskyQR2
  // (SFD_OPT_CQR2): a second transform + Gram + Cholesky of a stored panel, so the panel kept in
  // BF16 is orthonormal to BF16 precision, not only to that times its condition number
  const bool bf = h->precision == SFD_PRECISION_BF16;
  const PanelType pt = bf ? PanelType::BF16 : PanelType::F32;
  void* X = bf ? static_cast<void*>(ln.Xb) : static_cast<void*>(ln.X);
  void* Y = bf ? static_cast<void*>(ln.Yb) : static_cast<void*>(ln.Y);
  const bool cqr2_all = bf && h->cqr2 == SFD_CQR2_ALL;
  const bool cqr2_final = bf && h->cqr2 != SFD_CQR2_OFF;
  if (bf) CK(to_bf16(ln.X, d * L, ln.Xb, ln.st));
  // the first transform from the Gram of G itself (G T = G with T = I)
  CK(set_identity(ln.T, L, 1, ln.st));
  if ((rc = orth_out(h, ln, X, pt, d))) return rc;
  // the products' launch configurations before any capture (tuning synchronises); the transposed
  // product's candidates write P^T, which the last product overwrites
  if (ln.q > 0) {
    SpmmConfig c;
    const void* vr = bf ? static_cast<const void*>(ln.valb) : static_cast<const void*>(ln.val);
    const void* vc = bf ? static_cast<const void*>(ln.cscvalb) : static_cast<const void*>(ln.cscval);
    if ((rc = product_config(h, ln.st, ln.sr, ln.colidx, vr, bf, X, pt, Y, pt, ln.partial, d, ln.nnz, &c))) return rc;
    if ((rc = product_config(h, ln.st, ln.scs, ln.cscrow, vc, bf, Y, pt, ln.Pt, pt, ln.partial, m, ln.nnz, &c)))
      return rc;
  }
  // one iteration: Y = A' X T_x, X = A'^T Y T_y with their CholeskyQR steps -- the same launches
  // with the same arguments every time, so with SFD_OPT_GRAPHS it is captured once and replayed
  auto iteration = [&]() -> int {
    int r;
    if ((r = spmm_csr(h, ln, X, pt, Y, pt, bf))) return r;
    if ((r = orth_out(h, ln, Y, pt, m))) return r;
    if (cqr2_all && (r = orth_out(h, ln, Y, pt, m))) return r;
    if ((r = spmm_csc(h, ln, Y, pt, X, pt, bf))) return r;
    if ((r = orth_out(h, ln, X, pt, d))) return r;
    if (cqr2_all && (r = orth_out(h, ln, X, pt, d))) return r;
    return SFD_OK;
  };
  if ((rc = replay(h, ln.st, ln.q, iteration))) return rc;
  if ((rc = spmm_csr(h, ln, X, pt, Y, pt, bf))) return rc;
  if ((rc = orth_out(h, ln, Y, pt, m))) return rc;
  if (cqr2_final && (rc = orth_out(h, ln, Y, pt, m))) return rc;
  if ((rc = spmm_csc(h, ln, Y, pt, ln.Pt, PanelType::F32))) return rc;
  {
    // P^T <- P^T T_y and W = P P^T
    ProfScope ps(h, ln.st, SFD_PROF_GRAM, 8.0 * d * ell, 2.0 * d * ell * (ell + 1), 2);
    CK(xform_gram(ln.Pt, PanelType::F32, L, d, L, ln.T, ln.gram_part, ln.W, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_EIG, 16.0 * ell * ell, 0.0, 1);
    CK(eig_sym(ln.W, L, ell, ell, ln.evals, ln.evecs, ln.eig_work, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(ssh_post(ln.evals, ln.evecs, ell, L, kAlpha, ln.M64, ln.M32, ln.sc, ln.st));
  }
  return SFD_OK;
}

// VerifySpectral (Alg 6): t power steps from the sphere vector of (buffer, attempt); leaves
// ln ||C^t x|| in ln.sc.  Asynchronous.
int verify_spectral(sfd_t* h, Lane& ln, int attempt, int t) {
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  const int m = ln.m;
  ProfScope ps(h, ln.st, SFD_PROF_VS, t * (16.0 * ln.nnz + 8.0 * d * ell + 4.0 * (2.0 * m + 6.0 * d)),
               t * (4.0 * ln.nnz + 4.0 * d * ell), 8 * t + 3);
  CK(start_block(h->seed, ln.ss->stream_id, (uint64_t)ln.buffer, (uint64_t)attempt, (uint64_t)ln.px, d, 1, ln.vs_w,
                 1, ln.st));
  CK(vs_init(ln.vs_w, d, ln.vs_npart, ln.sc, ln.st));
  // one power step (the same launches every step: captured once and replayed with SFD_OPT_GRAPHS)
  auto power_step = [&]() -> int {
    CK(spmv(ln.rowptr, ln.colidx, ln.val, ln.sr, ln.vs_w, &ln.sc->inv_norm, ln.vs_z, ln.partial, ln.st));
    CK(panel_gemv_t(ln.Pt, L, L, d, ln.vs_w, &ln.sc->inv_norm, ln.vs_gpart, ln.st));
    CK(spmv(ln.cscptr, ln.cscrow, ln.cscval, ln.scs, ln.vs_z, nullptr, ln.vs_wraw, ln.partial, ln.st));
    CK(vs_small(ln.vs_gpart, gemv_blocks(d), ln.M64, ell, L, ln.vs_c2, ln.st));
    CK(vs_finish(ln.vs_wraw, ln.Pt, L, L, ell, ln.vs_c2, d, ln.vs_w, ln.vs_npart, ln.st));
    CK(vs_norm(ln.vs_npart, vs_finish_blocks(d), ln.sc, ln.st));
    return SFD_OK;
  };
  return replay(h, ln.st, t, power_step);
}

// Issue everything of a buffer step that does not depend on B or on the VerifySpectral counter.
int issue_shrink(sfd_t* h, Lane& ln) {
  int rc = prepare(h, ln);
  if (rc) return rc;
  if (ln.m <= h->ell) {
    // exact buffer (SparseShrink needs ell <= m): P^T = A'^T, M = I
    CK(dense_from_csc(ln.cscptr, ln.cscrow, ln.cscval, h->d, ln.Pt, h->L, h->L, ln.st));
    CK(ssh_identity(h->ell, h->L, ln.M64, ln.M32, ln.sc, ln.st));
    return SFD_OK;
  }
  ln.q = si_iterations(h, ln.m);
  return sparse_shrink(h, ln, 0);
}

// DenseShrink (Alg 5) of [B; B'] with B'^T = P^T M (M = I for an exact block); the stack is
// kept exactly when it has at most ell live rows.  B is read from `Bin`, the result goes to
// `out` (both d x L).  Waits for the previous DenseShrink and records its own completion.
int dense_shrink(sfd_t* h, Lane& ln, const float* Bin, const float* Pt, int lossless, float* out,
                 const double* M64 = nullptr) {
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  if (!M64) M64 = ln.M64;
  CK(hipStreamWaitEvent(ln.st, ln.ss->ev_dsh, 0));
  {
    // the symmetric Gram of the d x 2 ell stack [B^T | P^T]
    ProfScope ps(h, ln.st, SFD_PROF_GRAM, 8.0 * d * ell, 2.0 * d * ell * (2.0 * ell + 1), 2);
    CK(gram2(Bin, L, Pt, L, d, L, ln.gram_part, ln.W2, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(dsh_assemble(ln.W2, L, ell, M64, ln.SS, ln.evecs, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_EIG, 64.0 * ell * ell, 0.0, 1);
    // only the ell leading eigenvectors enter the new sketch
    CK(eig_sym(ln.SS, 2 * ell, 2 * ell, ell, ln.evals, ln.evecs, ln.eig_work, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(dsh_post(ln.evals, ln.evecs, ell, L, M64, lossless, ln.T2, ln.sc, ln.st));
  }
  {
    ProfScope ps(h, ln.st, SFD_PROF_XFORM, 12.0 * d * ell, 4.0 * d * ell * ell, 1);
    CK(panel_xform2(Bin, L, Pt, L, L, ln.T2, out, L, d, ln.st));
  }
  CK(hipEventRecord(ln.ss->ev_dsh, ln.st));
  return SFD_OK;
}

// The in-order part of a buffer step: BoostedSparseShrink's acceptance (Alg 4, with the
// VerifySpectral counter continued from vs_base) and the DenseShrink into `out`.
// *live = structural live rows of the result, *calls = VerifySpectral calls made.
// (a0 > 0: attempts 0 .. a0 - 1 were made and rejected elsewhere, with calls0 VerifySpectral
// calls; attempt a0's SparseShrink has been issued on the lane)
int finish_step(sfd_t* h, Lane& ln, int64_t vs_base, int live_in, const float* Bin, float* out, int* live,
                int64_t* calls, int a0 = 0, int64_t calls0 = 0) {
  const int ell = h->ell;
  int rc;
  *calls = calls0;
  int r_add;
  if (ln.m <= ell) {
    r_add = ln.m;
  } else {
    bool accepted = false;
    for (int a = a0;; ++a) {
      if ((rc = read_scalars(h, ln))) return rc;
      const DevScalars s = *ln.sc_host;
      sfd_stats_t& stats = ln.ss->stats;
      stats.attempts += 1;
      stats.last_q = ln.q;
      stats.last_fro2_buffer = s.fro2A;
      stats.last_lambda_ell2 = s.lam_ell2;
      stats.last_delta = 2.0 * s.half_delta;
      if (s.S <= 64.0 * kUnitRoundoff32 * ell * s.fro2A || !h->verify) {
        accepted = true;
        break;
      }
      *calls += 1;
      const int t = vs_steps(h, vs_base + *calls);
      if ((rc = verify_spectral(h, ln, a, t))) return rc;
      if ((rc = read_scalars(h, ln))) return rc;
      const double ln_norm = ln.sc_host->ln_norm;
      ln.ss->stats.last_t = t;
      ln.ss->stats.last_ln_norm = ln_norm;
      if (ln_norm <= 0.0) {
        accepted = true;
        break;
      }
      ln.ss->stats.vs_rejects += 1;
      if (a + 1 >= h->max_attempts) break;
      if ((rc = sparse_shrink(h, ln, a + 1))) return rc;
    }
    if (!accepted) return SFD_E_NOCONVERGE;
    r_add = ell - 1;
  }
  const int lossless = (live_in + r_add <= ell) ? 1 : 0;
  if ((rc = dense_shrink(h, ln, Bin, ln.Pt, lossless, out))) return rc;
  *live = lossless ? live_in + r_add : ell - 1;
  return SFD_OK;
}

// Group workspace for up to kmax buffers (batch handles).
int alloc_group(sfd_t* h, int kmax) {
  GroupWork& g = h->grp;
  const int64_t d = h->d, L = h->L, cap = h->cap;
  g.kmax = kmax;
  g.cap_rows = kmax * d;
  g.cap_nnz = kmax * cap;
  const int64_t tiles = (g.cap_nnz + 2047) / 2048;
  const int64_t max_chunks = g.cap_rows + g.cap_nnz / kSpmmChunk + 2;
  bool ok = true;
  ok = ok && dalloc(h, &g.rowptr, g.cap_rows + 1) && dalloc(h, &g.colidx, g.cap_nnz) && dalloc(h, &g.val, g.cap_nnz);
  ok = ok && dalloc(h, &g.cscptr, kmax * d + 1) && dalloc(h, &g.cscrow, g.cap_nnz) && dalloc(h, &g.cscval, g.cap_nnz);
  ok = ok && dalloc(h, &g.csc.counts, 1) && dalloc(h, &g.csc.rowid, g.cap_nnz);
  ok = ok && dalloc(h, &g.csc.keys0, g.cap_nnz) && dalloc(h, &g.csc.keys1, g.cap_nnz);
  ok = ok && dalloc(h, &g.csc.vals0, g.cap_nnz) && dalloc(h, &g.csc.vals1, g.cap_nnz);
  ok = ok && dalloc(h, &g.csc.hist, 256 * tiles + 1) && dalloc(h, &g.csc.part, 1024);
  ok = ok && dalloc(h, &g.scan_tmp, scan_tmp_ints(std::max<int64_t>(256 * tiles + 1, g.cap_rows + 1)) + 16);
  g.csc.scan_tmp = g.scan_tmp;
  for (Schedule* sch : {&g.sr, &g.scs}) {
    const int64_t rows = g.cap_rows + 1;
    ok = ok && dalloc(h, &sch->nch, rows) && dalloc(h, &sch->pslot, rows) && dalloc(h, &sch->desc, max_chunks) &&
         dalloc(h, &sch->long_rows, rows) && dalloc(h, &sch->counters, 4) && dalloc(h, &sch->regions, kXcdBands + 2) &&
         dalloc(h, &sch->queue, kXcdBands + 2);
    sch->max_chunks = max_chunks;
  }
  g.scs.transposed = true;
  ok = ok && dalloc(h, &g.partial, (2 * g.cap_nnz / kSpmmChunk + 16) * L);
  ok = ok && dalloc(h, &g.X, kmax * d * L) && dalloc(h, &g.Y, kmax * d * L) && dalloc(h, &g.Pt, kmax * d * L);
  ok = ok && dalloc(h, &g.gram_part, kmax * gram_partial_stride((int)L));
  ok = ok && dalloc(h, &g.W, kmax * L * L) && dalloc(h, &g.Wp, kmax * L * L) && dalloc(h, &g.T, kmax * L * L);
  ok = ok && dalloc(h, &g.evals, kmax * 2 * L) && dalloc(h, &g.evecs, kmax * 4 * L * L);
  ok = ok && dalloc(h, &g.M64, kmax * L * L) && dalloc(h, &g.M32, kmax * L * L) && dalloc(h, &g.sc, kmax);
  ok = ok && dalloc(h, &g.eig_work, kmax * eig_work_bytes(h->ell)) &&
       dalloc(h, &g.cholw, kmax * chol_work_doubles((int)L));
  ok = ok && dalloc(h, &g.segs_x, kmax) && dalloc(h, &g.segs_y, kmax) && dalloc(h, &g.seg_rows, kmax + 1) &&
       dalloc(h, &g.tsteps, kmax) && dalloc(h, &g.qdev, kmax + 1);
  ok = ok && dalloc(h, &g.vs_w, kmax * d) && dalloc(h, &g.vs_wraw, kmax * d) && dalloc(h, &g.vs_z, g.cap_rows) &&
       dalloc(h, &g.vs_c2, kmax * 2 * L) && dalloc(h, &g.vs_gpart, kmax * gemv_blocks(d) * L) &&
       dalloc(h, &g.vs_npart, kmax * 1024) && dalloc(h, &g.fro_part, fro2_part_doubles(kmax));
  if (!ok) return SFD_E_NOMEM;
  if (hipHostMalloc((void**)&g.sc_host, sizeof(DevScalars) * kmax) != hipSuccess) return SFD_E_NOMEM;
  const size_t hbytes = sizeof(GroupSeg) * 2 * kmax + sizeof(int64_t) * (kmax + 1) + sizeof(int) * 2 * kmax;
  if (hipHostMalloc((void**)&g.segs_host, hbytes) != hipSuccess) return SFD_E_NOMEM;
  if (hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking) != hipSuccess) return SFD_E_DEVICE;
  if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) return SFD_E_DEVICE;
  return SFD_OK;
}

// A buffer of a stream: a CSR view plus where its rows come from.
struct BufferView {
  StreamState* ss;
  const int* rowptr;      // int32 row pointers (if already rebased), else nullptr
  const int64_t* indptr;  // caller's int64 row pointers to rebase from (device), or nullptr
  int64_t r0;             // first row in indptr
  const int* colidx;
  const float* val;
  int m, nnz;
};

int bind(sfd_t* h, Lane& ln, const BufferView& v, int64_t buffer, int pg, int px) {
  ln.ss = v.ss;
  ln.m = v.m;
  ln.nnz = v.nnz;
  ln.colidx = v.colidx;
  ln.val = v.val;
  ln.buffer = buffer;
  ln.pg = pg;
  ln.px = px;
  if (v.rowptr) {
    ln.rowptr = v.rowptr;
  } else {
    CK(fill_i32(ln.own_rowptr, 1, 0, ln.st));
    CK(append_rowptr(v.indptr, v.r0, v.m, ln.own_rowptr, 0, 0, ln.st));
    ln.rowptr = ln.own_rowptr;
  }
  return SFD_OK;
}

// Run the buffer steps of `views` through the lanes.  Views of one stream are consecutive
// flushes of it, in order; the buffer steps finish (VerifySpectral, DenseShrink) in view order.
int run_flushes(sfd_t* h, const std::vector<BufferView>& views) {
  const int nbuf = (int)views.size();
  int rc;
  const int nl = h->nlanes;
  // flush index of each view: its stream's count so far plus the earlier views of the stream
  std::vector<int64_t> index((size_t)nbuf);
  {
    std::map<const StreamState*, int64_t> earlier;
    for (int b = 0; b < nbuf; ++b) index[(size_t)b] = views[b].ss->flushes + earlier[views[b].ss]++;
  }
  for (int b = 0; b < nbuf && b < nl; ++b) {
    Lane& ln = h->lanes[b % nl];
    if ((rc = bind(h, ln, views[b], index[(size_t)b], kPurposeSI, kPurposeVS))) return rc;
    if ((rc = issue_shrink(h, ln))) return rc;
  }
  for (int b = 0; b < nbuf; ++b) {
    Lane& ln = h->lanes[b % nl];
    StreamState& ss = *views[b].ss;
    int live = 0;
    int64_t calls = 0;
    if ((rc = finish_step(h, ln, ss.vs_calls, ss.live, ss.B, ss.B, &live, &calls))) return rc;
    ss.live = live;
    ss.vs_calls += calls;
    ss.flushes += 1;
    if (b + nl < nbuf) {
      // same lane: ordered after this buffer's DenseShrink by the stream
      if ((rc = bind(h, ln, views[b + nl], index[(size_t)(b + nl)], kPurposeSI, kPurposeVS))) return rc;
      if ((rc = issue_shrink(h, ln))) return rc;
    }
  }
  return SFD_OK;
}

// ------------------------------------------------------------------ lockstep groups
// One buffer of a group: the view, the key of its random draws, where its DenseShrink goes,
// and (after run_group) its results.
struct GroupItem {
  BufferView v;
  int64_t buffer;
  int pg, px;
  float* out;  // DenseShrink destination (the stream's B, or a query's panel)
  int live = 0;
  int64_t calls = 0;
};

// Buffer steps of K buffers of different streams (each with m > ell) in lockstep: one launch per
// step for all of them.  Every per-buffer result is bit for bit the one the single-buffer path
// gives (same chunks, Gram geometry and reductions per buffer).  Buffers whose q is reached keep
// their P^T and P P^T while the others go on; VerifySpectral runs max t steps with each buffer's
// log-norm frozen after its own t.  A rejected buffer retries alone on a lane (Alg 4).
int run_group(sfd_t* h, std::vector<GroupItem>& items) {
  GroupWork& g = h->grp;
  const int K = (int)items.size();
  const int64_t d = h->d;
  const int L = h->L, ell = h->ell;
  const int64_t LL = (int64_t)L * L;
  int rc;
  if (K == 0) return SFD_OK;
  hipStream_t st = g.st;
  // the lanes' previous DenseShrinks read Pt / M64 of the previous group
  for (int i = 0; i < h->nlanes; ++i) CK(hipStreamSynchronize(h->lanes[i].st));
  // ---- stack the buffers
  std::vector<int64_t> R((size_t)K + 1, 0), E((size_t)K + 1, 0);
  std::vector<int> q((size_t)K);
  int qmax = 0;
  for (int k = 0; k < K; ++k) {
    R[(size_t)k + 1] = R[(size_t)k] + items[(size_t)k].v.m;
    E[(size_t)k + 1] = E[(size_t)k] + items[(size_t)k].v.nnz;
    q[(size_t)k] = si_iterations(h, items[(size_t)k].v.m);
    qmax = std::max(qmax, q[(size_t)k]);
  }
  const int64_t M = R[(size_t)K], NNZ = E[(size_t)K];
  CK(fill_i32(g.rowptr, 1, 0, st));
  for (int k = 0; k < K; ++k) {
    const BufferView& v = items[(size_t)k].v;
    if (v.rowptr)
      CK(offset_copy(v.rowptr + 1, v.m, (int)E[(size_t)k], g.rowptr + R[(size_t)k] + 1, st));
    else
      CK(append_rowptr(v.indptr, v.r0, v.m, g.rowptr, (int)R[(size_t)k], (int)E[(size_t)k], st));
    CK(offset_copy(v.colidx, v.nnz, (int)(k * d), g.colidx + E[(size_t)k], st));
    if (v.nnz > 0)
      CK(hipMemcpyAsync(g.val + E[(size_t)k], v.val, sizeof(float) * v.nnz, hipMemcpyDeviceToDevice, st));
  }
  const int* keys = nullptr;
  CK(build_csc(g.rowptr, g.colidx, g.val, (int)M, (int)NNZ, (int64_t)K * d, g.cscptr, g.cscrow, g.cscval, g.csc,
               &keys, st));
  CK(fro2_segments(g.cscptr, keys, g.cscrow, g.cscval, d, K, g.fro_part, g.sc, st));
  g.sr.max_chunks = M + NNZ / kSpmmChunk + 2;
  g.scs.max_chunks = (int64_t)K * d + NNZ / kSpmmChunk + 2;
  CK(schedule_build(g.rowptr, (int)M, g.sr, g.scan_tmp, st));
  CK(schedule_build(g.cscptr, (int)(K * d), g.scs, g.scan_tmp, st));
  // ---- per-buffer geometry
  GroupSeg* hx = g.segs_host;
  GroupSeg* hy = hx + g.kmax;
  int64_t* hrows = reinterpret_cast<int64_t*>(hy + g.kmax);
  int* hsteps = reinterpret_cast<int*>(hrows + g.kmax + 1);
  CK(hipStreamSynchronize(st));  // the pinned staging may still be read by the previous group
  int nbx = 1, nby = 1;
  for (int k = 0; k < K; ++k) {
    GroupSeg& sx = hx[k];
    sx.row0 = k * d;
    sx.rows = d;
    gram_geometry(d, (int)L, &sx.nb, &sx.rpb);
    GroupSeg& sy = hy[k];
    sy.row0 = R[(size_t)k];
    sy.rows = items[(size_t)k].v.m;
    gram_geometry(sy.rows, (int)L, &sy.nb, &sy.rpb);
    nbx = std::max(nbx, sx.nb);
    nby = std::max(nby, sy.nb);
    hrows[k] = R[(size_t)k];
  }
  hrows[K] = M;
  CK(hipMemcpyAsync(g.segs_x, hx, sizeof(GroupSeg) * K, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(g.segs_y, hy, sizeof(GroupSeg) * K, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(g.seg_rows, hrows, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, st));
  // ---- SimultaneousIteration (Alg 1) of all buffers
  int* hq = hsteps + g.kmax;
  for (int k = 0; k < K; ++k) hq[k] = q[(size_t)k];
  CK(hipMemcpyAsync(g.qdev, hq, sizeof(int) * K, hipMemcpyHostToDevice, st));
  int* iter_dev = g.qdev + g.kmax;
  CK(fill_i32(iter_dev, 1, 0, st));
  CK(fill_f32(g.X, (int64_t)K * d * L, 0.f, st));
  for (int k = 0; k < K; ++k) {
    const GroupItem& it = items[(size_t)k];
    CK(start_block(h->seed, it.v.ss->stream_id, (uint64_t)it.buffer, 0, (uint64_t)it.pg, d, ell, g.X + k * d * L, L,
                   st));
    if (h->test_zero_row >= 0 && h->test_zero_row < d && h->test_zero_attempts > 0)
      CK(fill_f32(g.X + k * d * L + (int64_t)h->test_zero_row * L, L, 0.f, st));
  }
  CK(set_identity(g.T, L, K, st));
  CK(xform_gram_group(g.X, PanelType::F32, L, d, 0, nbx, g.segs_x, K, L, g.T, g.gram_part, g.W, st));
  CK(chol_inv_group(g.W, L, ell, L, kCholDropTol, g.T, g.sc, K, LL, g.cholw, st));
  // the products' launch configurations (tuned on first sight; the tuning runs write Y and P^T,
  // which the iteration overwrites before reading)
  SpmmConfig cfg_r, cfg_c;
  if ((rc = product_config(h, st, g.sr, g.colidx, g.val, false, g.X, PanelType::F32, g.Y, PanelType::F32, g.partial,
                           (int64_t)K * d, NNZ, &cfg_r)))
    return rc;
  if ((rc = product_config(h, st, g.scs, g.cscrow, g.cscval, false, g.Y, PanelType::F32, g.Pt, PanelType::F32,
                           g.partial, M, NNZ, &cfg_c)))
    return rc;
  // One iteration: Y = A' X T_x, X = A'^T Y T_y (with the Grams and Choleskys), the buffers at
  // their final product keep P^T = A'^T Y T_y and P P^T, the counter moves on.  Every iteration is
  // the same launches with the same arguments, so with SFD_OPT_GRAPHS it is captured once as a
  // HIP graph and replayed qmax + 1 times.
  auto iteration = [&]() -> int {
    CK(spmm(g.sr, g.colidx, g.val, false, g.X, PanelType::F32, L, g.Y, PanelType::F32, L, L, g.partial, cfg_r, st));
    CK(spmm_finish(g.sr, g.partial, g.Y, PanelType::F32, L, L, st));
    CK(xform_gram_group(g.Y, PanelType::F32, L, 0, 0, nby, g.segs_y, K, L, g.T, g.gram_part, g.W, st));
    CK(chol_inv_group(g.W, L, ell, L, kCholDropTol, g.T, g.sc, K, LL, g.cholw, st));
    CK(spmm(g.scs, g.cscrow, g.cscval, false, g.Y, PanelType::F32, L, g.X, PanelType::F32, L, L, g.partial, cfg_c,
            st));
    CK(spmm_finish(g.scs, g.partial, g.X, PanelType::F32, L, L, st));
    CK(xform_gram_group(g.X, PanelType::F32, L, d, 0, nbx, g.segs_x, K, L, g.T, g.gram_part, g.W, st));
    CK(group_snapshot(iter_dev, g.qdev, K, g.X, g.Pt, d * L, g.W, g.Wp, LL, st));
    CK(chol_inv_group(g.W, L, ell, L, kCholDropTol, g.T, g.sc, K, LL, g.cholw, st));
    CK(counter_add(iter_dev, 1, st));
    return SFD_OK;
  };
  if ((rc = replay(h, st, qmax + 1, iteration))) return rc;
  // ---- SparseShrink (Alg 3): eig of P P^T, M = H D, the scalars of Alg 4
  CK(eig_sym_group(g.Wp, L, ell, ell, g.evals, g.evecs, K, LL, 2 * L, 4 * LL, g.eig_work, eig_work_bytes(ell), st));
  CK(ssh_post_group(g.evals, g.evecs, ell, L, kAlpha, g.M64, g.M32, g.sc, K, 2 * L, 4 * LL, st));
  CK(hipMemcpyAsync(g.sc_host, g.sc, sizeof(DevScalars) * K, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  // ---- BoostedSparseShrink (Alg 4): lossless accept, else VerifySpectral (Alg 6)
  std::vector<char> verdict((size_t)K, 0);  // 1 accepted, 0 needs VerifySpectral, 2 rejected
  int tmax = 0;
  for (int k = 0; k < K; ++k) {
    const DevScalars sk = g.sc_host[k];
    StreamState& ss = *items[(size_t)k].v.ss;
    ss.stats.attempts += 1;
    ss.stats.last_q = q[(size_t)k];
    ss.stats.last_fro2_buffer = sk.fro2A;
    ss.stats.last_lambda_ell2 = sk.lam_ell2;
    ss.stats.last_delta = 2.0 * sk.half_delta;
    hsteps[k] = 0;
    if (sk.S <= 64.0 * kUnitRoundoff32 * ell * sk.fro2A || !h->verify) {
      verdict[(size_t)k] = 1;
    } else {
      items[(size_t)k].calls = 1;
      hsteps[k] = vs_steps(h, ss.vs_calls + 1);
      tmax = std::max(tmax, hsteps[k]);
    }
  }
  if (tmax > 0) {
    CK(hipMemcpyAsync(g.tsteps, hsteps, sizeof(int) * K, hipMemcpyHostToDevice, st));
    CK(fill_f32(g.vs_w, (int64_t)K * d, 0.f, st));
    for (int k = 0; k < K; ++k) {
      if (hsteps[k] == 0) continue;
      const GroupItem& it = items[(size_t)k];
      CK(start_block(h->seed, it.v.ss->stream_id, (uint64_t)it.buffer, 0, (uint64_t)it.px, d, 1, g.vs_w + k * d, 1,
                     st));
    }
    constexpr int kScStride = (int)(sizeof(DevScalars) / sizeof(double));
    CK(vs_init(g.vs_w, d, g.vs_npart, g.sc, st, K));
    // one power step for every buffer (a buffer past its own t is left as it is): the same
    // launches every step, captured once and replayed with SFD_OPT_GRAPHS
    auto power_step = [&]() -> int {
      CK(spmv(g.rowptr, g.colidx, g.val, g.sr, g.vs_w, &g.sc->inv_norm, g.vs_z, g.partial, st, g.seg_rows, K,
              kScStride));
      CK(panel_gemv_t(g.Pt, L, L, d, g.vs_w, &g.sc->inv_norm, g.vs_gpart, st, K, kScStride));
      CK(spmv(g.cscptr, g.cscrow, g.cscval, g.scs, g.vs_z, nullptr, g.vs_wraw, g.partial, st));
      CK(vs_small(g.vs_gpart, gemv_blocks(d), g.M64, ell, L, g.vs_c2, st, K));
      CK(vs_finish(g.vs_wraw, g.Pt, L, L, ell, g.vs_c2, d, g.vs_w, g.vs_npart, st, K));
      CK(vs_norm(g.vs_npart, vs_finish_blocks(d), g.sc, st, K, g.tsteps));
      return SFD_OK;
    };
    if ((rc = replay(h, st, tmax, power_step))) return rc;
    CK(hipMemcpyAsync(g.sc_host, g.sc, sizeof(DevScalars) * K, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int k = 0; k < K; ++k) {
      if (hsteps[k] == 0) continue;
      StreamState& ss = *items[(size_t)k].v.ss;
      const double ln_norm = g.sc_host[k].ln_norm;
      ss.stats.last_t = hsteps[k];
      ss.stats.last_ln_norm = ln_norm;
      if (ln_norm <= 0.0) {
        verdict[(size_t)k] = 1;
      } else {
        ss.stats.vs_rejects += 1;
        verdict[(size_t)k] = 2;
      }
    }
  }
  CK(hipEventRecord(g.done, st));
  // ---- DenseShrink (Alg 5) per buffer on the lanes; rejected buffers retry there (Alg 4)
  const int nl = h->nlanes;
  for (int k = 0; k < K; ++k) {
    GroupItem& it = items[(size_t)k];
    Lane& ln = h->lanes[k % nl];
    StreamState& ss = *it.v.ss;
    CK(hipStreamWaitEvent(ln.st, g.done, 0));
    if (verdict[(size_t)k] == 1) {
      ln.ss = &ss;
      const int r_add = ell - 1;
      const int lossless = (ss.live + r_add <= ell) ? 1 : 0;
      if ((rc = dense_shrink(h, ln, ss.B, g.Pt + k * d * L, lossless, it.out, g.M64 + k * LL))) return rc;
      it.live = lossless ? ss.live + r_add : ell - 1;
    } else {
      if (h->max_attempts <= 1) return SFD_E_NOCONVERGE;
      if ((rc = bind(h, ln, it.v, it.buffer, it.pg, it.px))) return rc;
      if ((rc = prepare(h, ln))) return rc;
      ln.q = q[(size_t)k];
      if ((rc = sparse_shrink(h, ln, 1))) return rc;
      if ((rc = finish_step(h, ln, ss.vs_calls, ss.live, ss.B, it.out, &it.live, &it.calls, 1, 1))) return rc;
    }
  }
  for (int i = 0; i < nl; ++i) CK(hipStreamSynchronize(h->lanes[i].st));
  return SFD_OK;
}

// Buffer steps of `views` (consecutive flushes per stream, any streams) for a batch handle:
// rounds of at most one buffer per stream (the r-th pending flush of each stream), each round in
// lockstep groups of at most kmax buffers; buffers of at most ell rows take the lane path.
int run_batched(sfd_t* h, const std::vector<BufferView>& views) {
  int rc;
  std::map<const StreamState*, int64_t> earlier;
  std::vector<std::vector<std::pair<BufferView, int64_t>>> rounds;
  for (const BufferView& v : views) {
    const int64_t r = earlier[v.ss]++;
    if ((int64_t)rounds.size() <= r) rounds.resize((size_t)r + 1);
    rounds[(size_t)r].push_back({v, v.ss->flushes + r});
  }
  for (auto& round : rounds) {
    std::vector<BufferView> small;
    std::vector<GroupItem> items;
    for (auto& e : round) {
      // lockstep groups run FP32 panels; the precision form's buffers take the lanes
      if (e.first.m <= h->ell || h->grp.kmax == 0 || h->precision == SFD_PRECISION_BF16 ||
          csc_hot(h, e.first.m, e.first.nnz)) {
        small.push_back(e.first);
        continue;
      }
      items.push_back({e.first, e.second, kPurposeSI, kPurposeVS, e.first.ss->B});
      if ((int)items.size() == h->grp.kmax) {
        if ((rc = run_group(h, items))) return rc;
        for (GroupItem& it : items) {
          it.v.ss->live = it.live;
          it.v.ss->vs_calls += it.calls;
          it.v.ss->flushes += 1;
        }
        items.clear();
      }
    }
    if (!items.empty()) {
      if ((rc = run_group(h, items))) return rc;
      for (GroupItem& it : items) {
        it.v.ss->live = it.live;
        it.v.ss->vs_calls += it.calls;
        it.v.ss->flushes += 1;
      }
    }
    if (!small.empty()) {
      if ((rc = run_flushes(h, small))) return rc;
      if ((rc = sync_all(h))) return rc;
    }
  }
  return SFD_OK;
}

// Query of stream ss on lane ln: B with the pending rows folded into the lane's copy (purposes
// 2/3, VerifySpectral counter from vs_calls + 1, nothing stored).  Returns the panel holding the
// result (asynchronous on the lane's stream when *panel != ss.B).
int query_issue(sfd_t* h, StreamState& ss, Lane& ln) {
  BufferView v{&ss, ss.prow, nullptr, 0, ss.pcol, ss.pval, ss.pm, ss.pnnz};
  int rc;
  if ((rc = bind(h, ln, v, ss.flushes, kPurposeQuerySI, kPurposeQueryVS))) return rc;
  return issue_shrink(h, ln);
}

int query(sfd_t* h, StreamState& ss, Lane& ln, const float** panel, int* live, int64_t* calls) {
  *calls = 0;
  int rc = sync_all(h);
  if (rc) return rc;
  if (ss.pm == 0) {
    *panel = ss.B;
    *live = ss.live;
    return SFD_OK;
  }
  if ((rc = query_issue(h, ss, ln))) return rc;
  if ((rc = finish_step(h, ln, ss.vs_calls, ss.live, ss.B, ln.Bq, live, calls))) return rc;
  if ((rc = sync_all(h))) return rc;
  *panel = ln.Bq;
  return SFD_OK;
}

int check_handle(sfd_t* h) {
  if (!h) return SFD_E_ARG;
  if (h->error) return SFD_E_STATE;
  return SFD_OK;
}

// Rows [r0, r1) (entries [p0, p1)) of a block appended to the stream's pending buffer.
int to_pending(sfd_t* h, StreamState& ss, bool host, const int64_t* indptr, const int32_t* indices,
               const float* values, int64_t r0, int64_t r1, int64_t p0, int64_t p1) {
  Lane& l0 = h->lanes[0];
  const int64_t cnt = r1 - r0, nz = p1 - p0;
  if (cnt <= 0) return SFD_OK;
  const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if (host) {
    std::vector<int> rp((size_t)cnt);
    for (int64_t i = 0; i < cnt; ++i) rp[(size_t)i] = (int)(indptr[r0 + 1 + i] - p0) + ss.pnnz;
    CK(hipMemcpyAsync(ss.prow + ss.pm + 1, rp.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, l0.st));
    if (nz > 0) {
      CK(hipMemcpyAsync(ss.pcol + ss.pnnz, indices + p0, sizeof(int32_t) * nz, kind, l0.st));
      CK(hipMemcpyAsync(ss.pval + ss.pnnz, values + p0, sizeof(float) * nz, kind, l0.st));
    }
    int rc = sync_lane(h, l0);  // the staging vector goes out of scope
    if (rc) return rc;
  } else {
    CK(append_rowptr(indptr, r0, cnt, ss.prow, ss.pm, ss.pnnz, l0.st));
    if (nz > 0) {
      CK(hipMemcpyAsync(ss.pcol + ss.pnnz, indices + p0, sizeof(int32_t) * nz, kind, l0.st));
      CK(hipMemcpyAsync(ss.pval + ss.pnnz, values + p0, sizeof(float) * nz, kind, l0.st));
    }
  }
  ss.pm += (int)cnt;
  ss.pnnz += (int)nz;
  return SFD_OK;
}

// Alg 2's rule on host row pointers (nrows rows, indptr[0] may be != 0), continuing the
// stream's pending buffer: the rows after which a flush happens.
void host_cuts(const sfd_t* h, const StreamState& ss, const int64_t* indptr, int64_t nrows,
               std::vector<int64_t>& cuts) {
  const int64_t budget = flush_nnz(h), row_limit = flush_rows(h);
  int64_t r = 0, m = ss.pm, z = ss.pnnz;
  while (r < nrows) {
    const int64_t target = budget - z + indptr[r];
    const int64_t* it = std::lower_bound(indptr + r + 1, indptr + nrows + 1, target);
    const int64_t by_nnz = (it - indptr) - 1;
    const int64_t by_rows = r + (row_limit - m) - 1;
    const int64_t cut = std::min(by_nnz, by_rows);
    if (cut >= nrows) break;
    cuts.push_back(cut);
    r = cut + 1;
    m = 0;
    z = 0;
  }
}

// One block of rows of one stream, validated: the cuts (rows after which a flush happens) and
// the entry offset after each cut.
struct Segment {
  StreamState* ss;
  const int64_t* indptr;  // the block's row pointers (nrows + 1, host or device)
  const int32_t* indices;
  const float* values;
  int64_t nrows, lo, hi;  // entries [lo, hi) of indices / values
  std::vector<int64_t> cuts, cut_ptr;
};

// Full buffers of a segment as views (the first one continues the stream's pending rows,
// which are copied; the others are read in place from the caller's device arrays), and the
// position where its remainder starts.
int segment_views(sfd_t* h, Segment& sg, std::vector<BufferView>& views, int64_t* r_rem, int64_t* p_rem) {
  int rc;
  int64_t r = 0, p = sg.lo;
  StreamState& ss = *sg.ss;
  for (size_t k = 0; k < sg.cuts.size(); ++k) {
    const int64_t r1 = sg.cuts[k] + 1, p1 = sg.cut_ptr[k];
    if (k == 0 && ss.pm > 0) {
      if ((rc = to_pending(h, ss, false, sg.indptr, sg.indices, sg.values, r, r1, p, p1))) return rc;
      views.push_back({&ss, ss.prow, nullptr, 0, ss.pcol, ss.pval, ss.pm, ss.pnnz});
    } else {
      views.push_back({&ss, nullptr, sg.indptr, r, sg.indices + p, sg.values + p, (int)(r1 - r), (int)(p1 - p)});
    }
    r = r1;
    p = p1;
  }
  *r_rem = r;
  *p_rem = p;
  return SFD_OK;
}

// Device block: entry range, validation (rows no longer than d, ids in [0, d)) and cuts.
int device_segment(sfd_t* h, Segment& sg) {
  Lane& l0 = h->lanes[0];
  int rc;
  int64_t* hv = h->i64_host;
  const int64_t nrows = sg.nrows;
  CK(hipMemcpyAsync(hv + 0, sg.indptr, sizeof(int64_t), hipMemcpyDeviceToHost, l0.st));
  CK(hipMemcpyAsync(hv + 1, sg.indptr + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, l0.st));
  if ((rc = sync_lane(h, l0))) return rc;
  sg.lo = hv[0];
  sg.hi = hv[1];
  if (sg.hi < sg.lo || sg.lo < 0) return SFD_E_ARG;
  if (sg.hi > sg.lo && (!sg.indices || !sg.values)) return SFD_E_ARG;
  CK(fill_i32(h->err_dev, 1, 0, l0.st));
  CK(validate_rows(sg.indptr, nrows, h->d, h->err_dev, l0.st));
  CK(validate_indices(sg.indices, sg.lo, sg.hi, h->d, h->err_dev, l0.st));
  int* e32 = reinterpret_cast<int*>(hv + 2);
  CK(hipMemcpyAsync(e32, h->err_dev, sizeof(int), hipMemcpyDeviceToHost, l0.st));
  if ((rc = sync_lane(h, l0))) return rc;
  if (*e32 & 1) return SFD_E_ARG;
  if (*e32 & 2) return SFD_E_INDEX;
  const int64_t max_cuts = (nrows + sg.ss->pm) / std::min<int64_t>(h->ell, flush_rows(h)) + 2;
  if (max_cuts > h->cut_cap) {
    int64_t* p = nullptr;
    if (!dalloc(h, &p, 1 + 2 * max_cuts)) return SFD_E_NOMEM;
    h->cut_dev = p;
    h->cut_cap = max_cuts;
  }
  CK(find_cuts(sg.indptr, nrows, sg.ss->pm, sg.ss->pnnz, flush_nnz(h), flush_rows(h), max_cuts, h->cut_dev + 1,
               h->cut_dev + 1 + h->cut_cap, h->cut_dev, l0.st));
  CK(hipMemcpyAsync(hv + 3, h->cut_dev, sizeof(int64_t), hipMemcpyDeviceToHost, l0.st));
  if ((rc = sync_lane(h, l0))) return rc;
  const int64_t ncuts = hv[3];
  sg.cuts.resize((size_t)ncuts);
  sg.cut_ptr.resize((size_t)ncuts);
  if (ncuts > 0) {
    CK(hipMemcpy(sg.cuts.data(), h->cut_dev + 1, sizeof(int64_t) * ncuts, hipMemcpyDeviceToHost));
    CK(hipMemcpy(sg.cut_ptr.data(), h->cut_dev + 1 + h->cut_cap, sizeof(int64_t) * ncuts, hipMemcpyDeviceToHost));
  }
  return SFD_OK;
}

// Host block: validation and cuts on the host.
int host_segment(sfd_t* h, Segment& sg) {
  const int64_t* indptr = sg.indptr;
  sg.lo = indptr[0];
  sg.hi = indptr[sg.nrows];
  if (sg.hi < sg.lo || sg.lo < 0) return SFD_E_ARG;
  if (sg.hi > sg.lo && (!sg.indices || !sg.values)) return SFD_E_ARG;
  for (int64_t r = 0; r < sg.nrows; ++r) {
    const int64_t len = indptr[r + 1] - indptr[r];
    if (len < 0 || len > h->d) return SFD_E_ARG;
  }
  for (int64_t k = sg.lo; k < sg.hi; ++k)
    if (sg.indices[k] < 0 || (int64_t)sg.indices[k] >= h->d) return SFD_E_INDEX;
  host_cuts(h, *sg.ss, indptr, sg.nrows, sg.cuts);
  for (int64_t c : sg.cuts) sg.cut_ptr.push_back(indptr[c + 1]);
  return SFD_OK;
}

// Append validated device segments (at most one per stream): run all their full buffers through
// the lanes, then move each remainder into its stream's pending buffer.
int append_device_segments(sfd_t* h, std::vector<Segment>& segs) {
  int rc;
  std::vector<BufferView> views;
  std::vector<int64_t> rrem(segs.size()), prem(segs.size());
  std::vector<char> flushed(segs.size(), 0);
  for (size_t i = 0; i < segs.size(); ++i) {
    if ((rc = segment_views(h, segs[i], views, &rrem[i], &prem[i]))) return rc;
    flushed[i] = !segs[i].cuts.empty();
  }
  if (!views.empty()) {
    if ((rc = h->grp.kmax > 0 ? run_batched(h, views) : run_flushes(h, views))) return rc;
    if ((rc = sync_all(h))) return rc;
  }
  for (size_t i = 0; i < segs.size(); ++i) {
    Segment& sg = segs[i];
    if (flushed[i]) sg.ss->pm = sg.ss->pnnz = 0;
    if ((rc = to_pending(h, *sg.ss, false, sg.indptr, sg.indices, sg.values, rrem[i], sg.nrows, prem[i], sg.hi)))
      return rc;
    sg.ss->stats.rows_seen += sg.nrows;
    sg.ss->stats.nnz_seen += sg.hi - sg.lo;
  }
  return sync_all(h);
}

// Append a validated host segment: each full buffer is staged through the pending buffer and run.
int append_host_segment(sfd_t* h, Segment& sg) {
  int rc;
  StreamState& ss = *sg.ss;
  int64_t r = 0, p = sg.lo;
  for (size_t k = 0; k < sg.cuts.size(); ++k) {
    const int64_t r1 = sg.cuts[k] + 1, p1 = sg.cut_ptr[k];
    if ((rc = to_pending(h, ss, true, sg.indptr, sg.indices, sg.values, r, r1, p, p1))) return rc;
    std::vector<BufferView> views{{&ss, ss.prow, nullptr, 0, ss.pcol, ss.pval, ss.pm, ss.pnnz}};
    if ((rc = run_flushes(h, views))) return rc;
    if ((rc = sync_all(h))) return rc;
    ss.pm = ss.pnnz = 0;
    r = r1;
    p = p1;
  }
  if ((rc = to_pending(h, ss, true, sg.indptr, sg.indices, sg.values, r, sg.nrows, p, sg.hi))) return rc;
  if ((rc = sync_all(h))) return rc;
  ss.stats.rows_seen += sg.nrows;
  ss.stats.nnz_seen += sg.hi - sg.lo;
  return SFD_OK;
}

int create_handle(int64_t d, int32_t ell, double eps, uint64_t seed, int nstreams, int lanes, sfd_t** out) {
  if (!out) return SFD_E_ARG;
  *out = nullptr;
  if (ell < 1 || d < ell || ell > kMaxEll) return SFD_E_ARG;
  if (!(eps > 0.0 && eps < 1.0)) return SFD_E_ARG;
  if ((int64_t)ell * d + d >= ((int64_t)1 << 31)) return SFD_E_ARG;
  sfd_t* h = new (std::nothrow) sfd_t();
  if (!h) return SFD_E_NOMEM;
  h->d = d;
  h->ell = ell;
  h->L = ell <= 32 ? 32 : ell <= 64 ? 64 : ell <= 128 ? 128 : 256;
  h->eps = eps;
  h->seed = seed;
  h->lanes_alloc = lanes;
  h->nlanes = lanes;
  h->streams.resize((size_t)nstreams);
  for (int s = 0; s < nstreams; ++s) h->streams[(size_t)s].stream_id = (uint64_t)s;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return SFD_E_DEVICE;
  }
  int rc = alloc_state(h);
  if (rc == SFD_OK) rc = reset_state(h);
  if (rc != SFD_OK) {
    free_all(h);
    delete h;
    return rc == SFD_E_NOMEM ? SFD_E_NOMEM : SFD_E_DEVICE;
  }
  *out = h;
  return SFD_OK;
}

// Counters of a stream restored to `old`; the last_* figures keep describing the last attempt made.
void restore_counters(StreamState& ss, const sfd_stats_t& old) {
  const sfd_stats_t cur = ss.stats;
  ss.stats = old;
  ss.stats.last_q = cur.last_q;
  ss.stats.last_t = cur.last_t;
  ss.stats.last_ln_norm = cur.last_ln_norm;
  ss.stats.last_delta = cur.last_delta;
  ss.stats.last_fro2_buffer = cur.last_fro2_buffer;
  ss.stats.last_lambda_ell2 = cur.last_lambda_ell2;
}

// The state of a single stream before an append, for its rollback when a buffer's
// BoostedSparseShrink exhausts its attempts (Alg 4): the host-side fields, the sketch (copied
// to Bsave) and, when the append could overwrite them, the pending buffer's rows.
struct StreamSnapshot {
  int live = 0;
  int64_t flushes = 0, vs_calls = 0;
  sfd_stats_t stats{};
  int pm = 0, pnnz = 0;
  bool pending_saved = false;
};

int snapshot_stream(sfd_t* h, StreamState& ss, bool save_pending, StreamSnapshot* snap) {
  Lane& l0 = h->lanes[0];
  snap->live = ss.live;
  snap->flushes = ss.flushes;
  snap->vs_calls = ss.vs_calls;
  snap->stats = ss.stats;
  snap->pm = ss.pm;
  snap->pnnz = ss.pnnz;
  CK(hipMemcpyAsync(h->Bsave, ss.B, sizeof(float) * h->d * h->L, hipMemcpyDeviceToDevice, l0.st));
  if (save_pending && ss.pm > 0) {
    if (!h->psave_row) {
      if (!dalloc(h, &h->psave_row, h->d + 1) || !dalloc(h, &h->psave_col, h->cap) ||
          !dalloc(h, &h->psave_val, h->cap))
        return SFD_E_NOMEM;
    }
    CK(hipMemcpyAsync(h->psave_row, ss.prow, sizeof(int) * (ss.pm + 1), hipMemcpyDeviceToDevice, l0.st));
    if (ss.pnnz > 0) {
      CK(hipMemcpyAsync(h->psave_col, ss.pcol, sizeof(int) * ss.pnnz, hipMemcpyDeviceToDevice, l0.st));
      CK(hipMemcpyAsync(h->psave_val, ss.pval, sizeof(float) * ss.pnnz, hipMemcpyDeviceToDevice, l0.st));
    }
    snap->pending_saved = true;
  }
  // every DenseShrink of this append waits for the stream's last one: now the copy
  CK(hipEventRecord(ss.ev_dsh, l0.st));
  return SFD_OK;
}

// Undo an append after SFD_E_NOCONVERGE: wait for the buffer steps still in flight on the
// lanes, then put back the sketch, the pending rows and the counters.
int rollback_stream(sfd_t* h, StreamState& ss, const StreamSnapshot& snap) {
  int rc = sync_all(h);
  if (rc) return rc;
  Lane& l0 = h->lanes[0];
  CK(hipMemcpyAsync(ss.B, h->Bsave, sizeof(float) * h->d * h->L, hipMemcpyDeviceToDevice, l0.st));
  if (snap.pending_saved) {
    CK(hipMemcpyAsync(ss.prow, h->psave_row, sizeof(int) * (snap.pm + 1), hipMemcpyDeviceToDevice, l0.st));
    if (snap.pnnz > 0) {
      CK(hipMemcpyAsync(ss.pcol, h->psave_col, sizeof(int) * snap.pnnz, hipMemcpyDeviceToDevice, l0.st));
      CK(hipMemcpyAsync(ss.pval, h->psave_val, sizeof(float) * snap.pnnz, hipMemcpyDeviceToDevice, l0.st));
    }
  }
  CK(hipEventRecord(ss.ev_dsh, l0.st));
  if ((rc = sync_lane(h, l0))) return rc;
  ss.live = snap.live;
  ss.flushes = snap.flushes;
  ss.vs_calls = snap.vs_calls;
  ss.pm = snap.pm;
  ss.pnnz = snap.pnnz;
  restore_counters(ss, snap.stats);
  return SFD_E_NOCONVERGE;
}

void fill_stats(const StreamState& ss, sfd_stats_t* out) {
  *out = ss.stats;
  out->flushes = ss.flushes;
  out->vs_calls = ss.vs_calls;
  out->live_rows = ss.live;
  out->pending_rows = ss.pm;
  out->pending_nnz = ss.pnnz;
}

}  // namespace

struct sfd_batch_s {
  sfd_t* core;
};

namespace {
// the queries of every stream of a batch handle into B_out (sfd_batch_sketch)
int batch_queries(sfd_t* h, float* B_out, int mem);
}  // namespace

extern "C" {

const char* sfd_strerror(int code) {
  switch (code) {
    case SFD_OK: return "ok";
    case SFD_E_ARG: return "invalid argument";
    case SFD_E_INDEX: return "column index out of range";
    case SFD_E_SHAPE: return "shape mismatch";
    case SFD_E_NOMEM: return "device allocation failed";
    case SFD_E_DEVICE: return "HIP runtime error";
    case SFD_E_NOCONVERGE: return "BoostedSparseShrink exhausted its attempts";
    case SFD_E_STATE: return "handle is in an error state";
    case SFD_E_TOOBIG: return "work exceeds the fixed scratch of a no-allocation call";
    default: return "unknown error";
  }
}

int sfd_create(int64_t d, int32_t ell, double eps, uint64_t seed, sfd_t** out) {
  // past ell = 128 the FP64 Cholesky and eigensolves of a buffer step (one workgroup each) set its
  // pace, so more buffer steps run side by side
  return create_handle(d, ell, eps, seed, 1, ell > 128 ? kLanesWide : kLanesSingle, out);
}

int sfd_destroy(sfd_t* h) {
  if (!h) return SFD_OK;
  DeviceGuard g(h->device);
  for (int i = 0; i < h->lanes_alloc; ++i)
    if (h->lanes[i].st) (void)hipStreamSynchronize(h->lanes[i].st);
  free_all(h);
  delete h;
  return SFD_OK;
}

int sfd_reset(sfd_t* h) {
  if (!h) return SFD_E_ARG;
  DeviceGuard g(h->device);
  return reset_state(h);
}

int sfd_set_option(sfd_t* h, int key, double value) {
  if (!h) return SFD_E_ARG;
  switch (key) {
    case SFD_OPT_DELTA:
      if (!(value > 0.0 && value < 1.0)) return SFD_E_ARG;
      h->delta = value;
      return SFD_OK;
    case SFD_OPT_Q:
      if (value > 1e6) return SFD_E_ARG;
      h->q_override = value > 0 ? (int)value : 0;
      return SFD_OK;
    case SFD_OPT_MAX_ATTEMPTS:
      if (!(value >= 1 && value <= 1e6)) return SFD_E_ARG;
      h->max_attempts = (int)value;
      return SFD_OK;
    case SFD_OPT_VERIFY:
      if (value != 0.0 && value != 1.0) return SFD_E_ARG;
      h->verify = (int)value;
      return SFD_OK;
    case SFD_OPT_PROFILE:
      if (value != 0.0 && value != 1.0) return SFD_E_ARG;
      h->prof = (int)value;
      if (h->prof) std::memset(&h->profile, 0, sizeof(h->profile));
      return SFD_OK;
    case SFD_OPT_STREAM_ID:
      if (h->streams.size() != 1) return SFD_E_ARG;  // a batch keys stream s as STREAM_ID = s
      if (!(value >= 0) || value > 9.0e15 || value != std::floor(value)) return SFD_E_ARG;
      h->streams[0].stream_id = (uint64_t)value;
      return SFD_OK;
    case SFD_OPT_PRECISION:
      if (value != SFD_PRECISION_FP32 && value != SFD_PRECISION_BF16) return SFD_E_ARG;
      h->precision = (int)value;
      return SFD_OK;
    case SFD_OPT_CQR2:
      if (value != SFD_CQR2_OFF && value != SFD_CQR2_FINAL && value != SFD_CQR2_ALL) return SFD_E_ARG;
      h->cqr2 = (int)value;
      return SFD_OK;
    case SFD_OPT_AUTOTUNE:
      if (value != 0 && value != 1) return SFD_E_ARG;
      h->autotune = (int)value;
      return SFD_OK;
    case SFD_OPT_GRAPHS:
      if (value != 0 && value != 1) return SFD_E_ARG;
      h->graphs = (int)value;
      return SFD_OK;
    case SFD_OPT_PRODUCT_LAUNCH:
      if (!(value >= 0 && value <= 3) || value != std::floor(value)) return SFD_E_ARG;
      h->launch = (int)value;
      return SFD_OK;
    case SFD_OPT_LANES: {
      if (!(value >= 1 && value <= kLanes) || value != std::floor(value)) return SFD_E_ARG;
      // lanes beyond those allocated get their workspaces now (after the work in flight)
      if ((int)value > h->lanes_alloc) {
        DeviceGuard g(h->device);
        int rc = sync_all(h);
        if (rc) return rc;
        for (int li = h->lanes_alloc; li < (int)value; ++li) {
          if ((rc = alloc_lane(h, h->lanes[li]))) return rc;
          h->lanes_alloc = li + 1;
        }
      }
      h->nlanes = (int)value;
      return SFD_OK;
    }
    case SFD_OPT_ALGORITHM:
      if (value != SFD_ALGO_SFD && value != SFD_ALGO_FD) return SFD_E_ARG;
      h->algorithm = (int)value;
      return SFD_OK;
    case SFD_OPT_CSC_BANDS:
      if (value != 0 && value != 1 && value != kXcdBands) return SFD_E_ARG;
      h->bands_opt = (int)value;
      return SFD_OK;
    case SFD_OPT_CSC_HOT_MIN:
      if (!(value >= 1 && value <= (double)(1 << 30)) || value != std::floor(value)) return SFD_E_ARG;
      h->hot_min = (int)value;
      return SFD_OK;
    case SFD_OPT_TEST_ZERO_ROW:
      if (!(value >= -1 && value < (double)h->d) || value != std::floor(value)) return SFD_E_ARG;
      h->test_zero_row = (int)value;
      return SFD_OK;
    case SFD_OPT_TEST_ZERO_ATTEMPTS:
      if (!(value >= 0 && value <= 1e6) || value != std::floor(value)) return SFD_E_ARG;
      h->test_zero_attempts = (int)value;
      return SFD_OK;
    default:
      return SFD_E_ARG;
  }
}

int sfd_set_stream(sfd_t* h, void* hip_stream) {
  if (!h) return SFD_E_ARG;
  DeviceGuard g(h->device);
  int rc = sync_all(h);
  if (rc) return rc;
  h->user_stream = static_cast<hipStream_t>(hip_stream);
  return SFD_OK;
}

int sfd_get_stats(const sfd_t* h, sfd_stats_t* out) {
  if (!h || !out) return SFD_E_ARG;
  fill_stats(h->streams[0], out);
  return SFD_OK;
}

int sfd_get_profile(const sfd_t* h, sfd_profile_t* out) {
  if (!h || !out) return SFD_E_ARG;
  *out = h->profile;
  return SFD_OK;
}

int sfd_append_csr(sfd_t* h, int64_t nrows, const int64_t* indptr, const int32_t* indices, const float* values,
                   int mem) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nrows < 0 || (mem != SFD_MEM_HOST && mem != SFD_MEM_DEVICE)) return SFD_E_ARG;
  if (nrows == 0) return SFD_OK;
  if (!indptr) return SFD_E_ARG;
  DeviceGuard g(h->device);
  if ((rc = order_after_caller(h))) return rc;
  std::vector<Segment> segs(1);
  Segment& sg = segs[0];
  sg.ss = &h->streams[0];
  sg.indptr = indptr;
  sg.indices = indices;
  sg.values = values;
  sg.nrows = nrows;
  if (mem == SFD_MEM_HOST) {
    if ((rc = host_segment(h, sg))) return rc;
  } else {
    if ((rc = device_segment(h, sg))) return rc;
  }
  // an append that flushes can end in SFD_E_NOCONVERGE: keep what it could change.  A host
  // block stages each full buffer through the pending buffer, so from its second flush on it
  // overwrites the rows pending before the call; a device block only appends after them.
  StreamSnapshot snap;
  const bool flushes = !sg.cuts.empty();
  if (flushes && (rc = snapshot_stream(h, *sg.ss, mem == SFD_MEM_HOST && sg.cuts.size() >= 2, &snap))) return rc;
  rc = mem == SFD_MEM_HOST ? append_host_segment(h, sg) : append_device_segments(h, segs);
  if (rc == SFD_E_NOCONVERGE && flushes) return rollback_stream(h, *sg.ss, snap);
  return rc;
}

int sfd_sketch(sfd_t* h, float* B_out, int mem, int32_t* live_rows) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!B_out || (mem != SFD_MEM_HOST && mem != SFD_MEM_DEVICE)) return SFD_E_ARG;
  DeviceGuard g(h->device);
  if ((rc = order_after_caller(h))) return rc;
  const float* panel;
  int live;
  int64_t calls;
  Lane& l0 = h->lanes[0];
  const sfd_stats_t before = h->streams[0].stats;
  if ((rc = query(h, h->streams[0], l0, &panel, &live, &calls))) {
    if (rc == SFD_E_NOCONVERGE) restore_counters(h->streams[0], before);
    return rc;
  }
  if (mem == SFD_MEM_DEVICE) {
    CK(transpose_out(panel, h->L, h->d, h->ell, B_out, l0.st));
  } else {
    CK(transpose_out(panel, h->L, h->d, h->ell, l0.X, l0.st));
    CK(hipMemcpyAsync(B_out, l0.X, sizeof(float) * h->d * h->ell, hipMemcpyDeviceToHost, l0.st));
  }
  if ((rc = sync_all(h))) return rc;
  if (live_rows) *live_rows = live;
  return SFD_OK;
}

int sfd_merge(sfd_t* dst, const sfd_t* src_c) {
  if (!dst || !src_c || dst == src_c) return SFD_E_ARG;
  // src's logical state (sketch, buffer, counters) is left as it was; its query runs in its own
  // lane workspaces, which are scratch between calls
  sfd_t* src = const_cast<sfd_t*>(src_c);
  int rc = check_handle(dst);
  if (rc) return rc;
  if ((rc = check_handle(src))) return rc;
  if (dst->d != src->d || dst->ell != src->ell) return SFD_E_SHAPE;
  if (dst->device != src->device) return SFD_E_ARG;
  if (dst->streams.size() != 1 || src->streams.size() != 1) return SFD_E_ARG;
  DeviceGuard g(dst->device);
  sfd_t* h = dst;
  if ((rc = order_after_caller(dst))) return rc;
  if ((rc = order_after_caller(src))) return rc;
  StreamState& sd = dst->streams[0];
  const sfd_stats_t src_before = src->streams[0].stats, dst_before = sd.stats;
  const float *ps, *pd;
  int live_s, live_d;
  int64_t calls_s, calls_d;
  rc = query(src, src->streams[0], src->lanes[0], &ps, &live_s, &calls_s);
  src->streams[0].stats = src_before;
  if (rc) return rc;
  if ((rc = query(dst, sd, dst->lanes[0], &pd, &live_d, &calls_d))) {
    if (rc == SFD_E_NOCONVERGE) restore_counters(sd, dst_before);
    return rc;
  }
  // stack [query(dst); query(src)], DenseShrink with M = I
  Lane& ln = h->lanes[0];
  ln.ss = &sd;
  CK(ssh_identity(h->ell, h->L, ln.M64, ln.M32, ln.sc, ln.st));
  const int lossless = (live_d + live_s <= h->ell) ? 1 : 0;
  if ((rc = dense_shrink(h, ln, pd, ps, lossless, sd.B))) return rc;
  if ((rc = sync_all(h))) return rc;
  sd.live = lossless ? live_d + live_s : h->ell - 1;
  sd.vs_calls += calls_d;
  sd.flushes += 1;
  sd.pm = sd.pnnz = 0;
  return SFD_OK;
}

int sfd_start_block(uint64_t seed, uint64_t stream_id, uint64_t buffer, uint64_t attempt, uint64_t purpose,
                    int64_t d, int32_t ell, float* G_out) {
  if (d < 1 || ell < 1 || !G_out) return SFD_E_ARG;
  if (start_block(seed, stream_id, buffer, attempt, purpose, d, ell, G_out, ell, nullptr) != hipSuccess)
    return SFD_E_DEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return SFD_E_DEVICE;
  return SFD_OK;
}

// ------------------------------------------------------------------ batched streams

int sfd_batch_create(int32_t nstreams, int64_t d, int32_t ell, double eps, uint64_t seed, sfd_batch_t** out) {
  if (!out) return SFD_E_ARG;
  *out = nullptr;
  if (nstreams < 1) return SFD_E_ARG;
  sfd_batch_t* b = new (std::nothrow) sfd_batch_t();
  if (!b) return SFD_E_NOMEM;
  int rc = create_handle(d, ell, eps, seed, nstreams, kLanes, &b->core);
  if (rc) {
    delete b;
    return rc;
  }
  if (nstreams > 1) {
    // lockstep groups of up to 128 buffers, within about 8 GiB of workspace (128 rather than 64:
    // 7.33 against 7.55 s for 4,096 streams at d = 2e4, ell = 32; fewer host round trips)
    sfd_t* h = b->core;
    const int64_t L = h->L;
    const int64_t per = h->cap * 40 + h->d * L * 4 * 3 + gram_partial_stride((int)L) * 4 + h->d * 64;
    int kmax = (int)std::min<int64_t>({(int64_t)nstreams, 128, std::max<int64_t>(1, ((int64_t)8 << 30) / per)});
    DeviceGuard g(h->device);
    if (kmax >= 2 && (rc = alloc_group(h, kmax)) != SFD_OK) {
      sfd_destroy(h);
      delete b;
      return rc;
    }
  }
  *out = b;
  return SFD_OK;
}

int sfd_batch_destroy(sfd_batch_t* b) {
  if (!b) return SFD_OK;
  int rc = sfd_destroy(b->core);
  delete b;
  return rc;
}

int sfd_batch_reset(sfd_batch_t* b) { return b ? sfd_reset(b->core) : SFD_E_ARG; }

int sfd_batch_set_option(sfd_batch_t* b, int key, double value) {
  if (!b || key == SFD_OPT_STREAM_ID) return SFD_E_ARG;
  return sfd_set_option(b->core, key, value);
}

int sfd_batch_set_stream(sfd_batch_t* b, void* hip_stream) { return b ? sfd_set_stream(b->core, hip_stream) : SFD_E_ARG; }

int sfd_batch_get_stats(const sfd_batch_t* b, int32_t stream, sfd_stats_t* out) {
  if (!b || !out || stream < 0 || stream >= (int32_t)b->core->streams.size()) return SFD_E_ARG;
  fill_stats(b->core->streams[(size_t)stream], out);
  return SFD_OK;
}

int sfd_batch_append_csr(sfd_batch_t* b, int32_t nseg, const int32_t* stream_of_seg, const int64_t* seg_row_start,
                         const int64_t* indptr, const int32_t* indices, const float* values, int mem) {
  if (!b) return SFD_E_ARG;
  sfd_t* h = b->core;
  int rc = check_handle(h);
  if (rc) return rc;
  if (nseg < 0 || (nseg > 0 && (!stream_of_seg || !seg_row_start || !indptr))) return SFD_E_ARG;
  if (mem != SFD_MEM_HOST && mem != SFD_MEM_DEVICE) return SFD_E_ARG;
  if (nseg == 0) return SFD_OK;
  // segment table: streams in range and each stream at most once, row ranges non-decreasing
  const int32_t ns = (int32_t)h->streams.size();
  std::vector<char> used((size_t)ns, 0);
  for (int32_t i = 0; i < nseg; ++i) {
    const int32_t s = stream_of_seg[i];
    if (s < 0 || s >= ns || used[(size_t)s]) return SFD_E_ARG;
    used[(size_t)s] = 1;
    if (seg_row_start[i] < 0 || seg_row_start[i + 1] < seg_row_start[i]) return SFD_E_ARG;
  }
  DeviceGuard g(h->device);
  if ((rc = order_after_caller(h))) return rc;
  std::vector<Segment> segs((size_t)nseg);
  for (int32_t i = 0; i < nseg; ++i) {
    Segment& sg = segs[(size_t)i];
    sg.ss = &h->streams[(size_t)stream_of_seg[i]];
    sg.indptr = indptr + seg_row_start[i];
    sg.indices = indices;
    sg.values = values;
    sg.nrows = seg_row_start[i + 1] - seg_row_start[i];
  }
  if (mem == SFD_MEM_HOST) {
    // validate every segment before any state changes, then stage them one at a time
    for (Segment& sg : segs)
      if ((rc = host_segment(h, sg))) return rc;
    for (Segment& sg : segs) {
      if (sg.nrows > 0 && (rc = append_host_segment(h, sg))) {
        if (rc == SFD_E_NOCONVERGE) h->error = rc;
        return rc;
      }
    }
    return SFD_OK;
  }
  for (Segment& sg : segs) {
    if (sg.nrows == 0) {
      sg.lo = sg.hi = 0;
      continue;
    }
    if ((rc = device_segment(h, sg))) return rc;
  }
  std::vector<Segment> live_segs;
  for (Segment& sg : segs)
    if (sg.nrows > 0) live_segs.push_back(std::move(sg));
  // the streams' buffer steps are interleaved, so a stream whose retries run out leaves the
  // others partly advanced: the batch goes to its error state (no rollback)
  rc = append_device_segments(h, live_segs);
  if (rc == SFD_E_NOCONVERGE) h->error = rc;
  return rc;
}

int sfd_batch_sketch(sfd_batch_t* b, float* B_out, int mem) {
  if (!b) return SFD_E_ARG;
  sfd_t* h = b->core;
  int rc = check_handle(h);
  if (rc) return rc;
  if (!B_out || (mem != SFD_MEM_HOST && mem != SFD_MEM_DEVICE)) return SFD_E_ARG;
  DeviceGuard g(h->device);
  if ((rc = order_after_caller(h))) return rc;
  if ((rc = sync_all(h))) return rc;
  std::vector<sfd_stats_t> before;
  for (const StreamState& ss : h->streams) before.push_back(ss.stats);
  rc = batch_queries(h, B_out, mem);
  if (rc == SFD_E_NOCONVERGE) {
    // queries change no state; their counters are put back (the streams' buffers are intact)
    (void)sync_all(h);
    for (size_t s = 0; s < h->streams.size(); ++s) restore_counters(h->streams[s], before[s]);
  }
  return rc;
}

}  // extern "C"

namespace {

int batch_queries(sfd_t* h, float* B_out, int mem) {
  int rc;
  const int64_t per = (int64_t)h->ell * h->d;
  const int nl = h->nlanes;
  Lane& l0 = h->lanes[0];
  // one query result (d x L panel) -> stream s's ell x d block of B_out
  auto emit = [&](const float* panel, int32_t s, hipStream_t st, float* stage) -> int {
    float* dst = mem == SFD_MEM_DEVICE ? B_out + s * per : stage;
    CK(transpose_out(panel, h->L, h->d, h->ell, dst, st));
    if (mem == SFD_MEM_HOST) {
      CK(hipMemcpyAsync(B_out + s * per, stage, sizeof(float) * per, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
    }
    return SFD_OK;
  };
  // streams without pending rows: B itself; pending buffers of more than ell rows: lockstep
  // groups (purposes 2/3, nothing stored) unless they take XCD-local pieces; the others: the lanes
  std::vector<int32_t> lane_q, grp_q;
  for (int32_t s = 0; s < (int32_t)h->streams.size(); ++s) {
    StreamState& ss = h->streams[(size_t)s];
    if (ss.pm == 0) {
      if ((rc = emit(ss.B, s, l0.st, l0.X))) return rc;
    } else if (ss.pm > h->ell && h->grp.kmax > 0 && !csc_hot(h, ss.pm, ss.pnnz)) {
      grp_q.push_back(s);
    } else {
      lane_q.push_back(s);
    }
  }
  if ((rc = sync_all(h))) return rc;
  for (size_t i0 = 0; i0 < grp_q.size(); i0 += (size_t)h->grp.kmax) {
    const size_t i1 = std::min(grp_q.size(), i0 + (size_t)h->grp.kmax);
    std::vector<GroupItem> items;
    for (size_t i = i0; i < i1; ++i) {
      StreamState& ss = h->streams[(size_t)grp_q[i]];
      BufferView v{&ss, ss.prow, nullptr, 0, ss.pcol, ss.pval, ss.pm, ss.pnnz};
      items.push_back({v, ss.flushes, kPurposeQuerySI, kPurposeQueryVS, h->grp.X + (int64_t)(i - i0) * h->d * h->L});
    }
    if ((rc = run_group(h, items))) return rc;
    for (size_t i = i0; i < i1; ++i)
      if ((rc = emit(items[i - i0].out, grp_q[i], h->grp.st, h->grp.Y))) return rc;
    CK(hipStreamSynchronize(h->grp.st));
  }
  const int nq = (int)lane_q.size();
  for (int k = 0; k < nq && k < nl; ++k)
    if ((rc = query_issue(h, h->streams[(size_t)lane_q[(size_t)k]], h->lanes[k % nl]))) return rc;
  for (int k = 0; k < nq; ++k) {
    Lane& ln = h->lanes[k % nl];
    StreamState& ss = h->streams[(size_t)lane_q[(size_t)k]];
    int live = 0;
    int64_t calls = 0;
    if ((rc = finish_step(h, ln, ss.vs_calls, ss.live, ss.B, ln.Bq, &live, &calls))) return rc;
    if ((rc = emit(ln.Bq, lane_q[(size_t)k], ln.st, ln.X))) return rc;
    if (k + nl < nq)
      if ((rc = query_issue(h, h->streams[(size_t)lane_q[(size_t)(k + nl)]], ln))) return rc;
  }
  return sync_all(h);
}

}  // namespace
