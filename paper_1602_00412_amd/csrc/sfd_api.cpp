// Host orchestrator and C ABI of the Sparse Frequent Directions library (declarations and
// conventions in include/sfd.h).
//
// Per handle the device holds: the buffer A' as CSR (and, per buffer step, its CSC copy), the
// panel C = [B^T | P^T] (d x 2L, row-major, L = ell rounded up to 32) whose left half is the
// sketch B stored transposed, the SimultaneousIteration panels X (d x L) and Y (m x L), and
// the small FP64 work of the shrink steps.  The buffer step (Alg 2's flush) runs:
//   CSC build -> G (Philox) -> q x { Y = orth(A' X); X = orth(A'^T Y) } -> Y = orth(A' X)
//   -> P^T = A'^T Y -> Gram of C -> eig(P P^T) -> M = H D (so B'^T = P^T M)
//   -> VerifySpectral (Alg 6) -> on reject retry with the next attempt's G (Alg 4)
//   -> DenseShrink (Alg 5) of [B; B'] through the Gram of C -> B^T = C T2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "sfd.h"
#include "sfd_internal.h"

using namespace sfd;

namespace {

constexpr double kAlpha = 6.0 / 41.0;          // alpha of Alg 4 / Theorem 3.1
constexpr double kUnitRoundoff32 = 1.0 / 16777216.0;  // 2^-24: the panels' arithmetic
constexpr double kCholDropTol = 1e-5;          // relative residual^2 below which a column is dependent
constexpr int kPurposeSI = 0, kPurposeVS = 1, kPurposeQuerySI = 2, kPurposeQueryVS = 3;

}  // namespace

struct sfd_s {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  int64_t d = 0;
  int ell = 0;
  int L = 0;
  double eps = 0.25;
  uint64_t seed = 0, stream_id = 0;
  double delta = 0.01;
  int q_override = 0;
  int max_attempts = 16;
  int verify = 1;
  // stream state
  int live = 0;
  int64_t flushes = 0, vs_calls = 0;
  int m = 0;    // pending rows
  int nnz = 0;  // pending stored entries
  int error = 0;
  sfd_stats_t stats{};
  int64_t cap = 0;
  // device memory
  int* rowptr = nullptr;
  int* colidx = nullptr;
  float* val = nullptr;
  int* cscptr = nullptr;
  int* cscrow = nullptr;
  float* cscval = nullptr;
  CscWork csc{};
  Schedule sr{}, sc_sched{};
  float* partial = nullptr;
  float *X = nullptr, *Y = nullptr, *C = nullptr, *Bq = nullptr;
  float* gram_part = nullptr;
  double* W = nullptr;
  double *evals = nullptr, *evecs = nullptr, *SS = nullptr, *M64 = nullptr;
  float *M32 = nullptr, *T = nullptr, *T2 = nullptr;
  float *vs_w = nullptr, *vs_wraw = nullptr, *vs_z = nullptr, *vs_c2 = nullptr, *vs_gpart = nullptr;
  double* vs_npart = nullptr;
  DevScalars* sc = nullptr;
  int* err_dev = nullptr;
  int64_t* cut_dev = nullptr;  // [0] count, then cuts, then cut_ptr
  int64_t cut_cap = 0;
  int* scan_tmp = nullptr;
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
  // pinned host staging
  DevScalars* sc_host = nullptr;
  int64_t* i64_host = nullptr;  // small readbacks
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
  if (h->sc_host) (void)hipHostFree(h->sc_host);
  if (h->i64_host) (void)hipHostFree(h->i64_host);
  h->sc_host = nullptr;
  h->i64_host = nullptr;
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  h->own_stream = nullptr;
}

int fail(sfd_t* h, int code) {
  if (code == SFD_E_DEVICE || code == SFD_E_NOCONVERGE) h->error = code;
  return code;
}

#define CK(expr)                                        \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return fail(h, SFD_E_DEVICE); \
  } while (0)

// Events bracketing the launches of one kernel class on the handle's stream.
struct ProfScope {
  sfd_t* h;
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
  ProfScope(sfd_t* h_, int cls_, double bytes_, double flops_ = 0.0, int launches_ = 1)
      : h(h_), cls(cls_), bytes(bytes_), flops(flops_), launches(launches_) {
    if (h->prof) {
      a = take(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~ProfScope() {
    if (!h->prof || !a) return;
    hipEvent_t b = take(h);
    if (!b) {
      h->ev_pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, h->stream);
    h->pending.push_back({cls, a, b, bytes, flops, launches});
  }
};

void prof_resolve(sfd_t* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->profile.ms[p.cls] += ms;
      h->profile.launches[p.cls] += p.launches;
      h->profile.bytes[p.cls] += p.bytes;
      h->profile.flops[p.cls] += p.flops;
    }
    h->ev_pool.push_back(p.a);
    h->ev_pool.push_back(p.b);
  }
  h->pending.clear();
}

int sync(sfd_t* h) {
  CK(hipStreamSynchronize(h->stream));
  if (!h->pending.empty()) prof_resolve(h);
  return SFD_OK;
}

int read_scalars(sfd_t* h) {
  CK(hipMemcpyAsync(h->sc_host, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
  return sync(h);
}

int alloc_state(sfd_t* h) {
  const int64_t d = h->d, L = h->L;
  const int64_t cap = h->ell * d + d;
  h->cap = cap;
  const int64_t tiles = (cap + 2047) / 2048;
  const int64_t max_chunks = d + cap / kSpmmChunk + 2;
  const int64_t slots = 2 * cap / kSpmmChunk + 16;
  bool ok = true;
  ok = ok && dalloc(h, &h->rowptr, d + 1) && dalloc(h, &h->colidx, cap) && dalloc(h, &h->val, cap);
  ok = ok && dalloc(h, &h->cscptr, d + 1) && dalloc(h, &h->cscrow, cap) && dalloc(h, &h->cscval, cap);
  ok = ok && dalloc(h, &h->csc.counts, d + 1) && dalloc(h, &h->csc.rowid, cap);
  ok = ok && dalloc(h, &h->csc.keys0, cap) && dalloc(h, &h->csc.keys1, cap);
  ok = ok && dalloc(h, &h->csc.vals0, cap) && dalloc(h, &h->csc.vals1, cap);
  ok = ok && dalloc(h, &h->csc.hist, 256 * tiles + 1) && dalloc(h, &h->csc.part, 1024);
  ok = ok && dalloc(h, &h->scan_tmp, scan_tmp_ints(std::max<int64_t>(256 * tiles + 1, d + 1)) + 16);
  h->csc.scan_tmp = h->scan_tmp;
  for (Schedule* s : {&h->sr, &h->sc_sched}) {
    ok = ok && dalloc(h, &s->nch, d + 1) && dalloc(h, &s->pslot, d + 1) && dalloc(h, &s->chunk_row, max_chunks) &&
         dalloc(h, &s->long_rows, d + 1) && dalloc(h, &s->counters, 4);
  }
  ok = ok && dalloc(h, &h->partial, slots * L);
  ok = ok && dalloc(h, &h->X, d * L) && dalloc(h, &h->Y, d * L) && dalloc(h, &h->C, d * 2 * L) &&
       dalloc(h, &h->Bq, d * L);
  ok = ok && dalloc(h, &h->gram_part, (int64_t)gram_max_blocks() * 4 * L * L) && dalloc(h, &h->W, 4 * L * L);
  ok = ok && dalloc(h, &h->evals, 2 * L) && dalloc(h, &h->evecs, 4 * L * L) && dalloc(h, &h->SS, 4 * L * L);
  ok = ok && dalloc(h, &h->M64, L * L) && dalloc(h, &h->M32, L * L) && dalloc(h, &h->T, L * L) &&
       dalloc(h, &h->T2, 2 * L * L);
  ok = ok && dalloc(h, &h->vs_w, d) && dalloc(h, &h->vs_wraw, d) && dalloc(h, &h->vs_z, d) &&
       dalloc(h, &h->vs_c2, 2 * L) && dalloc(h, &h->vs_gpart, (int64_t)gemv_blocks(d) * L) &&
       dalloc(h, &h->vs_npart, 2048);
  ok = ok && dalloc(h, &h->sc, 1) && dalloc(h, &h->err_dev, 4);
  if (!ok) return SFD_E_NOMEM;
  if (hipHostMalloc((void**)&h->sc_host, sizeof(DevScalars)) != hipSuccess) return SFD_E_NOMEM;
  if (hipHostMalloc((void**)&h->i64_host, sizeof(int64_t) * 16) != hipSuccess) return SFD_E_NOMEM;
  return SFD_OK;
}

int reset_state(sfd_t* h) {
  h->live = 0;
  h->flushes = 0;
  h->vs_calls = 0;
  h->m = 0;
  h->nnz = 0;
  h->error = 0;
  std::memset(&h->stats, 0, sizeof(h->stats));
  CK(fill_f32(h->C, h->d * 2 * h->L, 0.f, h->stream));
  CK(fill_i32(h->rowptr, 1, 0, h->stream));
  return sync(h);
}

int si_iterations(const sfd_t* h, int m) {
  if (h->q_override > 0) return h->q_override;
  return (int)std::ceil(std::log((double)m / h->eps) / h->eps);
}

int vs_steps(const sfd_t* h, int64_t i) {
  double di = h->delta / (2.0 * (double)i * (double)i);
  return (int)std::ceil(std::log2((double)h->d / di));
}

int build_schedule(sfd_t* h, const int* ptr, int rows, Schedule& s) {
  hipStream_t st = h->stream;
  CK(schedule_counts(ptr, rows, s, st));
  CK(scan_exclusive(s.nch, s.nch, rows, h->scan_tmp, st));
  CK(scan_exclusive(s.pslot, s.pslot, rows, h->scan_tmp, st));
  CK(schedule_finish(ptr, rows, s, st));
  int* hv = reinterpret_cast<int*>(h->i64_host);
  CK(hipMemcpyAsync(hv + 0, s.nch + rows, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(hv + 1, s.pslot + rows, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(hv + 2, s.counters, sizeof(int), hipMemcpyDeviceToHost, st));
  int rc = sync(h);
  if (rc) return rc;
  s.nchunks = hv[0];
  s.nslots = hv[1];
  s.nlong = hv[2];
  return SFD_OK;
}

// panel <- panel * R^{-1} with R the (pivoted) Cholesky factor of panel^T panel
int orth(sfd_t* h, float* panel, int64_t rows) {
  hipStream_t st = h->stream;
  const int L = h->L;
  const double ell = h->ell;
  {
    ProfScope ps(h, SFD_PROF_GRAM, 4.0 * rows * ell, 2.0 * rows * ell * ell, 2);
    CK(gram(panel, L, rows, L, h->gram_part, h->W, st));
  }
  {
    ProfScope ps(h, SFD_PROF_CHOL, 8.0 * ell * ell, ell * ell * ell, 1);
    CK(chol_inv(h->W, L, h->ell, L, kCholDropTol, h->T, h->sc, st));
  }
  {
    ProfScope ps(h, SFD_PROF_XFORM, 8.0 * rows * ell, 2.0 * rows * ell * ell, 1);
    CK(panel_xform(panel, L, L, h->T, panel, L, L, rows, st));
  }
  return SFD_OK;
}

// algorithmic bytes of one sparse product over the buffer: the stored entries (id + value)
// and row pointers once, the input panel read once, the output panel written once
double spmm_bytes(const sfd_t* h, bool transposed) {
  const double N = h->nnz, m = h->m, d = (double)h->d, ell = h->ell;
  return 8.0 * N + 4.0 * ((transposed ? d : m) + 1) + 4.0 * ell * (m + d);
}

int spmm_csr(sfd_t* h, const float* X, int ldx, float* Y, int ldy) {
  ProfScope ps(h, SFD_PROF_SPMM_CSR, spmm_bytes(h, false), 2.0 * h->nnz * h->ell, 1);
  CK(spmm(h->rowptr, h->colidx, h->val, h->m, h->sr, X, ldx, Y, ldy, h->L, h->partial, h->stream));
  return SFD_OK;
}

int spmm_csc(sfd_t* h, const float* Y, int ldy, float* X, int ldx) {
  ProfScope ps(h, SFD_PROF_SPMM_CSC, spmm_bytes(h, true), 2.0 * h->nnz * h->ell, 1);
  CK(spmm(h->cscptr, h->cscrow, h->cscval, (int)h->d, h->sc_sched, Y, ldy, X, ldx, h->L, h->partial, h->stream));
  return SFD_OK;
}

// SparseShrink (Alg 3) of the buffer with start block (buffer, attempt, purpose): leaves P^T in
// the right half of C, the Gram of C in W, M = H D and the scalars of Alg 4 on the device.
int sparse_shrink(sfd_t* h, int purpose, int64_t buffer, int attempt, int q) {
  hipStream_t st = h->stream;
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  const int m = h->m;
  int rc;
  {
    ProfScope ps(h, SFD_PROF_OTHER, 4.0 * d * ell, 0.0, 2);
    CK(fill_f32(h->X, d * L, 0.f, st));
    CK(start_block(h->seed, h->stream_id, (uint64_t)buffer, (uint64_t)attempt, (uint64_t)purpose, d, ell, h->X, L,
                   st));
  }
  if ((rc = orth(h, h->X, d))) return rc;
  for (int it = 0; it < q; ++it) {
    if ((rc = spmm_csr(h, h->X, L, h->Y, L))) return rc;
    if ((rc = orth(h, h->Y, m))) return rc;
    if ((rc = spmm_csc(h, h->Y, L, h->X, L))) return rc;
    if ((rc = orth(h, h->X, d))) return rc;
  }
  if ((rc = spmm_csr(h, h->X, L, h->Y, L))) return rc;
  if ((rc = orth(h, h->Y, m))) return rc;
  if ((rc = spmm_csc(h, h->Y, L, h->C + L, 2 * L))) return rc;
  {
    ProfScope ps(h, SFD_PROF_GRAM, 8.0 * d * ell, 8.0 * d * ell * ell, 2);
    CK(gram(h->C, 2 * L, d, 2 * L, h->gram_part, h->W, st));
  }
  {
    ProfScope ps(h, SFD_PROF_EIG, 16.0 * ell * ell, 0.0, 1);
    CK(eig_sym(h->W + (int64_t)L * 2 * L + L, 2 * L, ell, h->evals, h->evecs, st));
  }
  {
    ProfScope ps(h, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(ssh_post(h->evals, h->evecs, ell, L, kAlpha, h->M64, h->M32, h->sc, st));
  }
  return SFD_OK;
}

// VerifySpectral (Alg 6): t power steps from the sphere vector of (buffer, attempt, purpose);
// returns ln ||C^t x|| in *ln_norm.
int verify_spectral(sfd_t* h, int purpose, int64_t buffer, int attempt, int t, double* ln_norm) {
  hipStream_t st = h->stream;
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  const int m = h->m;
  const float* Pt = h->C + L;
  ProfScope ps(h, SFD_PROF_VS, t * (16.0 * h->nnz + 8.0 * d * ell + 4.0 * (2.0 * m + 6.0 * d)),
               t * (4.0 * h->nnz + 4.0 * d * ell), 6 * t + 3);
  CK(start_block(h->seed, h->stream_id, (uint64_t)buffer, (uint64_t)attempt, (uint64_t)purpose, d, 1, h->vs_w, 1, st));
  CK(vs_init(h->vs_w, d, h->vs_npart, h->sc, st));
  for (int s = 0; s < t; ++s) {
    CK(spmv(h->rowptr, h->colidx, h->val, m, h->sr, h->vs_w, &h->sc->inv_norm, h->vs_z, h->partial, st));
    CK(panel_gemv_t(Pt, 2 * L, L, d, h->vs_w, &h->sc->inv_norm, h->vs_gpart, st));
    CK(spmv(h->cscptr, h->cscrow, h->cscval, (int)d, h->sc_sched, h->vs_z, nullptr, h->vs_wraw, h->partial, st));
    CK(vs_small(h->vs_gpart, gemv_blocks(d), h->M64, ell, L, h->vs_c2, st));
    CK(vs_finish(h->vs_wraw, Pt, 2 * L, L, ell, h->vs_c2, d, h->vs_w, h->vs_npart, st));
    CK(vs_norm(h->vs_npart, vs_finish_blocks(d), h->sc, st));
  }
  return SFD_OK;
}

// Fold the pending buffer into B (Alg 2's flush, or a query's copy of it).  B is read from the
// left half of C; the result goes to `out` (pitch out_ld).  live/calls: results for the caller.
int fold(sfd_t* h, int purpose_g, int purpose_x, int64_t buffer, int64_t vs_base, float* out, int out_ld,
         int* live_out, int64_t* calls_out) {
  hipStream_t st = h->stream;
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  const int m = h->m;
  int rc;
  *calls_out = 0;
  {
    ProfScope ps(h, SFD_PROF_CSC_BUILD, 16.0 * h->nnz + 4.0 * (m + d), 0.0, 1);
    CK(build_csc(h->rowptr, h->colidx, h->val, m, h->nnz, d, h->cscptr, h->cscrow, h->cscval, h->csc, h->sc, st));
  }
  int r_add;
  if (m <= ell) {
    // exact buffer (SparseShrink needs ell <= m): P^T = A'^T, M = I
    CK(dense_from_csc(h->cscptr, h->cscrow, h->cscval, d, h->C + L, 2 * L, L, st));
    CK(ssh_identity(ell, L, h->M64, h->M32, h->sc, st));
    CK(gram(h->C, 2 * L, d, 2 * L, h->gram_part, h->W, st));
    r_add = m;
  } else {
    if ((rc = build_schedule(h, h->rowptr, m, h->sr))) return rc;
    if ((rc = build_schedule(h, h->cscptr, (int)d, h->sc_sched))) return rc;
    const int q = si_iterations(h, m);
    bool accepted = false;
    int64_t calls = 0;
    for (int a = 0; a < h->max_attempts && !accepted; ++a) {
      if ((rc = sparse_shrink(h, purpose_g, buffer, a, q))) return rc;
      if ((rc = read_scalars(h))) return rc;
      const DevScalars s = *h->sc_host;
      h->stats.attempts += 1;
      h->stats.last_q = q;
      h->stats.last_fro2_buffer = s.fro2A;
      h->stats.last_lambda_ell2 = s.lam_ell2;
      h->stats.last_delta = 2.0 * s.half_delta;
      if (s.S <= 64.0 * kUnitRoundoff32 * ell * s.fro2A || !h->verify) {
        accepted = true;
        break;
      }
      ++calls;
      const int t = vs_steps(h, vs_base + calls);
      double ln_norm = 0.0;
      if ((rc = verify_spectral(h, purpose_x, buffer, a, t, &ln_norm))) return rc;
      if ((rc = read_scalars(h))) return rc;
      ln_norm = h->sc_host->ln_norm;
      h->stats.last_t = t;
      h->stats.last_ln_norm = ln_norm;
      if (ln_norm <= 0.0)
        accepted = true;
      else
        h->stats.vs_rejects += 1;
    }
    *calls_out = calls;
    if (!accepted) return fail(h, SFD_E_NOCONVERGE);
    r_add = ell - 1;
  }
  const int lossless = (h->live + r_add <= ell) ? 1 : 0;
  {
    ProfScope ps(h, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(dsh_assemble(h->W, L, ell, h->M64, h->SS, st));
  }
  {
    ProfScope ps(h, SFD_PROF_EIG, 64.0 * ell * ell, 0.0, 1);
    CK(eig_sym(h->SS, 2 * ell, 2 * ell, h->evals, h->evecs, st));
  }
  {
    ProfScope ps(h, SFD_PROF_OTHER, 0.0, 0.0, 1);
    CK(dsh_post(h->evals, h->evecs, ell, L, h->M64, lossless, h->T2, h->sc, st));
  }
  {
    ProfScope ps(h, SFD_PROF_XFORM, 12.0 * d * ell, 4.0 * d * ell * ell, 1);
    CK(panel_xform(h->C, 2 * L, 2 * L, h->T2, out, out_ld, L, d, st));
  }
  *live_out = lossless ? h->live + r_add : ell - 1;
  return sync(h);
}

int flush(sfd_t* h) {
  int live = 0;
  int64_t calls = 0;
  int rc = fold(h, kPurposeSI, kPurposeVS, h->flushes, h->vs_calls, h->C, 2 * h->L, &live, &calls);
  if (rc) return rc;
  h->live = live;
  h->vs_calls += calls;
  h->flushes += 1;
  h->m = 0;
  h->nnz = 0;
  return SFD_OK;
}

// Query: fold the pending rows into a copy of B (left in Bq, pitch L), or point at B itself.
int query(sfd_t* h, const float** panel, int* ld, int* live, int64_t* calls) {
  *calls = 0;
  if (h->m == 0) {
    *panel = h->C;
    *ld = 2 * h->L;
    *live = h->live;
    return SFD_OK;
  }
  int rc = fold(h, kPurposeQuerySI, kPurposeQueryVS, h->flushes, h->vs_calls, h->Bq, h->L, live, calls);
  if (rc) return rc;
  *panel = h->Bq;
  *ld = h->L;
  return SFD_OK;
}

int check_handle(sfd_t* h) {
  if (!h) return SFD_E_ARG;
  if (h->error) return SFD_E_STATE;
  return SFD_OK;
}

// Append rows [r0, r1) of a block whose entries [p0, p1) are known on the host.
int copy_rows_device(sfd_t* h, const int64_t* indptr, const int32_t* indices, const float* values, int64_t r0,
                     int64_t r1, int64_t p0, int64_t p1) {
  hipStream_t st = h->stream;
  const int64_t cnt = r1 - r0, nz = p1 - p0;
  if (cnt <= 0) return SFD_OK;
  CK(append_rowptr(indptr, r0, cnt, h->rowptr, h->m, h->nnz, st));
  if (nz > 0) {
    CK(hipMemcpyAsync(h->colidx + h->nnz, indices + p0, sizeof(int32_t) * nz, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(h->val + h->nnz, values + p0, sizeof(float) * nz, hipMemcpyDeviceToDevice, st));
  }
  h->m += (int)cnt;
  h->nnz += (int)nz;
  return SFD_OK;
}

int copy_rows_host(sfd_t* h, const int64_t* indptr, const int32_t* indices, const float* values, int64_t r0,
                   int64_t r1) {
  hipStream_t st = h->stream;
  const int64_t cnt = r1 - r0;
  if (cnt <= 0) return SFD_OK;
  const int64_t p0 = indptr[r0], p1 = indptr[r1], nz = p1 - p0;
  std::vector<int> rp((size_t)cnt);
  for (int64_t i = 0; i < cnt; ++i) rp[(size_t)i] = (int)(indptr[r0 + 1 + i] - p0) + h->nnz;
  CK(hipMemcpyAsync(h->rowptr + h->m + 1, rp.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, st));
  if (nz > 0) {
    CK(hipMemcpyAsync(h->colidx + h->nnz, indices + p0, sizeof(int32_t) * nz, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->val + h->nnz, values + p0, sizeof(float) * nz, hipMemcpyHostToDevice, st));
  }
  int rc = sync(h);  // the staging vector goes out of scope
  if (rc) return rc;
  h->m += (int)cnt;
  h->nnz += (int)nz;
  return SFD_OK;
}

// Alg 2's rule, on the host: rows after which a flush happens.
void host_cuts(const sfd_t* h, const int64_t* indptr, int64_t nrows, std::vector<int64_t>& cuts) {
  const int64_t budget = (int64_t)h->ell * h->d;
  int64_t r = 0, m = h->m, z = h->nnz;
  while (r < nrows) {
    const int64_t target = budget - z + indptr[r];
    const int64_t* it = std::lower_bound(indptr + r + 1, indptr + nrows + 1, target);
    const int64_t by_nnz = (it - indptr) - 1;
    const int64_t by_rows = r + (h->d - m) - 1;
    const int64_t cut = std::min(by_nnz, by_rows);
    if (cut >= nrows) break;
    cuts.push_back(cut);
    r = cut + 1;
    m = 0;
    z = 0;
  }
}

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
    default: return "unknown error";
  }
}

int sfd_create(int64_t d, int32_t ell, double eps, uint64_t seed, sfd_t** out) {
  if (!out) return SFD_E_ARG;
  *out = nullptr;
  if (ell < 1 || d < ell || ell > kMaxEll) return SFD_E_ARG;
  if (!(eps > 0.0 && eps < 1.0)) return SFD_E_ARG;
  if ((int64_t)ell * d + d >= ((int64_t)1 << 31)) return SFD_E_ARG;
  sfd_t* h = new (std::nothrow) sfd_t();
  if (!h) return SFD_E_NOMEM;
  h->d = d;
  h->ell = ell;
  h->L = ((ell + 31) / 32) * 32;
  h->eps = eps;
  h->seed = seed;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return SFD_E_DEVICE;
  }
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return SFD_E_DEVICE;
  }
  h->stream = h->own_stream;
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

int sfd_destroy(sfd_t* h) {
  if (!h) return SFD_OK;
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
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
      if (!(value >= 0) || value > 9.0e15 || value != std::floor(value)) return SFD_E_ARG;
      h->stream_id = (uint64_t)value;
      return SFD_OK;
    default:
      return SFD_E_ARG;
  }
}

int sfd_set_stream(sfd_t* h, void* hip_stream) {
  if (!h) return SFD_E_ARG;
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
  h->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : h->own_stream;
  return SFD_OK;
}

int sfd_get_stats(const sfd_t* h, sfd_stats_t* out) {
  if (!h || !out) return SFD_E_ARG;
  *out = h->stats;
  out->flushes = h->flushes;
  out->vs_calls = h->vs_calls;
  out->live_rows = h->live;
  out->pending_rows = h->m;
  out->pending_nnz = h->nnz;
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
  hipStream_t st = h->stream;
  if (mem == SFD_MEM_HOST) {
    const int64_t lo = indptr[0], hi = indptr[nrows];
    if (hi < lo || lo < 0) return SFD_E_ARG;
    if (hi > lo && (!indices || !values)) return SFD_E_ARG;
    for (int64_t r = 0; r < nrows; ++r) {
      const int64_t len = indptr[r + 1] - indptr[r];
      if (len < 0 || len > h->d) return SFD_E_ARG;
    }
    for (int64_t k = lo; k < hi; ++k)
      if (indices[k] < 0 || (int64_t)indices[k] >= h->d) return SFD_E_INDEX;
    std::vector<int64_t> cuts;
    host_cuts(h, indptr, nrows, cuts);
    int64_t r = 0;
    for (int64_t c : cuts) {
      if ((rc = copy_rows_host(h, indptr, indices, values, r, c + 1))) return rc;
      if ((rc = flush(h))) return rc;
      r = c + 1;
    }
    if ((rc = copy_rows_host(h, indptr, indices, values, r, nrows))) return rc;
    h->stats.rows_seen += nrows;
    h->stats.nnz_seen += hi - lo;
    return SFD_OK;
  }
  // device block: read the ends, validate on the device, then find the cuts on the device
  int64_t* hv = h->i64_host;
  CK(hipMemcpyAsync(hv + 0, indptr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(hv + 1, indptr + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if ((rc = sync(h))) return rc;
  const int64_t lo = hv[0], hi = hv[1];
  if (hi < lo || lo < 0) return SFD_E_ARG;
  if (hi > lo && (!indices || !values)) return SFD_E_ARG;
  CK(fill_i32(h->err_dev, 1, 0, st));
  CK(validate_rows(indptr, nrows, h->d, h->err_dev, st));
  CK(validate_indices(indices, lo, hi, h->d, h->err_dev, st));
  int* hi32 = reinterpret_cast<int*>(hv + 2);
  CK(hipMemcpyAsync(hi32, h->err_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  if ((rc = sync(h))) return rc;
  if (*hi32 & 1) return SFD_E_ARG;
  if (*hi32 & 2) return SFD_E_INDEX;
  const int64_t max_cuts = (nrows + h->m) / h->ell + 2;
  if (max_cuts > h->cut_cap) {
    int64_t* p = nullptr;
    if (!dalloc(h, &p, 1 + 2 * max_cuts)) return SFD_E_NOMEM;
    h->cut_dev = p;
    h->cut_cap = max_cuts;
  }
  CK(find_cuts(indptr, nrows, h->m, h->nnz, (int64_t)h->ell * h->d, h->d, max_cuts, h->cut_dev + 1,
               h->cut_dev + 1 + max_cuts, h->cut_dev, st));
  CK(hipMemcpyAsync(hv + 3, h->cut_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if ((rc = sync(h))) return rc;
  const int64_t ncuts = hv[3];
  std::vector<int64_t> cuts((size_t)ncuts), cut_ptr((size_t)ncuts);
  if (ncuts > 0) {
    CK(hipMemcpy(cuts.data(), h->cut_dev + 1, sizeof(int64_t) * ncuts, hipMemcpyDeviceToHost));
    CK(hipMemcpy(cut_ptr.data(), h->cut_dev + 1 + max_cuts, sizeof(int64_t) * ncuts, hipMemcpyDeviceToHost));
  }
  int64_t r = 0, p = lo;
  for (int64_t k = 0; k < ncuts; ++k) {
    if ((rc = copy_rows_device(h, indptr, indices, values, r, cuts[(size_t)k] + 1, p, cut_ptr[(size_t)k]))) return rc;
    if ((rc = flush(h))) return rc;
    r = cuts[(size_t)k] + 1;
    p = cut_ptr[(size_t)k];
  }
  if ((rc = copy_rows_device(h, indptr, indices, values, r, nrows, p, hi))) return rc;
  if ((rc = sync(h))) return rc;
  h->stats.rows_seen += nrows;
  h->stats.nnz_seen += hi - lo;
  return SFD_OK;
}

int sfd_sketch(sfd_t* h, float* B_out, int mem, int32_t* live_rows) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!B_out || (mem != SFD_MEM_HOST && mem != SFD_MEM_DEVICE)) return SFD_E_ARG;
  DeviceGuard g(h->device);
  const float* panel;
  int ld, live;
  int64_t calls;
  if ((rc = query(h, &panel, &ld, &live, &calls))) return rc;
  if (mem == SFD_MEM_DEVICE) {
    CK(transpose_out(panel, ld, h->d, h->ell, B_out, h->stream));
  } else {
    CK(transpose_out(panel, ld, h->d, h->ell, h->X, h->stream));
    CK(hipMemcpyAsync(B_out, h->X, sizeof(float) * h->d * h->ell, hipMemcpyDeviceToHost, h->stream));
  }
  if ((rc = sync(h))) return rc;
  if (live_rows) *live_rows = live;
  return SFD_OK;
}

int sfd_merge(sfd_t* dst, sfd_t* src) {
  if (!dst || !src || dst == src) return SFD_E_ARG;
  int rc = check_handle(dst);
  if (rc) return rc;
  if ((rc = check_handle(src))) return rc;
  if (dst->d != src->d || dst->ell != src->ell) return SFD_E_SHAPE;
  if (dst->device != src->device) return SFD_E_ARG;
  DeviceGuard g(dst->device);
  sfd_t* h = dst;
  const float *ps, *pd;
  int lds, ldd, live_s, live_d;
  int64_t calls_s, calls_d;
  if ((rc = query(src, &ps, &lds, &live_s, &calls_s))) return rc;
  if ((rc = query(dst, &pd, &ldd, &live_d, &calls_d))) return rc;
  const int L = h->L, ell = h->ell;
  const int64_t d = h->d;
  hipStream_t st = h->stream;
  // C = [query(dst)^T | query(src)^T]; DenseShrink with M = I
  if (pd != h->C) CK(copy_panel(pd, ldd, h->C, 2 * L, d, L, st));
  CK(copy_panel(ps, lds, h->C + L, 2 * L, d, L, st));
  CK(ssh_identity(ell, L, h->M64, h->M32, h->sc, st));
  CK(gram(h->C, 2 * L, d, 2 * L, h->gram_part, h->W, st));
  const int lossless = (live_d + live_s <= ell) ? 1 : 0;
  CK(dsh_assemble(h->W, L, ell, h->M64, h->SS, st));
  CK(eig_sym(h->SS, 2 * ell, 2 * ell, h->evals, h->evecs, st));
  CK(dsh_post(h->evals, h->evecs, ell, L, h->M64, lossless, h->T2, h->sc, st));
  CK(panel_xform(h->C, 2 * L, 2 * L, h->T2, h->C, 2 * L, L, d, st));
  if ((rc = sync(h))) return rc;
  h->live = lossless ? live_d + live_s : ell - 1;
  h->vs_calls += calls_d;
  h->flushes += 1;
  h->m = 0;
  h->nnz = 0;
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

}  // extern "C"
