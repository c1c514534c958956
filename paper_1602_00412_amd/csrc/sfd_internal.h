// Internal interface between the host orchestrator (sfd_api.cpp) and the HIP kernels.
// Every launcher enqueues on `st` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfd {

constexpr int kMaxEll = 256;     // panels up to 256 wide; FP64 eigensolves up to 512 x 512
constexpr int kSpmmChunk = 256;  // entries per wave in the sparse products; longer rows are split
constexpr int kXcdBands = 8;     // row bands of the hot-column pieces (one per XCD)
constexpr int kHotCap = 32768;   // hot columns a transposed-product schedule holds at most (and <= d)
constexpr int kHotMinDefault = 160;  // entries from which a CSC column is cut into XCD-local pieces

// One buffer of a lockstep group (buffers of several streams running their SimultaneousIteration
// together, one launch per step for all of them): its segment of a stacked panel (first row,
// rows) and the Gram launch geometry a single-buffer launch over that many rows has, so every
// per-buffer result equals the single-buffer one.
struct GroupSeg {
  int64_t row0;
  int64_t rows;
  int rpb;  // rows per Gram block
  int nb;   // Gram blocks
};

// element type of a dense panel (FP32, or BF16 in the precision form: the upper 16 bits of an
// FP32 value, rounded to nearest even)
enum class PanelType { F32, BF16 };

// Small device-resident scalars of one buffer step.
struct DevScalars {
  double fro2A;       // ||A'||_F^2 (repeated entries summed)
  double fro2Bp;      // ||B'||_F^2 = sum_i (lambda_i^2 - lambda_ell^2)_+
  double S;           // fro2A - fro2Bp = trace(A'^T A' - B'^T B')
  double half_delta;  // Delta / 2, Delta = S / (alpha ell)
  double lam_ell2;    // lambda_ell^2
  double ln_norm;     // running ln ||C^s x|| of VerifySpectral
  double inv_norm;    // 1 / ||w|| of the last power step (scales the next input)
  double mu_ell;      // DenseShrink pivot mu_ell (0 when the stack is kept exactly)
  int zero_flag;      // a power step vector was exactly 0
  int dropped;        // directions dropped by the last pivoted Cholesky
  int pad[2];
};

// ---------------------------------------------------------------- utilities (sfd_util.hip)
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t st);
hipError_t fill_i32(int* p, int64_t n, int v, hipStream_t st);
// exclusive prefix sum of n int32 values; out[n] = total (out has n + 1 entries; may alias in)
hipError_t scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t st);
int64_t scan_tmp_ints(int64_t n);
// copy a d x w block between panels with pitches (elements)
hipError_t copy_panel(const float* src, int lds, float* dst, int ldd, int64_t rows, int w, hipStream_t st);
// K consecutive L x L identity matrices
hipError_t set_identity(float* T, int L, int K, hipStream_t st);
// dst[i] = BF16 rounding of src[i], n elements
hipError_t to_bf16(const float* src, int64_t n, uint16_t* dst, hipStream_t st);
// out (ell x d, row-major) = panel^T restricted to the first ell columns
hipError_t transpose_out(const float* panel, int ld, int64_t d, int ell, float* out, hipStream_t st);
// lockstep groups: for the K buffers with q[k] == *iter, Pt + k n <- X + k n (n floats) and
// Wp + k m <- W + k m (m doubles); iter and q in device memory
hipError_t group_snapshot(const int* iter, const int* q, int K, const float* X, float* Pt, int64_t n, const double* W,
                          double* Wp, int64_t m, hipStream_t st);
// *c += v (device counter, one thread)
hipError_t counter_add(int* c, int v, hipStream_t st);

// ---------------------------------------------------------------- ingest / CSC (sfd_ingest.hip)
// validation of a device CSR block: err |= 1 for a decreasing or over-long row, 2 for a bad index
hipError_t validate_rows(const int64_t* indptr, int64_t nrows, int64_t d, int* err, hipStream_t st);
hipError_t validate_indices(const int32_t* idx, int64_t lo, int64_t hi, int64_t d, int* err, hipStream_t st);
// flush cut rows of a device block (single thread): cuts[k] = last row of the k-th full buffer,
// cut_ptr[k] = indptr[cuts[k] + 1]; *ncuts = count
hipError_t find_cuts(const int64_t* indptr, int64_t nrows, int64_t buf_rows, int64_t buf_nnz, int64_t budget,
                     int64_t d, int64_t max_cuts, int64_t* cuts, int64_t* cut_ptr, int64_t* ncuts, hipStream_t st);
// rowptr[m0 + 1 + i] = indptr[r0 + 1 + i] - indptr[r0] + nnz0 for i < cnt
hipError_t append_rowptr(const int64_t* indptr, int64_t r0, int64_t cnt, int* rowptr, int m0, int nnz0,
                         hipStream_t st);
// CSR -> CSC by a stable LSD radix sort of the column ids
struct CscWork {
  int* counts;    // d + 1
  int* scan_tmp;
  int* rowid;     // cap
  int* keys0; int* keys1; int* vals0; int* vals1;  // cap each
  int* hist;      // 256 * tiles
  double* part;   // reduction partials
};
// *sorted_keys: the entries' sorted column ids, in one of w's arrays
hipError_t build_csc(const int* rowptr, const int* colidx, const float* val, int m, int nnz, int64_t d,
                     int* cscptr, int* cscrow, float* cscval, CscWork& w, const int** sorted_keys, hipStream_t st);
// ||A'||_F^2 with repeated (row, column) entries summed, for each of K column segments of d
// columns of a CSC (keys: its entries' sorted column ids, from build_csc) (the buffers of a group; K = 1 for one buffer) into sc[k].fro2A; part holds
// fro2_part_doubles(K) doubles
hipError_t fro2_segments(const int* cscptr, const int* keys, const int* cscrow, const float* cscval, int64_t d, int K,
                         double* part, DevScalars* sc, hipStream_t st);
int fro2_part_doubles(int K);
// dst[i] = src[i] + add, i < n
hipError_t offset_copy(const int* src, int64_t n, int add, int* dst, hipStream_t st);
// dense transpose of a small buffer (m <= L rows): out[j][r] = sum of A'[r][j], pitch ld, width L
hipError_t dense_from_csc(const int* cscptr, const int* cscrow, const float* cscval, int64_t d, float* out,
                          int ld, int L, hipStream_t st);

// ---------------------------------------------------------------- sparse products (sfd_spmm.hip)
struct Schedule {
  int* nch;          // rows + 1 : chunks per row -> scanned chunk start; nch[rows] = number of chunks
  int* pslot;        // output rows + 1 : partial slots per long output row -> scanned slot start
  int4* desc;        // chunk -> {output row, first entry, end entry, partial slot or -1 (whole row)}
  int* long_rows;    // output rows whose chunks write partial slots
  int* counters;     // [0] = number of long rows
  int* regions;      // kXcdBands + 2 chunk offsets: the chunk ranges the product kernels walk
  int rows;          // rows of the structure the schedule was built for
  int64_t max_chunks;  // capacity of desc (bounds the grid)
  // 0: one chunk range [regions[0], regions[1]) walked by every block.  kXcdBands (hot-column
  // pieces of a CSC, schedule_build_hot): range b < kXcdBands holds the pieces of the hot
  // columns whose entries lie in row band b, walked by the blocks with blockIdx % kXcdBands == b
  // (dispatched to XCD b, so the rows they gather stay in that XCD's L2); range kXcdBands holds
  // the other columns, walked by every block.
  int nlocal = 0;
  bool transposed = false;  // the CSC of a buffer (A'^T products); only names the kernels apart
  int* queue = nullptr;     // kXcdBands + 2 work-queue counters of the ranges (persistent products)
  // rows staged in LDS (CSR schedules of the products Y = A' X; stage_build): the column ids
  // with the staged ones encoded (nnz), the staged columns, {count, threshold, histogram[32]},
  // and the slot of every column (d)
  int* stage_idx = nullptr;
  int* hot_cols = nullptr;
  int* hot_n = nullptr;
  int* slot_of = nullptr;
};

// Launch configuration of a sparse product.  Every configuration sums each output row's entries
// in the same order, so the choice changes the time, never the bits.
struct SpmmConfig {
  int unroll = 0;     // FP32 panels: entries gathered per batch, 8 (0: default) or 4
  bool queue = false; // persistent grid fed by the schedule's work queues
  int occupancy = 4;  // persistent grid: blocks per CU
  bool stage = false; // Y = A' X with a queue grid: the most popular columns' rows of X in LDS
  int live = 0;       // 16-byte segments of each panel row to gather (0: all).  The columns past
                      // the sketch's ell are zero in every panel, so the segments wholly past the
                      // last 64-byte sector that holds a live column need not be fetched
};
// the segments of a panel row (elem_bytes per element) that reach the 64-byte sector holding
// column ell - 1: what SpmmConfig::live needs to gather
int live_segments(int ell, int elem_bytes);
// builds the chunk schedule of a CSR/CSC structure on the device (no host synchronisation)
hipError_t schedule_build(const int* ptr, int rows, Schedule& s, int* scan_tmp, hipStream_t st);
// staging of a buffer's CSR schedule s: the columns whose entry counts (from its CSC colptr) reach
// the largest power of two that keeps them within 32 KB of LDS rows (L wide, FP32 or BF16), and
// the column ids of colidx (nnz) with those encoded as -1 - slot, into s's staging arrays
hipError_t stage_build(const int* cscptr, int d, const int* colidx, int64_t nnz, int L, bool bf16, Schedule& s,
                       hipStream_t st);
// The schedule of a buffer's CSC (d columns, rows ascending in every column) with XCD-local
// pieces: the rows of the buffer (CSR rowptr, m rows, nnz entries) are cut into kXcdBands
// contiguous bands of about nnz / kXcdBands entries (row r in band floor(rowptr[r] kXcdBands /
// nnz)); a column of at least hot_min entries is cut at the band boundaries, and its pieces'
// chunks all write partial slots that the fix-up adds in band order, then chunk order.  s.nch
// holds (kXcdBands + 1) d + 1 ints, s.pslot d + 1, s.desc d + 2 nnz / kSpmmChunk + kXcdBands
// hot columns + 2 (hot_min >= nnz / H keeps the hot columns within H).
hipError_t schedule_build_hot(const int* cscptr, const int* cscrow, int d, const int* rowptr, int m, int nnz,
                              int hot_min, Schedule& s, int* scan_tmp, hipStream_t st);
// Y[r, :] = sum_k val[k] X[idx[k], :] over the structure of schedule s (its entries idx, val);
// rows of width L (32, 64, 128 or 256) with pitches ldx / ldy in elements; FP32 accumulation.
// (values, panel in -> panel out): (FP32, F32 -> F32), (BF16, BF16 -> BF16), (FP32, BF16 -> F32);
// val_bf16: val holds BF16 values (uint16).  This launches the main kernel only; spmm_finish
// completes the product.
hipError_t spmm(const Schedule& s, const int* idx, const void* val, bool val_bf16, const void* X, PanelType xt, int ldx,
                void* Y, PanelType yt, int ldy, int L, float* partial, const SpmmConfig& cfg, hipStream_t st);
// clears the schedule's work queues (the fix-up does this after every product; needed only
// between products launched back to back without one)
hipError_t spmm_queue_reset(const Schedule& s, hipStream_t st);
// the long rows' fix-up of a product
hipError_t spmm_finish(const Schedule& s, float* partial, void* Y, PanelType yt, int ldy, int L, hipStream_t st);
// z[r] = scale * sum_k val[k] y[idx[k]], scale = *scale_ptr (nullptr: 1); for a group's stacked
// structure (seg_rows: K + 1 row offsets, device) row r of buffer k is scaled by
// scale_ptr[k sstride]
hipError_t spmv(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* y,
                const double* scale_ptr, float* z, float* partial, hipStream_t st, const int64_t* seg_rows = nullptr,
                int K = 1, int sstride = 0);

// ---------------------------------------------------------------- dense panels (sfd_dense.hip)
// partial buffers of the Gram kernels hold at most gram_max_blocks() blocks of 4*L*L floats
int gram_max_blocks();
// P <- P T in place (rows x L, L in {32, 64, 128, 256}, FP32 or BF16; T: L x L f32, upper
// triangular: its zero blocks below the diagonal are skipped) and W = Gram of the result as
// stored (FP64, L x L)
hipError_t xform_gram(void* P, PanelType pt, int ld, int64_t rows, int L, const float* T, float* partials, double* W,
                      hipStream_t st);
// the same for the K buffers of a group: segs (device, K entries) give each buffer's rows of P;
// buffer k uses T + k L L, partials + k gram_partial_stride(L), W + k L L; nb = max segs[k].nb.
// With segs = nullptr and K = 1 it is the single-buffer launch over (rows, rpb, nb).
hipError_t xform_gram_group(void* P, PanelType pt, int ld, int64_t rows, int rpb, int nb, const GroupSeg* segs, int K,
                            int L, const float* T, float* partials, double* W, hipStream_t st);
void gram_geometry(int64_t rows, int L, int* nb, int* rpb);
// BF16 panels (sfd_bf16.hip): P <- P T on BF16 MFMA (T split into two BF16 parts when split) and
// the per-block partial Grams of the stored result (upper tiles, FP32), for the Gram reduction
hipError_t xform_gram_bf16_partials(uint16_t* P, int ld, int64_t rows, int rpb, int nb, const GroupSeg* segs, int K,
                                    int L, const float* T, float* partials, int64_t pstride, bool split,
                                    hipStream_t st);
int64_t gram_partial_stride(int L);
// Gram of the side-by-side panel [P1 | P2] (rows x 2L, each half L wide) into FP64 (2L x 2L)
hipError_t gram2(const float* P1, int ld1, const float* P2, int ld2, int64_t rows, int L, float* partials, double* W,
                 hipStream_t st);
// out[j, 0:L] = [P1[j, 0:L] | P2[j, 0:L]] * T2 (T2: 2L x L, f32); out may be P1 (row-wise in place)
hipError_t panel_xform2(const float* P1, int ld1, const float* P2, int ld2, int L, const float* T2, float* out,
                        int ldo, int64_t rows, hipStream_t st);
// partial sums of P^T y over row blocks: part[b][k] = sum_{j in block} P[j][k] * y[j] * scale
int gemv_blocks(int64_t rows);
// K > 1: buffer k reads P + k rows ld, y + k rows, scale_ptr + k sstride (doubles) and writes
// part + k gemv_blocks(rows) L
hipError_t panel_gemv_t(const float* P, int ld, int L, int64_t rows, const float* y, const double* scale_ptr,
                        float* part, hipStream_t st, int K = 1, int sstride = 0);
// Philox4x64-10 start block: out[row][col] for row < d, col < ell (pitch ld); pads untouched
hipError_t start_block(uint64_t seed, uint64_t stream_id, uint64_t buffer, uint64_t attempt, uint64_t purpose,
                       int64_t d, int ell, float* out, int ld, hipStream_t st);

// ---------------------------------------------------------------- small FP64 solvers (sfd_small.hip)
// pivoted Cholesky of the ell x ell Gram W (pitch ldw) and the inverse of its factor, T (L x L,
// f32, zero-padded); columns whose residual falls to tau * (their norm^2) are dropped
// (ell > 128: Rw holds chol_work_doubles(L) doubles per buffer, the factor between the passes)
hipError_t chol_inv(const double* W, int ldw, int ell, int L, double tau, float* T, DevScalars* sc, double* Rw,
                    hipStream_t st);
int64_t chol_work_doubles(int L);
// group launches (one workgroup per buffer k): chol_inv on W + k wstride -> T + k L L, sc + k;
// eig_sym on A + k astride -> evals + k estride, evecs + k vstride; ssh_post on evals + k estride,
// H + k vstride -> M64 / M32 + k L L, sc + k
hipError_t chol_inv_group(const double* W, int ldw, int ell, int L, double tau, float* T, DevScalars* sc, int K,
                          int64_t wstride, double* Rw, hipStream_t st);
// (n > 112: work holds eig_work_bytes(n) bytes per buffer, wstride bytes apart; n <= 512; the
// eigenvectors of the nvec largest eigenvalues are computed, the other columns may be zero)
hipError_t eig_sym_group(const double* A, int lda, int n, int nvec, double* evals, double* evecs, int K,
                         int64_t astride, int64_t estride, int64_t vstride, void* work, int64_t wstride,
                         hipStream_t st);
int64_t eig_work_bytes(int n);
// the tridiagonal solver (sfd_eig_tri.hip) behind eig_sym_group for 112 < n <= 512
hipError_t eig_tri_group(const double* A, int lda, int n, int nvec, double* evals, double* evecs, int K,
                         int64_t astride, int64_t estride, int64_t vstride, void* work, int64_t wstride,
                         hipStream_t st);
int64_t eig_tri_work_bytes(int n);
hipError_t ssh_post_group(const double* evals, const double* H, int ell, int L, double alpha, double* M64, float* M32,
                          DevScalars* sc, int K, int64_t estride, int64_t vstride, hipStream_t st);
// symmetric eigensolver (cyclic Jacobi, FP64) of the n x n matrix A (pitch lda), n <= 2*kMaxEll:
// evals descending, evecs column i <-> evals[i], pitch n (columns beyond the nvec largest may
// be zero); work: eig_work_bytes(n) bytes (may be null when that is 0)
hipError_t eig_sym(const double* A, int lda, int n, int nvec, double* evals, double* evecs, void* work,
                   hipStream_t st);
// SparseShrink tail: from the eigenpairs of P P^T: M = H D (ell x ell, FP64 and f32 L x L),
// ||B'||^2, S, Delta/2, lambda_ell^2
hipError_t ssh_post(const double* evals, const double* H, int ell, int L, double alpha, double* M64, float* M32,
                    DevScalars* sc, hipStream_t st);
// exact buffer: M = I
hipError_t ssh_identity(int ell, int L, double* M64, float* M32, DevScalars* sc, hipStream_t st);
// DenseShrink stack Gram: SS = diag(I, M^T) W2 diag(I, M) (2 ell x 2 ell) from W2 (2L x 2L);
// scratch: ell x ell doubles
hipError_t dsh_assemble(const double* W2, int L, int ell, const double* M64, double* SS, double* scratch,
                        hipStream_t st);
// DenseShrink factors: T2 (2L x L, f32) = diag(I, M) U_ell D; lossless: no shift
hipError_t dsh_post(const double* evals, const double* U, int ell, int L, const double* M64, int lossless,
                    float* T2, DevScalars* sc, hipStream_t st);

// ---------------------------------------------------------------- VerifySpectral (sfd_vs.hip)
// The VerifySpectral launches take K buffers of a group (K = 1: one buffer); buffer k uses
// vectors at k d, partials at k (blocks), M64 at k L L, c2 at k 2 L, scalars sc + k.
// x: gaussian vector already in w; sets sc->inv_norm = 1/||w||, ln_norm = 0, zero_flag = 0
hipError_t vs_init(const float* w, int64_t d, double* part, DevScalars* sc, hipStream_t st, int K = 1);
int vs_norm_blocks();
// c2 = M M^T c with c = sum of gemv partials (nb blocks)
hipError_t vs_small(const float* part, int nb, const double* M64, int ell, int L, float* c2, hipStream_t st,
                    int K = 1);
// w = w_raw - P c2; partial ||w||^2 per block
int vs_finish_blocks(int64_t d);
hipError_t vs_finish(const float* w_raw, const float* P, int ld, int L, int ell, const float* c2, int64_t d,
                     float* w, double* part, hipStream_t st, int K = 1);
// reduce ||w||^2, ln_norm += ln||w|| - ln(Delta/2), inv_norm = 1/||w||; in a group, tsteps[k]
// counts buffer k's remaining steps down (a buffer at 0 is left as it is), so every step is the
// same launch
hipError_t vs_norm(const double* part, int nb, DevScalars* sc, hipStream_t st, int K = 1, int* tsteps = nullptr);

}  // namespace sfd
