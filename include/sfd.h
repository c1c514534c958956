/*
 * sfd.h -- C ABI of the MI355X (gfx950) Sparse Frequent Directions library.
 *
 * Method: Ghashami, Liberty & Phillips, "Efficient Frequent Directions Algorithm for Sparse
 * Matrices" (arXiv:1602.00412).  Rows of a sparse matrix A (n x d) arrive one at a time; the
 * library keeps an ell x d sketch B with the covariance guarantee of Theorem 3.1.  Each call
 * below cites the passage that defines the operation it performs.
 *
 * Conventions for every call:
 *  - Ownership: the caller owns every pointer it passes.  Input arrays are consumed (copied
 *    or fully read) before the call returns; output arrays are written before it returns.
 *  - Memory kind: `mem` is SFD_MEM_HOST for host pointers and SFD_MEM_DEVICE for pointers to
 *    device memory of the handle's device (e.g. torch CUDA tensors).
 *  - Synchronisation: work runs on the handle's HIP stream (sfd_set_stream); every call
 *    returns after that work has completed.
 *  - Errors: functions return SFD_OK (0) or a negative SFD_E_* code; sfd_strerror() names it.
 *    Argument and input-validation errors leave the handle unchanged.  On an sfd_t, an
 *    exhausted BoostedSparseShrink loop (SFD_E_NOCONVERGE) also leaves the handle as it was
 *    before the call (sketch, buffer and counters; the stats' last_* figures then describe the
 *    last rejected attempt).  A device error, and SFD_E_NOCONVERGE from sfd_batch_append_csr,
 *    leave the handle in an error state in which every call but sfd_reset/sfd_destroy/
 *    sfd_get_stats returns SFD_E_STATE.
 *  - Threads: a handle must not be used by two threads at once.  Different handles are
 *    independent.
 *  - Sizes: 1 <= ell <= min(d, 256); ell*d + d < 2^31 (int32 buffer indices).
 *  - Streams: an sfd_t is one stream; an sfd_batch_t holds many (see the end of this file).
 */
#ifndef SFD_H
#define SFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfd_s sfd_t;
typedef struct sfd_batch_s sfd_batch_t;

enum {
  SFD_OK = 0,
  SFD_E_ARG = -1,        /* bad argument (size, null pointer, option value) */
  SFD_E_INDEX = -2,      /* a column index outside [0, d) */
  SFD_E_SHAPE = -3,      /* merge of handles with different (d, ell) */
  SFD_E_NOMEM = -4,      /* device allocation failed */
  SFD_E_DEVICE = -5,     /* a HIP runtime call failed */
  SFD_E_NOCONVERGE = -6, /* BoostedSparseShrink exhausted its attempts */
  SFD_E_STATE = -7,      /* handle is in an error state (see above) */
  SFD_E_TOOBIG = -8      /* the work of a no-allocation call exceeds its fixed scratch */
};

enum { SFD_MEM_HOST = 0, SFD_MEM_DEVICE = 1 };

enum { SFD_PRECISION_FP32 = 0, SFD_PRECISION_BF16 = 1 };

enum { SFD_ALGO_SFD = 0, SFD_ALGO_FD = 1 };

/* Option keys for sfd_set_option. */
enum {
  SFD_OPT_DELTA = 1,        /* failure probability delta of Alg 2 / Alg 6, in (0,1); default 0.01 */
  SFD_OPT_Q = 2,            /* power count q of Alg 1; <= 0 restores q = ceil(ln(m/eps)/eps) */
  SFD_OPT_MAX_ATTEMPTS = 3, /* cap on the BoostedSparseShrink loop (Alg 4); default 16 */
  SFD_OPT_VERIFY = 4,       /* 1: BoostedSparseShrink (Alg 4); 0: SparseShrink alone (Sec. 4) */
  SFD_OPT_STREAM_ID = 5,    /* second word of the random key; default 0 */
  SFD_OPT_PROFILE = 6,      /* 1: time every kernel class with HIP events and clear the
                               counters; 0: stop timing.  Default 0. */
  SFD_OPT_CSC_BANDS = 7,    /* XCD-local pieces in the transposed products A'^T Y: 0 automatic
                               (default: on when the gathered panel, rows(A') x panel width, is
                               4-64 MB), 1 off, 8 on.  On: the buffer's rows are cut into 8 bands
                               of about nnz/8 entries, every column with at least
                               SFD_OPT_CSC_HOT_MIN entries is cut at the band boundaries, and the
                               pieces of band b run on the workgroups dispatched to XCD b (its L2
                               then holds that band's rows of Y).  Results agree to rounding. */
  SFD_OPT_LANES = 8,        /* lanes (HIP streams) that run successive buffers' SparseShrink
                               concurrently, 1..16; default 4 (8 for ell > 128, where a buffer
                               step is paced by its one-workgroup FP64 solvers).  A lane beyond
                               those allocated gets its workspaces (one buffer's CSC, schedules
                               and panels: about 28 (ell d + d) + 20 d L bytes, L the panel
                               width 32/64/128/256, e.g. 0.35 GB at d = 1e5, ell = 50) when first
                               asked for, after the work in flight.  Results do not depend on it. */
  SFD_OPT_PRECISION = 9,    /* SFD_PRECISION_FP32 (default) or SFD_PRECISION_BF16: the products
                               1 .. 2q+1 of SimultaneousIteration (Alg 1) read BF16 copies of the
                               buffer's values and BF16 panels and write BF16 panels (FP32
                               accumulation), and the panel transforms and Grams of its
                               CholeskyQR run on BF16 MFMA (FP32 accumulation; the Cholesky
                               stays FP64).  The last product P^T = A'^T Y (Alg 3) reads the
                               FP32 values and the stored BF16 Y, takes its transform from that
                               Y's own Gram and writes FP32, so B'^T B' <= A'^T A' (Property 1)
                               still holds for the FP32 values.  Only the subspace quality
                               changes (cov-err, Sec. 4).  A batch handle runs such buffers on
                               its lanes rather than in lockstep groups. */
  SFD_OPT_ALGORITHM = 10,   /* SFD_ALGO_SFD (default): Alg 2's flush rule (rows(A') = d or
                               nnz(A') >= ell*d) and BoostedSparseShrink; SFD_ALGO_FD: the
                               paper's comparator FrequentDirections (Sec. 2.1) in batches of
                               ell rows -- the buffer flushes at ell rows and is folded exactly
                               by DenseShrink (Alg 5).  Applies to the flushes that follow. */
  SFD_OPT_CSC_HOT_MIN = 11, /* entries from which a column is cut into XCD-local pieces
                               (SFD_OPT_CSC_BANDS), >= 1; default 160.  Raised to
                               ceil(nnz(A') / min(d, 32768)) for a buffer, so at most
                               min(d, 32768) columns are cut. */
  SFD_OPT_TEST_ZERO_ROW = 12,      /* test hook, -1 (default) off: a column id j in [0, d) whose
                                      row of the start block G of SimultaneousIteration (Alg 1)
                                      is set to 0 in the attempts a < SFD_OPT_TEST_ZERO_ATTEMPTS
                                      of every buffer step (flushes and queries).  A direction
                                      that G misses stays out of span(Z) whatever q is, so a
                                      buffer whose dominant direction is e_j gets a SparseShrink
                                      that VerifySpectral (Alg 6) rejects: this runs the retry
                                      loop of BoostedSparseShrink (Alg 4) on purpose. */
  SFD_OPT_TEST_ZERO_ATTEMPTS = 13, /* attempts a < value that SFD_OPT_TEST_ZERO_ROW applies to,
                                      >= 0; default 1 (the first attempt of each buffer). */
  SFD_OPT_CQR2 = 14,               /* precision form only: CholeskyQR2 -- a second panel transform,
                                      Gram and Cholesky after the first, so a panel stored in BF16
                                      is orthonormal to BF16 precision rather than to that times
                                      its condition number.  SFD_CQR2_OFF, SFD_CQR2_FINAL
                                      (default: the final basis Y of Alg 1, whose span defines
                                      B'), SFD_CQR2_ALL (every product's panel). */
  SFD_OPT_AUTOTUNE = 15,           /* 1: the launch configuration of each sparse product
                                      of SimultaneousIteration (entries gathered per batch; a
                                      static grid or a persistent grid fed by a device work queue)
                                      is picked by timing the candidates on the first product of
                                      each shape (panel width, direction, element types, binary
                                      orders of magnitude of entries and rows), once per process;
                                      the environment variable SFD_TUNE_CACHE names a file that
                                      keeps the choices across processes.  Every candidate gives
                                      the same bits.  0 (default): the static grid, gathering 8
                                      entries per batch (4 for BF16 panels). */
  SFD_OPT_GRAPHS = 16,             /* 1 (default): the SimultaneousIteration step of each buffer
                                      step (of a lane, or of a batch handle's lockstep group) and
                                      its VerifySpectral power step are captured once as HIP graphs
                                      and replayed (q, resp. t times); 0 (and while SFD_OPT_PROFILE
                                      is on): issued launch by launch.  Same results. */
  SFD_OPT_PRODUCT_LAUNCH = 17     /* 0 (default): the sparse products' launches as SFD_OPT_AUTOTUNE
                                      decides; 1: static grid; 2: persistent grid fed by device
                                      work queues; 3: as 2, and the products Y = A' X of a lane
                                      stage the input rows of the buffer's most popular columns
                                      (up to 32 KB) in LDS.  Same results in every mode. */
};

enum { SFD_CQR2_OFF = 0, SFD_CQR2_FINAL = 1, SFD_CQR2_ALL = 2 };

/* Kernel classes of the per-phase profile (sfd_get_profile). */
enum {
  SFD_PROF_CSC_BUILD = 0, /* CSR -> CSC of a buffer */
  SFD_PROF_SPMM_CSR = 1,  /* Y = A' X (Alg 1 products with A') */
  SFD_PROF_SPMM_CSC = 2,  /* X = A'^T Y and P^T = A'^T Z (Alg 1, Alg 3) */
  SFD_PROF_GRAM = 3,      /* panel Gram matrices on MFMA */
  SFD_PROF_CHOL = 4,      /* ell x ell FP64 Cholesky + inverse */
  SFD_PROF_XFORM = 5,     /* panel x small-matrix row transforms */
  SFD_PROF_EIG = 6,       /* FP64 symmetric eigensolves */
  SFD_PROF_VS = 7,        /* VerifySpectral power steps (Alg 6) */
  SFD_PROF_OTHER = 8,     /* start blocks, shrink factors, copies */
  SFD_PROF_FIXUP = 9,     /* long-row and hot-column fix-ups that complete a sparse product */
  SFD_PROF_COUNT = 10
};

/* Accumulated per-class figures since profiling was switched on: kernel launches, device time
 * between HIP events recorded around the class's launches on the handle's stream, and the
 * class's algorithmic bytes and flops (what the method must read/write once, and compute). */
typedef struct {
  int64_t launches[16]; /* kernel launches */
  double ms[16];
  double bytes[16];
  double flops[16];
  int64_t calls[16];    /* timed calls (one product, one solve, ...), each of one or more launches */
} sfd_profile_t;

/* Per-handle counters and the last buffer step's figures. */
typedef struct {
  int64_t rows_seen;      /* rows appended so far */
  int64_t nnz_seen;       /* stored entries appended so far */
  int64_t flushes;        /* completed buffer steps (b) */
  int64_t vs_calls;       /* persistent VerifySpectral counter i (Alg 6) */
  int64_t attempts;       /* SparseShrink runs in total (Alg 4 loop iterations) */
  int64_t vs_rejects;     /* VerifySpectral calls that returned False */
  int32_t live_rows;      /* structural count of rows of B that may be non-zero */
  int32_t pending_rows;   /* rows in the buffer A' */
  int64_t pending_nnz;    /* stored entries in the buffer A' */
  int32_t last_q;         /* q of the last SparseShrink */
  int32_t last_t;         /* power steps of the last VerifySpectral */
  double last_ln_norm;    /* ln ||C^t x|| of the last VerifySpectral */
  double last_delta;      /* Delta of the last BoostedSparseShrink attempt */
  double last_fro2_buffer;/* ||A'||_F^2 of the last buffer */
  double last_lambda_ell2;/* lambda_ell^2 of the last SparseShrink */
} sfd_stats_t;

/* Create a stream sketch of width d and ell rows on the current HIP device (Alg 2 inputs).
 * eps is the accuracy of SimultaneousIteration (Alg 1; SparseShrink uses 1/4) and sets the
 * power count q = ceil(ln(m/eps)/eps) for an m-row buffer; seed is the first word of the
 * random key.  B starts at 0 (Alg 2).  Allocates all device memory the handle uses.
 * Errors: SFD_E_ARG (ell < 1, ell > min(d, 256), ell*d + d >= 2^31, eps not in (0,1),
 * out == NULL), SFD_E_NOMEM, SFD_E_DEVICE. */
int sfd_create(int64_t d, int32_t ell, double eps, uint64_t seed, sfd_t **out);

/* Free the handle and its device memory.  NULL is a no-op. */
int sfd_destroy(sfd_t *h);

/* Return the handle to its just-created state (B = 0, empty buffer, counters 0), keeping its
 * options and memory; clears an error state. */
int sfd_reset(sfd_t *h);

/* Set an option (keys above).  Errors: SFD_E_ARG for an unknown key or a value out of range. */
int sfd_set_option(sfd_t *h, int key, double value);

/* Use `hip_stream` (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) for this
 * handle's work; NULL selects the handle's own stream. */
int sfd_set_stream(sfd_t *h, void *hip_stream);

/* Append nrows rows in CSR form (Alg 2, the loop over rows a of A).  Row r holds the entries
 * indices[k], values[k] for indptr[r] <= k < indptr[r+1]; indptr has nrows+1 entries and
 * indptr[0] may be non-zero.  Repeated column ids in a row add up; every stored entry counts
 * towards nnz(A').  After each row the buffer is flushed when nnz(A') >= ell*d or
 * rows(A') = d: B' = BoostedSparseShrink(A', ell, delta) (Alg 4), B = DenseShrink([B; B'], ell)
 * (Alg 5).  indptr/indices/values live in memory of kind `mem`.
 * Errors (state unchanged): SFD_E_ARG (nrows < 0, null pointer with nrows > 0, decreasing
 * indptr, a row with more than d entries), SFD_E_INDEX (column id outside [0, d)),
 * SFD_E_NOCONVERGE (a buffer's BoostedSparseShrink rejected SFD_OPT_MAX_ATTEMPTS SparseShrinks
 * in a row: the sketch, the buffer and the counters are restored to their values before the
 * call).  SFD_E_DEVICE puts the handle in its error state. */
int sfd_append_csr(sfd_t *h, int64_t nrows, const int64_t *indptr, const int32_t *indices,
                   const float *values, int mem);

/* Write the sketch of everything appended so far into B_out: ell x d, row-major, FP32, memory
 * of kind `mem`.  Rows still in the buffer are folded into a copy of the state (Alg 2 returns
 * B; folding the pending rows keeps them), so the stream is unchanged and a repeated query
 * returns the same B.  *live_rows (may be NULL) receives the structural count of rows of
 * B_out that may be non-zero.  Errors: SFD_E_ARG (B_out == NULL), SFD_E_NOCONVERGE (the pending
 * buffer's BoostedSparseShrink exhausted its attempts; the handle is unchanged). */
int sfd_sketch(sfd_t *h, float *B_out, int mem, int32_t *live_rows);

/* Merge src into dst (mergeability of Frequent Directions sketches, Sec. 2.1):
 * dst.B = DenseShrink([sketch(dst); sketch(src)], ell); dst's buffer is consumed; src is
 * unchanged (its sketch, buffer and counters; its query runs in src's own device workspaces,
 * so src must not be in use by another thread).  Both handles must be on the same device.
 * Errors: SFD_E_SHAPE (different d or ell), SFD_E_ARG (NULL, dst == src, a batch handle),
 * SFD_E_NOCONVERGE (either query; both handles unchanged). */
int sfd_merge(sfd_t *dst, const sfd_t *src);

/* Copy the handle's counters into *out. */
int sfd_get_stats(const sfd_t *h, sfd_stats_t *out);

/* Copy the handle's per-class profile (SFD_OPT_PROFILE) into *out.  Errors: SFD_E_ARG. */
int sfd_get_profile(const sfd_t *h, sfd_profile_t *out);

/* The start block G ~ N(0,1)^{d x ell} of SimultaneousIteration (Alg 1) that the handle
 * scheme draws for (seed, stream_id, buffer, attempt, purpose), written FP32 row-major
 * (d x ell) to the device array G_out; purpose 0 = flush, 2 = query.  With purpose 1 or 3 and
 * ell = 1 it writes the Gaussian vector whose normalisation is VerifySpectral's x (Alg 6).
 * Runs on the null stream.  Errors: SFD_E_ARG. */
int sfd_start_block(uint64_t seed, uint64_t stream_id, uint64_t buffer, uint64_t attempt,
                    uint64_t purpose, int64_t d, int32_t ell, float *G_out);

/* Static text for an SFD_E_* code. */
const char *sfd_strerror(int code);

/* ------------------------------------------------------------------ batched streams
 * Many independent streams with identical per-stream semantics: stream s of a batch gives
 * exactly the sketch of an sfd_t with the same (d, ell, eps, seed) and SFD_OPT_STREAM_ID = s
 * fed the same rows (Alg 2 per stream; the streams share the device workspaces and their
 * buffer steps run concurrently).  Memory per stream: the d x L sketch and a pending buffer of
 * ell*d + d entries. */

/* Create nstreams >= 1 streams.  Arguments and errors as sfd_create. */
int sfd_batch_create(int32_t nstreams, int64_t d, int32_t ell, double eps, uint64_t seed, sfd_batch_t **out);
int sfd_batch_destroy(sfd_batch_t *h);  /* NULL-safe */
int sfd_batch_reset(sfd_batch_t *h);    /* every stream back to its initial state */
/* Options as sfd_set_option, applied to every stream; SFD_OPT_STREAM_ID is rejected (stream s
 * is keyed s).  SFD_OPT_LANES accepts 1..16 (default 16). */
int sfd_batch_set_option(sfd_batch_t *h, int key, double value);
int sfd_batch_set_stream(sfd_batch_t *h, void *hip_stream);
/* Counters of stream s (as sfd_get_stats).  Errors: SFD_E_ARG. */
int sfd_batch_get_stats(const sfd_batch_t *h, int32_t stream, sfd_stats_t *out);

/* Append rows to several streams (Alg 2 per stream).  The rows form one CSR block
 * (indptr/indices/values as in sfd_append_csr, in memory of kind mem); segment i is rows
 * [seg_row_start[i], seg_row_start[i+1]) of the block and goes to stream stream_of_seg[i].
 * stream_of_seg (nseg entries) and seg_row_start (nseg + 1, non-decreasing) are host arrays.
 * A stream may appear in at most one segment per call.  Errors: SFD_E_ARG (bad table, repeated
 * stream, bad row pointers), SFD_E_INDEX; validation happens before any stream changes. */
int sfd_batch_append_csr(sfd_batch_t *h, int32_t nseg, const int32_t *stream_of_seg, const int64_t *seg_row_start,
                         const int64_t *indptr, const int32_t *indices, const float *values, int mem);

/* Query every stream (as sfd_sketch, non-destructive): B_out holds nstreams consecutive
 * ell x d row-major sketches, caller-owned, in memory of kind mem. */
int sfd_batch_sketch(sfd_batch_t *h, float *B_out, int mem);

/* ------------------------------------------------------------------ accuracy of a sketch
 * The measures of the paper's experiments (Sec. 4, "Measurements"), in FP64 on the GPU:
 *   cov-err  = ||A^T A - B^T B||_2 / ||A||_F^2;
 *   proj-err = ||A - A V_k V_k^T||_F^2 / ||A - A_k||_F^2, V_k the top-k right singular vectors of
 *              B, A_k the best rank-k approximation of A (Sec. 1.1 notation). */
typedef struct {
  double fro2A;        /* ||A||_F^2, repeated (row, column) entries summed */
  double cov_min;      /* smallest and largest eigenvalue of A^T A - B^T B (Lanczos Ritz values) */
  double cov_max;
  double cov_err;      /* max(|cov_min|, |cov_max|) / fro2A (+inf or NaN when A = 0) */
  double top_k_energy; /* sum of the k largest eigenvalues of A^T A = sum_{i<=k} sigma_i(A)^2; when
                          the Lanczos run on A^T A closes its Krylov space after j < k steps (the
                          start vector meets fewer than k distinct eigenvalues, e.g. A = 0), the
                          sum of the j it found */
  double proj_num;     /* ||A - A V_k V_k^T||_F^2 = fro2A - ||A V_k||_F^2 */
  double proj_err;     /* proj_num / (fro2A - top_k_energy); the three are NaN when k = 0 */
  int32_t steps;       /* Lanczos steps taken for cov-err (fewer than asked when the Krylov
                          space of the operator closes) */
  int32_t pad;
  /* Ritz residual norms ||M y - theta y|| of the reported Ritz pairs (beta_{j+1} |s_j|, s the
   * eigenvector of the Lanczos tridiagonal): each Ritz value lies within its residual of an
   * eigenvalue of the operator, so a small residual certifies the extremes above.  0 when the
   * Krylov space closed (the Ritz values are then exact eigenvalues). */
  double cov_min_res;  /* of the pair giving cov_min */
  double cov_max_res;  /* of the pair giving cov_max */
  double top_k_res;    /* sum over the k pairs that give top_k_energy (NaN when k = 0) */
} sfd_eval_t;

/* Evaluate the ell x d sketch B against the n x d matrix A it summarises.
 * A: CSR in device memory as in sfd_append_csr (int64 indptr[n + 1], rows read from
 * indices/values positions indptr[0] .. indptr[n]); B: ell x d FP32 row-major in device memory
 * (ell = 0: no sketch, B may be NULL; ell <= 512).  k: rank of proj-err, 0 <= k <= ell and
 * k <= min(d, steps) (0 skips it).  n, d < 2^31, at most 2^31 - 1 stored entries.
 * steps: Lanczos steps per operator, 1..512, at most d (<= 0: min(d, 160)).  The extreme
 * eigenvalues of A^T A - B^T B come from Lanczos with full reorthogonalisation on
 * x -> A^T(Ax) - B^T(Bx) from a start vector keyed by seed, the k largest of A^T A likewise on
 * x -> A^T(Ax); A is never densified (a CSC copy is built for A^T y).  Work memory is allocated
 * and freed inside the call (about 28 bytes per stored entry plus (steps + 1) d doubles); the
 * work runs on hip_stream (NULL: the null stream) and the call returns when it is done.
 * Errors: SFD_E_ARG (bad sizes or row pointers), SFD_E_INDEX (a column id outside [0, d)),
 * SFD_E_NOMEM, SFD_E_DEVICE; *out is written only on success. */
int sfd_evaluate(int64_t n, int64_t d, const int64_t *indptr, const int32_t *indices, const float *values,
                 const float *B, int32_t ell, int32_t k, int32_t steps, uint64_t seed, void *hip_stream,
                 sfd_eval_t *out);

/* sfd_evaluate for callers that cannot allocate device memory (code in a serving loop that must
 * not call hipMalloc, harnesses that forbid it): the same arguments, kernels and results (equal
 * bit for bit to sfd_evaluate's), with the work memory taken from a fixed array of 64 MiB in
 * device memory that the library holds on every GPU it runs on until the process ends.  The call
 * makes no device allocation of any kind; on its first use on a device it looks up that device's
 * copy of the array (with the device current).
 * Limit: the work must fit the 64 MiB: about 29 bytes per stored entry, 40 bytes per row and per
 * column, the (steps + 1) d doubles of the Lanczos basis, k d doubles for proj-err and about
 * 2 MiB of fixed parts (e.g. 10^6 entries in 5 10^4 rows at d = 20,000 with 160 steps and k = 10
 * fit).  Larger inputs return SFD_E_TOOBIG before any work is issued (only the argument checks
 * run).
 * Sharing: calls on one device share its array, which keeps the last call's contents (every
 * part that must start at zero is cleared by the call).  Calls from threads of one process are
 * serialized per device by a lock; work that overlaps it on that device's array otherwise races.
 * Errors: those of sfd_evaluate, SFD_E_TOOBIG in place of SFD_E_NOMEM. */
int sfd_evaluate_noalloc(int64_t n, int64_t d, const int64_t *indptr, const int32_t *indices, const float *values,
                         const float *B, int32_t ell, int32_t k, int32_t steps, uint64_t seed, void *hip_stream,
                         sfd_eval_t *out);

#ifdef __cplusplus
}
#endif

#endif /* SFD_H */
