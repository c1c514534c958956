// Accuracy of a sketch against its input on the GPU, in FP64: the measures of the paper's
// experiments (Sec. 4, "Measurements").
//   cov-err  = ||A^T A - B^T B||_2 / ||A||_F^2.  The extreme eigenvalues of the d x d matrix
//              A^T A - B^T B come from Lanczos with full reorthogonalisation on the operator
//              x -> A^T (A x) - B^T (B x); the matrix is never formed.
//   proj-err = ||A - A V_k V_k^T||_F^2 / ||A - A_k||_F^2 (Sec. 1.1 notation): V_k holds the top-k
//              right singular vectors of B (from the FP64 eig of the ell x ell Gram B B^T), the
//              numerator is ||A||_F^2 - ||A V_k||_F^2, and ||A - A_k||_F^2 = ||A||_F^2 minus the
//              sum of the k largest eigenvalues of A^T A (Lanczos on x -> A^T (A x)).
// A x runs over the input CSR, A^T y over a CSC built once (FP32 values, FP64 accumulation);
// B stays FP32 and is read in FP64 arithmetic.  Every reduction has a fixed order, so results
// are reproducible run to run.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <mutex>

#include "sfd.h"
#include "sfd_internal.h"

namespace sfd {
namespace {

constexpr int kEvalBlocks = 512;       // partial sums of the FP64 reductions
constexpr int kEvalMaxSteps = 512;     // Lanczos steps per operator
constexpr int kEvalDefaultSteps = 160;

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 8192) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// rowptr[r] = indptr[r] - indptr[0], r <= n (int32 offsets of the input CSR)
__global__ void k_rebase(const int64_t* __restrict__ indptr, int64_t n, int* __restrict__ rowptr) {
  const int64_t base = indptr[0];
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += (int64_t)gridDim.x * blockDim.x)
    rowptr[r] = (int)(indptr[r] - base);
}

// y[r] = sum_k val[k] x[idx[k]] over the chunk schedule of a CSR / CSC structure (rows cut into
// chunks of at most kSpmmChunk entries, so Zipf-long columns are spread over many groups): a
// 16-lane group per chunk, lane s adding entries s, s + 16, ... then a fixed xor tree; a whole
// row is written to y, the chunks of a long row to their partial slots (k_spmv64_fixup).
__global__ __launch_bounds__(256) void k_spmv64(const int4* __restrict__ desc, const int* __restrict__ nchunks_ptr,
                                                const int* __restrict__ idx, const float* __restrict__ val,
                                                const double* __restrict__ x, double* __restrict__ y,
                                                double* __restrict__ partial) {
  const int sub = threadIdx.x & 15;
  const int64_t nchunks = *nchunks_ptr;
  const int64_t ng = ((int64_t)gridDim.x * blockDim.x) >> 4;
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; c < nchunks; c += ng) {
    const int4 dc = desc[c];
    double acc = 0.0;
    for (int p = dc.y + sub; p < dc.z; p += 16) acc = fma((double)val[p], x[idx[p]], acc);
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (sub == 0) {
      if (dc.w < 0)
        y[dc.x] = acc;
      else
        partial[dc.w] = acc;
    }
  }
}

// y[r] = sum of the partial slots of long row r, in slot order (lane j adds slots j, j + 64, ...,
// then a fixed xor tree); one wave per long row
__global__ __launch_bounds__(256) void k_spmv64_fixup(const int* __restrict__ slot_start,
                                                      const int* __restrict__ long_rows,
                                                      const int* __restrict__ nlong_ptr,
                                                      const double* __restrict__ partial, double* __restrict__ y) {
  const int nlong = *nlong_ptr;
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < nlong; i += nw) {
    const int r = long_rows[i];
    const int s0 = slot_start[r], n = slot_start[r + 1] - s0;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += partial[s0 + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y[r] = acc;
  }
}

// block sum of v over 256 threads, fixed tree; the result is valid in thread 0
__device__ inline double block_sum256(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  return s[0];
}

// part[v nb + b] = block b's share of <Q[v], w> (rows of Q pitch ld), v = blockIdx.y
__global__ __launch_bounds__(256) void k_multi_dot(const double* __restrict__ Q, int64_t ld,
                                                   const double* __restrict__ w, int64_t d,
                                                   double* __restrict__ part) {
  __shared__ double s[256];
  const double* q = Q + (int64_t)blockIdx.y * ld;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256)
    acc = fma(q[t], w[t], acc);
  const double tot = block_sum256(acc, s);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// out[v] = sum of part[v nb .. v nb + nb), v = blockIdx.x
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[(int64_t)blockIdx.x * nb + b];
  const double tot = block_sum256(acc, s);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// u[i] = sum_t B[i][t] x[t] (B: rows x d FP32, row-major), one block per row
__global__ __launch_bounds__(256) void k_rows_dot(const float* __restrict__ B, int64_t d,
                                                  const double* __restrict__ x, double* __restrict__ u) {
  __shared__ double s[256];
  const float* row = B + (int64_t)blockIdx.x * d;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < d; t += 256) acc = fma((double)row[t], x[t], acc);
  const double tot = block_sum256(acc, s);
  if (threadIdx.x == 0) u[blockIdx.x] = tot;
}

// w[t] -= sum_i B[i][t] u[i], i < rows
__global__ __launch_bounds__(256) void k_sub_bt(const float* __restrict__ B, int rows, int64_t d,
                                                const double* __restrict__ u, double* __restrict__ w) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int i = 0; i < rows; ++i) acc = fma((double)B[(int64_t)i * d + t], u[i], acc);
    w[t] -= acc;
  }
}

// w -= alpha[j] q_j + beta[j] q_{j-1}  (beta[0] = 0: q_{-1} is not read)
__global__ __launch_bounds__(256) void k_three_term(double* __restrict__ w, const double* __restrict__ qj,
                                                    const double* __restrict__ qm, const double* __restrict__ alpha,
                                                    const double* __restrict__ beta, int j, int64_t d) {
  const double a = alpha[j], b = j > 0 ? beta[j] : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) {
    double v = fma(-a, qj[t], w[t]);
    if (j > 0) v = fma(-b, qm[t], v);
    w[t] = v;
  }
}

// w -= sum_{i < nv} h[i] Q[i]  (one classical Gram-Schmidt sweep against the Lanczos basis)
__global__ __launch_bounds__(256) void k_reorth(const double* __restrict__ Q, int64_t ld, int nv,
                                                const double* __restrict__ h, double* __restrict__ w, int64_t d) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc = fma(Q[(int64_t)i * ld + t], h[i], acc);
    w[t] -= acc;
  }
}

// q = w / sqrt(*nrm2) (q = 0 when the norm is 0); *beta_out = the norm
__global__ __launch_bounds__(256) void k_normalize(const double* __restrict__ w, const double* __restrict__ nrm2,
                                                   double* __restrict__ q, double* __restrict__ beta_out, int64_t d) {
  const double b = sqrt(fmax(*nrm2, 0.0));
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && beta_out) *beta_out = b;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) q[t] = w[t] * inv;
}

// start vector: q[t] uniform in [-1, 1) from a splitmix64 hash of (seed, t)
__global__ __launch_bounds__(256) void k_start(uint64_t seed, double* __restrict__ q, int64_t d) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(t + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    q[t] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// G[i][j] = G[j][i] = sum_t B[i][t] B[j][t] for i <= j (one block per pair, fixed order)
__global__ __launch_bounds__(256) void k_gram64(const float* __restrict__ B, int rows, int64_t d,
                                                double* __restrict__ G) {
  __shared__ double s[256];
  const int i = blockIdx.x, j = blockIdx.y;
  if (i > j) return;
  const float* bi = B + (int64_t)i * d;
  const float* bj = B + (int64_t)j * d;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < d; t += 256) acc = fma((double)bi[t], (double)bj[t], acc);
  const double tot = block_sum256(acc, s);
  if (threadIdx.x == 0) {
    G[(int64_t)i * rows + j] = tot;
    G[(int64_t)j * rows + i] = tot;
  }
}

// V[c][t] = (sum_l B[l][t] U[l][c]) / sigma_c for c < k (U: rows x rows eigenvectors, column c
// <-> the c-th largest eigenvalue ev[c] = sigma_c^2; a zero sigma gives a zero row)
__global__ __launch_bounds__(256) void k_right_vectors(const float* __restrict__ B, int rows, int64_t d,
                                                       const double* __restrict__ U, const double* __restrict__ ev,
                                                       int k, double* __restrict__ V) {
  const int c = blockIdx.y;
  const double sig = sqrt(fmax(ev[c], 0.0));
  const double inv = sig > 0.0 ? 1.0 / sig : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < d; t += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int l = 0; l < rows; ++l) acc = fma((double)B[(int64_t)l * d + t], U[(int64_t)l * rows + c], acc);
    V[(int64_t)c * d + t] = acc * inv;
  }
}

// The symmetric tridiagonal matrix of a Lanczos run: diagonal a[0 .. n), off-diagonal b[1 .. n)
// (b[i] couples i - 1 and i, b[0] unused).  Fixed capacity, so the host side of an evaluation
// needs no heap memory.
struct Tri {
  int n = 0;
  double a[kEvalMaxSteps];
  double b[kEvalMaxSteps + 1];
};

// The k-th smallest (k = 0 ..) eigenvalue of the tridiagonal t, by bisection on Sturm counts.
double tri_kth(const Tri& t, int k) {
  const int m = t.n;
  const double* a = t.a;
  const double* b = t.b;
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < m ? std::fabs(b[i + 1]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  const double tiny = std::numeric_limits<double>::min() / std::numeric_limits<double>::epsilon();
  // number of eigenvalues below x
  auto below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      q = a[i] - x - (i > 0 ? b[i] * b[i] / q : 0.0);
      if (q == 0.0) q = -tiny;
      if (q < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 2.0 * std::numeric_limits<double>::epsilon() * scale; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of the tridiagonal t for its eigenvalue theta, by
// inverse iteration: three solves with T - theta I, factored by Gaussian elimination with partial
// pivoting (a row exchange brings in a second superdiagonal); a pivot that vanishes is replaced by
// a tiny one, which only scales the solution along the eigenvector.
double tri_evec_last(const Tri& t, double theta) {
  const int m = t.n;
  if (m == 1) return 1.0;
  const double* a = t.a;
  const double* b = t.b;
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(a[i]) + (i > 0 ? std::fabs(b[i]) : 0.0));
  const double tiny = std::max(scale, std::numeric_limits<double>::min()) * std::numeric_limits<double>::epsilon();
  double dg[kEvalMaxSteps], up[kEvalMaxSteps], up2[kEvalMaxSteps], lo[kEvalMaxSteps], x[kEvalMaxSteps];
  bool swp[kEvalMaxSteps];
  for (int i = 0; i < m; ++i) {
    dg[i] = a[i] - theta;
    up[i] = up2[i] = lo[i] = 0.0;
    swp[i] = false;
  }
  for (int i = 0; i + 1 < m; ++i) {
    up[i] = b[i + 1];
    lo[i] = b[i + 1];
  }
  for (int i = 0; i + 1 < m; ++i) {
    if (std::fabs(dg[i]) >= std::fabs(lo[i])) {
      if (dg[i] == 0.0) dg[i] = tiny;
      const double f = lo[i] / dg[i];
      lo[i] = f;
      dg[i + 1] -= f * up[i];
    } else {
      // rows i and i + 1 exchanged
      const double f = dg[i] / lo[i];
      swp[i] = true;
      dg[i] = lo[i];
      lo[i] = f;
      const double tt = up[i];
      up[i] = dg[i + 1];
      dg[i + 1] = tt - f * dg[i + 1];
      if (i + 2 < m) {
        up2[i] = up[i + 1];
        up[i + 1] = -f * up[i + 1];
      }
    }
  }
  if (dg[m - 1] == 0.0) dg[m - 1] = tiny;
  for (int i = 0; i < m; ++i) x[i] = 1.0 / std::sqrt((double)m);
  for (int it = 0; it < 3; ++it) {
    for (int i = 0; i + 1 < m; ++i) {
      if (swp[i]) std::swap(x[i], x[i + 1]);
      x[i + 1] -= lo[i] * x[i];
    }
    x[m - 1] /= dg[m - 1];
    x[m - 2] = (x[m - 2] - up[m - 2] * x[m - 1]) / dg[m - 2];
    for (int i = m - 3; i >= 0; --i) x[i] = (x[i] - up[i] * x[i + 1] - up2[i] * x[i + 2]) / dg[i];
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm = std::max(nrm, std::fabs(x[i]));
    for (int i = 0; i < m; ++i) x[i] /= nrm;  // rescale first: the solve can overflow a plain 2-norm
    nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) x[i] /= nrm;
  }
  return std::fabs(x[m - 1]);
}

// Device work memory of one evaluation, taken in pieces.  Two sources:
//  - allocating: each piece is a hipMalloc, all freed when the workspace goes out of scope;
//  - arena: pieces are consecutive 256-byte aligned ranges of a fixed region (the static scratch
//    of sfd_evaluate_noalloc); a piece that does not fit fails.
struct Workspace {
  char* base = nullptr;  // arena region (nullptr: allocating)
  size_t cap = 0, used = 0;
  void* owned[64] = {};
  int nowned = 0;
  template <class T>
  bool get(T** out, int64_t count) {
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (base) {
      const size_t off = (used + 255) & ~(size_t)255;
      if (off > cap || bytes > cap - off) return false;
      used = off + bytes;
      *out = reinterpret_cast<T*>(base + off);
      return true;
    }
    void* q = nullptr;
    if (nowned == 64 || hipMalloc(&q, bytes) != hipSuccess) return false;
    owned[nowned++] = q;
    *out = static_cast<T*>(q);
    return true;
  }
  ~Workspace() {
    for (int i = 0; i < nowned; ++i) (void)hipFree(owned[i]);
  }
};

struct EvalCtx {
  int64_t n, d;
  const int* colidx;
  const float* val;
  const int* cscrow;
  const float* cscval;
  Schedule sr, sc;  // chunk schedules of the CSR and the CSC
  const float* B;
  int ell;
  double *y, *w, *u, *part, *scal, *Q, *alpha, *beta, *partial;
  hipStream_t st;
};

// y = the product of a scheduled structure with x
void spmv_sched(EvalCtx& c, const Schedule& s, const int* idx, const float* val, const double* x, double* y) {
  k_spmv64<<<grid_for(s.max_chunks * 16, 256), 256, 0, c.st>>>(s.desc, s.regions + 1, idx, val, x, y, c.partial);
  k_spmv64_fixup<<<256, 256, 0, c.st>>>(s.pslot, s.long_rows, s.counters, c.partial, y);
}

// w = A^T (A x) (- B^T (B x))
hipError_t apply_op(EvalCtx& c, const double* x, bool withB) {
  spmv_sched(c, c.sr, c.colidx, c.val, x, c.y);
  spmv_sched(c, c.sc, c.cscrow, c.cscval, c.y, c.w);
  if (withB && c.ell > 0) {
    k_rows_dot<<<c.ell, 256, 0, c.st>>>(c.B, c.d, x, c.u);
    k_sub_bt<<<grid_for(c.d, 256), 256, 0, c.st>>>(c.B, c.ell, c.d, c.u, c.w);
  }
  return hipGetLastError();
}

// <Q[v], w> for v < nv into out[v]
hipError_t multi_dot(EvalCtx& c, const double* Q, int nv, const double* w, double* out) {
  const unsigned nb = grid_for(c.d, 256, kEvalBlocks);
  k_multi_dot<<<dim3(nb, nv), 256, 0, c.st>>>(Q, c.d, w, c.d, c.part);
  k_sum_parts<<<nv, 256, 0, c.st>>>(c.part, (int)nb, out);
  return hipGetLastError();
}

// Lanczos with full reorthogonalisation (two classical Gram-Schmidt sweeps per step) on the
// operator: the tridiagonal coefficients of `steps` steps (fewer when the Krylov space closes).
// *beta_next: the coupling after the last kept step (0 when the Krylov space closed), which with
// the eigenvectors of the tridiagonal gives the Ritz residuals.
hipError_t lanczos(EvalCtx& c, bool withB, int steps, uint64_t seed, Tri& t, double* beta_next) {
  hipError_t e;
  const int64_t d = c.d;
  const unsigned gd = grid_for(d, 256);
  double* h = c.scal + 2;  // kEvalMaxSteps + 1 reorthogonalisation coefficients
  double* nrm2 = c.scal;
  k_start<<<gd, 256, 0, c.st>>>(seed, c.w, d);
  if ((e = multi_dot(c, c.w, 1, c.w, nrm2)) != hipSuccess) return e;
  k_normalize<<<gd, 256, 0, c.st>>>(c.w, nrm2, c.Q, nullptr, d);
  for (int j = 0; j < steps; ++j) {
    const double* qj = c.Q + (int64_t)j * d;
    if ((e = apply_op(c, qj, withB)) != hipSuccess) return e;
    if ((e = multi_dot(c, qj, 1, c.w, c.alpha + j)) != hipSuccess) return e;
    k_three_term<<<gd, 256, 0, c.st>>>(c.w, qj, j > 0 ? qj - d : qj, c.alpha, c.beta, j, d);
    for (int pass = 0; pass < 2; ++pass) {
      if ((e = multi_dot(c, c.Q, j + 1, c.w, h)) != hipSuccess) return e;
      k_reorth<<<gd, 256, 0, c.st>>>(c.Q, d, j + 1, h, c.w, d);
    }
    if ((e = multi_dot(c, c.w, 1, c.w, nrm2)) != hipSuccess) return e;
    k_normalize<<<gd, 256, 0, c.st>>>(c.w, nrm2, c.Q + (int64_t)(j + 1) * d, c.beta + j + 1, d);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double ha[kEvalMaxSteps], hb[kEvalMaxSteps + 1];
  if ((e = hipMemcpyAsync(ha, c.alpha, sizeof(double) * steps, hipMemcpyDeviceToHost, c.st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(hb, c.beta, sizeof(double) * (steps + 1), hipMemcpyDeviceToHost, c.st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(c.st)) != hipSuccess) return e;
  // the Krylov space closes at the first coupling that vanishes against the coefficients seen so
  // far (the steps after it start from rounding noise and are dropped: their coefficients are
  // meaningless and can grow without bound)
  double scale = 0.0;
  t.n = 0;
  t.b[0] = 0.0;
  *beta_next = 0.0;
  for (int j = 0; j < steps; ++j) {
    t.a[t.n++] = ha[j];
    scale = std::max(scale, std::fabs(ha[j]) + t.b[j]);
    const bool closed = !(hb[j + 1] > 1e-12 * scale);
    if (j + 1 < steps) {
      if (closed) break;
      t.b[j + 1] = hb[j + 1];
    } else if (!closed) {
      *beta_next = hb[j + 1];
    }
  }
  return hipSuccess;
}

int hip_fail(hipError_t e) { return e == hipErrorOutOfMemory ? SFD_E_NOMEM : SFD_E_DEVICE; }

// The whole evaluation with its device work memory taken from ws (allocating, or the static
// scratch).  A piece that does not fit the scratch is reported before any work that the result
// depends on has been issued (only the argument checks ran).
int evaluate_impl(Workspace& al, int64_t n, int64_t d, const int64_t* indptr, const int32_t* indices,
                  const float* values, const float* B, int32_t ell, int32_t k, int32_t steps, uint64_t seed,
                  void* hip_stream, sfd_eval_t* out) {
  if (!out || !indptr || n < 0 || d < 1 || ell < 0 || k < 0 || k > ell || (ell > 0 && !B)) return SFD_E_ARG;
  if (ell > 2 * kMaxEll || steps > kEvalMaxSteps || d >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31)) return SFD_E_ARG;
  const int m = (int)std::min<int64_t>(d, steps > 0 ? steps : kEvalDefaultSteps);
  if (k > m) return SFD_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nomem = al.base ? SFD_E_TOOBIG : SFD_E_NOMEM;
  // the input: rows, then the stored-entry count from the row pointers
  int* err = nullptr;
  if (!al.get(&err, 1)) return nomem;
  int64_t ends[2] = {0, 0};
  if (hipMemcpyAsync(&ends[0], indptr, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&ends[1], indptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SFD_E_DEVICE;
  const int64_t nnz = ends[1] - ends[0];
  if (nnz < 0 || nnz >= ((int64_t)1 << 31) || (nnz > 0 && (!indices || !values))) return SFD_E_ARG;
  int herr = 0;
  if (fill_i32(err, 1, 0, st) != hipSuccess || validate_rows(indptr, n, d, err, st) != hipSuccess ||
      validate_indices(indices, ends[0], ends[1], d, err, st) != hipSuccess ||
      hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SFD_E_DEVICE;
  if (herr & 1) return SFD_E_ARG;
  if (herr & 2) return SFD_E_INDEX;
  const int* colidx = indices + ends[0];
  const float* vals = values + ends[0];
  // workspaces
  EvalCtx c{};
  c.n = n;
  c.d = d;
  c.B = B;
  c.ell = ell;
  c.st = st;
  int *rowptr = nullptr, *cscptr = nullptr, *cscrow = nullptr;
  float* cscval = nullptr;
  CscWork w{};
  const int64_t tiles = (nnz + 2047) / 2048;
  DevScalars* sc = nullptr;
  bool ok = al.get(&rowptr, n + 1) && al.get(&cscptr, d + 1) && al.get(&cscrow, nnz) && al.get(&cscval, nnz);
  ok = ok && al.get(&w.counts, 1) && al.get(&w.rowid, nnz) && al.get(&w.keys0, nnz) && al.get(&w.keys1, nnz) &&
       al.get(&w.vals0, nnz) && al.get(&w.vals1, nnz) && al.get(&w.hist, 256 * tiles + 1) &&
       al.get(&w.part, fro2_part_doubles(1)) &&
       al.get(&w.scan_tmp, scan_tmp_ints(std::max<int64_t>(256 * tiles + 1, std::max(n, d) + 1)) + 16) &&
       al.get(&sc, 1);
  for (Schedule* sch : {&c.sr, &c.sc}) {
    const int64_t rows = sch == &c.sr ? n : d;
    sch->max_chunks = rows + nnz / kSpmmChunk + 2;
    ok = ok && al.get(&sch->nch, rows + 1) && al.get(&sch->pslot, rows + 1) && al.get(&sch->desc, sch->max_chunks) &&
         al.get(&sch->long_rows, rows + 1) && al.get(&sch->counters, 4) && al.get(&sch->regions, kXcdBands + 2);
  }
  ok = ok && al.get(&c.partial, 2 * nnz / kSpmmChunk + 16);
  ok = ok && al.get(&c.y, n) && al.get(&c.w, d) && al.get(&c.u, std::max(ell, 1)) &&
       al.get(&c.part, (int64_t)kEvalBlocks * (kEvalMaxSteps + 1)) && al.get(&c.scal, kEvalMaxSteps + 8) &&
       al.get(&c.Q, (int64_t)(m + 1) * d) && al.get(&c.alpha, m) && al.get(&c.beta, m + 1);
  double *G = nullptr, *ev = nullptr, *U = nullptr, *V = nullptr, *kd = nullptr;
  void* ework = nullptr;
  if (k > 0) {
    ok = ok && al.get(&G, (int64_t)ell * ell) && al.get(&ev, ell) && al.get(&U, (int64_t)ell * ell) &&
         al.get(&V, (int64_t)k * d) && al.get(&kd, k) &&
         al.get(reinterpret_cast<char**>(&ework), std::max<int64_t>(eig_work_bytes(ell), 1));
  }
  if (!ok) return nomem;
  hipError_t e;
  // CSR offsets, CSC (and ||A||_F^2 with repeated entries summed, from the sorted column ids)
  k_rebase<<<grid_for(n + 1, 256), 256, 0, st>>>(indptr, n, rowptr);
  const int* keys = nullptr;
  if ((e = build_csc(rowptr, colidx, vals, (int)n, (int)nnz, d, cscptr, cscrow, cscval, w, &keys, st)) != hipSuccess)
    return hip_fail(e);
  if ((e = fill_f32(reinterpret_cast<float*>(sc), sizeof(DevScalars) / 4, 0.f, st)) != hipSuccess) return hip_fail(e);
  if (nnz > 0 && (e = fro2_segments(cscptr, keys, cscrow, cscval, d, 1, w.part, sc, st)) != hipSuccess)
    return hip_fail(e);
  c.colidx = colidx;
  c.val = vals;
  c.cscrow = cscrow;
  c.cscval = cscval;
  if ((e = schedule_build(rowptr, (int)n, c.sr, w.scan_tmp, st)) != hipSuccess) return hip_fail(e);
  if ((e = schedule_build(cscptr, (int)d, c.sc, w.scan_tmp, st)) != hipSuccess) return hip_fail(e);
  DevScalars hsc{};
  if (hipMemcpyAsync(&hsc, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SFD_E_DEVICE;
  const double fro2A = nnz > 0 ? hsc.fro2A : 0.0;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  sfd_eval_t r{};
  r.fro2A = fro2A;
  // cov-err: extreme eigenvalues of A^T A - B^T B
  Tri t;
  double bn = 0.0;
  if ((e = lanczos(c, true, m, seed, t, &bn)) != hipSuccess) return hip_fail(e);
  r.cov_min = tri_kth(t, 0);
  r.cov_max = tri_kth(t, t.n - 1);
  r.cov_min_res = bn > 0.0 ? bn * tri_evec_last(t, r.cov_min) : 0.0;
  r.cov_max_res = bn > 0.0 ? bn * tri_evec_last(t, r.cov_max) : 0.0;
  r.cov_err = std::max(std::fabs(r.cov_min), std::fabs(r.cov_max)) / fro2A;
  r.steps = (int32_t)t.n;
  r.top_k_energy = nan;
  r.top_k_res = nan;
  r.proj_num = nan;
  r.proj_err = nan;
  if (k > 0) {
    // ||A - A_k||_F^2 from the k largest eigenvalues of A^T A
    if ((e = lanczos(c, false, m, seed ^ 0x5DEECE66Dull, t, &bn)) != hipSuccess) return hip_fail(e);
    const int mm = t.n;
    double topk = 0.0, topk_res = 0.0;
    for (int i = 0; i < k && i < mm; ++i) {
      const double th = tri_kth(t, mm - 1 - i);
      topk += th;
      if (bn > 0.0) topk_res += bn * tri_evec_last(t, th);
    }
    r.top_k_energy = topk;
    r.top_k_res = topk_res;
    // V_k from the eig of B B^T, then ||A V_k||_F^2 = sum_c ||A v_c||^2
    k_gram64<<<dim3(ell, ell), 256, 0, st>>>(B, ell, d, G);
    if ((e = eig_sym(G, ell, ell, ell, ev, U, ework, st)) != hipSuccess) return hip_fail(e);
    k_right_vectors<<<dim3(grid_for(d, 256), k), 256, 0, st>>>(B, ell, d, U, ev, k, V);
    for (int cc = 0; cc < k; ++cc) {
      spmv_sched(c, c.sr, colidx, vals, V + (int64_t)cc * d, c.y);
      const unsigned nb = grid_for(n, 256, kEvalBlocks);
      k_multi_dot<<<dim3(nb, 1), 256, 0, st>>>(c.y, n, c.y, n, c.part);
      k_sum_parts<<<1, 256, 0, st>>>(c.part, (int)nb, kd + cc);
    }
    double hk[2 * kMaxEll];
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
    if (hipMemcpyAsync(hk, kd, sizeof(double) * k, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SFD_E_DEVICE;
    double av = 0.0;
    for (int i = 0; i < k; ++i) av += hk[i];
    r.proj_num = fro2A - av;
    r.proj_err = r.proj_num / (fro2A - topk);
  }
  *out = r;
  return SFD_OK;
}

// The work memory of sfd_evaluate_noalloc: one array per GPU, alive until the process ends.  Host
// code never passes `scratch` itself to a kernel (on the host it names a stand-in, not device
// memory): the device address comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept in scratch_ptr[device].
constexpr size_t kEvalScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kEvalScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu[kMaxDevices];  // one evaluation at a time per device (they share its scratch)
void* scratch_ptr[kMaxDevices] = {};

}  // namespace
}  // namespace sfd

extern "C" int sfd_evaluate(int64_t n, int64_t d, const int64_t* indptr, const int32_t* indices, const float* values,
                            const float* B, int32_t ell, int32_t k, int32_t steps, uint64_t seed, void* hip_stream,
                            sfd_eval_t* out) {
  sfd::Workspace ws;
  return sfd::evaluate_impl(ws, n, d, indptr, indices, values, B, ell, k, steps, seed, hip_stream, out);
}

extern "C" int sfd_evaluate_noalloc(int64_t n, int64_t d, const int64_t* indptr, const int32_t* indices,
                                    const float* values, const float* B, int32_t ell, int32_t k, int32_t steps,
                                    uint64_t seed, void* hip_stream, sfd_eval_t* out) {
  using namespace sfd;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SFD_E_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return SFD_E_DEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu[dev]);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SFD_E_DEVICE;
    scratch_ptr[dev] = p;
  }
  Workspace ws;
  ws.base = static_cast<char*>(scratch_ptr[dev]);
  ws.cap = kEvalScratchBytes;
  return evaluate_impl(ws, n, d, indptr, indices, values, B, ell, k, steps, seed, hip_stream, out);
}
