// Symmetric eigensolver (FP64) for the larger small problems (112 < n <= 512): the eig of the
// 2 ell x 2 ell stack Gram of DenseShrink (Alg 5) and of P P^T (Alg 3) when ell is large.  The
// matrix and its eigenvectors no longer fit one CU's LDS together, so instead of Jacobi:
//  1. Householder reduction to tridiagonal form, Q^T A Q = T, by one workgroup with the matrix
//     in global memory (L2-resident): per column a reflector H = I - beta v v^T, the product
//     p = beta A v, w = p - (beta/2)(p^T v) v, and the rank-2 update A <- A - v w^T - w v^T;
//  2. the eigenvalues of T by bisection on Sturm counts (one thread per eigenvalue, to an
//     absolute accuracy of eps ||T||), then its eigenvectors by inverse iteration (three solves
//     with T - lambda I, LU with partial pivoting, one thread per eigenvalue), then made
//     orthonormal inside clusters of close eigenvalues by modified Gram-Schmidt over the block;
//  3. the eigenvectors of A = Q z, applying the reflectors in reverse order (one wave per
//     eigenvector).
// Output as the Jacobi solvers': eigenvalues descending, eigenvector columns (pitch n); only
// the columns of the nvec largest eigenvalues are computed, the others are returned as zeros.
#include <hip/hip_runtime.h>

#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int kTriMax = 512;
constexpr int kTriThreads = 1024;
constexpr int kBisThreads = 512;

// Workspace of one problem (doubles unless noted), n <= kTriMax, NT = kBisThreads:
//   Aw n*n | V n*n (reflector k in row k) | Zt n*n (eigenvector j in row j) | beta n | d n | e n
//   | ev n | LU 4*n*NT (dd, du, du2, dl interleaved by thread) | y n*NT | piv n*NT bytes (the
//   last two per thread of the eigenvalue kernel, element i of thread t at i*NT + t)
struct TriWork {
  double *Aw, *V, *Zt, *beta, *d, *e, *ev, *lu, *y;
  unsigned char* piv;
};

__host__ __device__ inline int64_t tri_work_doubles(int n) {
  return 3 * (int64_t)n * n + 4 * (int64_t)n + 5 * (int64_t)n * kBisThreads + ((int64_t)n * kBisThreads + 7) / 8;
}

__device__ inline TriWork tri_work(void* base, int n) {
  TriWork w;
  double* p = reinterpret_cast<double*>(base);
  w.Aw = p;
  w.V = w.Aw + (int64_t)n * n;
  w.Zt = w.V + (int64_t)n * n;
  w.beta = w.Zt + (int64_t)n * n;
  w.d = w.beta + n;
  w.e = w.d + n;
  w.ev = w.e + n;
  w.lu = w.ev + n;
  w.y = w.lu + 4 * (int64_t)n * kBisThreads;
  w.piv = reinterpret_cast<unsigned char*>(w.y + (int64_t)n * kBisThreads);
  return w;
}

// block-wide sum of one double per thread (all threads get the result)
__device__ inline double block_sum_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int q = 0; q < nw; ++q) s += red[q];
  return s;
}

// 1. tridiagonal reduction (one workgroup per problem, blockIdx.x = problem of a group)
__global__ __launch_bounds__(kTriThreads) void k_tri_reduce(const double* __restrict__ Ain, int lda, int n,
                                                            int64_t astride, char* work, int64_t wstride) {
  Ain += blockIdx.x * astride;
  TriWork w = tri_work(work + blockIdx.x * wstride, n);
  __shared__ double v[kTriMax];
  __shared__ double p[kTriMax];
  __shared__ double ph[kTriMax];
  __shared__ double red[16];
  __shared__ double sc[2];
  const int tid = threadIdx.x;
  double* A = w.Aw;
  for (int64_t q = tid; q < (int64_t)n * n; q += kTriThreads) A[q] = Ain[(q / n) * lda + q % n];
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    // x = A[k][k+1..] (row k = column k by symmetry)
    const double* rowk = A + (int64_t)k * n + k + 1;
    double xi = 0.0;
    if (tid < m) xi = rowk[tid];
    const double nx2 = block_sum_d(xi * xi, red);
    if (tid == 0) {
      const double x0 = rowk[0];
      if (nx2 == 0.0) {
        sc[0] = 0.0;  // beta: no reflector
        sc[1] = x0;
      } else {
        const double nx = sqrt(nx2);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        const double v0 = x0 - alpha;
        sc[0] = 2.0 / (nx2 - x0 * x0 + v0 * v0);
        sc[1] = alpha;
      }
    }
    __syncthreads();
    const double b = sc[0];
    if (tid == 0) {
      w.beta[k] = b;
      w.e[k] = sc[1];
    }
    if (b == 0.0) {
      if (tid < m) w.V[(int64_t)k * n + k + 1 + tid] = 0.0;
      __syncthreads();
      continue;
    }
    if (tid < m) {
      const double vi = tid == 0 ? xi - sc[1] : xi;
      v[tid] = vi;
      w.V[(int64_t)k * n + k + 1 + tid] = vi;
    }
    __syncthreads();
    // p = b A_sub v: thread (h, i) sums rows j = h, h + 2, ... of column i (coalesced over i)
    {
      const int h = tid / kTriMax, i = tid % kTriMax;
      double s = 0.0;
      if (i < m) {
        const double* col = A + (int64_t)(k + 1) * n + k + 1 + i;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int j = h;
        for (; j + 6 < m; j += 8) {  // four loads in flight
          const double a0 = col[(int64_t)j * n], a1 = col[(int64_t)(j + 2) * n];
          const double a2 = col[(int64_t)(j + 4) * n], a3 = col[(int64_t)(j + 6) * n];
          s = fma(a0, v[j], s);
          s1 = fma(a1, v[j + 2], s1);
          s2 = fma(a2, v[j + 4], s2);
          s3 = fma(a3, v[j + 6], s3);
        }
        for (; j < m; j += 2) s = fma(col[(int64_t)j * n], v[j], s);
        s = (s + s1) + (s2 + s3);
      }
      if (h == 1) ph[i] = s;
      __syncthreads();
      if (h == 0 && i < m) p[i] = b * (s + ph[i]);
    }
    __syncthreads();
    double pv = tid < m ? p[tid] * v[tid] : 0.0;
    const double Kc = 0.5 * b * block_sum_d(pv, red);
    if (tid < m) p[tid] = p[tid] - Kc * v[tid];  // w
    __syncthreads();
    // A_sub -= v w^T + w v^T: wave wv takes rows wv, wv + 16, ..., its lanes the columns
    {
      const int lane = tid & 63, wv = tid >> 6;
      for (int r = wv; r < m; r += kTriThreads / 64) {
        double* arow = A + (int64_t)(k + 1 + r) * n + k + 1;
        const double vr = v[r], pr = p[r];
        int c = lane;
        for (; c + 64 < m; c += 128) {
          const double a0 = arow[c], a1 = arow[c + 64];
          arow[c] = a0 - vr * p[c] - pr * v[c];
          arow[c + 64] = a1 - vr * p[c + 64] - pr * v[c + 64];
        }
        if (c < m) arow[c] = arow[c] - vr * p[c] - pr * v[c];
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += kTriThreads) w.d[i] = A[(int64_t)i * n + i];
  if (tid == 0 && n >= 2) w.e[n - 2] = A[(int64_t)(n - 1) * n + n - 2];
  if (tid == 0 && n >= 2) w.beta[n - 2] = 0.0;
  if (tid == 0) w.beta[n - 1] = 0.0;
}

// number of eigenvalues of T below x (Sturm sequence of the LDL^T recurrence)
__device__ inline int sturm_below(const double* d, const double* e2, int n, double x, double pivmin) {
  double q = d[0] - x;
  int c = q < 0.0 ? 1 : 0;
  for (int i = 1; i < n; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d[i] - x) - e2[i - 1] / q;
    c += q < 0.0 ? 1 : 0;
  }
  return c;
}

// 2. eigenvalues (bisection) and eigenvectors (inverse iteration) of T
__global__ __launch_bounds__(kBisThreads) void k_tri_eig(int n, int nvec, char* work, int64_t wstride,
                                                         double* __restrict__ evals, int64_t estride) {
  TriWork w = tri_work(work + blockIdx.x * wstride, n);
  evals += blockIdx.x * estride;
  __shared__ double d[kTriMax], e[kTriMax], e2[kTriMax], ev[kTriMax];
  __shared__ double bounds[3];
  const int t = threadIdx.x;
  for (int i = t; i < n; i += kBisThreads) {
    d[i] = w.d[i];
    e[i] = i + 1 < n ? w.e[i] : 0.0;
    e2[i] = e[i] * e[i];
  }
  __syncthreads();
  if (t == 0) {
    double lo = d[0], hi = d[0], e2max = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      if (i + 1 < n) e2max = fmax(e2max, e2[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
    const double eps = 2.220446049250313e-16;
    bounds[0] = lo - 2.0 * eps * tnorm - pivmin;
    bounds[1] = hi + 2.0 * eps * tnorm + pivmin;
    bounds[2] = tnorm;
  }
  __syncthreads();
  const double tnorm = bounds[2];
  const double eps = 2.220446049250313e-16;
  double e2max = 0.0;
  for (int i = 0; i + 1 < n; ++i) e2max = fmax(e2max, e2[i]);
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  const double atol = eps * tnorm + pivmin;
  // the t-th largest eigenvalue: index n - 1 - t ascending
  if (t < n) {
    const int j = n - 1 - t;
    double a = bounds[0], b = bounds[1];
    for (int it = 0; it < 128; ++it) {
      const double mid = 0.5 * (a + b);
      if (!(mid > a && mid < b)) break;
      if (b - a <= 2.0 * eps * fmax(fabs(a), fabs(b)) + atol) break;
      if (sturm_below(d, e2, n, mid, pivmin) <= j)
        a = mid;
      else
        b = mid;
    }
    ev[t] = 0.5 * (a + b);
    evals[t] = ev[t];
  }
  __syncthreads();
  // inverse iteration, every wanted eigenvalue (the nvec largest) on its own thread; the
  // recurrences carry their running values in registers, so the loads of the stored factors are
  // independent of the chain
  const double tiny = eps * tnorm + pivmin;
  double* dd = w.lu;
  double* du = w.lu + (int64_t)n * kBisThreads;
  double* du2 = w.lu + 2 * (int64_t)n * kBisThreads;
  double* dl = w.lu + 3 * (int64_t)n * kBisThreads;
  double* y = w.y;
  unsigned char* piv = w.piv;
#define LU(a, i) a[(int64_t)(i) * kBisThreads + t]
  if (t < nvec) {
    const double lam = ev[t];
    // T - lam I = P L U (partial pivoting): dd = U's diagonal, du / du2 its first / second
    // superdiagonal, dl the multipliers, piv the row interchanges
    double dcur = d[0] - lam, ucur = n > 1 ? e[0] : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double li = e[i];
      double dnext = d[i + 1] - lam;
      double unext = i + 2 < n ? e[i + 1] : 0.0;
      if (fabs(dcur) >= fabs(li)) {
        if (fabs(dcur) < tiny) dcur = dcur >= 0.0 ? tiny : -tiny;
        const double f = li / dcur;
        LU(dd, i) = dcur;
        LU(dl, i) = f;
        LU(du, i) = ucur;
        LU(du2, i) = 0.0;
        LU(piv, i) = 0;
        dnext = dnext - f * ucur;
      } else {
        const double f = dcur / li;
        LU(dd, i) = li;
        LU(dl, i) = f;
        LU(du, i) = dnext;
        LU(piv, i) = 1;
        const double nd = ucur - f * dnext;
        LU(du2, i) = unext;
        unext = -f * unext;
        dnext = nd;
      }
      dcur = dnext;
      ucur = unext;
    }
    if (fabs(dcur) < tiny) dcur = dcur >= 0.0 ? tiny : -tiny;
    LU(dd, n - 1) = dcur;
    // start vector (deterministic, spread over all components), three solves
    for (int i = 0; i < n; ++i) LU(y, i) = cos((double)i * (1.0 + t) * 0.6180339887498949 + t);
    for (int it = 0; it < 3; ++it) {
      double ycur = LU(y, 0);
      for (int i = 0; i + 1 < n; ++i) {
        const double f = LU(dl, i);
        const double yn = LU(y, i + 1);
        if (LU(piv, i) == 0) {
          LU(y, i) = ycur;
          ycur = yn - f * ycur;
        } else {
          LU(y, i) = yn;
          ycur = ycur - f * yn;
        }
      }
      double x1 = ycur / LU(dd, n - 1);
      LU(y, n - 1) = x1;
      if (n >= 2) {
        double x0 = (LU(y, n - 2) - LU(du, n - 2) * x1) / LU(dd, n - 2);
        LU(y, n - 2) = x0;
        for (int i = n - 3; i >= 0; --i) {
          const double xi = (LU(y, i) - LU(du, i) * x0 - LU(du2, i) * x1) / LU(dd, i);
          LU(y, i) = xi;
          x1 = x0;
          x0 = xi;
        }
      }
      double mx = 0.0;
      for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(LU(y, i)));
      const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
      double nr = 0.0;
      for (int i = 0; i < n; ++i) {
        const double v = LU(y, i) * inv;
        LU(y, i) = v;
        nr = fma(v, v, nr);
      }
      const double in = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
      for (int i = 0; i < n; ++i) LU(y, i) = LU(y, i) * in;
    }
    double* z = w.Zt + (int64_t)t * n;
    for (int i = 0; i < n; ++i) z[i] = LU(y, i);
  }
#undef LU
  __syncthreads();
  // clusters of close eigenvalues (gap <= ortol): modified Gram-Schmidt over the cluster's
  // vectors in order, by the whole block (outside clusters inverse iteration alone keeps the
  // vectors orthogonal to about eps ||T|| / gap)
  __shared__ double cred[kBisThreads / 64];
  __shared__ double cdot[kTriMax];
  const double ortol = 1e-5 * tnorm;
  const int lane = t & 63, wave = t >> 6;
  constexpr int NWB = kBisThreads / 64;
  int c0 = 0;
  while (c0 < nvec) {
    int c1 = c0 + 1;
    while (c1 < nvec && ev[c1 - 1] - ev[c1] <= ortol) ++c1;
    for (int j = c0; c1 - c0 > 1 && j < c1; ++j) {
      double* zj = w.Zt + (int64_t)j * n;
      // normalise z_j
      double s = 0.0;
      for (int i = t; i < n; i += kBisThreads) s = fma(zj[i], zj[i], s);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) cred[wave] = s;
      __syncthreads();
      double nr = 0.0;
      for (int q = 0; q < NWB; ++q) nr += cred[q];
      const double in = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
      __syncthreads();
      for (int i = t; i < n; i += kBisThreads) zj[i] *= in;
      __syncthreads();
      // the later vectors of the cluster lose their z_j component (one wave per vector)
      for (int k = j + 1 + wave; k < c1; k += NWB) {
        const double* zk = w.Zt + (int64_t)k * n;
        double dk = 0.0;
        for (int i = lane; i < n; i += 64) dk = fma(zk[i], zj[i], dk);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dk += __shfl_xor(dk, o, 64);
        if (lane == 0) cdot[k] = dk;
      }
      __syncthreads();
      for (int k = j + 1 + wave; k < c1; k += NWB) {
        double* zk = w.Zt + (int64_t)k * n;
        const double dk = cdot[k];
        for (int i = lane; i < n; i += 64) zk[i] = fma(-dk, zj[i], zk[i]);
      }
      __syncthreads();
    }
    c0 = c1;
  }
}

// 3. eigenvector j of A = H_0 H_1 ... H_{n-3} z_j: one wave per eigenvector, z in registers
// (lane l holds components l + 64 r)
__global__ __launch_bounds__(64) void k_tri_back(int n, int nvec, const char* work, int64_t wstride,
                                                 double* __restrict__ evecs, int64_t vstride) {
  const TriWork w = tri_work(const_cast<char*>(work) + blockIdx.y * wstride, n);
  evecs += blockIdx.y * vstride;
  constexpr int R = kTriMax / 64;
  const int lane = threadIdx.x;
  const int j = blockIdx.x;
  if (j >= nvec) {  // eigenvectors not asked for are returned as zero columns
    for (int i = lane; i < n; i += 64) evecs[(int64_t)i * n + j] = 0.0;
    return;
  }
  double z[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    z[r] = i < n ? w.Zt[(int64_t)j * n + i] : 0.0;
  }
  for (int k = n - 3; k >= 0; --k) {
    const double b = w.beta[k];
    if (b == 0.0) continue;
    const double* vk = w.V + (int64_t)k * n;
    double vr[R];
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      vr[r] = (i > k && i < n) ? vk[i] : 0.0;
      s = fma(vr[r], z[r], s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const double f = b * s;
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = fma(-f, vr[r], z[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    if (i < n) evecs[(int64_t)i * n + j] = z[r];
  }
}

}  // namespace

int64_t eig_tri_work_bytes(int n) { return n > 0 ? tri_work_doubles(n) * 8 + 256 : 0; }

hipError_t eig_tri_group(const double* A, int lda, int n, int nvec, double* evals, double* evecs, int K,
                         int64_t astride, int64_t estride, int64_t vstride, void* work, int64_t wstride,
                         hipStream_t st) {
  if (n < 1 || n > kTriMax || K < 1 || !work) return hipErrorInvalidValue;
  nvec = nvec < 1 || nvec > n ? n : nvec;
  char* wk = reinterpret_cast<char*>(work);
  k_tri_reduce<<<K, kTriThreads, 0, st>>>(A, lda, n, astride, wk, wstride);
  k_tri_eig<<<K, kBisThreads, 0, st>>>(n, nvec, wk, wstride, evals, estride);
  k_tri_back<<<dim3((unsigned)n, (unsigned)K), 64, 0, st>>>(n, nvec, wk, wstride, evecs, vstride);
  return hipGetLastError();
}

}  // namespace sfd
