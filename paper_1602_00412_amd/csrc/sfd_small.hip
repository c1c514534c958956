// Small dense FP64 solvers of the buffer step, each in one workgroup:
//  - pivoted Cholesky of an ell x ell Gram and the inverse of its factor (CholeskyQR form of the
//    GramSchmidt step of Alg 1),
//  - symmetric eigensolver (cyclic Jacobi) for svd(P, ell) of Alg 3 and svd([B; B'], ell) of
//    Alg 5 through their Gram matrices,
//  - the shrink factors sqrt(Lambda^2 - lambda_ell^2 I) of Alg 3 / Alg 5 and Delta of Alg 4.
#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int kCholMax = 128;      // register-resident factor and inverse together
constexpr int kCholMaxWide = 256;  // factor and inverse in two passes of 8 waves each

// 1/sqrt(x) for x > 0: the hardware estimate refined by one Newton step (relative error
// about one unit in the last place).
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  const double r = fma(-h, y, 0.5);
  return fma(y, r, y);
}

// 1/x: the hardware estimate refined by two Newton steps.
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
// the Jacobi solver (A and V in LDS) takes n <= kEigMax; larger problems go to the tridiagonal
// solver (sfd_eig_tri.hip)
constexpr int kEigMax = 112;

__device__ inline double readlane_d(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)bits, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Right-looking Cholesky W = R^T R of the n x n leading block with the matrix in registers:
// thread (w, j) (wave w of NW, lane j) holds columns j + 64 u (u < CPL), rows i = NW s + w.  One
// pivot per step: the wave owning row k scales it into row k of R and publishes it in LDS; after
// one barrier every thread updates its rows below k, reading the published row as LDS
// broadcasts.  A pivot that has fallen to tau * W_kk (the column's own squared norm) marks column
// k as dependent on the earlier ones: its row of R is zero.  T = R^{-1} on the kept columns
// follows by right-looking back substitution, last row first: the wave owning row i finishes row
// i of T and publishes it; the rows above subtract R[l][i] T[i][:], R[l][i] being an entry of
// row l held in the same wave (a readlane).  Steps are unrolled, so register indices are static;
// the published rows alternate between two LDS buffers, so one barrier per step suffices.
// panel * T then has orthonormal kept columns spanning the panel's numerical column space.
// (a group launch runs one workgroup per buffer k = blockIdx.x on W + k wstride, T + k L L, sc + k)
template <int NW, int CPL>
__global__ __launch_bounds__(64 * NW) void k_chol_inv(const double* __restrict__ W, int ldw, int n, int L, double tau,
                                                      float* __restrict__ T, DevScalars* sc, int64_t wstride) {
  W += blockIdx.x * wstride;
  T += (int64_t)blockIdx.x * L * L;
  sc += blockIdx.x;
  constexpr int NMAX = 64 * CPL;
  constexpr int S = NMAX / NW;  // row slots per thread
  __shared__ double pub[2][NMAX];
  __shared__ int ndrop[NW];
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int col[CPL];
  bool cn[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    col[u] = j + 64 * u;
    cn[u] = col[u] < n;
  }
  double a[S][CPL], t[S][CPL], iv[S], d0[CPL];
  {
    // unconditional loads from clamped indices (all in flight together), then masked
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = NW * s + w;
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        const double x = W[(i < n ? i : 0) * ldw + (cn[u] ? col[u] : 0)];
        a[s][u] = (i < n && cn[u]) ? x : 0.0;
        t[s][u] = 0.0;
      }
      iv[s] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) d0[u] = W[(cn[u] ? col[u] : 0) * ldw + (cn[u] ? col[u] : 0)];  // W_jj
  }
  int drops = 0;
  // step k = NW sk + wk: the slot loop is unrolled (static register indices; the column half of
  // the pivot, k / 64 = NW sk / 64, is static too because NW divides 64), the wave loop is not
#pragma unroll
  for (int sk = 0; sk < S; ++sk) {
    const int uk = (NW * sk) / 64;
    for (int wk = 0; wk < NW; ++wk) {
      const int k = NW * sk + wk;
      if (k >= n) break;
      const int lk = k % 64;
      if (w == wk) {
        const double p = readlane_d(a[sk][uk], lk);
        const double dk = readlane_d(d0[uk], lk);
        const bool keep = (dk > 0.0) && (p > tau * dk);
        const double is = keep ? rsqrt_nr(p) : 0.0;
        iv[sk] = is;
        drops += keep ? 0 : 1;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const double r = (col[u] >= k && cn[u]) ? a[sk][u] * is : 0.0;
          a[sk][u] = r;  // row k of R
          pub[k & 1][col[u]] = r;
        }
      }
      __syncthreads();
      // branch-free update (masked multipliers), so the broadcast reads are issued together
      double rkj[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) rkj[u] = pub[k & 1][col[u]];
#pragma unroll
      for (int s = sk; s < S; ++s) {  // rows NW s + w > k
        const int i = NW * s + w;
        const double f = (i > k && i < n) ? pub[k & 1][i] : 0.0;
#pragma unroll
        for (int u = 0; u < CPL; ++u) a[s][u] = fma(-f, rkj[u], a[s][u]);
      }
    }
  }
  // T = R^{-1}: t[s][u] accumulates row i = NW s + w of T (column col[u]); rows i = NW si + wi
  // from the last
#pragma unroll
  for (int si = S - 1; si >= 0; --si) {
    const int ui = (NW * si) / 64;
    for (int wi = NW - 1; wi >= 0; --wi) {
      const int i = NW * si + wi;
      if (i >= n) continue;
      const int li = i % 64;
      if (w == wi) {
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          const double x = ((i == col[u]) ? 1.0 : 0.0) - t[si][u];
          const double ti = cn[u] ? x * iv[si] : 0.0;
          t[si][u] = ti;
          pub[i & 1][col[u]] = ti;
        }
      }
      __syncthreads();
      double tij[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) tij[u] = pub[i & 1][col[u]];
#pragma unroll
      for (int s = 0; s <= si; ++s) {  // rows NW s + w <= i
        const int l = NW * s + w;
        const double r = readlane_d(a[s][ui], li);  // R[l][i]
#pragma unroll
        for (int u = 0; u < CPL; ++u) t[s][u] = fma(l < i ? r : 0.0, tij[u], t[s][u]);
      }
    }
  }
  // T (L x L, zero-padded)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = NW * s + w;
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (i < L && col[u] < L) T[i * L + col[u]] = (i < n && cn[u]) ? (float)t[s][u] : 0.f;
  }
  if (j == 0) ndrop[w] = drops;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < NW; ++q) tot += ndrop[q];
    sc->dropped = tot;
  }
}

// The same Cholesky for 128 < n <= 256 in two passes, because the factor and its inverse no
// longer fit the registers together.  Thread (w, j) of NW waves holds columns c = j + 64 u
// (u < 4) and, of rows i = NW s + w, only the slots that can be on or above the diagonal of
// its column group (s < (64 / NW) (u + 1)).
// Pass 1 factors W = R^T R (dropping dependent columns as above) and writes R (pitch 256, zero
// below the diagonal) and 1 / R_kk to Rw, Rw + 256 * 256.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_chol_factor_wide(const double* __restrict__ W, int ldw, int n, double tau,
                                                              double* __restrict__ Rw, DevScalars* sc,
                                                              int64_t wstride, int64_t rstride) {
  W += blockIdx.x * wstride;
  Rw += blockIdx.x * rstride;
  sc += blockIdx.x;
  constexpr int CPL = 4, S = 256 / NW, LD = 256, SG = 64 / NW;  // SG: slots per column group
  __shared__ double pub[2][256];
  __shared__ int ndrop[NW];
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int col[CPL];
  bool cn[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    col[u] = j + 64 * u;
    cn[u] = col[u] < n;
  }
  double a[S][CPL], d0[CPL];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = NW * s + w;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      if (s >= SG * (u + 1)) continue;
      const double x = W[(i < n ? i : 0) * ldw + (cn[u] ? col[u] : 0)];
      a[s][u] = (i < n && cn[u]) ? x : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < CPL; ++u) d0[u] = W[(cn[u] ? col[u] : 0) * ldw + (cn[u] ? col[u] : 0)];
  int drops = 0;
#pragma clang loop unroll(full)  // static register indices need the whole loop unrolled
  for (int sk = 0; sk < S; ++sk) {
    const int uk = sk / SG;
    for (int wk = 0; wk < NW; ++wk) {
      const int k = NW * sk + wk;
      if (k >= n) break;
      const int lk = k % 64;
      if (w == wk) {
        const double p = readlane_d(a[sk][uk], lk);
        const double dk = readlane_d(d0[uk], lk);
        const bool keep = (dk > 0.0) && (p > tau * dk);
        const double is = keep ? rsqrt_nr(p) : 0.0;
        drops += keep ? 0 : 1;
        if (j == 0) Rw[LD * LD + k] = is;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          double r = 0.0;
          if (sk < SG * (u + 1)) {
            r = (col[u] >= k && cn[u]) ? a[sk][u] * is : 0.0;
            a[sk][u] = r;  // row k of R
          }
          pub[k & 1][col[u]] = r;
        }
      }
      __syncthreads();
      double rkj[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) rkj[u] = pub[k & 1][col[u]];
#pragma unroll
      for (int s = sk; s < S; ++s) {
        const int i = NW * s + w;
        const double f = (i > k && i < n) ? pub[k & 1][i] : 0.0;
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          if (s < SG * (u + 1)) a[s][u] = fma(-f, rkj[u], a[s][u]);
      }
    }
  }
  // R (rows of this thread's slots; below-diagonal entries and untracked slots are zero)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = NW * s + w;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      double r = 0.0;
      if (s < SG * (u + 1)) r = (i <= col[u] && i < n && cn[u]) ? a[s][u] : 0.0;
      Rw[i * LD + col[u]] = r;
    }
  }
  if (j == 0) ndrop[w] = drops;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < NW; ++q) tot += ndrop[q];
    sc->dropped = tot;
  }
}

// Pass 2: T = R^{-1} by right-looking back substitution as in k_chol_inv; R[l][i] is read from
// Rw (one address per wave and slot).
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_chol_inverse_wide(const double* __restrict__ Rw, int n, int L,
                                                               float* __restrict__ T, int64_t rstride) {
  Rw += blockIdx.x * rstride;
  T += (int64_t)blockIdx.x * L * L;
  constexpr int CPL = 4, S = 256 / NW, LD = 256, SG = 64 / NW;
  __shared__ double pub[2][256];
  const int j = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int col[CPL];
  bool cn[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    col[u] = j + 64 * u;
    cn[u] = col[u] < n;
  }
  double t[S][CPL];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (s < SG * (u + 1)) t[s][u] = 0.0;
  const double* ivd = Rw + LD * LD;
#pragma clang loop unroll(full)  // static register indices need the whole loop unrolled
  for (int si = S - 1; si >= 0; --si) {
    for (int wi = NW - 1; wi >= 0; --wi) {
      const int i = NW * si + wi;
      if (i >= n) continue;
      if (w == wi) {
        const double iv = ivd[i];
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
          double ti = 0.0;
          if (si < SG * (u + 1)) {
            const double x = ((i == col[u]) ? 1.0 : 0.0) - t[si][u];
            ti = cn[u] ? x * iv : 0.0;
            t[si][u] = ti;
          }
          pub[i & 1][col[u]] = ti;
        }
      }
      __syncthreads();
      double tij[CPL];
#pragma unroll
      for (int u = 0; u < CPL; ++u) tij[u] = pub[i & 1][col[u]];
#pragma unroll
      for (int s = 0; s <= si; ++s) {
        const int l = NW * s + w;
        const double r = l < i ? Rw[l * LD + i] : 0.0;  // R[l][i]
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          if (s < SG * (u + 1)) t[s][u] = fma(r, tij[u], t[s][u]);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = NW * s + w;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      if (i >= L || col[u] >= L) continue;
      float v = 0.f;
      if (s < SG * (u + 1)) v = (i < n && cn[u]) ? (float)t[s][u] : 0.f;
      T[i * L + col[u]] = v;
    }
  }
}

__device__ inline int packed_index(int i, int j, int N) {
  const int a = i < j ? i : j;
  const int b = i < j ? j : i;
  return a * N - ((a * (a - 1)) >> 1) + (b - a);
}

constexpr int kJacobiThreads = 1024;
constexpr int kJacobiMaxBlocksPerThread = (kEigMax / 2) * (kEigMax / 2 + 1) / 2 / kJacobiThreads + 1;

// Cyclic Jacobi with the round-robin ordering: in each round the N/2 index pairs are disjoint,
// so every thread updates whole 2 x 2 blocks of A (packed upper triangle in LDS) and pairs of
// entries of V (N x N in LDS) with two barriers per round.  The (pair, pair) blocks a thread
// owns and the V entries it rotates are fixed for the whole solve.  Sweeps repeat until no
// off-diagonal entry exceeds 1e-15 sqrt(|a_pp a_qq|) (and 1e-18 of the largest diagonal entry).
// An odd n is padded with a zero row and column, which is never rotated.
// (a group launch runs one workgroup per buffer k = blockIdx.x on Ain + k astride,
// evals + k estride, evecs + k vstride)
__global__ __launch_bounds__(kJacobiThreads) void k_eig_jacobi(const double* __restrict__ Ain, int lda, int n,
                                                    double* __restrict__ evals, double* __restrict__ evecs,
                                                    int64_t astride, int64_t estride, int64_t evstride) {
  extern __shared__ double lds[];
  Ain += blockIdx.x * astride;
  evals += blockIdx.x * estride;
  evecs += blockIdx.x * evstride;
  const int N = n + (n & 1);
  const int P = N / 2;
  double* A = lds;                           // N (N + 1) / 2
  double* V = A + (N * (N + 1)) / 2;         // N * N
  double* rc = V + N * N;                    // P
  double* rs = rc + P;                       // P
  int* rp = reinterpret_cast<int*>(rs + P);  // P
  int* rq = rp + P;                          // P
  __shared__ int flag;
  __shared__ double scale;
  const int tid = threadIdx.x;
  for (int e = tid; e < N * N; e += kJacobiThreads) {
    const int i = e / N, j = e - (e / N) * N;
    if (i <= j) A[packed_index(i, j, N)] = (i < n && j < n) ? Ain[i * lda + j] : 0.0;
  }
  for (int e = tid; e < N * N; e += kJacobiThreads) V[e] = (e / N == e % N) ? 1.0 : 0.0;
  // blocks (k1 <= k2) owned by this thread
  int nblk = 0;
  int bk1[kJacobiMaxBlocksPerThread], bk2[kJacobiMaxBlocksPerThread];
  {
    const int total = P * (P + 1) / 2;
    int k1 = 0, base = 0;  // blocks of row k1 are [base, base + P - k1)
    for (int b = tid; b < total; b += kJacobiThreads) {
      while (b >= base + (P - k1)) {
        base += P - k1;
        ++k1;
      }
#pragma unroll
      for (int r = 0; r < kJacobiMaxBlocksPerThread; ++r)
        if (r == nblk) {
          bk1[r] = k1;
          bk2[r] = k1 + (b - base);
        }
      ++nblk;
    }
  }
  // V entries: pair vk, rows vi0, vi0 + vstride, ...
  const int vstride = kJacobiThreads / P;
  const int vk = tid % P;
  const int vi0 = tid / P;
  const bool vactive = tid < vstride * P;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, fabs(A[packed_index(i, i, N)]));
    scale = m;
  }
  __syncthreads();
  const double abs_tol = 1e-18 * scale;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      if (tid < P) {
        const int k = tid;
        int p = k == 0 ? 0 : 1 + (k - 1 + r) % (N - 1);
        int q = 1 + (N - 2 - k + r) % (N - 1);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double app = A[packed_index(p, p, N)], aqq = A[packed_index(q, q, N)];
        const double apq = A[packed_index(p, q, N)];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > abs_tol && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
          const double theta = (aqq - app) * rcp_nr(2.0 * apq);
          const double h2 = fma(theta, theta, 1.0);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(theta) + h2 * rsqrt_nr(h2));
          c = rsqrt_nr(fma(t, t, 1.0));
          s = t * c;
          flag = 1;
        }
        rc[k] = c;
        rs[k] = s;
        rp[k] = p;
        rq[k] = q;
      }
      __syncthreads();
#pragma unroll
      for (int rr = 0; rr < kJacobiMaxBlocksPerThread; ++rr) {
        if (rr >= nblk) break;
        const int k1 = bk1[rr], k2 = bk2[rr];
        const double c1 = rc[k1], s1 = rs[k1], c2 = rc[k2], s2 = rs[k2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = rp[k1], q1 = rq[k1], p2 = rp[k2], q2 = rq[k2];
        if (k1 == k2) {
          const int ipp = packed_index(p1, p1, N), iqq = packed_index(q1, q1, N), ipq = packed_index(p1, q1, N);
          const double t = s1 / c1;
          const double apq = A[ipq];
          A[ipp] = A[ipp] - t * apq;
          A[iqq] = A[iqq] + t * apq;
          A[ipq] = 0.0;
        } else {
          const int i_pp = packed_index(p1, p2, N), i_pq = packed_index(p1, q2, N);
          const int i_qp = packed_index(q1, p2, N), i_qq = packed_index(q1, q2, N);
          const double a_pp = A[i_pp], a_pq = A[i_pq], a_qp = A[i_qp], a_qq = A[i_qq];
          const double up = c2 * a_pp - s2 * a_pq, uq = s2 * a_pp + c2 * a_pq;
          const double wp = c2 * a_qp - s2 * a_qq, wq = s2 * a_qp + c2 * a_qq;
          A[i_pp] = c1 * up - s1 * wp;
          A[i_pq] = c1 * uq - s1 * wq;
          A[i_qp] = s1 * up + c1 * wp;
          A[i_qq] = s1 * uq + c1 * wq;
        }
      }
      if (vactive) {
        const double c = rc[vk], s = rs[vk];
        if (s != 0.0) {
          const int p = rp[vk], q = rq[vk];
          for (int i = vi0; i < N; i += vstride) {
            const double vp = V[i * N + p], vq = V[i * N + q];
            V[i * N + p] = c * vp - s * vq;
            V[i * N + q] = s * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
    const int done = (flag == 0);
    __syncthreads();
    if (done) break;
  }
  // eigenvalues descending (ties by index), eigenvector columns follow
  for (int i = tid; i < n; i += kJacobiThreads) {
    const double li = A[packed_index(i, i, N)];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[packed_index(j, j, N)];
      rank += (lj > li) || (lj == li && j < i);
    }
    evals[rank] = li;
    for (int row = 0; row < n; ++row) evecs[row * n + rank] = V[row * N + i];
  }
}

// (a group launch: buffer k = blockIdx.x on evals + k estride, H + k vstride, M64 / M32 + k L L,
// sc + k)
__global__ __launch_bounds__(256) void k_ssh_post(const double* __restrict__ evals, const double* __restrict__ H,
                                                  int ell, int L, double alpha, double* __restrict__ M64,
                                                  float* __restrict__ M32, DevScalars* sc, int64_t estride,
                                                  int64_t vstride) {
  evals += blockIdx.x * estride;
  H += blockIdx.x * vstride;
  M64 += (int64_t)blockIdx.x * L * L;
  M32 += (int64_t)blockIdx.x * L * L;
  sc += blockIdx.x;
  __shared__ double D[kMaxEll];
  __shared__ double pivot;
  const int tid = threadIdx.x;
  if (tid == 0) pivot = fmax(evals[ell - 1], 0.0);
  __syncthreads();
  if (tid < ell) {
    double l2 = fmax(evals[tid], 0.0);
    D[tid] = l2 > pivot ? sqrt((l2 - pivot) / l2) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < ell * ell; e += 256) {
    int i = e / ell, j = e % ell;
    M64[e] = H[i * ell + j] * D[j];
  }
  for (int e = tid; e < L * L; e += 256) {
    int i = e / L, j = e % L;
    M32[e] = (i < ell && j < ell) ? (float)(H[i * ell + j] * D[j]) : 0.f;
  }
  if (tid == 0) {
    double fb = 0.0;
    for (int i = 0; i < ell; ++i) fb += fmax(fmax(evals[i], 0.0) - pivot, 0.0);
    sc->fro2Bp = fb;
    sc->S = sc->fro2A - fb;
    sc->lam_ell2 = pivot;
    sc->half_delta = 0.5 * sc->S / (alpha * ell);
  }
}

__global__ void k_ssh_identity(int ell, int L, double* __restrict__ M64, float* __restrict__ M32, DevScalars* sc) {
  const int tid = threadIdx.x;
  for (int e = tid; e < ell * ell; e += blockDim.x) M64[e] = (e / ell == e % ell) ? 1.0 : 0.0;
  for (int e = tid; e < L * L; e += blockDim.x) {
    int i = e / L, j = e % L;
    M32[e] = (i == j && i < ell) ? 1.f : 0.f;
  }
  if (tid == 0) {
    sc->fro2Bp = sc->fro2A;
    sc->S = 0.0;
    sc->lam_ell2 = 0.0;
    sc->half_delta = 0.0;
  }
}

// Q = W_PP M (ell x ell, into scratch), W_PP the lower-right block of W2 (pitch 2L)
__global__ __launch_bounds__(256) void k_dsh_q(const double* __restrict__ W2, int L, int ell,
                                               const double* __restrict__ M, double* __restrict__ Q) {
  const int ld = 2 * L;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < ell * ell; e += gridDim.x * 256) {
    const int i = e / ell, j = e % ell;
    double s = 0.0;
    for (int k = 0; k < ell; ++k) s += W2[(L + i) * ld + L + k] * M[k * ell + j];
    Q[e] = s;
  }
}

// SS = [[W_BB, W_BP M], [M^T W_PB, M^T W_PP M]] with W2 = [[W_BB, W_BP], [W_PB, W_PP]] the Gram
// of [B^T | P^T] (pitch 2L): the Gram of the stack [B; B'] with B' = M^T P.  Q = W_PP M.
__global__ __launch_bounds__(256) void k_dsh_assemble(const double* __restrict__ W2, int L, int ell,
                                                      const double* __restrict__ M, const double* __restrict__ Q,
                                                      double* __restrict__ SS) {
  const int ld = 2 * L;
  const int n = 2 * ell;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < ell * ell; e += gridDim.x * 256) {
    int i = e / ell, j = e % ell;
    SS[i * n + j] = W2[i * ld + j];
    double s = 0.0;
    for (int k = 0; k < ell; ++k) s += W2[i * ld + L + k] * M[k * ell + j];
    SS[i * n + ell + j] = s;
    SS[(ell + j) * n + i] = s;
    if (i <= j) {
      double t = 0.0;
      for (int k = 0; k < ell; ++k) t += M[k * ell + i] * Q[k * ell + j];
      SS[(ell + i) * n + ell + j] = t;
      SS[(ell + j) * n + ell + i] = t;
    }
  }
}

// (a grid of blocks over the entries of T2; every block derives the shrink factors itself)
__global__ __launch_bounds__(256) void k_dsh_post(const double* __restrict__ evals, const double* __restrict__ U,
                                                  int ell, int L, const double* __restrict__ M, int lossless,
                                                  float* __restrict__ T2, DevScalars* sc) {
  __shared__ double D[kMaxEll];
  __shared__ double shift;
  const int tid = threadIdx.x;
  const int n = 2 * ell;
  if (tid == 0) shift = lossless ? 0.0 : fmax(evals[ell - 1], 0.0);
  __syncthreads();
  for (int i = tid; i < ell; i += 256) {
    double mu = evals[i];
    D[i] = (mu > 0.0 && mu > shift) ? sqrt((mu - shift) / mu) : 0.0;
  }
  __syncthreads();
  for (int e = blockIdx.x * 256 + tid; e < 2 * L * L; e += gridDim.x * 256) {
    int r = e / L, i = e % L;
    double v = 0.0;
    if (i < ell) {
      if (r < ell) {
        v = U[r * n + i] * D[i];
      } else if (r >= L && r < L + ell) {
        double s = 0.0;
        for (int k = 0; k < ell; ++k) s += M[(r - L) * ell + k] * U[(ell + k) * n + i];
        v = s * D[i];
      }
    }
    T2[e] = (float)v;
  }
  if (blockIdx.x == 0 && tid == 0) sc->mu_ell = shift;
}

}  // namespace

hipError_t chol_inv(const double* W, int ldw, int ell, int L, double tau, float* T, DevScalars* sc, double* Rw,
                    hipStream_t st) {
  return chol_inv_group(W, ldw, ell, L, tau, T, sc, 1, 0, Rw, st);
}

// dynamic LDS of the Jacobi solver for an n x n problem: packed upper A, V, pair lists
size_t eig_lds_bytes(int n) {
  const int N = n + (n & 1);
  const int P = N / 2;
  return sizeof(double) * ((size_t)N * (N + 1) / 2 + (size_t)N * N + 2 * P) + sizeof(int) * 2 * P;
}

int64_t eig_work_bytes(int n) { return n <= kEigMax ? 0 : eig_tri_work_bytes(n); }

hipError_t eig_sym_group(const double* A, int lda, int n, int nvec, double* evals, double* evecs, int K,
                         int64_t astride, int64_t estride, int64_t vstride, void* work, int64_t wstride,
                         hipStream_t st) {
  if (n > kEigMax)
    return eig_tri_group(A, lda, n, nvec, evals, evecs, K, astride, estride, vstride, work, wstride, st);
  if (n < 1 || K < 1) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    // allow the largest problem's dynamic LDS (more than the default 64 KiB; gfx950 has 160 KiB)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_jacobi),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)eig_lds_bytes(kEigMax));
    attr_set = true;
  }
  k_eig_jacobi<<<K, kJacobiThreads, eig_lds_bytes(n), st>>>(A, lda, n, evals, evecs, astride, estride, vstride);
  return hipGetLastError();
}

hipError_t eig_sym(const double* A, int lda, int n, int nvec, double* evals, double* evecs, void* work,
                   hipStream_t st) {
  return eig_sym_group(A, lda, n, nvec, evals, evecs, 1, 0, 0, 0, work, eig_work_bytes(n), st);
}

hipError_t ssh_post(const double* evals, const double* H, int ell, int L, double alpha, double* M64, float* M32,
                    DevScalars* sc, hipStream_t st) {
  k_ssh_post<<<1, 256, 0, st>>>(evals, H, ell, L, alpha, M64, M32, sc, 0, 0);
  return hipGetLastError();
}

int64_t chol_work_doubles(int L) { return L > kCholMax ? 256 * 256 + 256 : 0; }

hipError_t chol_inv_group(const double* W, int ldw, int ell, int L, double tau, float* T, DevScalars* sc, int K,
                          int64_t wstride, double* Rw, hipStream_t st) {
  if (ell > kCholMaxWide || L > kCholMaxWide) return hipErrorInvalidValue;
  if (ell <= 64 && L <= 64) {
    k_chol_inv<4, 1><<<K, 256, 0, st>>>(W, ldw, ell, L, tau, T, sc, wstride);
  } else if (ell <= kCholMax && L <= kCholMax) {
    k_chol_inv<16, 2><<<K, 1024, 0, st>>>(W, ldw, ell, L, tau, T, sc, wstride);
  } else {
    if (!Rw) return hipErrorInvalidValue;
    k_chol_factor_wide<8><<<K, 512, 0, st>>>(W, ldw, ell, tau, Rw, sc, wstride, chol_work_doubles(L));
    k_chol_inverse_wide<8><<<K, 512, 0, st>>>(Rw, ell, L, T, chol_work_doubles(L));
  }
  return hipGetLastError();
}

hipError_t ssh_post_group(const double* evals, const double* H, int ell, int L, double alpha, double* M64, float* M32,
                          DevScalars* sc, int K, int64_t estride, int64_t vstride, hipStream_t st) {
  k_ssh_post<<<K, 256, 0, st>>>(evals, H, ell, L, alpha, M64, M32, sc, estride, vstride);
  return hipGetLastError();
}

hipError_t ssh_identity(int ell, int L, double* M64, float* M32, DevScalars* sc, hipStream_t st) {
  k_ssh_identity<<<1, 256, 0, st>>>(ell, L, M64, M32, sc);
  return hipGetLastError();
}

hipError_t dsh_assemble(const double* W2, int L, int ell, const double* M64, double* SS, double* scratch,
                        hipStream_t st) {
  const unsigned g = (unsigned)std::min(64, (ell * ell + 255) / 256);
  k_dsh_q<<<g, 256, 0, st>>>(W2, L, ell, M64, scratch);
  k_dsh_assemble<<<g, 256, 0, st>>>(W2, L, ell, M64, scratch, SS);
  return hipGetLastError();
}

hipError_t dsh_post(const double* evals, const double* U, int ell, int L, const double* M64, int lossless,
                    float* T2, DevScalars* sc, hipStream_t st) {
  k_dsh_post<<<(unsigned)std::min(64, (2 * L * L + 255) / 256), 256, 0, st>>>(evals, U, ell, L, M64, lossless, T2, sc);
  return hipGetLastError();
}

}  // namespace sfd
