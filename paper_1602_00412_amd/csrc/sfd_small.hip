// Small dense FP64 solvers of the buffer step, each in one workgroup:
//  - pivoted Cholesky of an ell x ell Gram and the inverse of its factor (CholeskyQR form of the
//    GramSchmidt step of Alg 1),
//  - symmetric eigensolver (cyclic Jacobi) for svd(P, ell) of Alg 3 and svd([B; B'], ell) of
//    Alg 5 through their Gram matrices,
//  - the shrink factors sqrt(Lambda^2 - lambda_ell^2 I) of Alg 3 / Alg 5 and Delta of Alg 4.
#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int kCholMax = 64;
constexpr int kEigMax = 2 * kMaxEll;

// Right-looking Cholesky W = R^T R on the ell x ell leading block, in LDS.  A pivot that has
// fallen to tau * W_kk (the column's own squared norm) marks column k as dependent on the
// earlier ones: its row of R is zeroed and it is skipped.  Then T = R^{-1} on the kept
// columns (zero rows/columns for dropped ones), so panel * T has orthonormal kept columns
// spanning the panel's numerical column space.
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ W, int ldw, int n, int L, double tau,
                                                  float* __restrict__ T, DevScalars* sc) {
  __shared__ double A[kCholMax][kCholMax + 1];
  __shared__ double Ti[kCholMax][kCholMax + 1];
  __shared__ double d0[kCholMax];
  __shared__ int drop[kCholMax];
  __shared__ int ndrop;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += 256) {
    int i = e / n, j = e % n;
    A[i][j] = W[i * ldw + j];
  }
  if (tid < n) {
    d0[tid] = W[tid * ldw + tid];
    drop[tid] = 0;
  }
  if (tid == 0) ndrop = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = A[k][k];
    const bool dk = !(d0[k] > 0.0) || !(piv > tau * d0[k]);
    if (dk) {
      for (int j = k + tid; j < n; j += 256) A[k][j] = 0.0;
      if (tid == 0) {
        drop[k] = 1;
        ++ndrop;
      }
    } else {
      const double rkk = sqrt(piv);
      for (int j = k + 1 + tid; j < n; j += 256) A[k][j] /= rkk;
    }
    __syncthreads();
    if (!dk) {
      if (tid == 0) A[k][k] = sqrt(piv);
      const int m = n - k - 1;
      for (int e = tid; e < m * m; e += 256) {
        int i = k + 1 + e / m, j = k + 1 + e % m;
        if (i <= j) A[i][j] -= A[k][i] * A[k][j];
      }
    }
    __syncthreads();
  }
  if (tid < n) {
    const int j = tid;
    for (int i = 0; i < n; ++i) Ti[i][j] = 0.0;
    if (!drop[j]) {
      Ti[j][j] = 1.0 / A[j][j];
      for (int i = j - 1; i >= 0; --i) {
        if (drop[i]) continue;
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s += A[i][k] * Ti[k][j];
        Ti[i][j] = -s / A[i][i];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < L * L; e += 256) {
    int i = e / L, j = e % L;
    T[e] = (i < n && j < n) ? (float)Ti[i][j] : 0.f;
  }
  if (tid == 0) sc->dropped = ndrop;
}

__device__ inline int packed_index(int i, int j, int N) {
  if (i > j) {
    int t = i;
    i = j;
    j = t;
  }
  return i * N - (i * (i - 1)) / 2 + (j - i);
}

// Cyclic Jacobi with the round-robin ordering: in each round the N/2 index pairs are disjoint,
// every workgroup thread updates whole 2 x 2 blocks of A (packed upper triangle in LDS) and
// pairs of entries of V (N x N in LDS), so one round needs two barriers.  Sweeps repeat until
// no off-diagonal entry is above 1e-15 sqrt(|a_pp a_qq|) (and above 1e-18 of the largest
// diagonal).  An odd n is padded with a zero row and column, which is never rotated.
__global__ __launch_bounds__(256) void k_eig_jacobi(const double* __restrict__ Ain, int lda, int n,
                                                    double* __restrict__ evals, double* __restrict__ evecs) {
  extern __shared__ double lds[];
  const int N = n + (n & 1);
  const int P = N / 2;
  double* A = lds;                                 // N (N + 1) / 2
  double* V = A + (N * (N + 1)) / 2;               // N * N
  double* rc = V + N * N;                          // P
  double* rs = rc + P;                             // P
  int* rp = reinterpret_cast<int*>(rs + P);        // P
  int* rq = rp + P;                                // P
  __shared__ int flag;
  __shared__ double scale;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += 256) {
    for (int j = i; j < N; ++j) A[packed_index(i, j, N)] = (i < n && j < n) ? Ain[i * lda + j] : 0.0;
  }
  for (int e = tid; e < N * N; e += 256) V[e] = (e / N == e % N) ? 1.0 : 0.0;
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
      for (int k = tid; k < P; k += 256) {
        int i0 = k, i1 = N - 1 - k;
        int p = i0 == 0 ? 0 : 1 + (i0 - 1 + r) % (N - 1);
        int q = 1 + (i1 - 1 + r) % (N - 1);
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        double app = A[packed_index(p, p, N)], aqq = A[packed_index(q, q, N)], apq = A[packed_index(p, q, N)];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > abs_tol && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
          double theta = (aqq - app) / (2.0 * apq);
          double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          flag = 1;
        }
        rc[k] = c;
        rs[k] = s;
        rp[k] = p;
        rq[k] = q;
      }
      __syncthreads();
      for (int b = tid; b < P * P; b += 256) {
        const int k1 = b / P, k2 = b % P;
        if (k1 > k2) continue;
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
      for (int e = tid; e < N * P; e += 256) {
        const int i = e / P, k = e % P;
        const double c = rc[k], s = rs[k];
        if (s == 0.0) continue;
        const int p = rp[k], q = rq[k];
        const double vp = V[i * N + p], vq = V[i * N + q];
        V[i * N + p] = c * vp - s * vq;
        V[i * N + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    __syncthreads();
    if (flag == 0) break;
    __syncthreads();
  }
  // eigenvalues descending (ties by index), eigenvector columns follow
  for (int i = tid; i < n; i += 256) {
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

__global__ __launch_bounds__(256) void k_ssh_post(const double* __restrict__ evals, const double* __restrict__ H,
                                                  int ell, int L, double alpha, double* __restrict__ M64,
                                                  float* __restrict__ M32, DevScalars* sc) {
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

// SS = [[W_BB, W_BP M], [M^T W_PB, M^T W_PP M]] with W2 = [[W_BB, W_BP], [W_PB, W_PP]] the Gram
// of [B^T | P^T] (pitch 2L): the Gram of the stack [B; B'] with B' = M^T P.
__global__ __launch_bounds__(256) void k_dsh_assemble(const double* __restrict__ W2, int L, int ell,
                                                      const double* __restrict__ M, double* __restrict__ SS) {
  __shared__ double Q[kMaxEll][kMaxEll + 1];  // W_PP M
  const int tid = threadIdx.x;
  const int ld = 2 * L;
  const int n = 2 * ell;
  for (int e = tid; e < ell * ell; e += 256) {
    int i = e / ell, j = e % ell;
    double s = 0.0;
    for (int k = 0; k < ell; ++k) s += W2[(L + i) * ld + L + k] * M[k * ell + j];
    Q[i][j] = s;
  }
  __syncthreads();
  for (int e = tid; e < ell * ell; e += 256) {
    int i = e / ell, j = e % ell;
    SS[i * n + j] = W2[i * ld + j];
    double s = 0.0;
    for (int k = 0; k < ell; ++k) s += W2[i * ld + L + k] * M[k * ell + j];
    SS[i * n + ell + j] = s;
    SS[(ell + j) * n + i] = s;
    if (i <= j) {
      double t = 0.0;
      for (int k = 0; k < ell; ++k) t += M[k * ell + i] * Q[k][j];
      SS[(ell + i) * n + ell + j] = t;
      SS[(ell + j) * n + ell + i] = t;
    }
  }
}

__global__ __launch_bounds__(256) void k_dsh_post(const double* __restrict__ evals, const double* __restrict__ U,
                                                  int ell, int L, const double* __restrict__ M, int lossless,
                                                  float* __restrict__ T2, DevScalars* sc) {
  __shared__ double D[kMaxEll];
  __shared__ double shift;
  const int tid = threadIdx.x;
  const int n = 2 * ell;
  if (tid == 0) shift = lossless ? 0.0 : fmax(evals[ell - 1], 0.0);
  __syncthreads();
  if (tid < ell) {
    double mu = evals[tid];
    D[tid] = (mu > 0.0 && mu > shift) ? sqrt((mu - shift) / mu) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 2 * L * L; e += 256) {
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
  if (tid == 0) sc->mu_ell = shift;
}

}  // namespace

hipError_t chol_inv(const double* W, int ldw, int ell, int L, double tau, float* T, DevScalars* sc,
                    hipStream_t st) {
  if (ell > kCholMax || L > kCholMax) return hipErrorInvalidValue;
  k_chol_inv<<<1, 256, 0, st>>>(W, ldw, ell, L, tau, T, sc);
  return hipGetLastError();
}

hipError_t eig_sym(const double* A, int lda, int n, double* evals, double* evecs, hipStream_t st) {
  if (n < 1 || n > kEigMax) return hipErrorInvalidValue;
  const int N = n + (n & 1);
  const int P = N / 2;
  size_t bytes = sizeof(double) * ((size_t)N * (N + 1) / 2 + (size_t)N * N + 2 * P) + sizeof(int) * 2 * P;
  static bool attr_set = false;
  if (!attr_set) {
    // allow more than the default 64 KiB of dynamic LDS (gfx950 has 160 KiB per workgroup)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_jacobi),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr_set = true;
  }
  k_eig_jacobi<<<1, 256, bytes, st>>>(A, lda, n, evals, evecs);
  return hipGetLastError();
}

hipError_t ssh_post(const double* evals, const double* H, int ell, int L, double alpha, double* M64, float* M32,
                    DevScalars* sc, hipStream_t st) {
  k_ssh_post<<<1, 256, 0, st>>>(evals, H, ell, L, alpha, M64, M32, sc);
  return hipGetLastError();
}

hipError_t ssh_identity(int ell, int L, double* M64, float* M32, DevScalars* sc, hipStream_t st) {
  k_ssh_identity<<<1, 256, 0, st>>>(ell, L, M64, M32, sc);
  return hipGetLastError();
}

hipError_t dsh_assemble(const double* W2, int L, int ell, const double* M64, double* SS, hipStream_t st) {
  k_dsh_assemble<<<1, 256, 0, st>>>(W2, L, ell, M64, SS);
  return hipGetLastError();
}

hipError_t dsh_post(const double* evals, const double* U, int ell, int L, const double* M64, int lossless,
                    float* T2, DevScalars* sc, hipStream_t st) {
  k_dsh_post<<<1, 256, 0, st>>>(evals, U, ell, L, M64, lossless, T2, sc);
  return hipGetLastError();
}

}  // namespace sfd
