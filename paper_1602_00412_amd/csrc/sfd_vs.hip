// VerifySpectral (Alg 6) on C = (A'^T A' - B'^T B') / (Delta/2): power steps
//   w = A'^T (A' y) - B'^T (B' y),  y <- w / ||w||,  ln||C^t x|| = sum (ln||w|| - ln(Delta/2)).
// B'^T = P^T M is never formed: B'^T (B' y) = P^T (M (M^T (P y))).  The sparse products use the
// chunked SpMV of the SimultaneousIteration schedule; the scalars live in DevScalars.
#include <math.h>

#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int kNormBlocks = 512;

// Group launches: buffer k = blockIdx.y (k_sumsq, k_vs_finish) or blockIdx.x (the one-block
// kernels) works on its own vectors, partials, matrices and scalars at fixed strides.
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double s[256];
  x += (int64_t)blockIdx.y * n;
  part += (int64_t)blockIdx.y * gridDim.x;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double v = x[i];
    acc += v * v;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__device__ double block_sum(const double* part, int nb, double* s) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += part[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  return s[0];
}

__global__ __launch_bounds__(256) void k_vs_init(const double* __restrict__ part, int nb, DevScalars* sc) {
  __shared__ double s[256];
  part += (int64_t)blockIdx.x * nb;
  sc += blockIdx.x;
  double tot = block_sum(part, nb, s);
  if (threadIdx.x == 0) {
    double nrm = sqrt(tot);
    sc->ln_norm = 0.0;
    sc->zero_flag = nrm > 0.0 ? 0 : 1;
    sc->inv_norm = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
}

// c = sum of the P y partials (FP64; wave w adds partials w, w + 4, ..., then the waves in
// order); c2 = M (M^T c)
__global__ __launch_bounds__(1024) void k_vs_small(const float* __restrict__ part, int nb,
                                                   const double* __restrict__ M, int ell, int L,
                                                   float* __restrict__ c2) {
  __shared__ double red[16][256];
  part += (int64_t)blockIdx.x * nb * L;
  M += (int64_t)blockIdx.x * L * L;
  c2 += (int64_t)blockIdx.x * 2 * L;
  __shared__ double c[kMaxEll];
  __shared__ double u[kMaxEll];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // columns lane + 64 h (L <= 256)
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int cc = lane + 64 * h;
    if (cc >= L) break;
    double s = 0.0;
    int b = wave;
    for (; b + 48 < nb; b += 64) {
      const float v0 = part[(int64_t)b * L + cc], v1 = part[(int64_t)(b + 16) * L + cc];
      const float v2 = part[(int64_t)(b + 32) * L + cc], v3 = part[(int64_t)(b + 48) * L + cc];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; b < nb; b += 16) s += part[(int64_t)b * L + cc];
    red[wave][cc] = s;
  }
  __syncthreads();
  if (tid < ell) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += red[w][tid];
    c[tid] = t;
  }
  __syncthreads();
  if (tid < ell) {
    double s = 0.0;
    for (int k = 0; k < ell; ++k) s += M[k * ell + tid] * c[k];
    u[tid] = s;
  }
  __syncthreads();
  if (tid < L) {
    double s = 0.0;
    if (tid < ell)
      for (int k = 0; k < ell; ++k) s += M[tid * ell + k] * u[k];
    c2[tid] = (float)s;
  }
}

// w[j] = w_raw[j] - P[j, :] . c2 and the block's partial of sum_j w[j]^2 (FP64), for j < d.  A row
// is read by L/4 lanes (one float4 each) and reduced over them with xor shuffles; a wave takes
// 64/(L/4) rows per pass and kVsUnroll passes at once, so that many rows' loads are in flight.
// Groups: buffer k = blockIdx.y (its w_raw, P, c2, w and partials at offsets k d, k d ld,
// k 2 L, k d, k gridDim.x).
constexpr int kVsUnroll = 4;
template <int L>
__global__ __launch_bounds__(256) void k_vs_finish(const float* __restrict__ w_raw, const float* __restrict__ P,
                                                   int ld, const float* __restrict__ c2, int64_t d,
                                                   float* __restrict__ w, double* __restrict__ part) {
  constexpr int LPR = L / 4;     // lanes per row
  constexpr int RPW = 64 / LPR;  // rows per wave and pass
  __shared__ double s[4];
  {
    const int64_t k = blockIdx.y;
    w_raw += k * d;
    P += k * d * ld;
    c2 += k * 2 * L;
    w += k * d;
    part += k * gridDim.x;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane % LPR, rw = lane / LPR;
  const float4 cc = reinterpret_cast<const float4*>(c2)[sub];
  double acc = 0.0;
  const int64_t step = (int64_t)gridDim.x * 4 * RPW * kVsUnroll;
  for (int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * RPW * kVsUnroll; j0 < d; j0 += step) {
    float4 p[kVsUnroll];
    float wr[kVsUnroll];
#pragma unroll
    for (int u = 0; u < kVsUnroll; ++u) {
      const int64_t j = j0 + u * RPW + rw;
      p[u] = j < d ? reinterpret_cast<const float4*>(P + j * ld)[sub] : make_float4(0.f, 0.f, 0.f, 0.f);
      wr[u] = (sub == 0 && j < d) ? w_raw[j] : 0.f;
    }
    float v[kVsUnroll];
#pragma unroll
    for (int u = 0; u < kVsUnroll; ++u) v[u] = ((p[u].x * cc.x + p[u].y * cc.y) + p[u].z * cc.z) + p[u].w * cc.w;
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1)
#pragma unroll
      for (int u = 0; u < kVsUnroll; ++u) v[u] += __shfl_xor(v[u], o, 64);
    if (sub == 0) {
#pragma unroll
      for (int u = 0; u < kVsUnroll; ++u) {
        const int64_t j = j0 + u * RPW + rw;
        if (j < d) {
          const float r = wr[u] - v[u];
          w[j] = r;
          acc += (double)r * (double)r;
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) s[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// steps: the step being taken and, for a group, each buffer's step count (a buffer past its
// count keeps its norm)
__global__ __launch_bounds__(256) void k_vs_norm(const double* __restrict__ part, int nb, DevScalars* sc,
                                                 int* __restrict__ tsteps) {
  __shared__ double s[256];
  part += (int64_t)blockIdx.x * nb;
  sc += blockIdx.x;
  if (tsteps && tsteps[blockIdx.x] <= 0) return;
  double tot = block_sum(part, nb, s);  // (its barriers order every thread's read of tsteps above)
  if (threadIdx.x == 0) {
    if (tsteps) tsteps[blockIdx.x] -= 1;
    double nrm = sqrt(tot);
    if (sc->zero_flag || !(nrm > 0.0)) {
      sc->zero_flag = 1;
      sc->ln_norm = -HUGE_VAL;
      sc->inv_norm = 0.0;
    } else {
      sc->ln_norm += log(nrm) - log(sc->half_delta);
      sc->inv_norm = 1.0 / nrm;
    }
  }
}

}  // namespace

hipError_t vs_init(const float* w, int64_t d, double* part, DevScalars* sc, hipStream_t st, int K) {
  k_sumsq<<<dim3(kNormBlocks, K), 256, 0, st>>>(w, d, part);
  k_vs_init<<<K, 256, 0, st>>>(part, kNormBlocks, sc);
  return hipGetLastError();
}

int vs_norm_blocks() { return kNormBlocks; }

hipError_t vs_small(const float* part, int nb, const double* M64, int ell, int L, float* c2, hipStream_t st, int K) {
  k_vs_small<<<K, 1024, 0, st>>>(part, nb, M64, ell, L, c2);
  return hipGetLastError();
}

int vs_finish_blocks(int64_t d) {
  int64_t nb = (d + 63) / 64;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t vs_finish(const float* w_raw, const float* P, int ld, int L, int ell, const float* c2, int64_t d,
                     float* w, double* part, hipStream_t st, int K) {
  (void)ell;
  const dim3 grid(vs_finish_blocks(d), K);
  if (L == 32)
    k_vs_finish<32><<<grid, 256, 0, st>>>(w_raw, P, ld, c2, d, w, part);
  else if (L == 64)
    k_vs_finish<64><<<grid, 256, 0, st>>>(w_raw, P, ld, c2, d, w, part);
  else if (L == 128)
    k_vs_finish<128><<<grid, 256, 0, st>>>(w_raw, P, ld, c2, d, w, part);
  else if (L == 256)
    k_vs_finish<256><<<grid, 256, 0, st>>>(w_raw, P, ld, c2, d, w, part);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t vs_norm(const double* part, int nb, DevScalars* sc, hipStream_t st, int K, int* tsteps) {
  k_vs_norm<<<K, 256, 0, st>>>(part, nb, sc, tsteps);
  return hipGetLastError();
}

}  // namespace sfd
