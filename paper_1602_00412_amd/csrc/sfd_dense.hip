// Dense panel kernels: the Gram matrices of the tall panels on MFMA (GramSchmidt of Alg 1 as
// CholeskyQR, svd(P, ell) of Alg 3 and svd([B; B'], ell) of Alg 5 through W^T W), row
// transforms panel * T, the panel-transpose matrix-vector product of VerifySpectral, and the
// counter-based start block G of Alg 1.
//
// Panels are row-major and tall (d x L or m x L, L = ell rounded up to 32, zero-padded), so
// every Gram has its contraction along the tall axis.
#include "sfd_internal.h"

namespace sfd {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kGramMaxBlocks = 512;

// Gram partial of a row block.  MFMA v_mfma_f32_16x16x4f32: A (16 x 4) and B (4 x 16) come one
// float per lane, lane l holding row-of-A / column-of-B (l % 16) at k = l / 16; the 16 x 16
// accumulator leaves 4 floats per lane, lane l holding column l % 16, rows 4*(l/16) .. +3.
// For W = P^T P both operands are the same 4-row slab of the panel: lane l loads
// P[k0 + l/16][16*s + l%16] for each 16-column strip s.
template <int W>
__global__ __launch_bounds__(256) void k_gram_partial(const float* __restrict__ P, int ld, int64_t rows, int rpb,
                                                      float* __restrict__ partials) {
  constexpr int S = W / 16;          // strips
  constexpr int NT = S * S;          // 16 x 16 tiles
  constexpr int TG = NT >= 64 ? 4 : 1;  // tile groups (waves split tiles)
  constexpr int KG = 4 / TG;            // k groups (waves split rows)
  constexpr int TPW = NT / TG;          // tiles per wave
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tg = wave % TG;
  const int kg = wave / TG;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  floatx4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lrow = lane >> 4;
  const int lcol = lane & 15;
  for (int64_t k0 = r0 + 4 * kg; k0 < r1; k0 += 4 * KG) {
    const int64_t row = k0 + lrow;
    float f[S];
    if (row < r1) {
      const float* pr = P + row * ld + lcol;
#pragma unroll
      for (int s = 0; s < S; ++s) f[s] = pr[16 * s];
    } else {
#pragma unroll
      for (int s = 0; s < S; ++s) f[s] = 0.f;
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = tg * TPW + t;
      const int ti = tile / S, tj = tile % S;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[ti], f[tj], acc[t], 0, 0, 0);
    }
  }
  float* out = partials + (int64_t)blockIdx.x * W * W;
  if constexpr (KG == 1) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = tg * TPW + t;
      const int ti = tile / S, tj = tile % S;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * ti + 4 * lrow + v) * W + 16 * tj + lcol] = acc[t][v];
    }
  } else {
    __shared__ float red[W * W];
    for (int g = 0; g < KG; ++g) {
      if (kg == g) {
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          const int tile = tg * TPW + t;
          const int ti = tile / S, tj = tile % S;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int e = (16 * ti + 4 * lrow + v) * W + 16 * tj + lcol;
            red[e] = (g == 0) ? acc[t][v] : red[e] + acc[t][v];
          }
        }
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < W * W; e += 256) out[e] = red[e];
  }
}

// W64[i][j] = sum over blocks (in block order, FP64) of the upper-triangle partial (i <= j),
// mirrored, so W64 is exactly symmetric.
__global__ void k_gram_reduce(const float* __restrict__ partials, int nb, int W, double* __restrict__ Wout) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= W * W) return;
  int i = e / W, j = e % W;
  int src = i <= j ? e : j * W + i;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += (double)partials[(int64_t)b * W * W + src];
  Wout[e] = s;
}

// out[j, 0:WOUT] = in[j, 0:WIN] * T.  One wave per row; lane c keeps column c of T in
// registers and gathers the input row through readlane broadcasts.
template <int WIN, int WOUT>
__global__ __launch_bounds__(256) void k_panel_xform(const float* in, int ldi, const float* __restrict__ T,
                                                     float* out, int ldo, int64_t rows) {
  static_assert((WIN == 32 || WIN == 64 || WIN == 128) && WOUT <= 64, "panel shape");
  constexpr int KA = WIN < 64 ? WIN : 64;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  float t[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) t[k] = lane < WOUT ? T[k * WOUT + lane] : 0.f;
  for (int64_t r = wave; r < rows; r += nwaves) {
    const float* ir = in + r * ldi;
    const float a = lane < KA ? ir[lane] : 0.f;
    float b = 0.f;
    if constexpr (WIN > 64) b = ir[64 + lane];
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < KA; ++k)
      acc = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), k)), t[k], acc);
    if constexpr (WIN > 64) {
#pragma unroll
      for (int k = 0; k < 64; ++k)
        acc = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(b), k)), t[64 + k], acc);
    }
    if (lane < WOUT) out[r * ldo + lane] = acc;
  }
}

__global__ __launch_bounds__(256) void k_panel_gemv_t(const float* __restrict__ P, int ld, int L, int64_t rows,
                                                      int rpb, const float* __restrict__ y,
                                                      const double* __restrict__ scale_ptr, float* __restrict__ part) {
  __shared__ float red[4][128];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  float a0 = 0.f, a1 = 0.f;
  for (int64_t r = r0 + wave; r < r1; r += 4) {
    float yv = y[r];
    const float* pr = P + r * ld;
    if (lane < L) a0 = fmaf(pr[lane], yv, a0);
    if (64 + lane < L) a1 = fmaf(pr[64 + lane], yv, a1);
  }
  red[wave][lane] = a0;
  red[wave][64 + lane] = a1;
  __syncthreads();
  if (threadIdx.x < 128 && threadIdx.x < L) {
    float s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    float sc = scale_ptr ? (float)(*scale_ptr) : 1.f;
    part[(int64_t)blockIdx.x * L + threadIdx.x] = s * sc;
  }
}

// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of
//   (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2, x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
// with the key bumped by the Weyl constants (W0, W1) between rounds.
__device__ inline void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    uint64_t lo0 = m0 * x[0], hi0 = __umul64hi(m0, x[0]);
    uint64_t lo1 = m1 * x[2], hi1 = __umul64hi(m1, x[2]);
    uint64_t n0 = hi1 ^ x[1] ^ k0;
    uint64_t n2 = hi0 ^ x[3] ^ k1;
    x[0] = n0;
    x[1] = lo1;
    x[2] = n2;
    x[3] = lo0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
}

// word -> (0, 1): ((w >> 12) + 1/2) * 2^-52, exact in FP64
__device__ inline double unit_open(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// Block j (counter (j, attempt, buffer, purpose), key (seed, stream)) gives elements 4j..4j+3 of
// the row-major d x ell start block through the Box-Muller transform on (u0, u1), (u2, u3).
__global__ void k_start_block(uint64_t seed, uint64_t sid, uint64_t buffer, uint64_t attempt, uint64_t purpose,
                              int64_t d, int ell, float* out, int ld) {
  const int64_t total = d * ell;
  const int64_t nblk = (total + 3) / 4;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double two_pi = 2.0 * 3.141592653589793;
  for (; j < nblk; j += stride) {
    uint64_t x[4] = {(uint64_t)j, attempt, buffer, purpose};
    philox4x64_10(x, seed, sid);
    double u0 = unit_open(x[0]), u1 = unit_open(x[1]), u2 = unit_open(x[2]), u3 = unit_open(x[3]);
    double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
    double ta = two_pi * u1, tb = two_pi * u3;
    double z[4] = {ra * cos(ta), ra * sin(ta), rb * cos(tb), rb * sin(tb)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t e = 4 * j + q;
      if (e < total) {
        int64_t row = e / ell;
        int col = (int)(e - row * ell);
        out[row * ld + col] = (float)z[q];
      }
    }
  }
}

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int gram_max_blocks() { return kGramMaxBlocks; }

hipError_t gram(const float* P, int ld, int64_t rows, int w, float* partials, double* W, hipStream_t st) {
  int64_t nb = (rows + 63) / 64;
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  if (nb < 1) nb = 1;
  int rpb = (int)((rows + nb - 1) / nb);
  rpb = (rpb + 3) & ~3;
  nb = rows > 0 ? (rows + rpb - 1) / rpb : 1;
  switch (w) {
    case 32: k_gram_partial<32><<<(unsigned)nb, 256, 0, st>>>(P, ld, rows, rpb, partials); break;
    case 64: k_gram_partial<64><<<(unsigned)nb, 256, 0, st>>>(P, ld, rows, rpb, partials); break;
    case 128: k_gram_partial<128><<<(unsigned)nb, 256, 0, st>>>(P, ld, rows, rpb, partials); break;
    default: return hipErrorInvalidValue;
  }
  k_gram_reduce<<<(unsigned)((w * w + 255) / 256), 256, 0, st>>>(partials, (int)nb, w, W);
  return hipGetLastError();
}

hipError_t panel_xform(const float* in, int ldi, int win, const float* T, float* out, int ldo, int wout,
                       int64_t rows, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  unsigned grid = grid_for(rows, 4, 8192);
  if (win == 32 && wout == 32)
    k_panel_xform<32, 32><<<grid, 256, 0, st>>>(in, ldi, T, out, ldo, rows);
  else if (win == 64 && wout == 64)
    k_panel_xform<64, 64><<<grid, 256, 0, st>>>(in, ldi, T, out, ldo, rows);
  else if (win == 64 && wout == 32)
    k_panel_xform<64, 32><<<grid, 256, 0, st>>>(in, ldi, T, out, ldo, rows);
  else if (win == 128 && wout == 64)
    k_panel_xform<128, 64><<<grid, 256, 0, st>>>(in, ldi, T, out, ldo, rows);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int gemv_blocks(int64_t rows) {
  int64_t nb = (rows + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t panel_gemv_t(const float* P, int ld, int L, int64_t rows, const float* y, const double* scale_ptr,
                        float* part, hipStream_t st) {
  int nb = gemv_blocks(rows);
  int rpb = (int)((rows + nb - 1) / nb);
  k_panel_gemv_t<<<nb, 256, 0, st>>>(P, ld, L, rows, rpb, y, scale_ptr, part);
  return hipGetLastError();
}

hipError_t start_block(uint64_t seed, uint64_t stream_id, uint64_t buffer, uint64_t attempt, uint64_t purpose,
                       int64_t d, int ell, float* out, int ld, hipStream_t st) {
  int64_t nblk = (d * ell + 3) / 4;
  k_start_block<<<grid_for(nblk, 256, 16384), 256, 0, st>>>(seed, stream_id, buffer, attempt, purpose, d, ell, out, ld);
  return hipGetLastError();
}

}  // namespace sfd
