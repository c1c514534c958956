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

constexpr int kGramMaxBlocks = 256;

// Gram partial of a row block.  MFMA v_mfma_f32_16x16x4f32: A (16 x 4) and B (4 x 16) come one
// float per lane, lane l holding row-of-A / column-of-B (l % 16) at k = l / 16; the 16 x 16
// accumulator leaves 4 floats per lane, lane l holding column l % 16, rows 4*(l/16) .. +3.
// For W = P^T P both operands are the same 4-row slab of the panel: lane l loads
// P[k0 + l/16][16*s + l%16] for each 16-column strip s.  Eight waves per block split the rows
// (and, for W = 128, the tiles); the next slab is loaded while the current one is multiplied.
constexpr int kGramThreads = 512;
constexpr int kGramWaves = kGramThreads / 64;

// TWO: the panel is [P | P2] side by side, each W/2 wide (strips of the right half from P2).
template <int W, bool TWO>
__global__ __launch_bounds__(kGramThreads) void k_gram_partial(const float* __restrict__ P, int ld,
                                                               const float* __restrict__ P2, int ld2, int64_t rows,
                                                               int rpb, float* __restrict__ partials) {
  constexpr int S = W / 16;                // strips
  constexpr int NT = S * S;                // 16 x 16 tiles
  constexpr int TG = NT >= 64 ? 4 : 1;     // tile groups (waves split tiles)
  constexpr int KG = kGramWaves / TG;      // k groups (waves split rows)
  constexpr int TPW = NT / TG;             // tiles per wave
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
  constexpr int SPLIT = TWO ? S / 2 : S;  // strips read from P; the rest from P2
  float f[S], g[S];
  int64_t k0 = r0 + 4 * kg;
  {
    const int64_t row = k0 + lrow;
    const bool ok = row < r1;
    const float* pr = P + (ok ? row : 0) * ld + lcol;
    const float* pr2 = P2 + (ok ? row : 0) * ld2 + lcol;
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = ok ? (s < SPLIT ? pr[16 * s] : pr2[16 * (s - SPLIT)]) : 0.f;
  }
  for (; k0 < r1; k0 += 4 * KG) {
    const int64_t nrow = k0 + 4 * KG + lrow;
    const bool ok = nrow < r1;
    const float* pr = P + (ok ? nrow : 0) * ld + lcol;
    const float* pr2 = P2 + (ok ? nrow : 0) * ld2 + lcol;
#pragma unroll
    for (int s = 0; s < S; ++s) g[s] = ok ? (s < SPLIT ? pr[16 * s] : pr2[16 * (s - SPLIT)]) : 0.f;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = tg * TPW + t;
      const int ti = tile / S, tj = tile % S;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[ti], f[tj], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = g[s];
  }
  float* out = partials + (int64_t)blockIdx.x * W * W;
  // each k group writes its sums to its own LDS region; then all threads add the regions in
  // k-group order (W = 64: 8 x 16 KiB, W = 128: 2 x 64 KiB)
  __shared__ float red[KG][W * W];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = tg * TPW + t;
    const int ti = tile / S, tj = tile % S;
#pragma unroll
    for (int v = 0; v < 4; ++v) red[kg][(16 * ti + 4 * lrow + v) * W + 16 * tj + lcol] = acc[t][v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < W * W; e += kGramThreads) {
    float sum = red[0][e];
#pragma unroll
    for (int g2 = 1; g2 < KG; ++g2) sum += red[g2][e];
    out[e] = sum;
  }
}

// W64[i][j] = sum over blocks of the upper-triangle partial (i <= j), mirrored, so W64 is exactly
// symmetric.  A block owns 16 entries; sixteen thread groups sum interleaved sixteenths of the
// partials (fixed order) and the group sums are added in group order.
__global__ __launch_bounds__(256) void k_gram_reduce(const float* __restrict__ partials, int nb, int W,
                                                     double* __restrict__ Wout) {
  __shared__ double red[16][16];
  const int q = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;
  const int e = blockIdx.x * 16 + q;
  const int WW = W * W;
  double s = 0.0;
  if (e < WW) {
    const int i = e / W, j = e % W;
    const int src = i <= j ? e : j * W + i;
    const float* p = partials + src;
    int b = grp;
    for (; b + 16 < nb; b += 32) {
      const float v0 = p[(int64_t)b * WW], v1 = p[(int64_t)(b + 16) * WW];
      s += (double)v0;
      s += (double)v1;
    }
    for (; b < nb; b += 16) s += (double)p[(int64_t)b * WW];
  }
  red[grp][q] = s;
  __syncthreads();
  if (threadIdx.x < 16 && e < WW) {
    double t = 0.0;
#pragma unroll
    for (int g2 = 0; g2 < 16; ++g2) t += red[g2][q];
    Wout[e] = t;
  }
}

// out[j, 0:L] = [P1[j, 0:L] | P2[j, 0:L]] * T2 (T2: 2L x L).  One wave per row; lane c keeps
// column c of T2 in registers and receives the row through readlane broadcasts.  The row is
// read before it is written, so out may be P1.
template <int L>
__global__ __launch_bounds__(256) void k_panel_xform2(const float* P1, int ld1, const float* P2, int ld2,
                                                      const float* __restrict__ T2, float* out, int ldo,
                                                      int64_t rows) {
  static_assert(L == 32 || L == 64, "panel width");
  constexpr int WIN = 2 * L;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  float t[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) t[k] = lane < L ? T2[k * L + lane] : 0.f;
  for (int64_t r = wave; r < rows; r += nwaves) {
    float a, b = 0.f;
    if constexpr (L == 64) {
      a = P1[r * ld1 + lane];
      b = P2[r * ld2 + lane];
    } else {
      a = lane < L ? P1[r * ld1 + lane] : P2[r * ld2 + (lane - L)];
    }
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 64 && k < WIN; ++k)
      acc = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), k)), t[k], acc);
    if constexpr (L == 64) {
#pragma unroll
      for (int k = 0; k < 64; ++k)
        acc = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(b), k)), t[64 + k], acc);
    }
    if (lane < L) out[r * ldo + lane] = acc;
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
  const int c0 = lane < L ? lane : 0;
  const int c1 = 64 + lane < L ? 64 + lane : 0;
  const float m0 = lane < L ? 1.f : 0.f, m1 = 64 + lane < L ? 1.f : 0.f;
  int64_t r = r0 + wave;
  for (; r + 12 < r1; r += 16) {
    float yv[4], p0[4], p1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      yv[u] = y[r + 4 * u];
      p0[u] = P[(r + 4 * u) * ld + c0];
      p1[u] = P[(r + 4 * u) * ld + c1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 = fmaf(p0[u] * m0, yv[u], a0);
      a1 = fmaf(p1[u] * m1, yv[u], a1);
    }
  }
  for (; r < r1; r += 4) {
    const float yv = y[r];
    a0 = fmaf(P[r * ld + c0] * m0, yv, a0);
    a1 = fmaf(P[r * ld + c1] * m1, yv, a1);
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

static void gram_grid(int64_t rows, int64_t& nb, int& rpb) {
  nb = (rows + 511) / 512;
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  if (nb < 1) nb = 1;
  rpb = (int)((rows + nb - 1) / nb);
  rpb = (rpb + 3) & ~3;
  nb = rows > 0 ? (rows + rpb - 1) / rpb : 1;
}

hipError_t gram(const float* P, int ld, int64_t rows, int w, float* partials, double* W, hipStream_t st) {
  int64_t nb;
  int rpb;
  gram_grid(rows, nb, rpb);
  switch (w) {
    case 32: k_gram_partial<32, false><<<(unsigned)nb, kGramThreads, 0, st>>>(P, ld, P, ld, rows, rpb, partials); break;
    case 64: k_gram_partial<64, false><<<(unsigned)nb, kGramThreads, 0, st>>>(P, ld, P, ld, rows, rpb, partials); break;
    case 128:
      k_gram_partial<128, false><<<(unsigned)nb, kGramThreads, 0, st>>>(P, ld, P, ld, rows, rpb, partials);
      break;
    default: return hipErrorInvalidValue;
  }
  k_gram_reduce<<<(unsigned)((w * w + 15) / 16), 256, 0, st>>>(partials, (int)nb, w, W);
  return hipGetLastError();
}

hipError_t gram2(const float* P1, int ld1, const float* P2, int ld2, int64_t rows, int L, float* partials, double* W,
                 hipStream_t st) {
  int64_t nb;
  int rpb;
  gram_grid(rows, nb, rpb);
  switch (L) {
    case 32: k_gram_partial<64, true><<<(unsigned)nb, kGramThreads, 0, st>>>(P1, ld1, P2, ld2, rows, rpb, partials); break;
    case 64:
      k_gram_partial<128, true><<<(unsigned)nb, kGramThreads, 0, st>>>(P1, ld1, P2, ld2, rows, rpb, partials);
      break;
    default: return hipErrorInvalidValue;
  }
  k_gram_reduce<<<(unsigned)((4 * L * L + 15) / 16), 256, 0, st>>>(partials, (int)nb, 2 * L, W);
  return hipGetLastError();
}

hipError_t panel_xform2(const float* P1, int ld1, const float* P2, int ld2, int L, const float* T2, float* out,
                        int ldo, int64_t rows, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const unsigned grid = grid_for(rows, 4, 8192);
  if (L == 32)
    k_panel_xform2<32><<<grid, 256, 0, st>>>(P1, ld1, P2, ld2, T2, out, ldo, rows);
  else if (L == 64)
    k_panel_xform2<64><<<grid, 256, 0, st>>>(P1, ld1, P2, ld2, T2, out, ldo, rows);
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
