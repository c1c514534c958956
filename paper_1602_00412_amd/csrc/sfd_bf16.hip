// The precision form's panel step on BF16 MFMA: P <- P T for a BF16 panel P (rows x L, row-major,
// L = 32, 64, 128 or 256) and an FP32 upper-triangular T (the inverse Cholesky factor of the panel
// the product read), and the per-block partial Gram of the stored (BF16-rounded) result, in one
// kernel.  This is CholeskyQR (the GramSchmidt step of Alg 1) with the panel in BF16: products of
// BF16 values are exact in FP32, so the Gram is that of the stored panel up to FP32 accumulation,
// and the FP64 Cholesky of it (sfd_small.hip) gives the next transform.
//
// MFMA v_mfma_f32_16x16x32_bf16: A (16 x 32) gives lane l the 8 consecutive k of row l % 16 starting
// at k = 8 (l / 16), B (32 x 16) the same 8 k of column l % 16, and the 16 x 16 FP32 accumulator
// leaves lane l rows 4 (l / 16) .. + 3 of column l % 16.
//  * Transform: a 32-row slab of P is staged in LDS (row pitch L + 8 elements, so the A-operand
//    reads of 16 rows spread over the banks).  Each wave owns one or two 16-column output strips
//    and keeps their column slices of T as B operands in registers.  T is split into two BF16
//    parts, T = T_hi + T_lo with T_lo the BF16 rounding of T - T_hi, and both are applied
//    (two MFMAs), so the transform carries about 16 bits of T rather than BF16's 8: the stored
//    panel then stays orthonormal to that precision, not to BF16's, whatever the conditioning of
//    the panel T was computed for.  T is upper triangular, so strip n needs k-steps
//    ks <= n / 2 only.
//  * The two 16-row halves of a slab leave each lane 8 values of one column (rows 4 (l / 16) + v
//    and 16 + 4 (l / 16) + v): rounded to BF16 they are exactly an A / B operand of the Gram over
//    those 32 rows (both operands use the same assignment of rows to k), so
//    Gram += out^T out needs no data movement beyond publishing each strip's operand in LDS.
//    The upper tiles (si <= sj) of the Gram are dealt to the waves round-robin.
//  * The rounded result goes through LDS to coalesced 16-byte stores, in place.
// Groups (segs != nullptr): buffer k = blockIdx.y owns rows [segs[k].row0, + segs[k].rows) of P with
// T + k L L and partials + k pstride, and the geometry (rpb, nb) of a single-buffer launch.
#include <stdint.h>

#include "sfd_internal.h"

namespace sfd {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_float(uint32_t b) { return __uint_as_float(b << 16); }

__device__ inline floatx4 mfma_bf16(u32x4 a, u32x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

template <int L>
struct Bf16Geom {
  static constexpr int S = L / 16;                    // 16-column strips
  static constexpr int NW = S < 8 ? S : 8;            // waves
  static constexpr int SPW = S / NW;                  // strips per wave (1, or 2 at L = 256)
  static constexpr int NT = 64 * NW;                  // threads
  static constexpr int SPI = 256 / L > 1 ? 256 / L : 1;  // 32-row slabs per iteration
  static constexpr int RPI = 32 * SPI;                // rows per iteration
  static constexpr int LP = L + 8;                    // LDS row pitch (elements)
  static constexpr int KS = L / 32 > 0 ? L / 32 : 1;  // k-steps of the transform
  // (strip, k-step) pairs a wave applies: strip n needs ks <= n / 2 (T upper triangular); with two
  // strips w and S - 1 - w that is S / 2 + 1 pairs for every w
  static constexpr int NKS = SPW == 2 ? S / 2 + 1 : KS;
  static constexpr int NU = S * (S + 1) / 2;          // upper Gram tiles
  static constexpr int TPW = (NU + NW - 1) / NW;      // Gram tiles per wave
  static constexpr int CH = L / 8;                    // 16-byte chunks per row
  static constexpr int NLD = RPI * CH / NT;           // chunks per thread per iteration
  static_assert(NLD * NT == RPI * CH, "whole chunks per thread");
};

// the strips of wave w: w, and S - 1 - w when a wave holds two (balances the triangular work)
template <int L>
__device__ inline int strip_of(int w, int e) {
  return e == 0 ? w : Bf16Geom<L>::S - 1 - w;
}

// pair j of wave w's (strip, k-step) list: with two strips (w needs k-steps 0 .. w / 2, S - 1 - w
// needs 0 .. (S - 1 - w) / 2), the pairs of the two strips alternate while both have k-steps left,
// so consecutive MFMAs go to different accumulators; with one strip, k-step j of strip w
template <int L>
__device__ inline void pair_of(int w, int j, int& e, int& ks) {
  if constexpr (Bf16Geom<L>::SPW == 2) {
    const int n0 = w / 2 + 1, n1 = Bf16Geom<L>::NKS - n0;
    const int m = n0 < n1 ? n0 : n1;
    if (j < 2 * m) {
      e = j & 1;
      ks = j >> 1;
    } else {
      e = n0 > n1 ? 0 : 1;
      ks = m + (j - 2 * m);
    }
  } else {
    e = 0;
    ks = j;
  }
}

// upper tile u of the S x S tile grid in row-major order -> (si, sj)
template <int S>
__device__ inline void upper_tile(int u, int& si, int& sj) {
  int i = 0;
  while (u >= S - i) {
    u -= S - i;
    ++i;
  }
  si = i;
  sj = i + u;
}

template <int L, bool SPLIT>
__global__ __launch_bounds__(Bf16Geom<L>::NT) void k_xform_gram_bf16(uint16_t* __restrict__ P, int ld, int64_t rows,
                                                                     int rpb, const float* __restrict__ T,
                                                                     float* __restrict__ partials,
                                                                     const GroupSeg* segs, int64_t pstride) {
  using G = Bf16Geom<L>;
  constexpr int S = G::S, NW = G::NW, SPW = G::SPW, NT = G::NT, SPI = G::SPI, RPI = G::RPI, LP = G::LP;
  constexpr int NKS = G::NKS, TPW = G::TPW, CH = G::CH, NLD = G::NLD, NU = G::NU;
  if (segs) {
    const GroupSeg g = segs[blockIdx.y];
    if ((int)blockIdx.x >= g.nb) return;
    P += (size_t)g.row0 * ld;
    rows = g.rows;
    rpb = g.rpb;
    T += (int64_t)blockIdx.y * L * L;
    partials += (int64_t)blockIdx.y * pstride;
  }
  __shared__ __align__(16) uint16_t sin_[RPI * LP];
  __shared__ __align__(16) uint16_t sout[RPI * LP];
  __shared__ u32x4 sop[SPI][S][64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  const int lm = lane & 15, lk = lane >> 4;
  // B operands: column slices of T (rows 32 ks + 8 lk .. + 7 of column 16 n + lm) for this wave's
  // (strip, k-step) pairs, split into BF16 parts
  u32x4 th[NKS], tl[NKS];
#pragma unroll
  for (int j = 0; j < NKS; ++j) {
    int e, ks;
    pair_of<L>(w, j, e, ks);
    const int n = strip_of<L>(w, e);
    uint32_t hb[8], lb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = 32 * ks + 8 * lk + i;
      const float t = r < L ? T[r * L + 16 * n + lm] : 0.f;
      hb[i] = bf16_bits(t);
      lb[i] = bf16_bits(t - bf16_float(hb[i]));
    }
    th[j] = u32x4{hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16), hb[4] | (hb[5] << 16), hb[6] | (hb[7] << 16)};
    tl[j] = u32x4{lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16), lb[4] | (lb[5] << 16), lb[6] | (lb[7] << 16)};
  }
  floatx4 g[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) g[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  const size_t pitch = (size_t)ld;
  u32x4 nxt[NLD];
  uint32_t ob[SPI][SPW][2][4];  // rounded results of the current iteration (Gram operands)
  auto load = [&](int64_t it0) {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      const int64_t row = it0 + c / CH;
      nxt[j] = row < r1 ? *reinterpret_cast<const u32x4*>(P + row * pitch + 8 * (c % CH)) : u32x4{0u, 0u, 0u, 0u};
    }
  };
  load(r0);
  for (int64_t it0 = r0; it0 < r1; it0 += RPI) {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      *reinterpret_cast<u32x4*>(sin_ + (c / CH) * LP + 8 * (c % CH)) = nxt[j];
    }
    __syncthreads();
    load(it0 + RPI);
#pragma unroll
    for (int s = 0; s < SPI; ++s) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // the T_hi and T_lo products go to separate accumulators (independent MFMA chains),
        // added once the k-steps are done
        floatx4 acc[SPW], accl[SPW];
#pragma unroll
        for (int e = 0; e < SPW; ++e) acc[e] = accl[e] = floatx4{0.f, 0.f, 0.f, 0.f};
        const uint16_t* arow = sin_ + (32 * s + 16 * h + lm) * LP + 8 * lk;
#pragma unroll
        for (int j = 0; j < NKS; ++j) {
          int e, ks;
          pair_of<L>(w, j, e, ks);
          if (ks > strip_of<L>(w, e) / 2) continue;  // T is upper triangular
          const u32x4 a = *reinterpret_cast<const u32x4*>(arow + 32 * ks);
#pragma unroll
          for (int ee = 0; ee < SPW; ++ee) {
            if (ee != e) continue;
            acc[ee] = mfma_bf16(a, th[j], acc[ee]);
            if constexpr (SPLIT) accl[ee] = mfma_bf16(a, tl[j], accl[ee]);
          }
        }
        if constexpr (SPLIT) {
#pragma unroll
          for (int e = 0; e < SPW; ++e) acc[e] += accl[e];
        }
#pragma unroll
        for (int e = 0; e < SPW; ++e) {
          const int n = strip_of<L>(w, e);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 32 * s + 16 * h + 4 * lk + v;
            const uint32_t b = it0 + lr < r1 ? bf16_bits(acc[e][v]) : 0u;
            ob[s][e][h][v] = b;
            sout[lr * LP + 16 * n + lm] = (uint16_t)b;
          }
        }
      }
#pragma unroll
      for (int e = 0; e < SPW; ++e) {
        const uint32_t(&o)[2][4] = ob[s][e];
        sop[s][strip_of<L>(w, e)][lane] =
            u32x4{o[0][0] | (o[0][1] << 16), o[0][2] | (o[0][3] << 16), o[1][0] | (o[1][1] << 16),
                  o[1][2] | (o[1][3] << 16)};
      }
    }
    __syncthreads();
    // the rounded result, coalesced, in place
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      const int64_t row = it0 + c / CH;
      if (row < r1)
        *reinterpret_cast<u32x4*>(P + row * pitch + 8 * (c % CH)) =
            *reinterpret_cast<const u32x4*>(sout + (c / CH) * LP + 8 * (c % CH));
    }
    // Gram of the stored rows: this wave's upper tiles
#pragma unroll
    for (int s = 0; s < SPI; ++s) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int u = w + NW * t;
        if (u < NU) {
          int si, sj;
          upper_tile<S>(u, si, sj);
          g[t] = mfma_bf16(sop[s][si][lane], sop[s][sj][lane], g[t]);
        }
      }
    }
  }
  float* out = partials + (int64_t)blockIdx.x * L * L;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int u = w + NW * t;
    if (u < NU) {
      int si, sj;
      upper_tile<S>(u, si, sj);
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * si + 4 * lk + v) * L + 16 * sj + lm] = g[t][v];
    }
  }
}

template <int L>
void launch_xform_gram_bf16(uint16_t* P, int ld, int64_t rows, int rpb, int nb, const GroupSeg* segs, int K,
                            const float* T, float* partials, int64_t pstride, bool split, hipStream_t st) {
  const dim3 grid((unsigned)nb, (unsigned)K);
  if (split)
    k_xform_gram_bf16<L, true><<<grid, Bf16Geom<L>::NT, 0, st>>>(P, ld, rows, rpb, T, partials, segs, pstride);
  else
    k_xform_gram_bf16<L, false><<<grid, Bf16Geom<L>::NT, 0, st>>>(P, ld, rows, rpb, T, partials, segs, pstride);
}

}  // namespace

hipError_t xform_gram_bf16_partials(uint16_t* P, int ld, int64_t rows, int rpb, int nb, const GroupSeg* segs, int K,
                                    int L, const float* T, float* partials, int64_t pstride, bool split,
                                    hipStream_t st) {
  switch (L) {
    case 32: launch_xform_gram_bf16<32>(P, ld, rows, rpb, nb, segs, K, T, partials, pstride, split, st); break;
    case 64: launch_xform_gram_bf16<64>(P, ld, rows, rpb, nb, segs, K, T, partials, pstride, split, st); break;
    case 128: launch_xform_gram_bf16<128>(P, ld, rows, rpb, nb, segs, K, T, partials, pstride, split, st); break;
    case 256: launch_xform_gram_bf16<256>(P, ld, rows, rpb, nb, segs, K, T, partials, pstride, split, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sfd
