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
//
// A block has eight waves and takes 32 G rows per iteration: G groups of S / 2 waves (S = L / 16
// column strips), each group one 32-row slab.  Wave p of a group owns the strips a = p and
// b = S - 1 - p, which balances the triangular work, and every wave runs the same instruction
// stream: no branch depends on the wave, so loads, MFMAs and waits schedule statically.
//  * Transform: the iteration's rows are staged in LDS (row pitch L + 8 elements, so the A-operand
//    reads of 16 rows spread over the banks).  T is split into two BF16 parts, T = T_hi + T_lo
//    with T_lo the BF16 rounding of T - T_hi, and both are applied (two MFMAs into separate
//    accumulators), so the transform carries about 16 bits of T rather than BF16's 8: the stored
//    panel stays orthonormal to that precision whatever the conditioning of the panel T was
//    computed for.  Strip n needs the k-steps ks <= n / 2 (T is upper triangular): strip a at
//    most the first half of them, strip b all of them.  Both strips take the first half and strip
//    b the second, with the column slices of T held in registers as B operands and the entries of
//    T below its diagonal read as zero, so the k-steps a strip does not need add exact zeros.
//  * The two 16-row halves of a slab leave each lane 8 values of one column (rows 4 (l / 16) + v
//    and 16 + 4 (l / 16) + v): rounded to BF16 they are exactly an A / B operand of the Gram over
//    those 32 rows (both operands use the same assignment of rows to k), so Gram += out^T out
//    needs no data movement beyond publishing each strip's operand in LDS.  Wave p forms the
//    upper tiles of its own columns, (si, b) for si <= b and (si, a) for si <= a: S + 1 tiles,
//    the B operand from its registers and the A operand from LDS.
//  * The rounded result goes through LDS to coalesced 16-byte stores, in place.  The block's rows
//    are addressed through a buffer resource that covers exactly them: rows past the end load as
//    zeros and their stores are dropped, with no branches around the memory operations.
//  * With G > 1 the groups' Gram sums are added in group order in LDS at the end.
// Groups (segs != nullptr): buffer k = blockIdx.y owns rows [segs[k].row0, + segs[k].rows) of P with
// T + k L L and partials + k pstride, and the geometry (rpb, nb) of a single-buffer launch.
#include <stdint.h>

#include "sfd_internal.h"

namespace sfd {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// word 3 of a raw buffer resource on gfx9-family GPUs (offsets in bytes, checked against the
// record count: loads past it return 0, stores past it are dropped)
constexpr int kRsrcWord3 = 0x00020000;

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
  static constexpr int S = L / 16;           // 16-column strips
  static constexpr int NW = S / 2;           // waves per slab (two strips each)
  static constexpr int G = 8 / NW;           // slabs per iteration
  static constexpr int NT = 512;             // threads
  static constexpr int RPI = 32 * G;         // rows per iteration
  static constexpr int LP = L + 8;           // LDS row pitch (elements)
  static constexpr int KS = L / 32;          // 32-deep k-steps of the transform
  static constexpr int P1 = (KS + 1) / 2;    // k-steps both strips take
  static constexpr int NJ = S + 1;           // Gram tiles per wave
  static constexpr int CH = L / 8;           // 16-byte chunks per row
  static constexpr int NLD = RPI * CH / NT;  // chunks per thread per iteration
  static_assert(NW * G == 8, "eight waves");
  static_assert(NLD * NT == RPI * CH, "whole chunks per thread");
  static_assert((KS - 1) / 2 < P1 || S == 2, "strip a fits the first k-steps");
};

// B operand of strip n, k-step ks for lane (lk, lm): T[32 ks + 8 lk + i][16 n + lm], i = 0..7, as
// its BF16 part hi and the BF16 rounding of the rest lo (entries below the diagonal are zero)
template <int L>
__device__ inline void t_operand(const float* __restrict__ T, int n, int ks, int lk, int lm, u32x4& hi, u32x4& lo) {
  uint32_t hb[8], lb[8];
  const int c = 16 * n + lm;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int r = 32 * ks + 8 * lk + i;
    const float t = r <= c ? T[r * L + c] : 0.f;
    hb[i] = bf16_bits(t);
    lb[i] = bf16_bits(t - bf16_float(hb[i]));
  }
  hi = u32x4{hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16), hb[4] | (hb[5] << 16), hb[6] | (hb[7] << 16)};
  lo = u32x4{lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16), lb[4] | (lb[5] << 16), lb[6] | (lb[7] << 16)};
}

template <int L, bool SPLIT>
__global__ __launch_bounds__(512) void k_xform_gram_bf16(uint16_t* __restrict__ P, int ld, int64_t rows, int rpb,
                                                         const float* __restrict__ T, float* __restrict__ partials,
                                                         const GroupSeg* segs, int64_t pstride) {
  using Gm = Bf16Geom<L>;
  constexpr int S = Gm::S, NW = Gm::NW, G = Gm::G, NT = Gm::NT, RPI = Gm::RPI, LP = Gm::LP, KS = Gm::KS;
  constexpr int P1 = Gm::P1, NJ = Gm::NJ, CH = Gm::CH, NLD = Gm::NLD;
  if (segs) {
    const GroupSeg g = segs[blockIdx.y];
    if ((int)blockIdx.x >= g.nb) return;
    P += (size_t)g.row0 * ld;
    rows = g.rows;
    rpb = g.rpb;
    T += (int64_t)blockIdx.y * L * L;
    partials += (int64_t)blockIdx.y * pstride;
  }
  // LDS: input rows and rounded output rows (RPI x LP each), the published Gram operands
  // [G][S][64]; after the loop, the groups' Gram sums [NW][NJ][64] (G > 1)
  constexpr int kRows = RPI * LP;
  constexpr int kStage = 4 * kRows + G * S * 64 * 16;
  constexpr int kRed = G > 1 ? NW * NJ * 64 * 16 : 0;
  __shared__ __align__(16) unsigned char lds[kStage > kRed ? kStage : kRed];
  uint16_t* const sin_ = reinterpret_cast<uint16_t*>(lds);
  uint16_t* const sout = sin_ + kRows;
  u32x4* const sop = reinterpret_cast<u32x4*>(lds + 4 * kRows);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  const int grp = w / NW, p = w % NW;
  const int sa = p, sb = S - 1 - p;
  const int lm = lane & 15, lk = lane >> 4;
  u32x4 tah[P1], tal[P1], tbh[KS], tbl[KS];
#pragma unroll
  for (int ks = 0; ks < P1; ++ks) t_operand<L>(T, sa, ks, lk, lm, tah[ks], tal[ks]);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) t_operand<L>(T, sb, ks, lk, lm, tbh[ks], tbl[ks]);
  floatx4 g[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) g[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int nr = (int)max((int64_t)0, min(rows, r0 + rpb) - r0);  // this block's rows
  const int pitch = ld * 2;                                        // bytes
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(P + (size_t)r0 * ld, (short)0, nr * pitch, kRsrcWord3);
  u32x4 nxt[NLD];
  auto load = [&](int it) {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      nxt[j] = __builtin_bit_cast(u32x4,
                                  __builtin_amdgcn_raw_buffer_load_b128(rs, (it + c / CH) * pitch + 16 * (c % CH), 0, 0));
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      *reinterpret_cast<u32x4*>(sin_ + (c / CH) * LP + 8 * (c % CH)) = nxt[j];
    }
  };
  const u32x4* const sopg = sop + grp * S * 64;
  load(0);
  stage();
  for (int it = 0; it < nr; it += RPI) {
    __syncthreads();
    // the next iteration's rows load while this one is transformed; they are staged at the end
    // of the pass, where the wait for them does not also cover the stores issued in between
    load(it + RPI);
    // out = slab * T for strips a and b, one 16-row half at a time
    uint32_t pa[4], pb[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      floatx4 ah = {0.f, 0.f, 0.f, 0.f}, al = ah, bh = ah, bl = ah;
      const uint16_t* arow = sin_ + (32 * grp + 16 * h + lm) * LP + 8 * lk;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(arow + 32 * ks);
        if (ks < P1) {
          ah = mfma_bf16(a, tah[ks], ah);
          if constexpr (SPLIT) al = mfma_bf16(a, tal[ks], al);
        }
        bh = mfma_bf16(a, tbh[ks], bh);
        if constexpr (SPLIT) bl = mfma_bf16(a, tbl[ks], bl);
      }
      if constexpr (SPLIT) {
        ah += al;
        bh += bl;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = 32 * grp + 16 * h + 4 * lk + v;  // row in the iteration
        const uint32_t keep = it + lr < nr ? 0xFFFFu : 0u;   // rows past the end add nothing
        const uint32_t ba = bf16_bits(ah[v]) & keep;
        const uint32_t bb = bf16_bits(bh[v]) & keep;
        sout[lr * LP + 16 * sa + lm] = (uint16_t)ba;
        sout[lr * LP + 16 * sb + lm] = (uint16_t)bb;
        if (v & 1) {
          pa[2 * h + (v >> 1)] |= ba << 16;
          pb[2 * h + (v >> 1)] |= bb << 16;
        } else {
          pa[2 * h + (v >> 1)] = ba;
          pb[2 * h + (v >> 1)] = bb;
        }
      }
    }
    const u32x4 opa = u32x4{pa[0], pa[1], pa[2], pa[3]};
    const u32x4 opb = u32x4{pb[0], pb[1], pb[2], pb[3]};
    sop[(grp * S + sa) * 64 + lane] = opa;
    sop[(grp * S + sb) * 64 + lane] = opb;
    __syncthreads();
    // the rounded rows, coalesced, in place (rows past the block's end are dropped)
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int c = j * NT + tid;
      __builtin_amdgcn_raw_buffer_store_b128(*reinterpret_cast<const u32x4*>(sout + (c / CH) * LP + 8 * (c % CH)), rs,
                                             (it + c / CH) * pitch + 16 * (c % CH), 0, 0);
    }
    // Gram tiles of this wave's columns: j < S - p: (j, b); otherwise (j - (S - p), a)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const bool colb = j <= S / 2 || j < S - p;
      const int si = colb ? j : j - (S - p);
      g[j] = mfma_bf16(sopg[si * 64 + lane], colb ? opb : opa, g[j]);
    }
    // the transform's reads of sin_ ended before the barrier above
    stage();
  }
  float* out = partials + (int64_t)blockIdx.x * L * L;
  auto write_tiles = [&](const floatx4* t) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const bool colb = j <= S / 2 || j < S - p;
      const int si = colb ? j : j - (S - p);
      const int sj = colb ? sb : sa;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * si + 4 * lk + v) * L + 16 * sj + lm] = t[j][v];
    }
  };
  if constexpr (G == 1) {
    write_tiles(g);
  } else {
    floatx4* const red = reinterpret_cast<floatx4*>(lds);  // [NW][NJ][64]
    __syncthreads();                                        // the last iteration's LDS reads are done
    for (int gg = 0; gg < G; ++gg) {
      if (grp == gg) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          floatx4& r = red[(p * NJ + j) * 64 + lane];
          r = gg == 0 ? g[j] : r + g[j];
        }
      }
      __syncthreads();
    }
    if (grp == 0) {
      floatx4 t[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) t[j] = red[(p * NJ + j) * 64 + lane];
      write_tiles(t);
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
