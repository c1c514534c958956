// Dense panel kernels: the Gram matrices of the tall panels on MFMA (GramSchmidt of Alg 1 as
// CholeskyQR, svd(P, ell) of Alg 3 and svd([B; B'], ell) of Alg 5 through W^T W), row
// transforms panel * T, the panel-transpose matrix-vector product of VerifySpectral, and the
// counter-based start block G of Alg 1.
//
// Panels are row-major and tall (d x L or m x L, L = 32, 64, 128 or 256 >= ell, zero-padded), so
// every Gram has its contraction along the tall axis.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "sfd_internal.h"

namespace sfd {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kGramMaxBlocks = 256;

// word 3 of a raw buffer resource on gfx9-family GPUs (stride 0: offsets are bytes, checked
// against the record count; loads past it return 0 and stores past it are dropped)
constexpr int kBufferRsrcWord3 = 0x00020000;
// (the raw buffer builtins move 32-bit integers: floats go through __float_as_uint, never a value
// conversion)

// Gram partial of a row block.  MFMA v_mfma_f32_16x16x4f32: A (16 x 4) and B (4 x 16) come one
// float per lane, lane l holding row-of-A / column-of-B (l % 16) at k = l / 16; the 16 x 16
// accumulator leaves 4 floats per lane, lane l holding column l % 16, rows 4*(l/16) .. +3.
// For W = P^T P both operands are the same 4-row slab of the panel: lane l loads
// P[k0 + l/16][16*s + l%16] for each 16-column strip s.  Only the tiles on and above the
// diagonal are formed (the reduction mirrors them).  Eight waves per block split the rows; each
// wave keeps kGramDepth slabs in flight: a slab's MFMAs
// run while the loads of the slabs after it are outstanding.
constexpr int kGramThreads = 512;
constexpr int kGramWaves = kGramThreads / 64;
constexpr int kGramDepth = 4;

// the tiles of the upper triangle of an S x S tile grid in row-major order: (ti[u], tj[u]), ti <= tj
template <int S>
struct UpperTiles {
  int ti[S * (S + 1) / 2];
  int tj[S * (S + 1) / 2];
  constexpr UpperTiles() : ti(), tj() {
    int u = 0;
    for (int i = 0; i < S; ++i)
      for (int j = i; j < S; ++j) {
        ti[u] = i;
        tj[u] = j;
        ++u;
      }
  }
};
template <int S>
constexpr UpperTiles<S> kUpper{};

// TWO: the panel is [P | P2] side by side, each W/2 wide (strips of the right half from P2).
template <int W, bool TWO>
__global__ __launch_bounds__(kGramThreads) void k_gram_partial(const float* __restrict__ P, int ld,
                                                               const float* __restrict__ P2, int ld2, int64_t rows,
                                                               int rpb, float* __restrict__ partials) {
  constexpr int S = W / 16;            // strips
  constexpr int NU = S * (S + 1) / 2;  // tiles on and above the diagonal, all formed by every wave
  constexpr int KG = kGramWaves;       // k groups (waves split rows)
  constexpr int TPW = NU;
  constexpr int D = kGramDepth;
  const int lane = threadIdx.x & 63;
  const int kg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  floatx4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int lrow = lane >> 4;
  const int lcol = lane & 15;
  constexpr int SPLIT = TWO ? S / 2 : S;  // strips read from P; the rest from P2
  const int64_t step = 4 * KG;
  float f[D][S];
#define SFD_GRAM_LOAD(dd, k)                                                                        \
  do {                                                                                              \
    const int64_t row_ = (k) + lrow;                                                                \
    const bool ok_ = row_ < r1;                                                                     \
    const float* pr_ = P + (ok_ ? row_ : 0) * ld;                                                    \
    const float* pr2_ = P2 + (ok_ ? row_ : 0) * ld2 + lcol;                                         \
    _Pragma("unroll") for (int s = 0; s < S; ++s) f[dd][s] =                                        \
        ok_ ? (s < SPLIT ? pr_[16 * s + lcol] : pr2_[16 * (s - SPLIT)]) : 0.f;                      \
  } while (0)
  int64_t k0 = r0 + 4 * kg;
#pragma unroll
  for (int dd = 0; dd < D; ++dd) SFD_GRAM_LOAD(dd, k0 + dd * step);
  for (; k0 < r1; k0 += D * step) {
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
#pragma unroll
      for (int t = 0; t < TPW; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[dd][kUpper<S>.ti[t]], f[dd][kUpper<S>.tj[t]], acc[t], 0, 0,
                                                      0);
      SFD_GRAM_LOAD(dd, k0 + (dd + D) * step);
    }
  }
#undef SFD_GRAM_LOAD
  // the k groups add their sums into one LDS copy in k-group order, then the block writes it
  __shared__ float red[W * W];
  for (int g2 = 0; g2 < KG; ++g2) {
    if (kg == g2) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = (16 * kUpper<S>.ti[t] + 4 * lrow + v) * W + 16 * kUpper<S>.tj[t] + lcol;
          red[e] = g2 == 0 ? acc[t][v] : red[e] + acc[t][v];
        }
      }
    }
    __syncthreads();
  }
  float* out = partials + (int64_t)blockIdx.x * W * W;
  for (int e = threadIdx.x; e < W * W; e += kGramThreads) {
    const int i = e / W, j = e % W;
    if (i / 16 <= j / 16) out[e] = red[e];
  }
}

// P <- P T in place (rows x L FP32 panel, pitch ld; T: L x L FP32) and the per-block partial
// Gram of the result, for k_gram_reduce (BF16 panels: sfd_bf16.hip).  This applies the inverse
// Cholesky factor of a product's input panel to the product's output (A'(X T) = (A' X) T), so the
// sparse products need no per-row epilogue.  Both the transform and the Gram run on MFMA
// (v_mfma_f32_16x16x4f32), 16 rows at a time per wave (wave w of a block: tiles w, w + 8, ...):
//  * the block's rows are addressed through a buffer resource that covers exactly them, so a
//    tile's rows past the block's end load as zeros and their stores are dropped by the hardware:
//    no branches around the memory operations, and the loop's wait for the next tile's loads does
//    not also wait for the current tile's stores;
//  * the tile is loaded coalesced and staged in LDS (row pitch L + 4 floats: the A-operand reads
//    below hit 64 distinct banks);
//  * out (16 x L) = tile (16 x L) * T: k-step ks, strip n: A[m][k] = tile[m][4 ks + k] (lane l:
//    m = l % 16, k = l / 16), B[k][n'] = T[4 ks + k][16 n + n'] (held in registers), C lane l:
//    out[4 (l / 16) + v][16 n + l % 16]; T is upper triangular (an inverse Cholesky factor), so
//    strip n needs the k-steps ks < 4 (n + 1) only;
//  * the accumulator of strip n at fixed v is itself an A / B operand over the four rows
//    4 k + v (k = l / 16), so Gram += out^T out is formed from the registers directly: for
//    v = 0..3 and each upper tile (si, sj), MFMA(C_si[v], C_sj[v]).  Rows past the end are zero
//    and add nothing.
// Groups (segs != nullptr): buffer k = blockIdx.y owns rows [segs[k].row0, + segs[k].rows) of P
// with its own T (T + k L L) and partials (partials + k pstride), and the block geometry a
// single-buffer launch over that many rows has (segs[k].rpb, .nb), so its result is the same.
template <int L>
__global__ __launch_bounds__(kGramThreads) void k_xform_gram(float* __restrict__ P, int ld, int64_t rows, int rpb,
                                                             const float* __restrict__ T,
                                                             float* __restrict__ partials, const GroupSeg* segs,
                                                             int64_t pstride) {
  if (segs) {
    const GroupSeg g = segs[blockIdx.y];
    if ((int)blockIdx.x >= g.nb) return;
    P += (size_t)g.row0 * ld;
    rows = g.rows;
    rpb = g.rpb;
    T += (int64_t)blockIdx.y * L * L;
    partials += (int64_t)blockIdx.y * pstride;
  }
  static_assert(L == 32 || L == 64, "panel width");
  constexpr int S = L / 16;            // column strips
  constexpr int KS = L / 4;            // k-steps of the transform
  constexpr int NU = S * (S + 1) / 2;  // upper tiles of the Gram
  constexpr int NW = kGramWaves;
  constexpr int LP = L + 4;            // LDS row pitch (floats)
  constexpr int EPL = 4;               // elements per lane per load (16 bytes)
  constexpr int LPRW = L / EPL;        // lanes per row in a load pass
  constexpr int RPP = 64 / LPRW;       // rows per load pass
  constexpr int NP = 16 / RPP;         // load passes per 16-row tile
  __shared__ float tile[NW][16 * LP];
  __shared__ float red[L * L];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  float tb[KS][S];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int n = 0; n < S; ++n) tb[ks][n] = T[(4 * ks + lk) * L + 16 * n + lm];
  // T is in registers before the tile loop, whose waits then cover only the loop's own loads
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int n = 0; n < S; ++n) asm volatile("" : "+v"(tb[ks][n]));
  floatx4 g[NU];
#pragma unroll
  for (int t = 0; t < NU; ++t) g[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int nr = (int)max((int64_t)0, min(rows, r0 + rpb) - r0);  // this block's rows
  const int pitch = ld * 4;
  // rows [r0, r0 + nr) as one buffer: offsets past nr * pitch bytes read 0 and are not written
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(P + (size_t)r0 * ld, (short)0, nr * pitch, kBufferRsrcWord3);
  const int prow = lane / LPRW, pcol = (lane % LPRW) * EPL;  // this lane's part of a load pass
  float* my = tile[wave];
  floatx4 nxt[NP];
  auto load_tile = [&](int t0) {
#pragma unroll
    for (int ip = 0; ip < NP; ++ip)
      nxt[ip] = __builtin_bit_cast(
          floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, (t0 + ip * RPP + prow) * pitch + pcol * 4, 0, 0));
  };
  auto stage = [&]() {
#pragma unroll
    for (int ip = 0; ip < NP; ++ip) *reinterpret_cast<floatx4*>(my + (ip * RPP + prow) * LP + pcol) = nxt[ip];
  };
  int t0 = 16 * wave;
  load_tile(t0);
  stage();
  for (; t0 < nr; t0 += 16 * NW) {
    // start loading the next tile; it is staged at the end of this pass, where the wait for
    // its loads does not cover the stores issued in between
    load_tile(t0 + 16 * NW);
    __builtin_amdgcn_wave_barrier();
    // out = tile * T
    floatx4 o[S];
#pragma unroll
    for (int n = 0; n < S; ++n) o[n] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float a = my[lm * LP + 4 * ks + lk];
      // T is upper triangular: rows 4 ks .. 4 ks + 3 of strip n are zero once ks >= 4 (n + 1)
#pragma unroll
      for (int n = 0; n < S; ++n)
        if (ks < 4 * (n + 1)) o[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, tb[ks][n], o[n], 0, 0, 0);
    }
    // store (rows past the block's end are dropped), and add the Gram of the tile
#pragma unroll
    for (int n = 0; n < S; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[n][v]), rs, (t0 + 4 * lk + v) * pitch + (16 * n + lm) * 4, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int t = 0; t < NU; ++t)
        g[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(o[kUpper<S>.ti[t]][v], o[kUpper<S>.tj[t]][v], g[t], 0, 0, 0);
    __builtin_amdgcn_wave_barrier();
    stage();
  }
  // the waves add their sums into one LDS copy in wave order, then the block writes it
  for (int g2 = 0; g2 < NW; ++g2) {
    if (wave == g2) {
#pragma unroll
      for (int t = 0; t < NU; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = (16 * kUpper<S>.ti[t] + 4 * lk + q) * L + 16 * kUpper<S>.tj[t] + lm;
          red[e] = g2 == 0 ? g[t][q] : red[e] + g[t][q];
        }
      }
    }
    __syncthreads();
  }
  float* out = partials + (int64_t)blockIdx.x * L * L;
  for (int e = threadIdx.x; e < L * L; e += kGramThreads) {
    const int i = e / L, j = e % L;
    if (i / 16 <= j / 16) out[e] = red[e];
  }
}

// Wide FP32 panels (L = 128 or 256): out <- Pin T (rows x L, T: L x L FP32, pitch ldt), and with
// ACC out <- out + Pin T (used for [P1 | P2] T2 as two passes).  The blocks stride over the
// 16-row tiles (block b takes tiles b, b + gridDim.x, ...), so a block loads its part of T once.
// Wave w computes output strip sw = strip_of_wave(w) (columns 16 sw .. 16 sw + 15) and keeps that
// strip of T as MFMA B operands in registers (lane l: T[4 ks + l / 16][16 sw + l % 16]); the
// 16-row input tile is loaded by the whole block (16 bytes per thread), staged in LDS as FP32
// (pitch L + 4, two buffers, so one barrier per tile), and read as A operands by every wave.  A
// tile is read completely before any of it is written, so out may be Pin.  UPPER: T is upper
// triangular (an inverse Cholesky factor), so strip sw needs the k-steps ks < 4 (sw + 1) only.
// Each wave runs two MFMA chains (even and odd k-steps) and adds them at the end.  The memory
// operations go through a buffer resource covering the tile's rows, so a tile's rows past the end
// load as zeros and are not written, with no branches.
// Groups: buffer k = blockIdx.z owns rows [segs[k].row0, + segs[k].rows) with T + k L L.
template <int L>
__device__ __forceinline__ int strip_of_wave(int w) {
  // waves w, w + 4, w + 8, ... run on one SIMD; strips {s, 7 - s, 8 + s, 15 - s, ...} give every
  // SIMD the same number of k-steps when T is triangular
  const int s = w & 3, j = w >> 2;
  return (j & 1) ? 4 * (j + 1) - 1 - s : 4 * j + s;
}

template <int L, bool ACC, bool UPPER>
__global__ __launch_bounds__(L * 4) void k_xform_strips(const float* Pin, int ldi, float* out, int ldo, int64_t rows,
                                                        const float* __restrict__ T, int ldt,
                                                        const GroupSeg* segs) {
  static_assert(L == 128 || L == 256, "strip-per-wave transform");
  constexpr int KS = L / 4;
  constexpr int LP = L + 4;
  if (segs) {
    const GroupSeg g = segs[blockIdx.z];
    Pin += (size_t)g.row0 * ldi;
    out += (size_t)g.row0 * ldo;
    rows = g.rows;
    T += (int64_t)blockIdx.z * L * L;
  }
  const int64_t ntiles = (rows + 15) / 16;
  if ((int64_t)blockIdx.x >= ntiles) return;
  __shared__ float tile[2][16 * LP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  const int lm = lane & 15, lk = lane >> 4;
  const int sw = strip_of_wave<L>(w);
  const int kmax = UPPER ? 4 * (sw + 1) : KS;
  float tb[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) tb[ks] = ks < kmax ? T[(4 * ks + lk) * ldt + 16 * sw + lm] : 0.f;
  // T is in registers before the tile loop, whose waits then cover only the loop's own loads
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) asm volatile("" : "+v"(tb[ks]));
  const int ipitch = ldi * 4, opitch = ldo * 4;
  // this thread's 4 elements of a tile: row tid / (L / 4), columns 4 (tid % (L / 4)) .. + 3
  const int trow = tid / (L / 4), tcol = 4 * (tid % (L / 4));
  auto rows_of = [&](int64_t t) -> int { return (int)max((int64_t)0, min((int64_t)16, rows - 16 * t)); };
  auto load = [&](int64_t t) -> floatx4 {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(Pin) + (size_t)min(t, ntiles) * 16 * ldi, (short)0, rows_of(t) * ipitch, kBufferRsrcWord3);
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, trow * ipitch + tcol * 4, 0, 0));
  };
  int64_t t = blockIdx.x;
  floatx4 nxt = load(t);
  int buf = 0;
  *reinterpret_cast<floatx4*>(tile[0] + trow * LP + tcol) = nxt;
  for (; t < ntiles; t += gridDim.x, buf ^= 1) {
    __syncthreads();  // tile[buf] staged; every wave is done with tile[buf ^ 1]
    nxt = load(t + gridDim.x);
    const __amdgpu_buffer_rsrc_t ro =
        __builtin_amdgcn_make_buffer_rsrc(out + (size_t)t * 16 * ldo, (short)0, rows_of(t) * opitch, kBufferRsrcWord3);
    floatx4 o0 = floatx4{0.f, 0.f, 0.f, 0.f}, o1 = o0;
    if constexpr (ACC) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        o0[v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                              ro, (4 * lk + v) * opitch + (16 * sw + lm) * 4, 0, 0));
    }
    // k-steps in groups of four (kmax is a multiple of 4); the A operands of the next group are
    // read from LDS before the current group's MFMAs are issued
    const float* tl = tile[buf] + lm * LP + lk;
    float a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = tl[4 * j];
#pragma unroll
    for (int kg = 0; kg < KS / 4; ++kg) {
      if (4 * kg < kmax) {
        float an[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) an[j] = kg + 1 < KS / 4 ? tl[16 * (kg + 1) + 4 * j] : 0.f;
        o0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], tb[4 * kg], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], tb[4 * kg + 1], o1, 0, 0, 0);
        o0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], tb[4 * kg + 2], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], tb[4 * kg + 3], o1, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = an[j];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o0[v] + o1[v]), ro, (4 * lk + v) * opitch + (16 * sw + lm) * 4, 0, 0);
    // the next tile into the other buffer (its last readers were before this pass's barrier)
    *reinterpret_cast<floatx4*>(tile[buf ^ 1] + trow * LP + tcol) = nxt;
  }
}

// Gram partials of wide panels by 64 x 64 output tiles: block (x, y, z) forms tile pair
// y = (I, J), I <= J, of the W x W Gram of the panel [P | P2] (64-column slices; slices below
// SPLIT = W1 / 64 come from P, the rest from P2) over row block x, for buffer z of a group.
// Four waves split the rows in 4-row slabs (MFMA operands as in k_gram_partial); their sums are
// added in wave order and the tile is written at its place in the block's W x W partial.
__global__ __launch_bounds__(256) void k_gram_tiles(const float* __restrict__ P, int ld, const float* __restrict__ P2,
                                                    int ld2, int W1, int W, int64_t rows, int rpb,
                                                    float* __restrict__ partials, const GroupSeg* segs,
                                                    int64_t pstride) {
  if (segs) {
    const GroupSeg g = segs[blockIdx.z];
    if ((int)blockIdx.x >= g.nb) return;
    P += (size_t)g.row0 * ld;
    rows = g.rows;
    rpb = g.rpb;
    partials += (int64_t)blockIdx.z * pstride;
  }
  // tile pair y -> (I, J) in row-major order of the upper triangle of the slice grid
  const int ns = W / 64;
  int I = 0, rem = blockIdx.y;
  while (rem >= ns - I) {
    rem -= ns - I;
    ++I;
  }
  const int J = I + rem;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lrow = lane >> 4, lcol = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  const int split = W1 / 64;
  // the two slices' column bases and sources
  const float* baseI = I < split ? P + 64 * I : P2 + 64 * (I - split);
  const float* baseJ = J < split ? P + 64 * J : P2 + 64 * (J - split);
  const int64_t pitchI = I < split ? ld : ld2;
  const int64_t pitchJ = J < split ? ld : ld2;
  floatx4 acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  constexpr int D = 2;  // slabs in flight per wave
  float fi[D][4], fj[D][4];
  auto load = [&](int dd, int64_t k) {
    const int64_t row = k + lrow;
    const bool ok = row < r1;
    const int64_t rr = ok ? row : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      fi[dd][s] = ok ? baseI[rr * pitchI + 16 * s + lcol] : 0.f;
      fj[dd][s] = ok ? baseJ[rr * pitchJ + 16 * s + lcol] : 0.f;
    }
  };
  const int64_t step = 16;  // four waves x 4 rows
  int64_t k0 = r0 + 4 * wave;
#pragma unroll
  for (int dd = 0; dd < D; ++dd) load(dd, k0 + dd * step);
  for (; k0 < r1; k0 += D * step) {
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[4 * a + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fi[dd][a], fj[dd][b], acc[4 * a + b], 0, 0, 0);
      load(dd, k0 + (dd + D) * step);
    }
  }
  __shared__ float red[64 * 64];
  for (int g2 = 0; g2 < 4; ++g2) {
    if (wave == g2) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int e = (16 * a + 4 * lrow + v) * 64 + 16 * b + lcol;
            red[e] = g2 == 0 ? acc[4 * a + b][v] : red[e] + acc[4 * a + b][v];
          }
    }
    __syncthreads();
  }
  float* outp = partials + (int64_t)blockIdx.x * W * W;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    outp[(int64_t)(64 * I + i) * W + 64 * J + j] = red[e];
  }
}

// W64[i][j] = W64[j][i] = sum over blocks of the partials' entry (i, j), i <= j (the partials hold
// the tiles on and above the diagonal), so W64 is exactly symmetric and each upper entry is read
// once per partial.  Block (x, i) owns row i, columns 16 x .. 16 x + 15 (blocks wholly below the
// diagonal return); sixteen thread groups sum interleaved sixteenths of the partials, four loads
// in flight each, in a fixed order, and the group sums are added in group order.  Groups: buffer
// k = blockIdx.z with segs[k].nb partials at partials + k pstride.
__global__ __launch_bounds__(256) void k_gram_reduce(const float* __restrict__ partials, int nb, int W,
                                                     double* __restrict__ Wout, const GroupSeg* segs,
                                                     int64_t pstride) {
  __shared__ double red[16][16];
  const int i = blockIdx.y;
  const int j0 = blockIdx.x * 16;
  if (j0 + 15 < i) return;
  if (segs) {
    nb = segs[blockIdx.z].nb;
    partials += (int64_t)blockIdx.z * pstride;
    Wout += (int64_t)blockIdx.z * W * W;
  }
  const int q = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;
  const int j = j0 + q;
  const bool mine = j >= i && j < W;
  const int64_t WW = (int64_t)W * W;
  double s = 0.0;
  if (mine) {
    const float* p = partials + (int64_t)i * W + j;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = grp;
    for (; b + 48 < nb; b += 64) {
      const float v0 = p[b * WW], v1 = p[(b + 16) * WW], v2 = p[(b + 32) * WW], v3 = p[(b + 48) * WW];
      s0 += (double)v0;
      s1 += (double)v1;
      s2 += (double)v2;
      s3 += (double)v3;
    }
    for (; b < nb; b += 16) s0 += (double)p[b * WW];
    s = (s0 + s1) + (s2 + s3);
  }
  red[grp][q] = s;
  __syncthreads();
  if (threadIdx.x < 16 && mine) {
    double t = 0.0;
#pragma unroll
    for (int g2 = 0; g2 < 16; ++g2) t += red[g2][q];
    Wout[(int64_t)i * W + j] = t;
    Wout[(int64_t)j * W + i] = t;
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

// Groups: buffer k = blockIdx.y has panel P + k rows ld, vector y + k rows, scale
// scale_ptr + k sstride and partials part + k gridDim.x L.
template <int CPL>
__global__ __launch_bounds__(256) void k_panel_gemv_t(const float* __restrict__ P, int ld, int L, int64_t rows,
                                                      int rpb, const float* __restrict__ y,
                                                      const double* __restrict__ scale_ptr, float* __restrict__ part,
                                                      int sstride) {
  __shared__ float red[4][64 * CPL];
  {
    const int64_t k = blockIdx.y;
    P += k * rows * ld;
    y += k * rows;
    if (scale_ptr) scale_ptr += k * sstride;
    part += k * gridDim.x * L;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min(rows, r0 + rpb);
  float a[CPL], m[CPL];
  int c[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    a[q] = 0.f;
    c[q] = 64 * q + lane < L ? 64 * q + lane : 0;
    m[q] = 64 * q + lane < L ? 1.f : 0.f;
  }
  int64_t r = r0 + wave;
  for (; r + 12 < r1; r += 16) {
    float yv[4], pv[4][CPL];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      yv[u] = y[r + 4 * u];
#pragma unroll
      for (int q = 0; q < CPL; ++q) pv[u][q] = P[(r + 4 * u) * ld + c[q]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < CPL; ++q) a[q] = fmaf(pv[u][q] * m[q], yv[u], a[q]);
  }
  for (; r < r1; r += 4) {
    const float yv = y[r];
#pragma unroll
    for (int q = 0; q < CPL; ++q) a[q] = fmaf(P[r * ld + c[q]] * m[q], yv, a[q]);
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) red[wave][64 * q + lane] = a[q];
  __syncthreads();
  for (int col = threadIdx.x; col < 64 * CPL && col < L; col += 256) {
    float s = red[0][col] + red[1][col] + red[2][col] + red[3][col];
    float sc = scale_ptr ? (float)(*scale_ptr) : 1.f;
    part[(int64_t)blockIdx.x * L + col] = s * sc;
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

// Blocks of a strip transform (k_xform_strips) over `tiles` 16-row tiles per buffer for K buffers:
// at most 64 (L = 256) or 128 (L = 128) blocks in all, shared out among the buffers; each block
// strides over its buffer's tiles and loads its part of T (up to 256 KB) once.  Fewer, longer
// blocks cost less compute-unit time in all than one block per CU, and compute-unit time is what
// paces a step when several lanes share the GPU (their kernels fill the CUs these leave free).
static int64_t strip_blocks(int L, int64_t tiles, int K) {
  const int64_t cap = L == 256 ? 64 : 128;
  int64_t g = std::min(tiles, std::max<int64_t>(1, cap / std::max(1, K)));
  return std::max<int64_t>(g, 1);
}

// Row blocks of a Gram (and of the fused transform + Gram): about 512 rows per block (1,024 for
// the fused BF16 kernel of 128- and 256-wide panels, whose blocks load both BF16 parts of T), at
// most kGramMaxBlocks.  Smaller blocks finish a lone transform sooner (128-row blocks: 19.9 against
// 23.8 us on a 10^5 x 64 panel) but spend more compute-unit time on loading T and on per-block
// partial Grams, and with several lanes on the GPU that time is what paces the step.
static void gram_grid(int64_t rows, int L, int64_t& nb, int& rpb, bool bf16 = false) {
  const int64_t per = bf16 && L >= 128 ? 1024 : 512;
  nb = (rows + per - 1) / per;
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  if (nb < 1) nb = 1;
  rpb = (int)((rows + nb - 1) / nb);
  rpb = (rpb + 3) & ~3;
  nb = rows > 0 ? (rows + rpb - 1) / rpb : 1;
}

hipError_t xform_gram(void* P, PanelType pt, int ld, int64_t rows, int L, const float* T, float* partials, double* W,
                      hipStream_t st) {
  int64_t nb;
  int rpb;
  gram_grid(rows, L, nb, rpb, pt == PanelType::BF16);
  return xform_gram_group(P, pt, ld, rows, rpb, (int)nb, nullptr, 1, L, T, partials, W, st);
}

void gram_geometry(int64_t rows, int L, int* nb, int* rpb) {
  int64_t n;
  gram_grid(rows, L, n, *rpb);
  *nb = (int)n;
}

int64_t gram_partial_stride(int L) { return (int64_t)kGramMaxBlocks * L * L; }

hipError_t xform_gram_group(void* P, PanelType pt, int ld, int64_t rows, int rpb, int nb, const GroupSeg* segs, int K,
                            int L, const float* T, float* partials, double* W, hipStream_t st) {
  const bool bf = pt == PanelType::BF16;
  const int64_t ps = gram_partial_stride(L);
  const dim3 grid((unsigned)nb, (unsigned)K);
  if (bf) {
    // BF16 panels: transform and Gram on BF16 MFMA (sfd_bf16.hip)
    hipError_t e = xform_gram_bf16_partials(static_cast<uint16_t*>(P), ld, rows, rpb, nb, segs, K, L, T, partials, ps,
                                            true, st);
    if (e != hipSuccess) return e;
  } else if (L == 32) {
    k_xform_gram<32><<<grid, kGramThreads, 0, st>>>(static_cast<float*>(P), ld, rows, rpb, T, partials, segs, ps);
  } else if (L == 64) {
    k_xform_gram<64><<<grid, kGramThreads, 0, st>>>(static_cast<float*>(P), ld, rows, rpb, T, partials, segs, ps);
  } else if (L == 128 || L == 256) {
    // transform in place, then the Gram of the stored result by 64 x 64 tiles
    float* Pf = static_cast<float*>(P);
    const dim3 gx((unsigned)strip_blocks(L, (int64_t)nb * 32, K), 1, (unsigned)K);
    const int ns = L / 64;
    const dim3 gg((unsigned)nb, (unsigned)(ns * (ns + 1) / 2), (unsigned)K);
    if (L == 128)
      k_xform_strips<128, false, true><<<gx, 512, 0, st>>>(Pf, ld, Pf, ld, rows, T, L, segs);
    else
      k_xform_strips<256, false, true><<<gx, 1024, 0, st>>>(Pf, ld, Pf, ld, rows, T, L, segs);
    k_gram_tiles<<<gg, 256, 0, st>>>(Pf, ld, nullptr, 0, L, L, rows, rpb, partials, segs, ps);
  } else {
    return hipErrorInvalidValue;
  }
  k_gram_reduce<<<dim3((unsigned)((L + 15) / 16), (unsigned)L, (unsigned)K), 256, 0, st>>>(partials, nb, L, W, segs,
                                                                                           ps);
  return hipGetLastError();
}

hipError_t gram2(const float* P1, int ld1, const float* P2, int ld2, int64_t rows, int L, float* partials, double* W,
                 hipStream_t st) {
  int64_t nb;
  int rpb;
  gram_grid(rows, 2 * L, nb, rpb);
  switch (L) {
    case 32:
      k_gram_partial<64, true><<<(unsigned)nb, kGramThreads, 0, st>>>(P1, ld1, P2, ld2, rows, rpb, partials);
      break;
    case 64:
      k_gram_partial<128, true><<<(unsigned)nb, kGramThreads, 0, st>>>(P1, ld1, P2, ld2, rows, rpb, partials);
      break;
    case 128:
    case 256: {
      // [P1 | P2] is 2L wide: 2L / 64 slices and their upper tile pairs
      const int ns = 2 * L / 64;
      k_gram_tiles<<<dim3((unsigned)nb, (unsigned)(ns * (ns + 1) / 2), 1), 256, 0, st>>>(
          P1, ld1, P2, ld2, L, 2 * L, rows, rpb, partials, nullptr, 0);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  k_gram_reduce<<<dim3((unsigned)((2 * L + 15) / 16), (unsigned)(2 * L), 1), 256, 0, st>>>(partials, (int)nb, 2 * L, W,
                                                                                         nullptr, 0);
  return hipGetLastError();
}

hipError_t panel_xform2(const float* P1, int ld1, const float* P2, int ld2, int L, const float* T2, float* out,
                        int ldo, int64_t rows, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const unsigned grid = grid_for(rows, 4, 8192);
  if (L == 32) {
    k_panel_xform2<32><<<grid, 256, 0, st>>>(P1, ld1, P2, ld2, T2, out, ldo, rows);
  } else if (L == 64) {
    k_panel_xform2<64><<<grid, 256, 0, st>>>(P1, ld1, P2, ld2, T2, out, ldo, rows);
  } else if (L == 128 || L == 256) {
    // out = P1 T2[0:L] (out may be P1), then out += P2 T2[L:2L]
    const unsigned nb = (unsigned)strip_blocks(L, (rows + 15) / 16, 1);
    if (L == 128) {
      k_xform_strips<128, false, false><<<nb, 512, 0, st>>>(P1, ld1, out, ldo, rows, T2, L, nullptr);
      k_xform_strips<128, true, false><<<nb, 512, 0, st>>>(P2, ld2, out, ldo, rows, T2 + L * L, L, nullptr);
    } else {
      k_xform_strips<256, false, false><<<nb, 1024, 0, st>>>(P1, ld1, out, ldo, rows, T2, L, nullptr);
      k_xform_strips<256, true, false><<<nb, 1024, 0, st>>>(P2, ld2, out, ldo, rows, T2 + L * L, L, nullptr);
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int gemv_blocks(int64_t rows) {
  int64_t nb = (rows + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t panel_gemv_t(const float* P, int ld, int L, int64_t rows, const float* y, const double* scale_ptr,
                        float* part, hipStream_t st, int K, int sstride) {
  int nb = gemv_blocks(rows);
  int rpb = (int)((rows + nb - 1) / nb);
  if (L <= 128)
    k_panel_gemv_t<2><<<dim3((unsigned)nb, (unsigned)K), 256, 0, st>>>(P, ld, L, rows, rpb, y, scale_ptr, part, sstride);
  else
    k_panel_gemv_t<4><<<dim3((unsigned)nb, (unsigned)K), 256, 0, st>>>(P, ld, L, rows, rpb, y, scale_ptr, part, sstride);
  return hipGetLastError();
}

hipError_t start_block(uint64_t seed, uint64_t stream_id, uint64_t buffer, uint64_t attempt, uint64_t purpose,
                       int64_t d, int ell, float* out, int ld, hipStream_t st) {
  int64_t nblk = (d * ell + 3) / 4;
  k_start_block<<<grid_for(nblk, 256, 16384), 256, 0, st>>>(seed, stream_id, buffer, attempt, purpose, d, ell, out, ld);
  return hipGetLastError();
}

}  // namespace sfd
