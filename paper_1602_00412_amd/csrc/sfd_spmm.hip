// Sparse x dense products of SimultaneousIteration (Alg 1: the factors A' and A'^T of
// A'(A'^T A')^q G) and the matrix-vector products of VerifySpectral (Alg 6).
//
// Work decomposition: a row of the CSR (or CSC) structure is cut into chunks of at most
// kSpmmChunk stored entries, each described by {row, first entry, end entry, partial slot}.
// Short rows are one chunk and are written directly; the chunks of a long row (Zipf-hot
// columns in the CSC) write partial rows that a fix-up pass adds in chunk order, so results do
// not depend on scheduling.  In the dense products an L/4-lane group owns one chunk at a time
// and reads each dense row of width L as float4 (lane s: columns 4s..4s+3).
#include <algorithm>
#include <utility>

#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int64_t kSpmmMaxBlocks = 16384;  // 64 four-wave blocks per CU at most

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// chunks per row: one for a short row (also an empty one, whose output row is then written as
// zeros, unless skip_empty), ceil(len / kSpmmChunk) for a long row
__global__ void k_sched_counts(const int* ptr, int rows, int skip_empty, int* nch, int* pslot) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  for (; r < rows; r += stride) {
    int len = ptr[r + 1] - ptr[r];
    int c = len <= kSpmmChunk ? (len > 0 || !skip_empty ? 1 : 0) : (len + kSpmmChunk - 1) / kSpmmChunk;
    nch[r] = c;
    pslot[r] = c > 1 ? c : 0;
  }
}

__global__ void k_sched_desc(const int* ptr, int rows, const int* chunk_start, const int* slot_start, int4* desc,
                             int* long_rows, int* counters) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  for (; r < rows; r += stride) {
    const int c0 = chunk_start[r], c1 = chunk_start[r + 1];
    const int b = ptr[r], e = ptr[r + 1];
    for (int c = c0; c < c1; ++c) {
      const int k = c - c0;
      const int bb = b + k * kSpmmChunk;
      desc[c] = make_int4(r, bb, min(e, bb + kSpmmChunk), c1 - c0 > 1 ? slot_start[r] + k : -1);
    }
    if (c1 - c0 > 1) long_rows[atomicAdd(&counters[0], 1)] = r;
  }
}

// BF16 storage of panels: the upper 16 bits of an FP32 value, rounded to nearest even.
__device__ inline uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// value of lane J of this lane's LPR-lane group: for LPR = 4 .. 32 (groups never straddle a
// 32-lane half) ds_swizzle in bit-mask mode, source = (lane & 31 & ~(LPR - 1)) | J; for LPR = 64
// (the whole wave) a readlane
template <int LPR, int J>
__device__ inline int bcast_i(int v) {
  static_assert(LPR == 4 || LPR == 8 || LPR == 16 || LPR == 32 || LPR == 64, "group width");
  if constexpr (LPR == 64) {
    return __builtin_amdgcn_readlane(v, J);
  } else {
    constexpr int and_mask = 0x1F & ~(LPR - 1);
    return __builtin_amdgcn_ds_swizzle(v, and_mask | (J << 5));
  }
}
template <int LPR, int J>
__device__ inline float bcast_f(float v) {
  return __int_as_float(bcast_i<LPR, J>(__float_as_int(v)));
}

// A panel row segment of one lane: VEC consecutive columns, FP32 (VEC = 4, one float4) or BF16
// (VEC = 8, one 16-byte word).
template <bool BF>
struct Seg;
template <>
struct Seg<false> {
  static constexpr int VEC = 4;
  using raw = float4;
  __device__ static inline void fma(float v, const raw& x, float* a) {
    a[0] = fmaf(v, x.x, a[0]);
    a[1] = fmaf(v, x.y, a[1]);
    a[2] = fmaf(v, x.z, a[2]);
    a[3] = fmaf(v, x.w, a[3]);
  }
};
template <>
struct Seg<true> {
  static constexpr int VEC = 8;
  using raw = uint4;
  __device__ static inline void fma(float v, const raw& x, float* a) {
    a[0] = fmaf(v, bf16_lo(x.x), a[0]);
    a[1] = fmaf(v, bf16_hi(x.x), a[1]);
    a[2] = fmaf(v, bf16_lo(x.y), a[2]);
    a[3] = fmaf(v, bf16_hi(x.y), a[3]);
    a[4] = fmaf(v, bf16_lo(x.z), a[4]);
    a[5] = fmaf(v, bf16_hi(x.z), a[5]);
    a[6] = fmaf(v, bf16_lo(x.w), a[6]);
    a[7] = fmaf(v, bf16_hi(x.w), a[7]);
  }
};

// store VEC FP32 values of a row segment as FP32 or BF16
template <int VEC, bool BF>
__device__ inline void store_seg(void* row, int sub, const float* o) {
  if constexpr (!BF) {
    float4* d = reinterpret_cast<float4*>(row) + (VEC / 4) * sub;
#pragma unroll
    for (int q = 0; q < VEC / 4; ++q) d[q] = make_float4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else if constexpr (VEC == 8) {
    uint4 w;
    w.x = f32_to_bf16(o[0]) | (f32_to_bf16(o[1]) << 16);
    w.y = f32_to_bf16(o[2]) | (f32_to_bf16(o[3]) << 16);
    w.z = f32_to_bf16(o[4]) | (f32_to_bf16(o[5]) << 16);
    w.w = f32_to_bf16(o[6]) | (f32_to_bf16(o[7]) << 16);
    reinterpret_cast<uint4*>(row)[sub] = w;
  } else {
    uint2 w;
    w.x = f32_to_bf16(o[0]) | (f32_to_bf16(o[1]) << 16);
    w.y = f32_to_bf16(o[2]) | (f32_to_bf16(o[3]) << 16);
    reinterpret_cast<uint2*>(row)[sub] = w;
  }
}

// U entries of the group's current block, starting at entry T0 of the block: broadcast their
// ids and values from the lanes that loaded them, gather the U dense row segments, accumulate.
template <int LPR, int U, int T0, bool BF>
__device__ inline void gather_block(int ci, float vi, const typename Seg<BF>::raw* __restrict__ Xs, int lds, int sub,
                                    float* acc) {
  int c[U];
  float v[U];
  typename Seg<BF>::raw x[U];
  [&]<int... u>(std::integer_sequence<int, u...>) {
    ((c[u] = bcast_i<LPR, T0 + u>(ci), v[u] = bcast_f<LPR, T0 + u>(vi)), ...);
  }(std::make_integer_sequence<int, U>{});
#pragma unroll
  for (int u = 0; u < U; ++u) x[u] = Xs[(int64_t)c[u] * lds + sub];
#pragma unroll
  for (int u = 0; u < U; ++u) Seg<BF>::fma(v[u], x[u], acc);
}

// Y[r, :] = sum_k val[k] X[idx[k], :] over chunk descriptors, X and Y FP32 or BF16
// panels (BIN / BOUT), FP32 accumulation.  A group of L/VEC lanes owns a chunk at a time (lane s
// holds columns VEC s .. VEC s + VEC - 1) and walks it in blocks of L/VEC entries: lane s of the
// group loads entry s of the block (coalesced), then the entries are broadcast inside the group
// and their dense row segments gathered.  The next block's ids and values, and the next chunk's
// descriptor, are loaded before the current block's gathers, so one memory latency per block is
// exposed instead of three.  A group's chunks are c, c + S, c + 2S, ... in its band's chunk
// range (S = all groups of the band).
// Bands (bands > 1, banded CSC): band b's chunks run on the blocks with blockIdx % bands == b;
// workgroups are dispatched round-robin over the 8 XCDs, so with 8 bands each XCD gathers from
// its own band's rows of X only.
// Output: a whole row goes to out[r], the chunks of a long row to their FP32 partial slots (the
// fix-up adds them in chunk order).  The inverse Cholesky factor of the input panel is applied to
// the output afterwards (xform_gram), together with the output's Gram.
template <int L, int U, bool TRANSPOSED, bool BIN, bool BOUT>
__global__ __launch_bounds__(256) void k_spmm(const int4* __restrict__ desc, const int* __restrict__ chunk_start,
                                              int bands, int band_rows, const int* __restrict__ idx,
                                              const float* __restrict__ val, const void* __restrict__ X, int ldx,
                                              void* __restrict__ out, int ldo, float* __restrict__ partial) {
  using S = Seg<BIN>;
  constexpr int VEC = S::VEC;
  constexpr int LPR = L / VEC;  // lanes per group
  constexpr int G = 64 / LPR;   // groups per wave
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int band = blockIdx.x % bands;
  const int slot = blockIdx.x / bands;
  const int c0 = chunk_start[(int64_t)band * band_rows];
  const int c1 = chunk_start[(int64_t)(band + 1) * band_rows];
  const int64_t stride = (int64_t)(gridDim.x / bands) * 4 * G;
  const typename S::raw* Xs = reinterpret_cast<const typename S::raw*>(X);
  const int lds = ldx / VEC;  // row pitch in segments
  const size_t out_row_bytes = (size_t)ldo * (BOUT ? 2 : 4);
  int64_t cc = c0 + ((int64_t)slot * 4 + wave) * G + grp;
  int4 dc = cc < c1 ? desc[cc] : make_int4(0, 0, 0, -1);
  int64_t ncc = cc + stride;
  int4 dn = ncc < c1 ? desc[ncc] : make_int4(0, 0, 0, -1);
  int p = dc.y;
  int ci = 0;
  float vi = 0.f;
  if (cc < c1 && p + sub < dc.z) {
    ci = idx[p + sub];
    vi = val[p + sub];
  }
  float acc[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) acc[q] = 0.f;
  while (cc < c1) {
    // where the next block starts: later in this chunk, or at the group's next chunk
    const bool same = p + LPR < dc.z;
    const int np = same ? p + LPR : dn.y;
    const int nend = same ? dc.z : dn.z;
    int ci2 = 0;
    float vi2 = 0.f;
    if ((same || ncc < c1) && np + sub < nend) {
      ci2 = idx[np + sub];
      vi2 = val[np + sub];
    }
    // entries beyond the chunk have id 0 and value 0: whole U-blocks past the end are skipped
    const int cnt = min(LPR, dc.z - p);
    [&]<int... b>(std::integer_sequence<int, b...>) {
      ((cnt > b * U ? gather_block<LPR, U, b * U, BIN>(ci, vi, Xs, lds, sub, acc) : void()), ...);
    }(std::make_integer_sequence<int, LPR / U>{});
    if (!same) {
      float o[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) o[q] = acc[q];
      if constexpr (BOUT) {
        if (dc.w < 0)
          store_seg<VEC, true>(reinterpret_cast<char*>(out) + (size_t)dc.x * out_row_bytes, sub, o);
        else
          store_seg<VEC, false>(partial + (int64_t)dc.w * L, sub, o);
      } else {
        float* dst = dc.w < 0 ? reinterpret_cast<float*>(reinterpret_cast<char*>(out) + (size_t)dc.x * out_row_bytes)
                              : partial + (int64_t)dc.w * L;
        store_seg<VEC, false>(dst, sub, o);
      }
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] = 0.f;
      cc = ncc;
      dc = dn;
      ncc += stride;
      dn = ncc < c1 ? desc[ncc] : make_int4(0, 0, 0, -1);
    }
    p = np;
    ci = ci2;
    vi = vi2;
  }
}

// One block per long row: wave w adds the row's partials w, w + 4, ... (in order), then the
// four wave sums are added in wave order.
template <int L, bool BOUT>
__global__ __launch_bounds__(256) void k_spmm_fixup(const int* __restrict__ chunk_start,
                                                    const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, const int* __restrict__ nlong_ptr,
                                                    const float* __restrict__ partial, void* __restrict__ Y,
                                                    int ldy) {
  constexpr int CPL = (L + 63) / 64;  // columns per lane
  __shared__ float red[4][L];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nlong = *nlong_ptr;
  for (int li = blockIdx.x; li < nlong; li += gridDim.x) {
  const int r = long_rows[li];
  const int n = chunk_start[r + 1] - chunk_start[r];
  const float* base = partial + (int64_t)slot_start[r] * L;
  float acc[CPL];
#pragma unroll
  for (int u = 0; u < CPL; ++u) acc[u] = 0.f;
  int j = wave;
  for (; j + 4 < n; j += 8) {
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      if (col < L) {
        const float a = base[(int64_t)j * L + col], b = base[(int64_t)(j + 4) * L + col];
        acc[u] += a;
        acc[u] += b;
      }
    }
  }
  for (; j < n; j += 4) {
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      if (col < L) acc[u] += base[(int64_t)j * L + col];
    }
  }
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int col = lane + 64 * u;
    if (col < L) red[wave][col] = acc[u];
  }
  __syncthreads();
  for (int col = threadIdx.x; col < L; col += 256) {
    const float v = ((red[0][col] + red[1][col]) + red[2][col]) + red[3][col];
    if constexpr (BOUT)
      reinterpret_cast<uint16_t*>(Y)[(int64_t)r * ldy + col] = (uint16_t)f32_to_bf16(v);
    else
      reinterpret_cast<float*>(Y)[(int64_t)r * ldy + col] = v;
  }
  __syncthreads();
  }
}

// Four chunks per wave, one per 16-lane group; a group strides its chunk's entries and
// reduces with a 16-lane xor tree.
// In a group (seg_rows != nullptr) row r belongs to the buffer k with seg_rows[k] <= r <
// seg_rows[k + 1] and is scaled by scale_ptr[k sstride].
__global__ __launch_bounds__(256) void k_spmv(const int4* __restrict__ desc, const int* __restrict__ nchunks_ptr,
                                              const int* __restrict__ idx, const float* __restrict__ val,
                                              const float* __restrict__ y, const double* __restrict__ scale_ptr,
                                              float* __restrict__ z, float* __restrict__ partial,
                                              const int64_t* __restrict__ seg_rows, int K, int sstride) {
  const int nchunks = *nchunks_ptr;
  const int lane = threadIdx.x & 63;
  const int sub = lane & 15;
  const int grp = lane >> 4;
  const float scale1 = (scale_ptr && !seg_rows) ? (float)(*scale_ptr) : 1.f;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t base = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * 4; base < nchunks; base += nwaves * 4) {
    const int64_t cc = base + grp;
    const bool active = cc < nchunks;
    const int4 dc = active ? desc[cc] : make_int4(0, 0, 0, -1);
    float acc = 0.f;
    int p = dc.y + sub;
    for (; p + 16 < dc.z; p += 32) {
      const int c0 = idx[p], c1 = idx[p + 16];
      const float v0 = val[p], v1 = val[p + 16];
      acc = fmaf(v0, y[c0], acc);
      acc = fmaf(v1, y[c1], acc);
    }
    if (p < dc.z) acc = fmaf(val[p], y[idx[p]], acc);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (active && sub == 0) {
      float scale = scale1;
      if (scale_ptr && seg_rows) {
        int lo = 0, hi = K;  // last k with seg_rows[k] <= row
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (seg_rows[mid] <= dc.x) lo = mid; else hi = mid;
        }
        scale = (float)scale_ptr[(int64_t)lo * sstride];
      }
      const float v = acc * scale;
      if (dc.w < 0)
        z[dc.x] = v;
      else
        partial[dc.w] = v;
    }
  }
}

// One wave per long row: lane j adds partials j, j + 64, ...; then an xor-tree over the wave.
__global__ __launch_bounds__(256) void k_spmv_fixup(const int* __restrict__ chunk_start,
                                                    const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, const int* __restrict__ nlong_ptr,
                                                    const float* __restrict__ partial, float* __restrict__ z) {
  const int nlong = *nlong_ptr;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t ii = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; ii < nlong; ii += nwaves) {
    const int i = (int)ii;
    const int r = long_rows[i];
    const int n = chunk_start[r + 1] - chunk_start[r];
    const int s0 = slot_start[r];
    float s = 0.f;
    for (int j = lane; j < n; j += 64) s += partial[s0 + j];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) z[r] = s;
  }
}

// Y[j, :] = (sum over bands b, in order, of part[b * band_rows + j, :]) * T; a band in which
// row j has no entries (no chunk) adds nothing.  One wave per output row; lane c < L holds
// column c, lanes 0..bands-1 fetch the bands' chunk counts.
template <int L>
__global__ __launch_bounds__(256) void k_band_reduce(const int* __restrict__ chunk_start, int bands, int band_rows,
                                                     const float* __restrict__ part, const float* __restrict__ T,
                                                     float* __restrict__ Y, int ldy) {
  static_assert(L <= 64, "one lane per column");
  __shared__ float tl[L * L];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (T) {
    for (int e = threadIdx.x; e < L * L; e += 256) tl[e] = T[e];
  }
  __syncthreads();
  const int col = lane < L ? lane : 0;
  for (int64_t j = (int64_t)blockIdx.x * 4 + wave; j < band_rows; j += (int64_t)gridDim.x * 4) {
    int n = 0;
    if (lane < bands) {
      const int64_t r = (int64_t)lane * band_rows + j;
      n = chunk_start[r + 1] - chunk_start[r];
    }
    float v[kMaxBands];
#pragma unroll
    for (int b = 0; b < kMaxBands; ++b) {
      const int nb = b < bands ? __builtin_amdgcn_readlane(n, b) : 0;
      v[b] = nb > 0 ? part[((int64_t)b * band_rows + j) * L + col] : 0.f;
    }
    float acc = 0.f;
#pragma unroll
    for (int b = 0; b < kMaxBands; ++b) acc += v[b];
    float o = acc;
    if (T) {
      o = 0.f;
#pragma unroll
      for (int kk = 0; kk < L; ++kk)
        o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc), kk)), tl[kk * L + col], o);
    }
    if (lane < L) Y[j * ldy + lane] = o;
  }
}

// z[j] = sum over bands b, in order, of zpart[b * band_rows + j] (bands with no entry in row j
// add nothing)
__global__ __launch_bounds__(256) void k_band_reduce_vec(const int* __restrict__ chunk_start, int bands,
                                                         int band_rows, const float* __restrict__ zpart,
                                                         float* __restrict__ z) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < band_rows; j += (int64_t)gridDim.x * 256) {
    float acc = 0.f;
    for (int b = 0; b < bands; ++b) {
      const int64_t r = (int64_t)b * band_rows + j;
      if (chunk_start[r + 1] > chunk_start[r]) acc += zpart[r];
    }
    z[j] = acc;
  }
}

template <int L, int U, bool BIN, bool BOUT>
void launch_spmm(const Schedule& s, const int* idx, const float* val, const void* X, int ldx, void* out, int ldo,
                 float* partial, hipStream_t st) {
  constexpr int G = 64 / (L / Seg<BIN>::VEC);
  // about four chunks per group; the grid is not persistent (finished blocks make room for
  // waiting ones, which balances uneven chunks), and a multiple of the band count
  int64_t per = ((int64_t)s.max_chunks / s.bands + 16 * G - 1) / (16 * G);
  per = std::max<int64_t>(1, std::min<int64_t>(per, kSpmmMaxBlocks / s.bands));
  const unsigned grid = (unsigned)(per * s.bands);
  const int band_rows = s.bands > 1 ? s.band_rows : s.rows;
  // TRANSPOSED (CSC products) only gives the two products different kernel names
  if (s.transposed)
    k_spmm<L, U, true, BIN, BOUT><<<grid, 256, 0, st>>>(s.desc, s.nch, s.bands, band_rows, idx, val, X, ldx, out,
                                                        ldo, partial);
  else
    k_spmm<L, U, false, BIN, BOUT><<<grid, 256, 0, st>>>(s.desc, s.nch, s.bands, band_rows, idx, val, X, ldx, out,
                                                         ldo, partial);
}

template <int L>
hipError_t spmm_l(const Schedule& s, const int* idx, const float* val, const void* X, PanelType xt, int ldx, void* Y,
                  PanelType yt, int ldy, float* partial, hipStream_t st) {
  const bool xb = xt == PanelType::BF16, yb = yt == PanelType::BF16;
  if (s.bands > 1) {
    // FP32 per-band rows; spmm_finish fixes up long rows in place and adds the bands
    if (xb || yb) return hipErrorInvalidValue;
    launch_spmm<L, 4, false, false>(s, idx, val, X, ldx, s.bandbuf, L, partial, st);
  } else if (!xb && !yb) {
    launch_spmm<L, 8, false, false>(s, idx, val, X, ldx, Y, ldy, partial, st);
  } else if (xb && yb) {
    launch_spmm<L, 4, true, true>(s, idx, val, X, ldx, Y, ldy, partial, st);
  } else if (xb && !yb) {
    launch_spmm<L, 4, true, false>(s, idx, val, X, ldx, Y, ldy, partial, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t schedule_build(const int* ptr, int rows, Schedule& s, int* scan_tmp, hipStream_t st) {
  hipError_t e;
  if (rows > 0)
    k_sched_counts<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.bands > 1 ? 1 : 0, s.nch, s.pslot);
  if ((e = scan_exclusive(s.nch, s.nch, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(s.pslot, s.pslot, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = fill_i32(s.counters, 1, 0, st)) != hipSuccess) return e;
  if (rows > 0)
    k_sched_desc<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.nch, s.pslot, s.desc, s.long_rows,
                                                             s.counters);
  s.rows = rows;
  return hipGetLastError();
}

hipError_t spmm(const Schedule& s, const int* idx, const float* val, const void* X, PanelType xt, int ldx, void* Y,
                PanelType yt, int ldy, int L, float* partial, hipStream_t st) {
  if (L == 32) return spmm_l<32>(s, idx, val, X, xt, ldx, Y, yt, ldy, partial, st);
  if (L == 64) return spmm_l<64>(s, idx, val, X, xt, ldx, Y, yt, ldy, partial, st);
  if (L == 128 && s.bands == 1) return spmm_l<128>(s, idx, val, X, xt, ldx, Y, yt, ldy, partial, st);
  if (L == 256 && s.bands == 1) return spmm_l<256>(s, idx, val, X, xt, ldx, Y, yt, ldy, partial, st);
  return hipErrorInvalidValue;
}

namespace {

template <int L>
void launch_fixup(const Schedule& s, float* partial, void* Y, bool yb, int ldy, hipStream_t st) {
  if (yb)
    k_spmm_fixup<L, true><<<256, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.counters, partial, Y, ldy);
  else
    k_spmm_fixup<L, false><<<256, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.counters, partial, Y, ldy);
}

}  // namespace

hipError_t spmm_finish(const Schedule& s, float* partial, void* Y, PanelType yt, int ldy, int L, hipStream_t st) {
  const bool yb = yt == PanelType::BF16;
  if (s.bands > 1) {
    // long rows fixed up in place in the band buffer, then the bands added
    if (yb || (L != 32 && L != 64)) return hipErrorInvalidValue;
    const unsigned gr = (unsigned)std::max<int64_t>(1, std::min<int64_t>((s.band_rows + 3) / 4, 8192));
    if (L == 32) {
      launch_fixup<32>(s, partial, s.bandbuf, false, 32, st);
      k_band_reduce<32><<<gr, 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, nullptr,
                                            reinterpret_cast<float*>(Y), ldy);
    } else {
      launch_fixup<64>(s, partial, s.bandbuf, false, 64, st);
      k_band_reduce<64><<<gr, 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, nullptr,
                                            reinterpret_cast<float*>(Y), ldy);
    }
  } else if (L == 32) {
    launch_fixup<32>(s, partial, Y, yb, ldy, st);
  } else if (L == 64) {
    launch_fixup<64>(s, partial, Y, yb, ldy, st);
  } else if (L == 128) {
    launch_fixup<128>(s, partial, Y, yb, ldy, st);
  } else if (L == 256) {
    launch_fixup<256>(s, partial, Y, yb, ldy, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t spmv(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* y,
                const double* scale_ptr, float* z, float* partial, hipStream_t st, const int64_t* seg_rows, int K,
                int sstride) {
  (void)ptr;
  const int* nchunks = s.nch + s.rows;
  int64_t g = ((int64_t)s.max_chunks + 15) / 16;
  if (g > kSpmmMaxBlocks) g = kSpmmMaxBlocks;
  if (g < 1) g = 1;
  float* zo = s.bands > 1 ? s.bandbuf : z;
  k_spmv<<<(unsigned)g, 256, 0, st>>>(s.desc, nchunks, idx, val, y, scale_ptr, zo, partial, seg_rows, K, sstride);
  k_spmv_fixup<<<64, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.counters, partial, zo);
  if (s.bands > 1)
    k_band_reduce_vec<<<grid_for(s.band_rows, 256, 4096), 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, z);
  return hipGetLastError();
}

}  // namespace sfd
