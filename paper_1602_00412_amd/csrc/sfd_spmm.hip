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

__device__ inline float4 fma4(float v, float4 x, float4 a) {
  a.x = fmaf(v, x.x, a.x);
  a.y = fmaf(v, x.y, a.y);
  a.z = fmaf(v, x.z, a.z);
  a.w = fmaf(v, x.w, a.w);
  return a;
}

// value of lane J of this lane's LPR-lane group (LPR = 8 or 16; groups never straddle a 32-lane
// half): ds_swizzle in bit-mask mode, source = (lane & ~(LPR - 1) & 31) | J
template <int LPR, int J>
__device__ inline int bcast_i(int v) {
  static_assert(LPR == 8 || LPR == 16, "group width");
  constexpr int and_mask = LPR == 16 ? 0x10 : 0x18;
  return __builtin_amdgcn_ds_swizzle(v, and_mask | (J << 5));
}
template <int LPR, int J>
__device__ inline float bcast_f(float v) {
  return __int_as_float(bcast_i<LPR, J>(__float_as_int(v)));
}

// U entries of the group's current block, starting at entry T0 of the block: broadcast their
// ids and values from the lanes that loaded them, gather the U dense rows, accumulate.
template <int LPR, int U, int T0>
__device__ inline void gather_block(int ci, float vi, const float4* __restrict__ X4, int ldx4, int sub, float4& acc) {
  int c[U];
  float v[U];
  float4 x[U];
  [&]<int... u>(std::integer_sequence<int, u...>) {
    ((c[u] = bcast_i<LPR, T0 + u>(ci), v[u] = bcast_f<LPR, T0 + u>(vi)), ...);
  }(std::make_integer_sequence<int, U>{});
#pragma unroll
  for (int u = 0; u < U; ++u) x[u] = X4[(int64_t)c[u] * ldx4 + sub];
#pragma unroll
  for (int u = 0; u < U; ++u) acc = fma4(v[u], x[u], acc);
}

// Y[r, :] = (sum_k val[k] X[idx[k], :]) [* T] over chunk descriptors.  Each L/4-lane group owns
// a chunk at a time and walks it in blocks of L/4 entries: lane s of the group loads entry s of
// the block (coalesced), then the entries are broadcast inside the group and their dense rows
// gathered as float4 (lane s holds columns 4s..4s+3).  The next block's ids and values, and the
// next chunk's descriptor, are loaded before the current block's gathers, so one memory latency
// per block is exposed instead of three.  A group's chunks are c, c + S, c + 2S, ... in its
// band's chunk range (S = all groups of the band).
// Bands (bands > 1, banded CSC): band b's chunks run on the blocks with blockIdx % bands == b;
// workgroups are dispatched round-robin over the 8 XCDs, so with 8 bands each XCD gathers from
// its own band's rows of X only.  Output: a whole row goes to out[r] (times T when XF, T in LDS,
// applied through in-group broadcasts), the chunks of a long row to their partial slots
// (untransformed; the fix-up adds them and applies T).
template <int L, bool XF, int U, bool TRANSPOSED>
__global__ __launch_bounds__(256) void k_spmm(const int4* __restrict__ desc, const int* __restrict__ chunk_start,
                                              int bands, int band_rows, const int* __restrict__ idx,
                                              const float* __restrict__ val, const float* __restrict__ X, int ldx,
                                              float* __restrict__ out, int ldo, float* __restrict__ partial,
                                              const float* __restrict__ T) {
  constexpr int LPR = L / 4;   // lanes per group
  constexpr int G = 64 / LPR;  // groups per wave
  __shared__ float4 tl4[XF ? L * L / 4 : 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int band = blockIdx.x % bands;
  const int slot = blockIdx.x / bands;
  const int c0 = chunk_start[(int64_t)band * band_rows];
  const int c1 = chunk_start[(int64_t)(band + 1) * band_rows];
  const int64_t stride = (int64_t)(gridDim.x / bands) * 4 * G;
  if (XF) {
    const float4* T4 = reinterpret_cast<const float4*>(T);
    for (int e = threadIdx.x; e < L * L / 4; e += 256) tl4[e] = T4[e];
    __syncthreads();
  }
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const int ldx4 = ldx / 4;
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
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
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
    if (cnt > 0) gather_block<LPR, U, 0>(ci, vi, X4, ldx4, sub, acc);
    if constexpr (LPR > U) {
      if (cnt > U) gather_block<LPR, U, U>(ci, vi, X4, ldx4, sub, acc);
    }
    if constexpr (LPR > 2 * U) {
      if (cnt > 2 * U) gather_block<LPR, U, 2 * U>(ci, vi, X4, ldx4, sub, acc);
    }
    if constexpr (LPR > 3 * U) {
      if (cnt > 3 * U) gather_block<LPR, U, 3 * U>(ci, vi, X4, ldx4, sub, acc);
    }
    if (!same) {
      float* dst = dc.w < 0 ? out + (int64_t)dc.x * ldo : partial + (int64_t)dc.w * L;
      if (XF) {
        // o[4 sub + q] = sum_k acc_k T[k][4 sub + q]; acc_k sits in lane k / 4 of the group
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        [&]<int... j>(std::integer_sequence<int, j...>) {
          ((o = fma4(bcast_f<LPR, j>(acc.x), tl4[(4 * j + 0) * (L / 4) + sub], o),
            o = fma4(bcast_f<LPR, j>(acc.y), tl4[(4 * j + 1) * (L / 4) + sub], o),
            o = fma4(bcast_f<LPR, j>(acc.z), tl4[(4 * j + 2) * (L / 4) + sub], o),
            o = fma4(bcast_f<LPR, j>(acc.w), tl4[(4 * j + 3) * (L / 4) + sub], o)),
           ...);
        }(std::make_integer_sequence<int, LPR>{});
        reinterpret_cast<float4*>(dst)[sub] = o;
      } else {
        reinterpret_cast<float4*>(dst)[sub] = acc;
      }
      acc = make_float4(0.f, 0.f, 0.f, 0.f);
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
template <int L>
__global__ __launch_bounds__(256) void k_spmm_fixup(const int* __restrict__ chunk_start,
                                                    const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, const int* __restrict__ nlong_ptr,
                                                    const float* __restrict__ partial, float* __restrict__ Y,
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
  for (int col = threadIdx.x; col < L; col += 256)
    Y[(int64_t)r * ldy + col] = ((red[0][col] + red[1][col]) + red[2][col]) + red[3][col];
  __syncthreads();
  }
}

// Four chunks per wave, one per 16-lane group; a group strides its chunk's entries and
// reduces with a 16-lane xor tree.
__global__ __launch_bounds__(256) void k_spmv(const int4* __restrict__ desc, const int* __restrict__ nchunks_ptr,
                                              const int* __restrict__ idx, const float* __restrict__ val,
                                              const float* __restrict__ y, const double* __restrict__ scale_ptr,
                                              float* __restrict__ z, float* __restrict__ partial) {
  const int nchunks = *nchunks_ptr;
  const int lane = threadIdx.x & 63;
  const int sub = lane & 15;
  const int grp = lane >> 4;
  const float scale = scale_ptr ? (float)(*scale_ptr) : 1.f;
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

template <int L, bool XF, int U>
void launch_spmm(const Schedule& s, const int* idx, const float* val, const float* X, int ldx, float* out, int ldo,
                 float* partial, const float* T, hipStream_t st) {
  constexpr int G = 64 / (L / 4);
  // about four chunks per group; the grid is not persistent (finished blocks make room for
  // waiting ones, which balances uneven chunks), and a multiple of the band count
  int64_t per = ((int64_t)s.max_chunks / s.bands + 16 * G - 1) / (16 * G);
  per = std::max<int64_t>(1, std::min<int64_t>(per, kSpmmMaxBlocks / s.bands));
  const unsigned grid = (unsigned)(per * s.bands);
  const int band_rows = s.bands > 1 ? s.band_rows : s.rows;
  // TRANSPOSED (CSC products) only gives the two products different kernel names
  if (s.transposed)
    k_spmm<L, XF, U, true><<<grid, 256, 0, st>>>(s.desc, s.nch, s.bands, band_rows, idx, val, X, ldx, out, ldo,
                                                 partial, T);
  else
    k_spmm<L, XF, U, false><<<grid, 256, 0, st>>>(s.desc, s.nch, s.bands, band_rows, idx, val, X, ldx, out, ldo,
                                                  partial, T);
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

hipError_t spmm(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* X, int ldx, float* Y,
                int ldy, int L, float* partial, const float* T, hipStream_t st) {
  (void)ptr;
  if (L != 32 && L != 64) return hipErrorInvalidValue;
  if (s.bands > 1) {
    // raw per-band rows; spmm_finish fixes up long rows in place and adds the bands times T
    if (L == 32)
      launch_spmm<32, false, 4>(s, idx, val, X, ldx, s.bandbuf, 32, partial, nullptr, st);
    else
      launch_spmm<64, false, 4>(s, idx, val, X, ldx, s.bandbuf, 64, partial, nullptr, st);
    return hipGetLastError();
  }
  if (L == 32) {
    if (T)
      launch_spmm<32, true, 8>(s, idx, val, X, ldx, Y, ldy, partial, T, st);
    else
      launch_spmm<32, false, 8>(s, idx, val, X, ldx, Y, ldy, partial, nullptr, st);
  } else {
    if (T)
      launch_spmm<64, true, 8>(s, idx, val, X, ldx, Y, ldy, partial, T, st);
    else
      launch_spmm<64, false, 8>(s, idx, val, X, ldx, Y, ldy, partial, nullptr, st);
  }
  return hipGetLastError();
}

hipError_t spmm_finish(const Schedule& s, float* partial, const float* T, float* Y, int ldy, int L, hipStream_t st) {
  if (L != 32 && L != 64) return hipErrorInvalidValue;
  const int* nlong = s.counters;
  const unsigned gfix = 256;
  if (s.bands > 1) {
    const unsigned gr = (unsigned)std::max<int64_t>(1, std::min<int64_t>((s.band_rows + 3) / 4, 8192));
    if (L == 32) {
      k_spmm_fixup<32><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, s.bandbuf, 32);
      k_band_reduce<32><<<gr, 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, T, Y, ldy);
    } else {
      k_spmm_fixup<64><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, s.bandbuf, 64);
      k_band_reduce<64><<<gr, 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, T, Y, ldy);
    }
  } else if (L == 32) {
    k_spmm_fixup<32><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
  } else {
    k_spmm_fixup<64><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
  }
  return hipGetLastError();
}

hipError_t spmv(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* y,
                const double* scale_ptr, float* z, float* partial, hipStream_t st) {
  (void)ptr;
  const int* nchunks = s.nch + s.rows;
  int64_t g = ((int64_t)s.max_chunks + 15) / 16;
  if (g > kSpmmMaxBlocks) g = kSpmmMaxBlocks;
  if (g < 1) g = 1;
  float* zo = s.bands > 1 ? s.bandbuf : z;
  k_spmv<<<(unsigned)g, 256, 0, st>>>(s.desc, nchunks, idx, val, y, scale_ptr, zo, partial);
  k_spmv_fixup<<<64, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.counters, partial, zo);
  if (s.bands > 1)
    k_band_reduce_vec<<<grid_for(s.band_rows, 256, 4096), 256, 0, st>>>(s.nch, s.bands, s.band_rows, s.bandbuf, z);
  return hipGetLastError();
}

}  // namespace sfd
