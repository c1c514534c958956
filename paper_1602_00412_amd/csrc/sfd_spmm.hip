// Sparse x dense products of SimultaneousIteration (Alg 1: the factors A' and A'^T of
// A'(A'^T A')^q G) and the matrix-vector products of VerifySpectral (Alg 6).
//
// Work decomposition: a row of the CSR (or CSC) structure is cut into chunks of at most
// kSpmmChunk stored entries; one wavefront owns one chunk.  Short rows are one chunk and are
// written directly; the chunks of a long row (Zipf-hot columns in the CSC) write partial rows
// that a fix-up pass adds in chunk order, so results do not depend on scheduling.
// Inside a wave the dense row of width L is read as float4 by L/4 lanes; the 64 lanes hold
// 256/L stored entries at a time and their partial rows are combined with cross-lane xor
// shuffles at the end.
#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int64_t kSpmmMaxBlocks = 2048;  // persistent grid: 8 four-wave blocks per CU

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

__global__ void k_sched_counts(const int* ptr, int rows, int* nch, int* pslot) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  for (; r < rows; r += stride) {
    int len = ptr[r + 1] - ptr[r];
    int c = len <= kSpmmChunk ? 1 : (len + kSpmmChunk - 1) / kSpmmChunk;
    nch[r] = c;
    pslot[r] = c > 1 ? c : 0;
  }
}

__global__ void k_sched_rows(int rows, const int* chunk_start, int* chunk_row, int* long_rows, int* counters) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int stride = gridDim.x * blockDim.x;
  for (; r < rows; r += stride) {
    int c0 = chunk_start[r], c1 = chunk_start[r + 1];
    for (int c = c0; c < c1; ++c) chunk_row[c] = r;
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

// Persistent waves: wave w takes chunks w, w + nwaves, ...  With T != nullptr the output row
// (or partial row) is multiplied by the L x L matrix T before it is stored: T sits in LDS, lane c
// computes output column c and receives the row's entries through readlane broadcasts (L <= 64).
template <int L>
__global__ __launch_bounds__(256) void k_spmm(const int* __restrict__ ptr, const int* __restrict__ idx,
                                              const float* __restrict__ val, const int* __restrict__ chunk_start,
                                              const int* __restrict__ slot_start,
                                              const int* __restrict__ chunk_row, const int* __restrict__ nchunks_ptr,
                                              const float* __restrict__ X, int ldx, float* __restrict__ Y, int ldy,
                                              float* __restrict__ partial, const float* __restrict__ T) {
  const int nchunks = *nchunks_ptr;
  constexpr int LPR = L / 4;   // lanes per dense row
  constexpr int G = 64 / LPR;  // stored entries in flight per wave step
  constexpr int TR = L <= 64 ? L : 4;
  __shared__ float tl[TR * TR];
  const int lane = threadIdx.x & 63;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const int ldx4 = ldx / 4;
  const bool xf = (T != nullptr) && (L <= 64);
  if (xf) {
    for (int e = threadIdx.x; e < TR * TR; e += 256) tl[e] = T[e];
  }
  __syncthreads();
  const int tc = lane < TR ? lane : 0;
  for (int64_t cc = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; cc < nchunks; cc += nwaves) {
    const int c = (int)cc;
    const int r = chunk_row[c];
    const int cs = chunk_start[r];
    const int k = c - cs;
    const int nch = chunk_start[r + 1] - cs;
    const int b = ptr[r] + k * kSpmmChunk;
    const int e = min(ptr[r + 1], b + kSpmmChunk);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int p = b + grp;
    for (; p + 3 * G < e; p += 4 * G) {
      const int c0 = idx[p], c1 = idx[p + G], c2 = idx[p + 2 * G], c3 = idx[p + 3 * G];
      const float v0 = val[p], v1 = val[p + G], v2 = val[p + 2 * G], v3 = val[p + 3 * G];
      const float4 x0 = X4[(int64_t)c0 * ldx4 + sub];
      const float4 x1 = X4[(int64_t)c1 * ldx4 + sub];
      const float4 x2 = X4[(int64_t)c2 * ldx4 + sub];
      const float4 x3 = X4[(int64_t)c3 * ldx4 + sub];
      acc = fma4(v0, x0, acc);
      acc = fma4(v1, x1, acc);
      acc = fma4(v2, x2, acc);
      acc = fma4(v3, x3, acc);
    }
    for (; p < e; p += G) {
      const int c0 = idx[p];
      const float v0 = val[p];
      acc = fma4(v0, X4[(int64_t)c0 * ldx4 + sub], acc);
    }
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
      acc.z += __shfl_xor(acc.z, o, 64);
      acc.w += __shfl_xor(acc.w, o, 64);
    }
    float* dst = (nch == 1) ? Y + (int64_t)r * ldy : partial + (int64_t)(slot_start[r] + k) * L;
    if (xf) {
      // every lane with the same `sub` holds entries 4 sub .. 4 sub + 3 of the row
      float o = 0.f;
#pragma unroll
      for (int kk = 0; kk < TR; kk += 4) {
        o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.x), kk / 4)), tl[kk * TR + tc], o);
        o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.y), kk / 4)), tl[(kk + 1) * TR + tc], o);
        o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.z), kk / 4)), tl[(kk + 2) * TR + tc], o);
        o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.w), kk / 4)), tl[(kk + 3) * TR + tc], o);
      }
      if (lane < L) dst[lane] = o;
    } else if (grp == 0) {
      reinterpret_cast<float4*>(dst)[sub] = acc;
    }
  }
}

// Row-packed variant for structures whose rows are short and of similar length (the CSR of a
// buffer): each L/4-lane group of a wave owns one chunk, so a wave advances 64/(L/4) chunks at
// once and needs no cross-group reduction.  Same output and transform as k_spmm.
template <int L>
__global__ __launch_bounds__(256) void k_spmm_rows(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                   const float* __restrict__ val,
                                                   const int* __restrict__ chunk_start,
                                                   const int* __restrict__ slot_start,
                                                   const int* __restrict__ chunk_row,
                                                   const int* __restrict__ nchunks_ptr, const float* __restrict__ X,
                                                   int ldx, float* __restrict__ Y, int ldy,
                                                   float* __restrict__ partial, const float* __restrict__ T) {
  constexpr int LPR = L / 4;   // lanes per group
  constexpr int G = 64 / LPR;  // chunks per wave
  constexpr int TR = L <= 64 ? L : 4;
  __shared__ float tl[TR * TR];
  const int nchunks = *nchunks_ptr;
  const int lane = threadIdx.x & 63;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const int ldx4 = ldx / 4;
  const bool xf = (T != nullptr) && (L <= 64);
  if (xf) {
    for (int e = threadIdx.x; e < TR * TR; e += 256) tl[e] = T[e];
  }
  __syncthreads();
  const int tc = lane < TR ? lane : 0;
  for (int64_t base = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * G; base < nchunks; base += nwaves * G) {
    const int64_t cc = base + grp;
    const bool active = cc < nchunks;
    int r = 0, k = 0, nch = 1, b = 0, e = 0;
    if (active) {
      r = chunk_row[cc];
      const int cs = chunk_start[r];
      k = (int)cc - cs;
      nch = chunk_start[r + 1] - cs;
      b = ptr[r] + k * kSpmmChunk;
      e = min(ptr[r + 1], b + kSpmmChunk);
    }
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int p = b;
    for (; p + 3 < e; p += 4) {
      const int c0 = idx[p], c1 = idx[p + 1], c2 = idx[p + 2], c3 = idx[p + 3];
      const float v0 = val[p], v1 = val[p + 1], v2 = val[p + 2], v3 = val[p + 3];
      const float4 x0 = X4[(int64_t)c0 * ldx4 + sub];
      const float4 x1 = X4[(int64_t)c1 * ldx4 + sub];
      const float4 x2 = X4[(int64_t)c2 * ldx4 + sub];
      const float4 x3 = X4[(int64_t)c3 * ldx4 + sub];
      acc = fma4(v0, x0, acc);
      acc = fma4(v1, x1, acc);
      acc = fma4(v2, x2, acc);
      acc = fma4(v3, x3, acc);
    }
    for (; p < e; ++p) acc = fma4(val[p], X4[(int64_t)idx[p] * ldx4 + sub], acc);
    float* dst = (nch == 1) ? Y + (int64_t)r * ldy : partial + (int64_t)(slot_start[(nch == 1) ? 0 : r] + k) * L;
    if (xf) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int lead = g * LPR;
        if (!__builtin_amdgcn_readlane((int)active, lead)) continue;
        float o = 0.f;
#pragma unroll
        for (int kk = 0; kk < TR; kk += 4) {
          const int src = lead + kk / 4;
          o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.x), src)), tl[kk * TR + tc], o);
          o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.y), src)), tl[(kk + 1) * TR + tc], o);
          o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.z), src)), tl[(kk + 2) * TR + tc], o);
          o = fmaf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.w), src)), tl[(kk + 3) * TR + tc], o);
        }
        const int64_t dlo = (int64_t)__builtin_amdgcn_readlane((int)(uintptr_t)dst, lead);
        const int64_t dhi = (int64_t)__builtin_amdgcn_readlane((int)((uintptr_t)dst >> 32), lead);
        float* dg = reinterpret_cast<float*>((uintptr_t)((dhi << 32) | (dlo & 0xffffffffll)));
        if (lane < L) dg[lane] = o;
      }
    } else if (active) {
      reinterpret_cast<float4*>(dst)[sub] = acc;
    }
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
__global__ __launch_bounds__(256) void k_spmv(const int* __restrict__ ptr, const int* __restrict__ idx,
                                              const float* __restrict__ val, const int* __restrict__ chunk_start,
                                              const int* __restrict__ slot_start,
                                              const int* __restrict__ chunk_row, const int* __restrict__ nchunks_ptr,
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
    int r = 0, k = 0, nch = 1, b = 0, e = 0;
    if (active) {
      r = chunk_row[cc];
      const int cs = chunk_start[r];
      k = (int)cc - cs;
      nch = chunk_start[r + 1] - cs;
      b = ptr[r] + k * kSpmmChunk;
      e = min(ptr[r + 1], b + kSpmmChunk);
    }
    float acc = 0.f;
    int p = b + sub;
    for (; p + 16 < e; p += 32) {
      const int c0 = idx[p], c1 = idx[p + 16];
      const float v0 = val[p], v1 = val[p + 16];
      acc = fmaf(v0, y[c0], acc);
      acc = fmaf(v1, y[c1], acc);
    }
    if (p < e) acc = fmaf(val[p], y[idx[p]], acc);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (active && sub == 0) {
      const float v = acc * scale;
      if (nch == 1)
        z[r] = v;
      else
        partial[slot_start[r] + k] = v;
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

}  // namespace

hipError_t schedule_build(const int* ptr, int rows, Schedule& s, int* scan_tmp, hipStream_t st) {
  hipError_t e;
  if (rows > 0) k_sched_counts<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.nch, s.pslot);
  if ((e = scan_exclusive(s.nch, s.nch, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(s.pslot, s.pslot, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = fill_i32(s.counters, 1, 0, st)) != hipSuccess) return e;
  if (rows > 0) k_sched_rows<<<grid_for(rows, 256, 8192), 256, 0, st>>>(rows, s.nch, s.chunk_row, s.long_rows,
                                                                           s.counters);
  s.rows = rows;
  return hipGetLastError();
}

hipError_t spmm(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* X, int ldx, float* Y,
                int ldy, int L, float* partial, const float* T, hipStream_t st) {
  if (T && L > 64) return hipErrorInvalidValue;
  const int* nchunks = s.nch + s.rows;
  const int* nlong = s.counters;
  int64_t g = ((int64_t)s.max_chunks + 3) / 4;
  if (g > kSpmmMaxBlocks) g = kSpmmMaxBlocks;
  if (g < 1) g = 1;
  const unsigned grid = (unsigned)g;
  const unsigned gfix = 256;
  if (s.row_packed && L <= 64) {
    int64_t gp = ((int64_t)s.max_chunks + 4 * (256 / L) - 1) / (4 * (256 / L));
    if (gp > kSpmmMaxBlocks) gp = kSpmmMaxBlocks;
    if (gp < 1) gp = 1;
    if (L == 32)
      k_spmm_rows<32><<<(unsigned)gp, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, X, ldx, Y,
                                                    ldy, partial, T);
    else
      k_spmm_rows<64><<<(unsigned)gp, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, X, ldx, Y,
                                                    ldy, partial, T);
    if (L == 32)
      k_spmm_fixup<32><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
    else
      k_spmm_fixup<64><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
    return hipGetLastError();
  }
  switch (L) {
    case 32:
      k_spmm<32><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, X, ldx, Y, ldy, partial, T);
      k_spmm_fixup<32><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
      break;
    case 64:
      k_spmm<64><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, X, ldx, Y, ldy, partial, T);
      k_spmm_fixup<64><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
      break;
    case 128:
      k_spmm<128><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, X, ldx, Y, ldy, partial,
                                        T);
      k_spmm_fixup<128><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, nlong, partial, Y, ldy);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t spmv(const int* ptr, const int* idx, const float* val, const Schedule& s, const float* y,
                const double* scale_ptr, float* z, float* partial, hipStream_t st) {
  const int* nchunks = s.nch + s.rows;
  int64_t g = ((int64_t)s.max_chunks + 15) / 16;
  if (g > kSpmmMaxBlocks) g = kSpmmMaxBlocks;
  if (g < 1) g = 1;
  k_spmv<<<(unsigned)g, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, nchunks, y, scale_ptr, z, partial);
  k_spmv_fixup<<<64, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.counters, partial, z);
  return hipGetLastError();
}

}  // namespace sfd
