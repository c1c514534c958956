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

template <int L>
__global__ __launch_bounds__(256) void k_spmm(const int* __restrict__ ptr, const int* __restrict__ idx,
                                              const float* __restrict__ val, const int* __restrict__ chunk_start,
                                              const int* __restrict__ slot_start,
                                              const int* __restrict__ chunk_row, int nchunks,
                                              const float* __restrict__ X, int ldx, float* __restrict__ Y, int ldy,
                                              float* __restrict__ partial) {
  constexpr int LPR = L / 4;   // lanes per dense row
  constexpr int G = 64 / LPR;  // stored entries in flight per wave step
  const int c = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  if (c >= nchunks) return;
  const int lane = threadIdx.x & 63;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int r = chunk_row[c];
  const int cs = chunk_start[r];
  const int k = c - cs;
  const int nch = chunk_start[r + 1] - cs;
  const int b = ptr[r] + k * kSpmmChunk;
  const int e = min(ptr[r + 1], b + kSpmmChunk);
  const float4* X4 = reinterpret_cast<const float4*>(X);
  const int ldx4 = ldx / 4;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  int p = b + grp;
  for (; p + 3 * G < e; p += 4 * G) {
    int c0 = idx[p], c1 = idx[p + G], c2 = idx[p + 2 * G], c3 = idx[p + 3 * G];
    float v0 = val[p], v1 = val[p + G], v2 = val[p + 2 * G], v3 = val[p + 3 * G];
    float4 x0 = X4[(int64_t)c0 * ldx4 + sub];
    float4 x1 = X4[(int64_t)c1 * ldx4 + sub];
    float4 x2 = X4[(int64_t)c2 * ldx4 + sub];
    float4 x3 = X4[(int64_t)c3 * ldx4 + sub];
    acc = fma4(v0, x0, acc);
    acc = fma4(v1, x1, acc);
    acc = fma4(v2, x2, acc);
    acc = fma4(v3, x3, acc);
  }
  for (; p < e; p += G) {
    int c0 = idx[p];
    float v0 = val[p];
    acc = fma4(v0, X4[(int64_t)c0 * ldx4 + sub], acc);
  }
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1) {
    acc.x += __shfl_xor(acc.x, o, 64);
    acc.y += __shfl_xor(acc.y, o, 64);
    acc.z += __shfl_xor(acc.z, o, 64);
    acc.w += __shfl_xor(acc.w, o, 64);
  }
  if (grp == 0) {
    float* dst = (nch == 1) ? Y + (int64_t)r * ldy : partial + (int64_t)(slot_start[r] + k) * L;
    reinterpret_cast<float4*>(dst)[sub] = acc;
  }
}

template <int L>
__global__ __launch_bounds__(256) void k_spmm_fixup(const int* __restrict__ chunk_start,
                                                    const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, int nlong,
                                                    const float* __restrict__ partial, float* __restrict__ Y,
                                                    int ldy) {
  const int i = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  if (i >= nlong) return;
  const int lane = threadIdx.x & 63;
  const int r = long_rows[i];
  const int n = chunk_start[r + 1] - chunk_start[r];
  const int s0 = slot_start[r];
  for (int col = lane; col < L; col += 64) {
    float s = 0.f;
    for (int j = 0; j < n; ++j) s += partial[(int64_t)(s0 + j) * L + col];
    Y[(int64_t)r * ldy + col] = s;
  }
}

__global__ __launch_bounds__(256) void k_spmv(const int* __restrict__ ptr, const int* __restrict__ idx,
                                              const float* __restrict__ val, const int* __restrict__ chunk_start,
                                              const int* __restrict__ slot_start,
                                              const int* __restrict__ chunk_row, int nchunks,
                                              const float* __restrict__ y, const double* __restrict__ scale_ptr,
                                              float* __restrict__ z, float* __restrict__ partial) {
  const int c = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  if (c >= nchunks) return;
  const int lane = threadIdx.x & 63;
  const int r = chunk_row[c];
  const int cs = chunk_start[r];
  const int k = c - cs;
  const int nch = chunk_start[r + 1] - cs;
  const int b = ptr[r] + k * kSpmmChunk;
  const int e = min(ptr[r + 1], b + kSpmmChunk);
  float acc = 0.f;
  for (int p = b + lane; p < e; p += 64) acc = fmaf(val[p], y[idx[p]], acc);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    float s = scale_ptr ? (float)(*scale_ptr) : 1.f;
    float v = acc * s;
    if (nch == 1)
      z[r] = v;
    else
      partial[slot_start[r] + k] = v;
  }
}

__global__ void k_spmv_fixup(const int* __restrict__ chunk_start, const int* __restrict__ slot_start,
                             const int* __restrict__ long_rows, int nlong, const float* __restrict__ partial,
                             float* __restrict__ z) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlong) return;
  int r = long_rows[i];
  int n = chunk_start[r + 1] - chunk_start[r];
  int s0 = slot_start[r];
  float s = 0.f;
  for (int j = 0; j < n; ++j) s += partial[s0 + j];
  z[r] = s;
}

}  // namespace

hipError_t schedule_counts(const int* ptr, int rows, Schedule& s, hipStream_t st) {
  if (rows > 0) k_sched_counts<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.nch, s.pslot);
  return hipGetLastError();
}

hipError_t schedule_finish(const int* ptr, int rows, Schedule& s, hipStream_t st) {
  (void)ptr;
  hipError_t e = fill_i32(s.counters, 1, 0, st);
  if (e != hipSuccess) return e;
  if (rows > 0) k_sched_rows<<<grid_for(rows, 256, 8192), 256, 0, st>>>(rows, s.nch, s.chunk_row, s.long_rows,
                                                                           s.counters);
  return hipGetLastError();
}

hipError_t spmm(const int* ptr, const int* idx, const float* val, int rows, const Schedule& s, const float* X,
                int ldx, float* Y, int ldy, int L, float* partial, hipStream_t st) {
  (void)rows;
  if (s.nchunks <= 0) return hipSuccess;
  unsigned grid = (unsigned)((s.nchunks + 3) / 4);
  unsigned gfix = (unsigned)((s.nlong + 3) / 4);
  switch (L) {
    case 32:
      k_spmm<32><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, s.nchunks, X, ldx, Y, ldy, partial);
      if (s.nlong) k_spmm_fixup<32><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.nlong, partial, Y, ldy);
      break;
    case 64:
      k_spmm<64><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, s.nchunks, X, ldx, Y, ldy, partial);
      if (s.nlong) k_spmm_fixup<64><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.nlong, partial, Y, ldy);
      break;
    case 128:
      k_spmm<128><<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, s.nchunks, X, ldx, Y, ldy,
                                        partial);
      if (s.nlong) k_spmm_fixup<128><<<gfix, 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.nlong, partial, Y, ldy);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t spmv(const int* ptr, const int* idx, const float* val, int rows, const Schedule& s, const float* y,
                const double* scale_ptr, float* z, float* partial, hipStream_t st) {
  (void)rows;
  if (s.nchunks <= 0) return hipSuccess;
  unsigned grid = (unsigned)((s.nchunks + 3) / 4);
  k_spmv<<<grid, 256, 0, st>>>(ptr, idx, val, s.nch, s.pslot, s.chunk_row, s.nchunks, y, scale_ptr, z, partial);
  if (s.nlong) k_spmv_fixup<<<grid_for(s.nlong, 256), 256, 0, st>>>(s.nch, s.pslot, s.long_rows, s.nlong, partial, z);
  return hipGetLastError();
}

}  // namespace sfd
