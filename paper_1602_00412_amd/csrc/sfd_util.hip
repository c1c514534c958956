// Utility kernels: fills, device-wide exclusive scan, panel copies and the output transpose.
#include <algorithm>

#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_i32(int* p, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the block total.
__device__ int block_exclusive_scan(int v, int* s_wave, int& total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  int before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    int t = s_wave[w];
    if (w < wave) before += t;
    total += t;
  }
  __syncthreads();
  return x - v + before;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* in, int64_t n, int* bsum) {
  __shared__ int s_wave[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) s += in[i];
  }
  int total;
  block_exclusive_scan(s, s_wave, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Single block: exclusive scan of nb block sums in place (looping over tiles with a carry).
__global__ __launch_bounds__(kScanThreads) void k_scan_blocksums(int* bsum, int64_t nb) {
  __shared__ int s_wave[kScanThreads / 64];
  int carry = 0;
  for (int64_t t0 = 0; t0 < nb; t0 += kScanTile) {
    int64_t base = t0 + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      v[k] = i < nb ? bsum[i] : 0;
      s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, s_wave, total) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      if (i < nb) bsum[i] = ex;
      ex += v[k];
    }
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int* in, int* out, int64_t n, const int* boff,
                                                             int64_t nb) {
  __shared__ int s_wave[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int total;
  int ex = block_exclusive_scan(s, s_wave, total) + boff[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
  // the last block also writes the grand total to out[n]
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = boff[blockIdx.x] + total;
  (void)nb;
}

__global__ void k_copy_panel(const float* src, int lds, float* dst, int ldd, int64_t rows, int w) {
  int64_t total = rows * w;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    int64_t r = i / w;
    int c = (int)(i - r * w);
    dst[r * ldd + c] = src[r * lds + c];
  }
}

// out[i][j] = panel[j][i] for i < ell, j < d, through a 64 x 65 LDS tile.
__global__ __launch_bounds__(256) void k_transpose_out(const float* panel, int ld, int64_t d, int ell, float* out) {
  __shared__ float tile[64][65];
  int64_t j0 = (int64_t)blockIdx.x * 64;
  int i0 = blockIdx.y * 64;
  for (int t = threadIdx.x; t < 64 * 64; t += 256) {
    int jj = t / 64, ii = t % 64;  // read along the panel row (consecutive columns)
    int64_t j = j0 + jj;
    int i = i0 + ii;
    tile[jj][ii] = (j < d && i < ell) ? panel[j * ld + i] : 0.f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * 64; t += 256) {
    int ii = t / 64, jj = t % 64;  // write along the output row
    int64_t j = j0 + jj;
    int i = i0 + ii;
    if (j < d && i < ell) out[(int64_t)i * d + j] = tile[jj][ii];
  }
}

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

__global__ void k_to_bf16(const float* __restrict__ src, int64_t n, uint16_t* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t u = __float_as_uint(src[i]);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    dst[i] = (uint16_t)(u >> 16);
  }
}

__global__ void k_set_identity(float* __restrict__ T, int L, int K) {
  const int64_t n = (int64_t)K * L * L;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % ((int64_t)L * L);
    T[e] = (r / L == r % L) ? 1.f : 0.f;
  }
}

// Buffers k of a lockstep group whose SimultaneousIteration ends at the current iteration
// (q[k] == *iter) keep their panel and Gram: Pt_k <- X_k (n floats), Wp_k <- W_k (m doubles).
// Block (x, k) copies its share of buffer k.
__global__ __launch_bounds__(256) void k_group_snapshot(const int* __restrict__ iter, const int* __restrict__ q,
                                                        const float* __restrict__ X, float* __restrict__ Pt,
                                                        const double* __restrict__ W, double* __restrict__ Wp,
                                                        int64_t n, int64_t m) {
  const int k = blockIdx.y;
  if (q[k] != *iter) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n; i += stride) Pt[k * n + i] = X[k * n + i];
  for (int64_t i = i0; i < m; i += stride) Wp[k * m + i] = W[k * m + i];
}

__global__ void k_counter_add(int* c, int v) {
  if (threadIdx.x == 0) *c += v;
}

}  // namespace

hipError_t group_snapshot(const int* iter, const int* q, int K, const float* X, float* Pt, int64_t n, const double* W,
                          double* Wp, int64_t m, hipStream_t st) {
  int64_t nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  k_group_snapshot<<<dim3((unsigned)nb, (unsigned)K), 256, 0, st>>>(iter, q, X, Pt, W, Wp, n, m);
  return hipGetLastError();
}

hipError_t counter_add(int* c, int v, hipStream_t st) {
  k_counter_add<<<1, 64, 0, st>>>(c, v);
  return hipGetLastError();
}

hipError_t set_identity(float* T, int L, int K, hipStream_t st) {
  const int64_t n = (int64_t)K * L * L;
  k_set_identity<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, st>>>(T, L, K);
  return hipGetLastError();
}

hipError_t to_bf16(const float* src, int64_t n, uint16_t* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  k_to_bf16<<<(unsigned)g, 256, 0, st>>>(src, n, dst);
  return hipGetLastError();
}

hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_f32<<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, int64_t n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

int64_t scan_tmp_ints(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t st) {
  if (n <= 0) {
    return fill_i32(out, 1, 0, st);
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  k_scan_reduce<<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, tmp);
  k_scan_blocksums<<<1, kScanThreads, 0, st>>>(tmp, nb);
  k_scan_apply<<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, tmp, nb);
  return hipGetLastError();
}

hipError_t copy_panel(const float* src, int lds, float* dst, int ldd, int64_t rows, int w, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  k_copy_panel<<<grid_for(rows * w, 256), 256, 0, st>>>(src, lds, dst, ldd, rows, w);
  return hipGetLastError();
}

hipError_t transpose_out(const float* panel, int ld, int64_t d, int ell, float* out, hipStream_t st) {
  dim3 grid((unsigned)((d + 63) / 64), (unsigned)((ell + 63) / 64));
  k_transpose_out<<<grid, 256, 0, st>>>(panel, ld, d, ell, out);
  return hipGetLastError();
}

}  // namespace sfd
