// Sparse x dense products of SimultaneousIteration (Alg 1: the factors A' and A'^T of
// A'(A'^T A')^q G) and the matrix-vector products of VerifySpectral (Alg 6).
//
// Work decomposition: a row of the CSR (or CSC) structure is cut into chunks of at most
// kSpmmChunk stored entries, each described by {row, first entry, end entry, partial slot}.
// Short rows are one chunk and are written directly; the chunks of a long row (Zipf-hot
// columns in the CSC) write partial rows that a fix-up pass adds in chunk order, so results do
// not depend on scheduling.  In the dense products an L/VEC-lane group owns one chunk at a time
// and reads each dense row of width L as 16-byte segments (lane s: columns VEC s .. VEC s +
// VEC - 1).
//
// XCD-local pieces (transposed products of large buffers): the gathered panel Y (m x L) is
// larger than one XCD's L2, and a gather of a random row of it runs at the Infinity-Cache /
// HBM rate.  The buffer's rows are cut into one band per XCD, and the hot columns (at least
// hot_min entries) are cut at the band boundaries: the pieces of band b run only on the blocks
// dispatched to XCD b, whose L2 then holds that band's rows of Y.  Short columns would pay
// more for the pieces' partial rows than they save and keep one chunk range for all blocks.
#include <algorithm>
#include <utility>

#include "sfd_internal.h"

namespace sfd {

namespace {

constexpr int64_t kSpmmMaxBlocks = 16384;  // 64 four-wave blocks per CU at most
constexpr int kQueueTicket = 8;            // chunks a group takes from a work queue per atomic

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// chunks per row: one for a short row (also an empty one, whose output row is then written as
// zeros), ceil(len / kSpmmChunk) for a long row
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

// regions[k] = chunk_start[k * span], k = 0 .. nreg (the chunk ranges of a schedule); the work
// queue counters of the ranges start at 0
__global__ void k_sched_regions(const int* chunk_start, int64_t span, int nreg, int* regions, int* queue) {
  const int k = threadIdx.x;
  if (k <= nreg) regions[k] = chunk_start[(int64_t)k * span];
  if (queue && k < kXcdBands + 2) queue[k] = 0;
}

// rb[b] = first row of row band b (b = 0 .. kXcdBands; rb[kXcdBands] = m); row r is in band
// min(kXcdBands - 1, floor(rowptr[r] kXcdBands / nnz)), so the bands are contiguous and hold
// about nnz / kXcdBands entries each (a band may be empty).
__global__ void k_band_rows(const int* rowptr, int m, int nnz, int* rb) {
  auto band_of = [&](int r) {
    const int b = (int)(((int64_t)rowptr[r] * kXcdBands) / nnz);
    return b < kXcdBands - 1 ? b : kXcdBands - 1;
  };
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (; r < m; r += stride) {
    const int br = band_of(r);
    const int bp = r > 0 ? band_of(r - 1) : -1;
    for (int b = bp + 1; b <= br; ++b) rb[b] = r;
    if (r == m - 1)
      for (int b = br + 1; b <= kXcdBands; ++b) rb[b] = m;
  }
}

// first position in [lo, hi) of the ascending rows a[] whose row is >= key
__device__ inline int lower_row(const int* a, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Chunk counts of the CSC with XCD-local pieces: "row" b d + j (b < kXcdBands) holds the chunks
// of hot column j's piece in row band b, "row" kXcdBands d + j those of a short column j (one
// at least, so an empty column is written as zeros).  pslot[j] = partial slots of column j.
__global__ void k_hot_counts(const int* ptr, const int* rowid, int d, int hot_min, const int* rb, int* nch,
                             int* pslot) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (; j < d; j += stride) {
    const int b = ptr[j], e = ptr[j + 1], len = e - b;
    if (len >= hot_min) {
      int lo = b, tot = 0;
      for (int k = 0; k < kXcdBands; ++k) {
        const int hi = k == kXcdBands - 1 ? e : lower_row(rowid, lo, e, rb[k + 1]);
        const int c = (hi - lo + kSpmmChunk - 1) / kSpmmChunk;
        nch[(int64_t)k * d + j] = c;
        tot += c;
        lo = hi;
      }
      nch[(int64_t)kXcdBands * d + j] = 0;
      pslot[j] = tot > 1 ? tot : 0;
    } else {
      for (int k = 0; k < kXcdBands; ++k) nch[(int64_t)k * d + j] = 0;
      const int c = len <= kSpmmChunk ? 1 : (len + kSpmmChunk - 1) / kSpmmChunk;
      nch[(int64_t)kXcdBands * d + j] = c;
      pslot[j] = c > 1 ? c : 0;
    }
  }
}

// Descriptors of the CSC with XCD-local pieces: a hot column's chunks take its partial slots in
// band order, then chunk order (the order the fix-up adds them).
__global__ void k_hot_desc(const int* ptr, const int* rowid, int d, int hot_min, const int* rb,
                           const int* chunk_start, const int* slot_start, int4* desc, int* long_rows,
                           int* counters) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (; j < d; j += stride) {
    const int b = ptr[j], e = ptr[j + 1], len = e - b;
    const int s0 = slot_start[j];
    const bool split = slot_start[j + 1] > s0;  // the column's chunks write partial slots
    if (len >= hot_min) {
      int lo = b, done = 0;
      for (int k = 0; k < kXcdBands; ++k) {
        const int hi = k == kXcdBands - 1 ? e : lower_row(rowid, lo, e, rb[k + 1]);
        const int c0 = chunk_start[(int64_t)k * d + j], c1 = chunk_start[(int64_t)k * d + j + 1];
        for (int c = c0; c < c1; ++c) {
          const int first = lo + (c - c0) * kSpmmChunk;
          desc[c] = make_int4(j, first, min(hi, first + kSpmmChunk), split ? s0 + done + (c - c0) : -1);
        }
        done += c1 - c0;
        lo = hi;
      }
    } else {
      const int64_t v = (int64_t)kXcdBands * d + j;
      const int c0 = chunk_start[v], c1 = chunk_start[v + 1];
      for (int c = c0; c < c1; ++c) {
        const int first = b + (c - c0) * kSpmmChunk;
        desc[c] = make_int4(j, first, min(e, first + kSpmmChunk), split ? s0 + (c - c0) : -1);
      }
    }
    if (split) long_rows[atomicAdd(&counters[0], 1)] = j;
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
// ids from the lanes that loaded them and gather their dense row segments.  A lane whose columns
// are all past the sketch's ell (live == false) holds zeros in every panel row: it reads segment 0
// of the row instead (a sector the group's first lane fetches anyway), so the row's tail sectors
// are never fetched and no load sits behind a branch; what it sums is discarded when its output
// is stored (zeros in its place).
// STAGE: an id c < 0 names row -1 - c of the rows staged in LDS (hot, pitch LPR segments).
template <int LPR, int U, int T0, bool BF, bool STAGE>
__device__ inline void gather_load(int ci, const typename Seg<BF>::raw* __restrict__ Xs, int lds, int sub, bool live,
                                   const typename Seg<BF>::raw* hot, typename Seg<BF>::raw* x) {
  int c[U];
  [&]<int... u>(std::integer_sequence<int, u...>) {
    ((c[u] = bcast_i<LPR, T0 + u>(ci)), ...);
  }(std::make_integer_sequence<int, U>{});
  const int s = live ? sub : 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (STAGE)
      x[u] = c[u] < 0 ? hot[(-1 - c[u]) * LPR + sub] : Xs[(int64_t)c[u] * lds + s];
    else
      x[u] = Xs[(int64_t)c[u] * lds + s];
  }
}

// ... and add them: acc += value * segment, in entry order
template <int LPR, int U, int T0, bool BF>
__device__ inline void gather_add(float vi, const typename Seg<BF>::raw* x, float* acc) {
  float v[U];
  [&]<int... u>(std::integer_sequence<int, u...>) {
    ((v[u] = bcast_f<LPR, T0 + u>(vi)), ...);
  }(std::make_integer_sequence<int, U>{});
#pragma unroll
  for (int u = 0; u < U; ++u) Seg<BF>::fma(v[u], x[u], acc);
}

template <int LPR, int U, int T0, bool BF, bool STAGE>
__device__ inline void gather_block(int ci, float vi, const typename Seg<BF>::raw* __restrict__ Xs, int lds, int sub,
                                    bool live, const typename Seg<BF>::raw* hot, float* acc) {
  typename Seg<BF>::raw x[U];
  gather_load<LPR, U, T0, BF, STAGE>(ci, Xs, lds, sub, live, hot, x);
  gather_add<LPR, U, T0, BF>(vi, x, acc);
}

// Y[r, :] = sum_k val[k] X[idx[k], :] over the chunk descriptors [c0, c1): this lane's group
// takes chunks c0 + first, + stride, ...  A group of L/VEC lanes owns a chunk at a time (lane s
// holds columns VEC s .. VEC s + VEC - 1) and walks it in blocks of L/VEC entries: lane s of the
// group loads entry s of the block (coalesced), then the entries are broadcast inside the group
// and their dense row segments gathered.  The next chunk's descriptor is loaded a chunk ahead and
// the next block's ids and values right after the current block's first gathers, so their
// latency overlaps the gathers instead of adding to them.
// Output: a whole row goes to out[r], the chunks of a long row to their FP32 partial slots (the
// fix-up adds them in slot order).  VB: the stored values are BF16 (the precision form's products
// 1 .. 2q+1), widened to FP32 exactly.
template <bool VB>
__device__ inline float load_val(const void* __restrict__ val, int q) {
  if constexpr (VB)
    return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(val)[q] << 16);
  else
    return reinterpret_cast<const float*>(val)[q];
}

// QUEUE: the group takes its chunks from a work queue (the counter *queue of the range; the
// group's first lane takes a ticket of kQueueTicket consecutive chunks per atomic, since one
// counter serves every group of the grid) instead of first, first + stride, ...; the group holds
// one chunk ahead, so the descriptor of the next chunk is loaded before the current one's gathers
// either way.
template <int L, int U, bool BIN, bool BOUT, bool VB, bool QUEUE, bool STAGE>
__device__ __forceinline__ void spmm_range(const int4* __restrict__ desc, int64_t c0, int64_t c1, int64_t first,
                                           int64_t stride, int* __restrict__ queue, const int* __restrict__ idx,
                                           const void* __restrict__ val, const void* __restrict__ X, int ldx,
                                           void* __restrict__ out, int ldo, float* __restrict__ partial,
                                           const typename Seg<BIN>::raw* hot, int nlive) {
  using S = Seg<BIN>;
  constexpr int VEC = S::VEC;
  constexpr int LPR = L / VEC;  // lanes per group
  const int sub = (threadIdx.x & 63) % LPR;
  const bool live = sub < nlive;  // this lane's columns reach below ell
  const typename S::raw* Xs = reinterpret_cast<const typename S::raw*>(X);
  const int lds = ldx / VEC;  // row pitch in segments
  const size_t out_row_bytes = (size_t)ldo * (BOUT ? 2 : 4);
  // the group's next chunk: from its current ticket or a new one (the first lane takes it, the
  // group shares it), or the next of the static sequence
  int64_t tk_next = 0, tk_end = 0;
  auto next_chunk = [&](int64_t cur) -> int64_t {
    if constexpr (QUEUE) {
      if (tk_next >= tk_end) {
        int t = 0;
        if (sub == 0) t = atomicAdd(queue, kQueueTicket);
        tk_next = c0 + bcast_i<LPR, 0>(t);
        tk_end = tk_next + kQueueTicket;
      }
      return tk_next++;
    } else {
      return cur + stride;
    }
  };
  int64_t cc = QUEUE ? next_chunk(0) : c0 + first;
  int4 dc = cc < c1 ? desc[cc] : make_int4(0, 0, 0, -1);
  int64_t ncc = cc < c1 ? next_chunk(cc) : c1;
  int4 dn = ncc < c1 ? desc[ncc] : make_int4(0, 0, 0, -1);
  int p = dc.y;
  int ci = 0;
  float vi = 0.f;
  if (cc < c1 && p + sub < dc.z) {
    ci = idx[p + sub];
    vi = load_val<VB>(val, p + sub);
  }
  float acc[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) acc[q] = 0.f;
  while (cc < c1) {
    // where the next block starts: later in this chunk, or at the group's next chunk
    const bool same = p + LPR < dc.z;
    const int np = same ? p + LPR : dn.y;
    const int nend = same ? dc.z : dn.z;
    // entries beyond the chunk have id 0 and value 0.  The block's first U entries are gathered
    // whatever its length (an empty row's chunk adds zeros: 0 times a row of X); then the next
    // block's ids and values are loaded, after those gathers, so the wait for the gathers does
    // not also wait for these loads; they load unconditionally, from the descriptors for an
    // entry past the end (then taken as id 0, value 0), so the waits count them exactly.
    typename Seg<BIN>::raw x0[U];
    gather_load<LPR, U, 0, BIN, STAGE>(ci, Xs, lds, sub, live, hot, x0);
    const bool nok = (same || ncc < c1) && np + sub < nend;
    const char* const ip = nok ? reinterpret_cast<const char*>(idx + (np + sub)) : reinterpret_cast<const char*>(desc);
    const char* const vp = nok ? reinterpret_cast<const char*>(val) + (size_t)(np + sub) * (VB ? 2 : 4)
                               : reinterpret_cast<const char*>(desc);
    int ci2 = *reinterpret_cast<const int*>(ip);
    float vi2 = load_val<VB>(vp, 0);
    ci2 = nok ? ci2 : 0;
    vi2 = nok ? vi2 : 0.f;
    gather_add<LPR, U, 0, BIN>(vi, x0, acc);
    // the block's other U-blocks: whole U-blocks past the chunk's end are skipped
    const int cnt = min(LPR, dc.z - p);
    [&]<int... b>(std::integer_sequence<int, b...>) {
      ((cnt > (b + 1) * U ? gather_block<LPR, U, (b + 1) * U, BIN, STAGE>(ci, vi, Xs, lds, sub, live, hot, acc)
                          : void()),
       ...);
    }(std::make_integer_sequence<int, LPR / U - 1>{});
    if (!same) {
      float o[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) o[q] = live ? acc[q] : 0.f;
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
      ncc = cc < c1 ? next_chunk(cc) : c1;
      dn = ncc < c1 ? desc[ncc] : make_int4(0, 0, 0, -1);
    }
    p = np;
    ci = ci2;
    vi = vi2;
  }
}

// The product over a schedule's chunk ranges.  nlocal = 0: every block walks [regions[0],
// regions[1]).  nlocal = kXcdBands: a block first walks the pieces of its XCD's row band
// (range blockIdx % nlocal, shared with the other blocks of that XCD), then its share of the
// short columns' range (range nlocal, shared with all blocks); gridDim.x is a multiple of nlocal.
// QUEUE: a persistent grid (a few blocks per CU) whose groups take chunks from the ranges' work
// queues (queue[range]); otherwise a grid of about four chunks per group walked statically.
// Either way each chunk is summed by one group in entry order, so the results are the same bits.
// STAGE (products Y = A' X with a queue grid): each block first copies the input rows of the
// buffer's most popular columns (hot_cols[0 .. *hot_n), at most kStageBytes of them) to LDS; idx
// then holds -1 - slot for the entries of those columns (the staged encoding of the column ids).
constexpr int kStageBytes = 32768;

template <int L, bool BIN>
constexpr int stage_rows() {
  return kStageBytes / (L * (BIN ? 2 : 4));
}

template <int L, int U, bool TRANSPOSED, bool BIN, bool BOUT, bool VB, bool QUEUE, bool STAGE>
__global__ __launch_bounds__(256) void k_spmm(const int4* __restrict__ desc, const int* __restrict__ regions,
                                              int nlocal, int* __restrict__ queue, const int* __restrict__ idx,
                                              const void* __restrict__ val, const void* __restrict__ X, int ldx,
                                              void* __restrict__ out, int ldo, float* __restrict__ partial,
                                              const int* __restrict__ hot_cols, const int* __restrict__ hot_n,
                                              int nlive) {
  using raw = typename Seg<BIN>::raw;
  constexpr int LPR = L / Seg<BIN>::VEC;
  constexpr int G = 64 / LPR;  // groups per wave
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane / LPR;
  __shared__ raw hot[STAGE ? stage_rows<L, BIN>() * LPR : 1];
  if constexpr (STAGE) {
    const int nh = min(*hot_n, stage_rows<L, BIN>());
    const raw* Xs = reinterpret_cast<const raw*>(X);
    const int lds = ldx / Seg<BIN>::VEC;
    for (int i = threadIdx.x; i < nh * LPR; i += 256) hot[i] = Xs[(int64_t)hot_cols[i / LPR] * lds + i % LPR];
    __syncthreads();
  }
  if (nlocal > 0) {
    const int band = blockIdx.x % nlocal;
    const int64_t slot = blockIdx.x / nlocal;
    spmm_range<L, U, BIN, BOUT, VB, QUEUE, STAGE>(desc, regions[band], regions[band + 1], (slot * 4 + wave) * G + grp,
                                                  (int64_t)(gridDim.x / nlocal) * 4 * G, queue + band, idx, val, X,
                                                  ldx, out, ldo, partial, hot, nlive);
  }
  spmm_range<L, U, BIN, BOUT, VB, QUEUE, STAGE>(desc, regions[nlocal], regions[nlocal + 1],
                                                ((int64_t)blockIdx.x * 4 + wave) * G + grp, (int64_t)gridDim.x * 4 * G,
                                                queue + nlocal, idx, val, X, ldx, out, ldo, partial, hot, nlive);
}

// One block per long row (rows whose chunks went to partial slots: long rows and XCD-local
// pieces; a Zipf-hot column of a 5 * 10^6-entry buffer has over a thousand): wave w adds the
// slots w, w + 4, w + 8, ... of each column, eight of them in flight at once (slot w + 4 i into
// sum i % 8); the eight sums are added as a fixed tree, then the four wave sums in wave order.
// The order is fixed, so results do not depend on scheduling.
// The product's work queues are cleared here for the next product over the schedule (the
// product has completed: the fix-up runs after it on the same stream).
template <int L, bool BOUT>
__global__ __launch_bounds__(256) void k_spmm_fixup(const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, const int* __restrict__ nlong_ptr,
                                                    const float* __restrict__ partial, void* __restrict__ Y,
                                                    int ldy, int* __restrict__ queue) {
  constexpr int CPL = (L + 63) / 64;  // columns per lane
  constexpr int ILP = 8;              // slots in flight per wave
  __shared__ float red[4][L];
  if (queue && blockIdx.x == 0 && threadIdx.x < kXcdBands + 2) queue[threadIdx.x] = 0;
  const int nlong = *nlong_ptr;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int li = blockIdx.x; li < nlong; li += gridDim.x) {
    const int r = long_rows[li];
    const int s0 = slot_start[r];
    const int n = slot_start[r + 1] - s0;
    const float* base = partial + (int64_t)s0 * L;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      if (col >= L) continue;
      const float* pc = base + col;
      float a[ILP];
#pragma unroll
      for (int k = 0; k < ILP; ++k) a[k] = 0.f;
      int j = wave;
      for (; j + 4 * (ILP - 1) < n; j += 4 * ILP) {
#pragma unroll
        for (int k = 0; k < ILP; ++k) a[k] += pc[(int64_t)(j + 4 * k) * L];
      }
#pragma unroll
      for (int k = 0; k < ILP - 1; ++k)
        if (j + 4 * k < n) a[k] += pc[(int64_t)(j + 4 * k) * L];
      red[wave][col] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
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

// Four chunks per wave, one per 16-lane group; a group strides its chunk's entries (lane s takes
// s, s + 16, ...) and reduces with a 16-lane xor tree.
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
  // the lane's entries p, p + 16, ... of a chunk in rounds of four: a round's ids and values are
  // loaded together, then its four gathers, then the products are added in entry order.  A wave
  // takes four chunks at a time (one per group) and loads the descriptors and the first round of
  // its next four before the current ones are reduced and stored.
  auto load_round = [&](int p, int end, int* c, float* v) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool in = p + 16 * k < end;
      c[k] = in ? idx[p + 16 * k] : 0;
      v[k] = in ? val[p + 16 * k] : 0.f;
    }
  };
  auto add_round = [&](int p, int end, const int* c, const float* v, float& acc) {
    float yv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) yv[k] = p + 16 * k < end ? y[c[k]] : 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (p + 16 * k < end) acc = fmaf(v[k], yv[k], acc);
  };
  int64_t base = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * 4;
  int4 dc = base + grp < nchunks ? desc[base + grp] : make_int4(0, 0, 0, -1);
  int c[4];
  float v[4];
  load_round(dc.y + sub, dc.z, c, v);
  for (; base < nchunks; base += nwaves * 4) {
    const int64_t nb = base + nwaves * 4;
    const int4 dn = nb + grp < nchunks ? desc[nb + grp] : make_int4(0, 0, 0, -1);
    float acc = 0.f;
    add_round(dc.y + sub, dc.z, c, v, acc);
    for (int p = dc.y + sub + 64; p < dc.z; p += 64) {
      int c2[4];
      float v2[4];
      load_round(p, dc.z, c2, v2);
      add_round(p, dc.z, c2, v2, acc);
    }
    load_round(dn.y + sub, dn.z, c, v);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (base + grp < nchunks && sub == 0) {
      float scale = scale1;
      if (scale_ptr && seg_rows) {
        int lo = 0, hi = K;  // last k with seg_rows[k] <= row
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (seg_rows[mid] <= dc.x) lo = mid; else hi = mid;
        }
        scale = (float)scale_ptr[(int64_t)lo * sstride];
      }
      const float val_out = acc * scale;
      if (dc.w < 0)
        z[dc.x] = val_out;
      else
        partial[dc.w] = val_out;
    }
    dc = dn;
  }
}

// One wave per long row: lane j adds partials j, j + 64, ...; then an xor-tree over the wave.
__global__ __launch_bounds__(256) void k_spmv_fixup(const int* __restrict__ slot_start,
                                                    const int* __restrict__ long_rows, const int* __restrict__ nlong_ptr,
                                                    const float* __restrict__ partial, float* __restrict__ z) {
  const int nlong = *nlong_ptr;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t ii = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; ii < nlong; ii += nwaves) {
    const int i = (int)ii;
    const int r = long_rows[i];
    const int n = slot_start[r + 1] - slot_start[r];
    const int s0 = slot_start[r];
    float s = 0.f;
    for (int j = lane; j < n; j += 64) s += partial[s0 + j];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) z[r] = s;
  }
}

// ---- rows staged in LDS for the products Y = A' X: the buffer's most popular columns
// hist[b] = columns whose entry count lies in [2^b, 2^(b+1))
__global__ void k_stage_hist(const int* __restrict__ cscptr, int d, int* __restrict__ hist) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d; c += gridDim.x * blockDim.x) {
    const int len = cscptr[c + 1] - cscptr[c];
    if (len >= 2) atomicAdd(&hist[31 - __clz(len)], 1);
  }
}

// the count threshold 2^b: the columns from the top bin down whose total stays within cap;
// hot_n[0] = 0 (filled by k_stage_slots), hot_n[1] = threshold (INT_MAX: none)
__global__ void k_stage_threshold(const int* __restrict__ hist, int cap, int* __restrict__ hot_n) {
  if (threadIdx.x != 0) return;
  int cum = 0, tau = 0x7FFFFFFF;
  for (int b = 31; b >= 1; --b) {
    if (cum + hist[b] > cap) break;
    cum += hist[b];
    if (hist[b] > 0) tau = 1 << b;
  }
  hot_n[0] = 0;
  hot_n[1] = tau;
}

// slot_of[c] = the LDS slot of column c (-1: not staged), hot_cols[slot] = c (slot order is that
// of the atomics; it only places rows in LDS, the products' sums do not depend on it)
__global__ void k_stage_slots(const int* __restrict__ cscptr, int d, int* __restrict__ hot_n,
                              int* __restrict__ hot_cols, int* __restrict__ slot_of) {
  const int tau = hot_n[1];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d; c += gridDim.x * blockDim.x) {
    const int len = cscptr[c + 1] - cscptr[c];
    int slot = -1;
    if (len >= tau) {
      slot = atomicAdd(&hot_n[0], 1);
      hot_cols[slot] = c;
    }
    slot_of[c] = slot;
  }
}

// enc[k] = -1 - slot of a staged column, else the column id
__global__ void k_stage_encode(const int* __restrict__ colidx, int64_t nnz, const int* __restrict__ slot_of,
                               int* __restrict__ enc) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    const int c = colidx[k];
    const int s = slot_of[c];
    enc[k] = s >= 0 ? -1 - s : c;
  }
}

int device_cus() {
  static int cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

template <int L, int U, bool BIN, bool BOUT, bool VB, bool QUEUE, bool STAGE = false>
void launch_spmm(const Schedule& s, const int* idx, const void* val, const void* X, int ldx, void* out, int ldo,
                 float* partial, int occupancy, int nlive, hipStream_t st) {
  constexpr int G = 64 / (L / Seg<BIN>::VEC);
  // static: about four chunks per group (finished blocks make room for waiting ones, which
  // balances uneven chunks); queue: `occupancy` blocks per CU at most.  A multiple of the XCD
  // count when the schedule has XCD-local pieces.
  int64_t grid = ((int64_t)s.max_chunks + 16 * G - 1) / (16 * G);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, kSpmmMaxBlocks));
  if (QUEUE) grid = std::min<int64_t>(grid, (int64_t)device_cus() * std::max(occupancy, 1));
  if (s.nlocal > 0) grid = (grid + s.nlocal - 1) / s.nlocal * s.nlocal;
  // TRANSPOSED (CSC products) only gives the two products different kernel names
  if (s.transposed)
    k_spmm<L, U, true, BIN, BOUT, VB, QUEUE, false><<<(unsigned)grid, 256, 0, st>>>(
        s.desc, s.regions, s.nlocal, s.queue, idx, val, X, ldx, out, ldo, partial, nullptr, nullptr, nlive);
  else
    k_spmm<L, U, false, BIN, BOUT, VB, QUEUE, STAGE><<<(unsigned)grid, 256, 0, st>>>(
        s.desc, s.regions, s.nlocal, s.queue, STAGE ? s.stage_idx : idx, val, X, ldx, out, ldo, partial, s.hot_cols,
        s.hot_n, nlive);
}

template <int L, int U, bool BIN, bool BOUT, bool VB>
void launch_spmm_cfg(const Schedule& s, const int* idx, const void* val, const void* X, int ldx, void* out, int ldo,
                     float* partial, const SpmmConfig& cfg, hipStream_t st) {
  constexpr int LPR = L / Seg<BIN>::VEC;
  const int nlive = cfg.live > 0 && cfg.live < LPR ? cfg.live : LPR;
  if (cfg.queue && cfg.stage)
    launch_spmm<L, U, BIN, BOUT, VB, true, true>(s, idx, val, X, ldx, out, ldo, partial, cfg.occupancy, nlive, st);
  else if (cfg.queue)
    launch_spmm<L, U, BIN, BOUT, VB, true>(s, idx, val, X, ldx, out, ldo, partial, cfg.occupancy, nlive, st);
  else
    launch_spmm<L, U, BIN, BOUT, VB, false>(s, idx, val, X, ldx, out, ldo, partial, 0, nlive, st);
}

template <int L>
hipError_t spmm_l(const Schedule& s, const int* idx, const void* val, bool vb, const void* X, PanelType xt, int ldx,
                  void* Y, PanelType yt, int ldy, float* partial, const SpmmConfig& cfg, hipStream_t st) {
  const bool xb = xt == PanelType::BF16, yb = yt == PanelType::BF16;
  // FP32 form: FP32 values and panels (entries gathered in batches of 8, or 4).  Precision form:
  // BF16 values and panels in the products 1 .. 2q+1, FP32 values and output in the last
  // (P^T = A'^T Y); batches of 4
  if (!xb && !yb && !vb) {
    if (cfg.unroll == 4)
      launch_spmm_cfg<L, 4, false, false, false>(s, idx, val, X, ldx, Y, ldy, partial, cfg, st);
    else
      launch_spmm_cfg<L, 8, false, false, false>(s, idx, val, X, ldx, Y, ldy, partial, cfg, st);
  } else if (xb && yb && vb) {
    launch_spmm_cfg<L, 4, true, true, true>(s, idx, val, X, ldx, Y, ldy, partial, cfg, st);
  } else if (xb && !yb && !vb) {
    launch_spmm_cfg<L, 4, true, false, false>(s, idx, val, X, ldx, Y, ldy, partial, cfg, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// blocks of the fix-up: a block per long row, striding over the rows
constexpr unsigned kFixupBlocks = 1024;

template <int L>
void launch_fixup(const Schedule& s, float* partial, void* Y, bool yb, int ldy, hipStream_t st) {
  if (yb)
    k_spmm_fixup<L, true><<<kFixupBlocks, 256, 0, st>>>(s.pslot, s.long_rows, s.counters, partial, Y, ldy, s.queue);
  else
    k_spmm_fixup<L, false><<<kFixupBlocks, 256, 0, st>>>(s.pslot, s.long_rows, s.counters, partial, Y, ldy,
                                                         s.queue);
}

}  // namespace

hipError_t schedule_build(const int* ptr, int rows, Schedule& s, int* scan_tmp, hipStream_t st) {
  hipError_t e;
  if (rows > 0) k_sched_counts<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.nch, s.pslot);
  if ((e = scan_exclusive(s.nch, s.nch, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(s.pslot, s.pslot, rows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = fill_i32(s.counters, 1, 0, st)) != hipSuccess) return e;
  if (rows > 0)
    k_sched_desc<<<grid_for(rows, 256, 8192), 256, 0, st>>>(ptr, rows, s.nch, s.pslot, s.desc, s.long_rows,
                                                             s.counters);
  k_sched_regions<<<1, 64, 0, st>>>(s.nch, rows, 1, s.regions, s.queue);
  s.rows = rows;
  s.nlocal = 0;
  return hipGetLastError();
}

hipError_t stage_build(const int* cscptr, int d, const int* colidx, int64_t nnz, int L, bool bf16, Schedule& s,
                       hipStream_t st) {
  if (!s.stage_idx || !s.hot_cols || !s.hot_n || !s.slot_of) return hipErrorInvalidValue;
  const int cap = kStageBytes / (L * (bf16 ? 2 : 4));
  hipError_t e;
  if ((e = fill_i32(s.hot_n + 2, 32, 0, st)) != hipSuccess) return e;
  k_stage_hist<<<grid_for(d, 256, 4096), 256, 0, st>>>(cscptr, d, s.hot_n + 2);
  k_stage_threshold<<<1, 64, 0, st>>>(s.hot_n + 2, cap, s.hot_n);
  k_stage_slots<<<grid_for(d, 256, 4096), 256, 0, st>>>(cscptr, d, s.hot_n, s.hot_cols, s.slot_of);
  k_stage_encode<<<grid_for(nnz, 256, 16384), 256, 0, st>>>(colidx, nnz, s.slot_of, s.stage_idx);
  return hipGetLastError();
}

hipError_t schedule_build_hot(const int* cscptr, const int* cscrow, int d, const int* rowptr, int m, int nnz,
                              int hot_min, Schedule& s, int* scan_tmp, hipStream_t st) {
  if (d <= 0 || m <= 0 || nnz <= 0 || hot_min < 1) return hipErrorInvalidValue;
  hipError_t e;
  const int64_t vrows = (int64_t)(kXcdBands + 1) * d;
  // the band boundaries live in the regions array until the regions are written last
  int* rb = s.regions;
  k_band_rows<<<grid_for(m, 256, 8192), 256, 0, st>>>(rowptr, m, nnz, rb);
  k_hot_counts<<<grid_for(d, 256, 8192), 256, 0, st>>>(cscptr, cscrow, d, hot_min, rb, s.nch, s.pslot);
  if ((e = scan_exclusive(s.nch, s.nch, vrows, scan_tmp, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(s.pslot, s.pslot, d, scan_tmp, st)) != hipSuccess) return e;
  if ((e = fill_i32(s.counters, 1, 0, st)) != hipSuccess) return e;
  k_hot_desc<<<grid_for(d, 256, 8192), 256, 0, st>>>(cscptr, cscrow, d, hot_min, rb, s.nch, s.pslot, s.desc,
                                                      s.long_rows, s.counters);
  k_sched_regions<<<1, 64, 0, st>>>(s.nch, d, kXcdBands + 1, s.regions, s.queue);
  s.rows = d;
  s.nlocal = kXcdBands;
  return hipGetLastError();
}

hipError_t spmm(const Schedule& s, const int* idx, const void* val, bool val_bf16, const void* X, PanelType xt, int ldx,
                void* Y, PanelType yt, int ldy, int L, float* partial, const SpmmConfig& cfg, hipStream_t st) {
  if (cfg.queue && !s.queue) return hipErrorInvalidValue;
  if (cfg.stage && (!cfg.queue || s.transposed || !s.stage_idx || !s.hot_cols || !s.hot_n)) return hipErrorInvalidValue;
  if (L == 32) return spmm_l<32>(s, idx, val, val_bf16, X, xt, ldx, Y, yt, ldy, partial, cfg, st);
  if (L == 64) return spmm_l<64>(s, idx, val, val_bf16, X, xt, ldx, Y, yt, ldy, partial, cfg, st);
  if (L == 128) return spmm_l<128>(s, idx, val, val_bf16, X, xt, ldx, Y, yt, ldy, partial, cfg, st);
  if (L == 256) return spmm_l<256>(s, idx, val, val_bf16, X, xt, ldx, Y, yt, ldy, partial, cfg, st);
  return hipErrorInvalidValue;
}

int live_segments(int ell, int elem_bytes) {
  const int bytes = (ell * elem_bytes + 63) / 64 * 64;
  return bytes / 16;
}

hipError_t spmm_queue_reset(const Schedule& s, hipStream_t st) {
  if (!s.queue) return hipSuccess;
  return fill_i32(s.queue, kXcdBands + 2, 0, st);
}

hipError_t spmm_finish(const Schedule& s, float* partial, void* Y, PanelType yt, int ldy, int L, hipStream_t st) {
  const bool yb = yt == PanelType::BF16;
  if (L == 32) {
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
  // every chunk of the schedule, in descriptor order: [regions[0], regions[nlocal + 1])
  const int* nchunks = s.regions + s.nlocal + 1;
  // about eight chunks per group of 16 lanes (16 groups per block)
  int64_t g = ((int64_t)s.max_chunks + 127) / 128;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  k_spmv<<<(unsigned)g, 256, 0, st>>>(s.desc, nchunks, idx, val, y, scale_ptr, z, partial, seg_rows, K, sstride);
  k_spmv_fixup<<<64, 256, 0, st>>>(s.pslot, s.long_rows, s.counters, partial, z);
  return hipGetLastError();
}

}  // namespace sfd
