// Deterministic device primitives: exclusive scan, stable LSD radix sort,
// stream compaction.
#include "prims.hpp"

namespace hef {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(const int32_t *in, int32_t *out, int32_t *tile_sums, int64_t n) {
  __shared__ int32_t sh[kScanThreads];
  const int tid = threadIdx.x;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(tid) * kScanItems;
  int32_t v[kScanItems];
  int32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int32_t t = (base + i < n) ? in[base + i] : 0;
    v[i] = sum;
    sum += t;
  }
  sh[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t x = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  const int32_t excl = sh[tid] - sum;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] = v[i] + excl;
  if (tid == kScanThreads - 1) tile_sums[blockIdx.x] = sh[tid];
}

// One block scans the tile sums in place (exclusive) and writes the total.
__global__ void __launch_bounds__(1024)
k_scan_sums(int32_t *sums, int64_t ntiles, int32_t *total) {
  __shared__ int32_t sh[1024];
  __shared__ int32_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < ntiles; c0 += 1024) {
    int64_t i = c0 + tid;
    int32_t v = i < ntiles ? sums[i] : 0;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int32_t x = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += x;
      __syncthreads();
    }
    if (i < ntiles) sums[i] = carry + sh[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(int32_t *out, const int32_t *tile_off, int64_t n) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  const int32_t add = tile_off[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    int64_t j = base + i;
    if (j < n) out[j] += add;
  }
}

// Adds to every item of tile t the sum of the tiles before it, a block
// reduction over tile_sums[0, t) (integer sums, so the order does not
// matter); the last tile's block also writes the total to out[n].  Up to
// kFinishTiles tiles this replaces the two kernels above: re-reading the
// earlier sums (at most kFinishTiles^2 / 2 reads, from L2) costs less than a
// launch.
constexpr int64_t kFinishTiles = 2048;
__global__ void __launch_bounds__(kScanThreads)
k_scan_finish(int32_t *out, const int32_t *tile_sums, int64_t n, int64_t ntiles) {
  __shared__ int32_t red[kScanThreads / 64];
  const int tid = threadIdx.x;
  const int64_t t = blockIdx.x;
  int32_t acc = 0;
  for (int64_t j = tid; j < t; j += kScanThreads) acc += tile_sums[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  int32_t add = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) add += red[w];
  const int64_t base = t * kScanTile;
  for (int i = tid; i < kScanTile; i += kScanThreads) {
    const int64_t q = base + i;
    if (q < n) out[q] += add;
  }
  if (t == ntiles - 1 && tid == 0) out[n] = add + tile_sums[t];
}

constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 16;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;

__global__ void __launch_bounds__(kRadixThreads)
k_radix_hist(const uint32_t *keys, int64_t n, int shift, int32_t *hist, int nblocks) {
  __shared__ int32_t cnt[kBins];
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRadixTile;
  for (int r = 0; r < kRadixRounds; ++r) {
    int64_t i = base + int64_t(r) * kRadixThreads + tid;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kBins - 1)], 1);
  }
  __syncthreads();
  hist[int64_t(tid) * nblocks + blockIdx.x] = cnt[tid];
}

// The histogram scan folded into the scatter: when the histogram has at most
// kRadixScanTiles scan tiles, it is scanned within tiles only (k_scan_tiles)
// and each scatter block adds the tile prefixes itself, from an exclusive
// scan of the tile sums in LDS (each thread takes a run of kTileRun sums).
constexpr int kTileRun = 8;
constexpr int kRadixScanTiles = kRadixThreads * kTileRun;

// Each block re-reads its tile and places every item at
// offset[digit][block] + (items of the same digit earlier in the tile).
// offs holds the exclusive scan of the histogram (digit-major), or with
// tile_sums given its scan within scan tiles, to which the block adds the
// sum of the scan tiles before each entry's.
__global__ void __launch_bounds__(kRadixThreads)
k_radix_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                uint32_t *vout, int64_t n, int shift, const int32_t *offs, int nblocks,
                const int32_t *tile_sums, int ntiles) {
  __shared__ int32_t base_cnt[kBins];
  __shared__ int32_t wcnt[kRadixThreads / 64][kBins];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t hidx = int64_t(tid) * nblocks + blockIdx.x;
  base_cnt[tid] = offs[hidx];
  if (tile_sums) {
    // exclusive prefix of the tile sums: a run of kTileRun per thread, a
    // scan of the run totals (in wcnt[0], free until the rounds below),
    // then each run's prefixes
    __shared__ int32_t tpre[kRadixScanTiles];
    int32_t run[kTileRun];
    int32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kTileRun; ++q) {
      const int t = tid * kTileRun + q;
      run[q] = tot;
      tot += t < ntiles ? tile_sums[t] : 0;
    }
    wcnt[0][tid] = tot;
    __syncthreads();
    for (int off = 1; off < kRadixThreads; off <<= 1) {
      const int32_t x = tid >= off ? wcnt[0][tid - off] : 0;
      __syncthreads();
      wcnt[0][tid] += x;
      __syncthreads();
    }
    const int32_t before = wcnt[0][tid] - tot;
#pragma unroll
    for (int q = 0; q < kTileRun; ++q) tpre[tid * kTileRun + q] = before + run[q];
    __syncthreads();
    base_cnt[tid] += tpre[hidx / kScanTile];
  }
  const int64_t base = int64_t(blockIdx.x) * kRadixTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRadixRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kRadixThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t i = base + int64_t(r) * kRadixThreads + tid;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t d = (k >> shift) & (kBins - 1);
    uint64_t peer = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peer &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peer & lt);
    if (valid && rank == 0) wcnt[wv][d] = __popcll(peer);
    __syncthreads();
    if (valid) {
      int32_t pos = base_cnt[d] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = vin[i];
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < kRadixThreads / 64; ++w) add += wcnt[w][tid];
    base_cnt[tid] += add;
    __syncthreads();
  }
}

__global__ void k_compact(const int32_t *flag, const int32_t *pos, int32_t *idx_out,
                          int32_t *count_dev, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) idx_out[pos[i]] = int32_t(i);
  if (i == 0) *count_dev = pos[n];
}

// 256 threads = 8 columns x 32 row lanes.
__global__ void __launch_bounds__(256)
k_reduce_cols(const double *__restrict__ in0, int64_t nrows0, double *__restrict__ out0,
              const double *__restrict__ in1, int64_t nrows1, double *__restrict__ out1,
              int64_t nbc, int64_t ncols) {
  __shared__ double red[32][9];
  // workgroups [0, nbc) reduce side 0, the rest side 1
  const bool second = int64_t(blockIdx.x) >= nbc;
  const double *__restrict__ in = second ? in1 : in0;
  const int64_t nrows = second ? nrows1 : nrows0;
  double *__restrict__ out = second ? out1 : out0;
  const int cl = threadIdx.x & 7, rl = threadIdx.x >> 3;
  const int64_t c = (int64_t(blockIdx.x) - (second ? nbc : 0)) * 8 + cl;
  // eight independent loads in flight per row lane
  double acc[8] = {};
  if (c < ncols) {
    int64_t r = rl;
    for (; r + 7 * 32 < nrows; r += 8 * 32) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = in[(r + 32 * q) * ncols + c];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += t[q];
    }
#pragma unroll
    for (int q = 0; q < 7; ++q)
      if (r + 32 * q < nrows) acc[q] += in[(r + 32 * q) * ncols + c];
  }
  red[rl][cl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  for (int off = 16; off > 0; off >>= 1) {
    if (rl < off) red[rl][cl] += red[rl + off][cl];
    __syncthreads();
  }
  if (rl == 0 && c < ncols) out[c] = red[0][cl];
}

// 4-byte words when the pointer and the size allow it, else bytes.
__global__ void k_zero_words(uint32_t *p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

__global__ void k_zero_bytes(uint8_t *p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

__global__ void k_flag_copy(const int32_t *flag, int32_t *out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = flag[i] ? 1 : 0;
}

}  // namespace

hef_status zero_async(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return HEF_OK;
  const bool words = ((reinterpret_cast<uintptr_t>(p) | bytes) & 3) == 0;
  const int64_t n = int64_t(words ? bytes / 4 : bytes);
  const int64_t nb = std::min<int64_t>(cdiv(n, 256), 4096);
  if (words)
    k_zero_words<<<nb, 256, 0, s>>>(static_cast<uint32_t *>(p), n);
  else
    k_zero_bytes<<<nb, 256, 0, s>>>(static_cast<uint8_t *>(p), n);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status reduce_cols_f64(const double *in, int64_t nrows, int64_t ncols, double *out,
                           hipStream_t s) {
  if (ncols <= 0) return HEF_OK;
  k_reduce_cols<<<cdiv(ncols, 8), 256, 0, s>>>(in, nrows, out, nullptr, 0, nullptr,
                                                cdiv(ncols, 8), ncols);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

hef_status reduce_cols_f64_pair(const double *in0, int64_t nrows0, double *out0,
                                const double *in1, int64_t nrows1, double *out1, int64_t ncols,
                                hipStream_t s) {
  if (ncols <= 0) return HEF_OK;
  const int64_t nbc = cdiv(ncols, 8);
  k_reduce_cols<<<2 * nbc, 256, 0, s>>>(in0, nrows0, out0, in1, nrows1, out1, nbc, ncols);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

size_t scan_ws_bytes(int64_t n) {
  Arena a;
  a.take<int32_t>(cdiv(n, kScanTile) + 1);
  return a.mark();
}

hef_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, Arena &ws,
                              hipStream_t s) {
  const int64_t ntiles = cdiv(n, kScanTile);
  const size_t mk = ws.mark();
  int32_t *sums = ws.take<int32_t>(ntiles + 1);
  HEF_WS_CHECK(ws);
  if (n == 0) {
    HEF_TRY(zero_async(out, sizeof(int32_t), s));
    ws.reset(mk);
    return HEF_OK;
  }
  k_scan_tiles<<<ntiles, kScanThreads, 0, s>>>(in, out, sums, n);
  if (ntiles <= kFinishTiles) {
    k_scan_finish<<<ntiles, kScanThreads, 0, s>>>(out, sums, n, ntiles);
  } else {
    k_scan_sums<<<1, 1024, 0, s>>>(sums, ntiles, out + n);
    k_scan_add<<<ntiles, kScanThreads, 0, s>>>(out, sums, n);
  }
  HEF_LAUNCH_CHECK();
  ws.reset(mk);
  return HEF_OK;
}

size_t radix_ws_bytes(int64_t n) {
  const int64_t nb = cdiv(n, kRadixTile);
  Arena a;
  a.take<int32_t>(nb * kBins + 1);
  return a.mark() + scan_ws_bytes(nb * kBins) + 512;
}

hef_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_out,
                            uint32_t *vals_out, int64_t n, int bits, Arena &ws,
                            hipStream_t s) {
  if (n == 0) return HEF_OK;
  const int64_t nb = cdiv(n, kRadixTile);
  const size_t mk = ws.mark();
  int32_t *hist = ws.take<int32_t>(nb * kBins + 1);
  HEF_WS_CHECK(ws);
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  uint32_t *ka = keys, *va = vals, *kb = keys_out, *vb = vals_out;
  // the histogram's scan tiles: when there are at most kRadixScanTiles
  // (n up to 64M keys) the scatter adds their prefixes itself
  const int64_t htiles = cdiv(nb * kBins, kScanTile);
  int32_t *tsum = htiles <= kRadixScanTiles ? ws.take<int32_t>(htiles) : nullptr;
  HEF_WS_CHECK(ws);
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    k_radix_hist<<<nb, kRadixThreads, 0, s>>>(ka, n, shift, hist, int(nb));
    if (tsum) {
      k_scan_tiles<<<htiles, kScanThreads, 0, s>>>(hist, hist, tsum, nb * kBins);
    } else {
      HEF_TRY(exclusive_scan_i32(hist, hist, nb * kBins, ws, s));
    }
    k_radix_scatter<<<nb, kRadixThreads, 0, s>>>(ka, va, kb, vb, n, shift, hist, int(nb), tsum,
                                                 int(htiles));
    HEF_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys_out) {
    HEF_HIP(hipMemcpyAsync(keys_out, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    HEF_HIP(hipMemcpyAsync(vals_out, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
  ws.reset(mk);
  return HEF_OK;
}

hef_status compact_flags(const int32_t *flag, int32_t *scratch, int32_t *idx_out,
                         int32_t *count_dev, int64_t n, Arena &ws, hipStream_t s) {
  if (n == 0) {
    HEF_TRY(zero_async(count_dev, sizeof(int32_t), s));
    return HEF_OK;
  }
  k_flag_copy<<<cdiv(n, 256), 256, 0, s>>>(flag, scratch, n);
  HEF_TRY(exclusive_scan_i32(scratch, scratch, n, ws, s));
  k_compact<<<cdiv(n, 256), 256, 0, s>>>(flag, scratch, idx_out, count_dev, n);
  HEF_LAUNCH_CHECK();
  return HEF_OK;
}

}  // namespace hef
