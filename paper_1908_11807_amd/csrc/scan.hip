// Exclusive scan of per-query hit counts into CSR offsets (section 2.2: after
// the counting pass the storage for the results is allocated; section 2.3:
// offsets[i] is where query i's results start in `indices`).
//
// Reduce-then-scan in three launches: tile sums (int64), one workgroup scans
// the tile sums, each tile rescans itself with its prefix.  Totals are kept
// in int64 so that an int32 overflow of the result count is detected.
#include "abx_internal.h"

namespace abx {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;
constexpr int kWaves = kBlock / kWave;

__device__ int64_t block_sum_i64(int64_t x, int64_t *s_tmp) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_down(x, o, kWave);
  if (lane == 0) s_tmp[wave] = x;
  __syncthreads();
  int64_t t = 0;
  for (int w = 0; w < kWaves; ++w) t += s_tmp[w];
  __syncthreads();
  return t;
}

__device__ int64_t block_exclusive_i64(int64_t x, int64_t *s_tmp, int64_t *total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int64_t inc = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) s_tmp[wave] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) before += s_tmp[w];
    all += s_tmp[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

__global__ __launch_bounds__(kBlock) void k_tile_sums(const int32_t *__restrict__ c, int64_t m,
                                                      int64_t *__restrict__ sums) {
  __shared__ int64_t s_tmp[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  int64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < m) acc += c[i];
  }
  acc = block_sum_i64(acc, s_tmp);
  if (threadIdx.x == 0) sums[blockIdx.x] = acc;
}

// one workgroup: exclusive scan of the tile sums in place, grand total out
__global__ __launch_bounds__(kBlock) void k_scan_sums(int64_t *sums, int64_t tiles,
                                                      int64_t *__restrict__ d_total) {
  __shared__ int64_t s_tmp[kWaves];
  int64_t carry = 0;
  for (int64_t b = 0; b < tiles; b += kBlock) {
    const int64_t i = b + threadIdx.x;
    const int64_t x = i < tiles ? sums[i] : 0;
    int64_t tot;
    const int64_t e = block_exclusive_i64(x, s_tmp, &tot);
    if (i < tiles) sums[i] = carry + e;
    carry += tot;
  }
  if (threadIdx.x == 0) *d_total = carry;
}

// Each thread owns kItems consecutive counts (blocked), scans them serially,
// and the thread totals are scanned across the workgroup.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t *__restrict__ c, int64_t m,
                                                       const int64_t *__restrict__ sums,
                                                       const int64_t *__restrict__ d_total,
                                                       int32_t *__restrict__ off) {
  __shared__ int64_t s_tmp[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int32_t v[kItems];
  int64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r;
    v[r] = i < m ? c[i] : 0;
    acc += v[r];
  }
  int64_t tot;
  int64_t run = sums[blockIdx.x] + block_exclusive_i64(acc, s_tmp, &tot);
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r;
    if (i < m) off[i] = (int32_t)(run < INT32_MAX ? run : INT32_MAX);
    run += v[r];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t t = *d_total;
    off[m] = (int32_t)(t < INT32_MAX ? t : INT32_MAX);
  }
}

__global__ void k_zero_total(int32_t *off, int64_t *d_total) {
  off[0] = 0;
  *d_total = 0;
}

}  // namespace

size_t scan_scratch_bytes(int64_t m) {
  const int64_t tiles = (m + kTile - 1) / kTile;
  return align_up((size_t)(tiles > 0 ? tiles : 1) * 8, 256);
}

abx_status exclusive_scan(const int32_t *counts, int64_t m, int32_t *offsets, int64_t *d_total,
                          void *scratch, size_t scratch_bytes, hipStream_t s) {
  if (m == 0)
    return launch("scan_empty", s, [&] { k_zero_total<<<1, 1, 0, s>>>(offsets, d_total); });
  if (scratch_bytes < scan_scratch_bytes(m)) return ABX_ERR_INVALID_ARG;
  const int64_t tiles = (m + kTile - 1) / kTile;
  int64_t *sums = static_cast<int64_t *>(scratch);
  ABX_TRY(launch("scan_tile_sums", s, [&] {
    k_tile_sums<<<(unsigned)tiles, kBlock, 0, s>>>(counts, m, sums);
  }));
  ABX_TRY(launch("scan_sums", s, [&] { k_scan_sums<<<1, kBlock, 0, s>>>(sums, tiles, d_total); }));
  return launch("scan_tiles", s, [&] {
    k_scan_tiles<<<(unsigned)tiles, kBlock, 0, s>>>(counts, m, sums, d_total, offsets);
  });
}

}  // namespace abx
