// Stable LSD radix sort of (key, int32 value) pairs for gfx950.
//
// Used for the Morton codes of the primitives (section 2.1 "Sort the
// bounding boxes using their Morton code") and of the queries (section 2.2
// "Query ordering").  Design: one read pass builds the digit histograms of
// every pass; then each 8-bit pass is a single kernel ("onesweep"): a
// workgroup takes the next tile from an atomic counter, publishes its
// per-digit counts (an LDS histogram), ranks its keys with wave64 ballots
// (stable: rank order = input order), resolves the prefix of the preceding
// tiles by decoupled look-back on one status word per (tile, digit), stages
// the keys in LDS in sorted order and writes them out in digit runs.
//
// Cross-workgroup communication is only through the status words; each word
// carries its own payload (2-bit flag + 30-bit count), so relaxed atomics at
// agent scope (coherent across the XCDs' L2s) suffice: no cache flushes.
// Forward progress: a tile index is taken after the workgroup is resident,
// so every tile waited on belongs to a running workgroup.  The wait is still
// bounded; a tile that gives up sets the caller's error word, publishes the
// prefix it has (never more than the true one, so every store stays inside
// the output) and lets its pass finish; the later passes see the word and
// do nothing.  The result is then invalid and the callers act on the word
// (the build fails, a query order falls back to the input order).
#include <atomic>

#include "abx_internal.h"

namespace abx {

// look-back polls of a predecessor that has published nothing, before the
// tile gives up (abx_set_sort_spin_limit; 0 gives up at once, for tests)
std::atomic<uint32_t> g_sort_spin_limit{1u << 26};

namespace {

constexpr int kBlock = 256;                 // 4 waves
// Threads of a onesweep workgroup (the digit work runs on the first kRadix)
// and keys per thread, by key width.  Swept at 1e7 keys: 64-bit keys, 8
// passes, 0.866 ms in 256 x 24 (6144-key tiles, two workgroups of 4
// wavefronts per CU by LDS), 0.74 in 512 x 9, 0.70 in 1024 x 5, 0.692 in
// 768 x 7 (5376-key tiles, two workgroups of 12 wavefronts); 32-bit keys, 4
// passes, 0.355 ms in 256 x 16, 0.337 in 512 x 8, 0.333 in 1024 x 5.  More
// wavefronts per tile shorten each tile's ranking, which a tile's successors
// wait on, and keep more loads in flight per CU.
template <typename K>
constexpr int kSweepOf = sizeof(K) == 8 ? 768 : 1024;
template <typename K>
constexpr int kItemsOf = sizeof(K) == 8 ? 7 : 5;
template <typename K>
constexpr int kTileOf = kSweepOf<K> * kItemsOf<K>;
constexpr int kWaves = kBlock / kWave;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;     // == kBlock: one digit per thread
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagPre = 2u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1;
constexpr int kHistBlocks = 1024;
constexpr int kLookWindow = 4;              // predecessors read per look-back round trip
static_assert(kRadix == kBlock, "one digit per thread");

int num_passes(int key_bits) { return (key_bits + kRadixBits - 1) / kRadixBits; }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & (kWave - 1);
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// exclusive scan of one value per thread over a B-thread block
template <int B>
__device__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *s_tmp /*[B / kWave]*/) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) s_tmp[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += s_tmp[w];
  __syncthreads();
  return before + inc - x;
}

// Histograms of all passes in one read of the keys.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_hist(const K *__restrict__ keys, int64_t n, int passes,
                                                 int key_bits, uint32_t *__restrict__ hist) {
  __shared__ uint32_t s_h[8][kRadix];
  for (int i = threadIdx.x; i < 8 * kRadix; i += kBlock) (&s_h[0][0])[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const K k = keys[i];
    for (int p = 0; p < passes; ++p) {
      const uint32_t d = (uint32_t)(k >> (p * kRadixBits)) & (kRadix - 1);
      atomicAdd(&s_h[p][d], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p) {
    const uint32_t c = s_h[p][threadIdx.x];
    if (c) atomicAdd(&hist[p * kRadix + threadIdx.x], c);
  }
  (void)key_bits;
}

// In place: hist[p][d] <- sum of hist[p][d'] for d' < d.
__global__ __launch_bounds__(kBlock) void k_hist_scan(uint32_t *hist) {
  __shared__ uint32_t s_tmp[kWaves];
  uint32_t *h = hist + blockIdx.x * kRadix;
  const uint32_t x = h[threadIdx.x];
  const uint32_t e = block_exclusive_scan<kBlock>(x, s_tmp);
  h[threadIdx.x] = e;
}

template <typename K, bool kIota>
__global__ __launch_bounds__(kSweepOf<K>) void k_onesweep(const K *__restrict__ kin,
                                                     const int32_t *__restrict__ vin,
                                                     K *__restrict__ kout, int32_t *__restrict__ vout,
                                                     int64_t n, int shift, int nbits,
                                                     const uint32_t *__restrict__ digit_start,
                                                     uint32_t *status, uint32_t *tile_ctr,
                                                     uint32_t spin_limit, int pass,
                                                     uint32_t *fail_pass, uint32_t *err,
                                                     uint32_t err_bit) {
  constexpr int kItems = kItemsOf<K>, kTile = kTileOf<K>;
  constexpr int kT = kSweepOf<K>, kW = kT / kWave;
  static_assert(kT >= kRadix && kT % kWave == 0, "a digit per thread among the first kRadix");
  __shared__ uint32_t s_cnt[kW][kRadix];
  __shared__ uint32_t s_loc[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_tmp[kW];
  __shared__ uint32_t s_hist[kRadix];
  __shared__ K s_keys[kTile];
  __shared__ int32_t s_vals[kTile];
  __shared__ uint32_t s_tile;

  // After a pass gave up, its output is no permutation of the keys the
  // digit histograms were taken from, so the scatter positions of a later
  // pass would not stay inside [0, n): the later passes do nothing.  (The
  // other tiles of the failing pass itself carry on: their successors wait
  // for their counts.)  *fail_pass is 0, or 1 + the pass that gave up.
  {
    const uint32_t f = __hip_atomic_load(fail_pass, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (f != 0 && f <= (uint32_t)pass) return;
  }
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < kW * kRadix; i += kT) (&s_cnt[0][0])[i] = 0;
  if (tid < kRadix) s_hist[tid] = 0;
  if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const int64_t base = (int64_t)tile * kTile;
  const int64_t wbase = base + (int64_t)wave * (kWave * kItems);
  const uint32_t dmask = (1u << nbits) - 1u;

  K k[kItems];
  int32_t v[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = wbase + r * kWave + lane;
    const bool ok = i < n;
    k[r] = ok ? kin[i] : (K)0;
    v[r] = ok ? (kIota ? (int32_t)i : vin[i]) : 0;
  }
  // The tile's digit counts go out first (a histogram in LDS), so the tiles
  // after this one find them while this one ranks its keys: taking them
  // from the ranking made each tile wait a ranking's time for its
  // predecessor (1e7 64-bit keys: 0.111 -> 0.103 ms a pass).  Resolving the
  // prefix before the ranking as well was slower (0.114 ms): the wait then
  // sits in front of the ranking instead of overlapping it.
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = wbase + r * kWave + lane;
    if (i < n) atomicAdd(&s_hist[(uint32_t)(k[r] >> shift) & dmask], 1u);
  }
  __syncthreads();
  uint32_t *st = status + (size_t)tile * kRadix + tid;
  const uint32_t total = tid < kRadix ? s_hist[tid] : 0u;
  if (tid < kRadix)
    __hip_atomic_store(st, (tile == 0 ? kFlagPre : kFlagAgg) | total, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);

  // Wave ranking: lanes holding the same digit find each other through one
  // ballot per digit bit; the lowest such lane bumps the wave's running
  // count for the digit and broadcasts the old value.
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = wbase + r * kWave + lane;
    const bool ok = i < n;
    const uint32_t d = (uint32_t)(k[r] >> shift) & dmask;
    uint64_t m = __ballot(ok);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int leader = ok ? (__ffsll((unsigned long long)m) - 1) : 0;
    uint32_t old = 0;
    if (ok && lane == leader) {
      old = s_cnt[wave][d];
      s_cnt[wave][d] = old + (uint32_t)__popcll(m);
    }
    old = __shfl(old, leader, kWave);
    rank[r] = old + (uint32_t)__popcll(m & lt);
  }
  __syncthreads();

  // per digit (one per thread): exclusive prefix over waves (the sum over
  // the waves is the tile's count, published above)
  const int d = tid;
  if (tid < kRadix) {
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
      const uint32_t c = s_cnt[w][d];
      s_cnt[w][d] = acc;
      acc += c;
    }
  }
  const uint32_t loc = block_exclusive_scan<kT>(total, s_tmp);
  if (tid < kRadix) s_loc[d] = loc;

  // decoupled look-back over the preceding tiles for digit d
  uint32_t excl = 0;
  if (tid < kRadix && tile != 0) {
    int64_t j = (int64_t)tile - 1;
    // Every awaited tile belongs to a resident workgroup, so the wait ends;
    // the spin bound (far above any real wait) only guarantees termination,
    // and giving up is recorded (the failed-pass word, and *err if given).
    // The words of kLookWindow predecessors are read together (one round
    // trip to the coherence point for several tiles: with counts published
    // before the ranking, a look-back often passes tiles that have their
    // counts out but not yet their prefix) and taken in order up to the
    // first unpublished one or the first inclusive prefix.
    for (uint32_t spins = 0;;) {
      if (spins >= spin_limit) {
        atomicMax(fail_pass, (uint32_t)pass + 1u);
        if (err) atomicOr(err, err_bit);
        break;
      }
      uint32_t w[kLookWindow];
#pragma unroll
      for (int u = 0; u < kLookWindow; ++u)
        w[u] = j - u >= 0 ? __hip_atomic_load(status + (size_t)(j - u) * kRadix + d, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                          : 0u;
      int used = 0;
      bool found = false;
#pragma unroll
      for (int u = 0; u < kLookWindow; ++u) {
        if (found || used < u || j - u < 0 || (w[u] & ~kCountMask) == 0) continue;
        excl += w[u] & kCountMask;
        ++used;
        if (w[u] & kFlagPre) found = true;
      }
      if (found) break;
      if (used == 0) {
        ++spins;
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      j -= used;
    }
    __hip_atomic_store(st, kFlagPre | (excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid < kRadix) s_gbase[d] = digit_start[d] + excl - loc;
  __syncthreads();

  // stage in LDS in sorted order
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = wbase + r * kWave + lane;
    if (i < n) {
      const uint32_t dd = (uint32_t)(k[r] >> shift) & dmask;
      const uint32_t pos = s_loc[dd] + s_cnt[wave][dd] + rank[r];
      s_keys[pos] = k[r];
      s_vals[pos] = v[r];
    }
  }
  __syncthreads();
  const int64_t rem = n - base;
  const int cnt = rem < kTile ? (int)rem : kTile;
  for (int i = tid; i < cnt; i += kT) {
    const K kk = s_keys[i];
    const uint32_t dd = (uint32_t)(kk >> shift) & dmask;
    const uint32_t o = s_gbase[dd] + (uint32_t)i;
    // o < n whenever this pass's input is a permutation of the histogrammed
    // keys (a tile that gave up publishes too small a prefix, never too
    // large); the test keeps every store in bounds regardless
    if (o < (uint64_t)n) {
      kout[o] = kk;
      vout[o] = s_vals[i];
    }
  }
}

template <typename K>
__global__ void k_copy_pairs(const K *__restrict__ kin, const int32_t *__restrict__ vin,
                             K *__restrict__ kout, int32_t *__restrict__ vout, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    kout[i] = kin[i];
    vout[i] = vin ? vin[i] : (int32_t)i;
  }
}

// the identity order when the sort that produced `order` gave up; the
// workgroups exit after one load when it did not
__global__ void k_order_guard(const uint32_t *__restrict__ err, int32_t *__restrict__ order,
                              int64_t m) {
  if (*err == 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    order[i] = (int32_t)i;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

struct SortLayout {
  size_t hist, ctr, err, status, tmp_keys, tmp_vals, total;
  int64_t tiles;
  int passes;
};

SortLayout sort_layout(int64_t n, int key_bits) {
  SortLayout L{};
  const size_t ksz = key_bits <= 32 ? 4 : 8;
  L.passes = num_passes(key_bits);
  const int64_t tile = ksz == 4 ? kTileOf<uint32_t> : kTileOf<uint64_t>;
  L.tiles = (n + tile - 1) / tile;
  size_t off = 0;
  L.hist = off;
  off = align_up(off + (size_t)L.passes * kRadix * 4, 256);
  L.ctr = off;
  off = align_up(off + (size_t)L.passes * 4, 256);
  L.err = off;  // 0, or 1 + the pass that gave up; cleared with the counters
  off = align_up(off + 4, 256);
  L.status = off;
  off = align_up(off + (size_t)L.passes * L.tiles * kRadix * 4, 256);
  L.tmp_keys = off;
  off = align_up(off + (size_t)n * ksz, 256);
  L.tmp_vals = off;
  off = align_up(off + (size_t)n * 4, 256);
  L.total = off;
  return L;
}

template <typename K>
abx_status sort_impl(const K *kin, const int32_t *vin, int64_t n, int key_bits, K *kout,
                     int32_t *vout, char *scratch, uint32_t *err, uint32_t err_bit, hipStream_t s) {
  if (n <= 1) {
    if (n == 1)
      ABX_TRY(launch("sort_copy", s, [&] {
        k_copy_pairs<K><<<1, 64, 0, s>>>(kin, vin, kout, vout, n);
      }));
    return ABX_OK;
  }
  const SortLayout L = sort_layout(n, key_bits);
  uint32_t *hist = reinterpret_cast<uint32_t *>(scratch + L.hist);
  uint32_t *ctr = reinterpret_cast<uint32_t *>(scratch + L.ctr);
  uint32_t *status = reinterpret_cast<uint32_t *>(scratch + L.status);
  K *tk = reinterpret_cast<K *>(scratch + L.tmp_keys);
  int32_t *tv = reinterpret_cast<int32_t *>(scratch + L.tmp_vals);
  uint32_t *fail_pass = reinterpret_cast<uint32_t *>(scratch + L.err);
  const uint32_t spin_limit = g_sort_spin_limit.load(std::memory_order_relaxed);
  // zero histograms, tile counters, the failed-pass word and status words in one fill
  ABX_TRY(fill_u32(hist, 0, (L.tmp_keys - L.hist) / 4, s));
  const unsigned hb = (unsigned)std::min<int64_t>(kHistBlocks, grid_for(n, kBlock * 8));
  ABX_TRY(launch("sort_hist", s, [&] {
    k_hist<K><<<hb, kBlock, 0, s>>>(kin, n, L.passes, key_bits, hist);
  }));
  ABX_TRY(launch("sort_hist_scan", s, [&] {
    k_hist_scan<<<L.passes, kBlock, 0, s>>>(hist);
  }));
  const K *src_k = kin;
  const int32_t *src_v = vin;
  for (int p = 0; p < L.passes; ++p) {
    const bool to_out = ((L.passes - 1 - p) % 2) == 0;
    K *dk = to_out ? kout : tk;
    int32_t *dv = to_out ? vout : tv;
    const int shift = p * kRadixBits;
    const int nbits = std::min(kRadixBits, key_bits - shift);
    const uint32_t *ds = hist + p * kRadix;
    uint32_t *stp = status + (size_t)p * L.tiles * kRadix;
    const unsigned g = (unsigned)L.tiles;
    if (p == 0 && src_v == nullptr) {
      ABX_TRY(launch("sort_onesweep", s, [&] {
        k_onesweep<K, true><<<g, kSweepOf<K>, 0, s>>>(src_k, nullptr, dk, dv, n, shift, nbits, ds, stp,
                                                 ctr + p, spin_limit, p, fail_pass, err, err_bit);
      }));
    } else {
      ABX_TRY(launch("sort_onesweep", s, [&] {
        k_onesweep<K, false><<<g, kSweepOf<K>, 0, s>>>(src_k, src_v, dk, dv, n, shift, nbits, ds, stp,
                                                  ctr + p, spin_limit, p, fail_pass, err, err_bit);
      }));
    }
    src_k = dk;
    src_v = dv;
  }
  return ABX_OK;
}

}  // namespace

abx_status fill_u32(void *p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return ABX_OK;
  const unsigned g = (unsigned)std::min<size_t>(4096, (count + 255) / 256);
  return launch("fill", s, [&] {
    k_fill_u32<<<g, 256, 0, s>>>(reinterpret_cast<uint32_t *>(p), value, count);
  });
}

size_t radix_sort_scratch_bytes(int64_t n, int key_bits) { return sort_layout(n, key_bits).total; }

abx_status order_guard(const uint32_t *err, int32_t *order, int64_t m, hipStream_t s) {
  if (!err || m <= 0) return ABX_OK;
  const unsigned g = (unsigned)std::min<int64_t>(256, grid_for(m, 256));
  return launch("order_guard", s, [&] { k_order_guard<<<g, 256, 0, s>>>(err, order, m); });
}

uint32_t *radix_sort_err_word(void *scratch, int64_t n, int key_bits) {
  if (n <= 1) return nullptr;  // no look-back: nothing can give up
  return reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) + sort_layout(n, key_bits).err);
}

abx_status radix_sort(const void *keys_in, const int32_t *vals_in, int64_t n, int key_bits,
                      void *keys_out, int32_t *vals_out, void *scratch, size_t scratch_bytes,
                      hipStream_t s, uint32_t *err, uint32_t err_bit) {
  if (n < 0 || key_bits < 1 || key_bits > 64) return ABX_ERR_INVALID_ARG;
  if (n >= (int64_t)kCountMask) return ABX_ERR_OVERFLOW;
  if (n > 0 && (!keys_in || !keys_out || !vals_out)) return ABX_ERR_INVALID_ARG;
  if (n > 0 && (keys_in == keys_out || (vals_in && (const void *)vals_in == (void *)vals_out)))
    return ABX_ERR_INVALID_ARG;
  if (n > 1 && (!scratch || scratch_bytes < radix_sort_scratch_bytes(n, key_bits)))
    return ABX_ERR_INVALID_ARG;
  if (key_bits <= 32)
    return sort_impl<uint32_t>(static_cast<const uint32_t *>(keys_in), vals_in, n, key_bits,
                               static_cast<uint32_t *>(keys_out), vals_out,
                               static_cast<char *>(scratch), err, err_bit, s);
  return sort_impl<uint64_t>(static_cast<const uint64_t *>(keys_in), vals_in, n, key_bits,
                             static_cast<uint64_t *>(keys_out), vals_out,
                             static_cast<char *>(scratch), err, err_bit, s);
}

}  // namespace abx
