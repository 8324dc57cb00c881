// LBVH construction kernels (ArborX paper, section 2.1):
//   scene box  -> "Calculate the scene bounding box" (reduction of corners)
//   Morton     -> "Assign Morton codes for each AABB"
//   (sort)     -> "Sort the bounding boxes using their Morton code" (sort.hip)
//   Karras     -> "Generate the bounding volume hierarchy" (Karras 2012)
//   refit      -> "Calculate internal nodes bounding boxes" (bottom-up, one
//                 thread per leaf, the second child to arrive continues)
//   quantise   -> 16-bit node boxes rounded outward (bandwidth reduction the
//                 paper cites from the literature; not the paper's own step)
#include <algorithm>
#include <atomic>

#include "abx_internal.h"

namespace abx {

constexpr int kBuildBlock = 256;
constexpr int kScenePartials = 1024;

// ------------------------------------------------------------ scene box
template <int KIND>
__global__ __launch_bounds__(kBuildBlock) void k_scene_partial(const float *__restrict__ p,
                                                               int64_t n,
                                                               float *__restrict__ partial) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float l = KIND == ABX_PRIM_POINTS ? p[3 * i + a] : p[6 * i + a];
      const float h = KIND == ABX_PRIM_POINTS ? l : p[6 * i + 3 + a];
      bad |= !__builtin_isfinite(l) || !__builtin_isfinite(h) || !(l <= h);
      lo[a] = fminf(lo[a], l);
      hi[a] = fmaxf(hi[a], h);
    }
  }
  __shared__ float s[kBuildBlock / kWave][7];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_down(lo[a], o, kWave));
      hi[a] = fmaxf(hi[a], __shfl_down(hi[a], o, kWave));
    }
    bad |= __shfl_down(bad, o, kWave);
  }
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      s[wave][a] = lo[a];
      s[wave][3 + a] = hi[a];
    }
    s[wave][6] = (float)bad;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int a = threadIdx.x;
    float v = s[0][a];
    for (int w = 1; w < kBuildBlock / kWave; ++w)
      v = a < 3 ? fminf(v, s[w][a]) : fmaxf(v, s[w][a]);
    partial[blockIdx.x * 8 + a] = v;
  }
}

// One thread per axis (plus one for the flag): final reduction and the Q16
// grid.  The grid step s is the smallest float with
// fmaf(65535, s, lo) >= hi, so the top code covers the scene box.
constexpr int kSceneFinalThreads = 256;

__global__ __launch_bounds__(kSceneFinalThreads) void k_scene_final(const float *__restrict__ partial,
                                                                    int blocks,
                                                                    TreeHeader *__restrict__ hdr) {
  // min / max / or over the partials (exact in any order), then the header
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int b = threadIdx.x; b < blocks; b += kSceneFinalThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], partial[b * 8 + a]);
      hi[a] = fmaxf(hi[a], partial[b * 8 + 3 + a]);
    }
    bad |= partial[b * 8 + 6] != 0.0f;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_down(lo[a], o, kWave));
      hi[a] = fmaxf(hi[a], __shfl_down(hi[a], o, kWave));
    }
    bad |= __shfl_down(bad, o, kWave);
  }
  __shared__ float s[kSceneFinalThreads / kWave][7];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      s[wave][a] = lo[a];
      s[wave][3 + a] = hi[a];
    }
    s[wave][6] = (float)bad;
  }
  __syncthreads();
  const int a = threadIdx.x;
  if (a < 3) {
    float l = s[0][a], h = s[0][3 + a];
    for (int w = 1; w < kSceneFinalThreads / kWave; ++w) {
      l = fminf(l, s[w][a]);
      h = fmaxf(h, s[w][3 + a]);
    }
    hdr->scene[a] = l;
    hdr->scene[3 + a] = h;
    const float ext = h - l;
    hdr->inv_ext[a] = ext > 0.0f ? 1.0f / ext : 0.0f;
    float sc = 0.0f;
    int overflow = 0;
    if (ext > 0.0f) {
      if (!__builtin_isfinite(ext)) {
        overflow = 1;
      } else {
        sc = ext / (float)kQ16Max;
        while (__fmaf_rn((float)kQ16Max, sc, l) < h) sc = nextafterf(sc, INFINITY);
      }
    }
    hdr->q_origin[a] = l;
    hdr->q_scale[a] = sc;
    if (overflow) atomicOr(&hdr->bad, 2);
  } else if (a == 3) {
    int any = 0;
    for (int w = 0; w < kSceneFinalThreads / kWave; ++w) any |= s[w][6] != 0.0f;
    if (any) atomicOr(&hdr->bad, 1);
    hdr->height = 0;
  }
}

__global__ void k_header_init(TreeHeader *hdr) {
  if (threadIdx.x == 0) {
    hdr->bad = 0;
    hdr->height = 0;
    hdr->root = 0;  // Karras numbering; the agglomerative build overwrites it
    hdr->node_count = 0;  // set by the 4-wide emission (binary trees: n - 1)
  }
}

// ------------------------------------------------------------ Morton codes
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// quantised coordinate of c on `bits` bits: scaled by the scene box into
// [0,1] (float32: inverse extent, clamp), truncated, clamped to 2^bits - 1
__device__ __forceinline__ uint32_t quantise_axis(float c, float lo, float inv, int bits) {
  float u = (c - lo) * inv;
  u = u > 0.0f ? u : 0.0f;
  u = u > 1.0f ? 1.0f : u;
  const uint32_t q = (uint32_t)(u * (float)(1u << bits));
  const uint32_t qmax = (1u << bits) - 1u;
  return q > qmax ? qmax : q;
}

template <int KIND, typename K>
__global__ __launch_bounds__(kBuildBlock) void k_morton(const float *__restrict__ p, int64_t n,
                                                        const float *__restrict__ scene, int bits,
                                                        K *__restrict__ codes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = scene[a];
    const float ext = scene[3 + a] - lo;
    const float inv = ext > 0.0f ? 1.0f / ext : 0.0f;
    const float c = KIND == ABX_PRIM_POINTS ? p[3 * i + a] : 0.5f * (p[6 * i + a] + p[6 * i + 3 + a]);
    q[a] = quantise_axis(c, lo, inv, bits);
  }
  if (bits <= 10)
    codes[i] = (K)((spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]));
  else
    codes[i] = (K)((spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]));
}

// A node's parent word: parent << 1 | side in the low half, the far end j of
// the parent's leaf range [min(parent, j), max(parent, j)] in the high half,
// so one load names the next node of a climb and whether its range leaves the
// current chunk or group.
__device__ __forceinline__ uint64_t parent_word(int64_t parent, int side, int64_t j) {
  return ((uint64_t)(uint32_t)j << 32) | (uint32_t)((parent << 1) | side);
}

// ------------------------------------------------------------ Karras 2012
// Common-prefix length of the index-augmented codes at sorted positions i
// and j (-1 outside [0, n)).  Equal codes fall back to the positions, which
// makes every augmented code unique (section 2.1: codes "augmented with an
// index").
template <typename K>
__device__ __forceinline__ int delta(const K *__restrict__ keys, int64_t n, int64_t i, K ki,
                                     int64_t j) {
  if (j < 0 || j >= n) return -1;
  const K kj = keys[j];
  if (ki != kj) return sizeof(K) == 8 ? __clzll((long long)(ki ^ kj)) : __clz((int)(ki ^ kj));
  return (int)(8 * sizeof(K)) + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// The same with the keys of positions [lo, hi) staged in LDS (a probe
// outside the window reads global memory; the value is the same).
template <typename K>
struct KeyWindow {
  const K *keys;
  const K *lds;
  int64_t lo, hi;
  __device__ __forceinline__ K at(int64_t j) const {
    return j >= lo && j < hi ? lds[j - lo] : keys[j];
  }
};

template <typename K>
__device__ __forceinline__ int delta(const KeyWindow<K> &w, int64_t n, int64_t i, K ki, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const K kj = w.at(j);
  if (ki != kj) return sizeof(K) == 8 ? __clzll((long long)(ki ^ kj)) : __clz((int)(ki ^ kj));
  return (int)(8 * sizeof(K)) + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// A workgroup stages the keys of its nodes and kKarrasHalo positions either
// side in LDS: most ranges are short, so most searches probe only there; the
// few long ones leave the window for their outer probes.
constexpr int kKarrasHalo = 768;
constexpr int kKarrasWindow = kBuildBlock + 2 * kKarrasHalo;

// One thread per internal node i: direction from the neighbours, range end
// by exponential then binary search, split by binary search on the prefix,
// children at gamma / gamma+1 (leaf when the child range has one element).
// Writes the children's parent words (parent << 1 | side, and the far end j
// of this node's range [min(i,j), max(i,j)]), its own range end and clears
// its arrival counter.  The child references are written by the refit, which
// emits each node whole.
template <typename K>
__global__ __launch_bounds__(kBuildBlock) void k_karras(const K *__restrict__ keys, int64_t n,
                                                        uint64_t *__restrict__ pw_leaf,
                                                        uint64_t *__restrict__ pw_int,
                                                        int32_t *__restrict__ other_end,
                                                        uint32_t *__restrict__ flags,
                                                        const TreeHeader *__restrict__ hdr) {
  __shared__ K s_keys[kKarrasWindow];
  // the searches stay inside [i, j] only over sorted keys: after a failed
  // sort nothing is built (the refit skips as well); the flag is the same
  // for the whole workgroup, which leaves before its barrier
  if (hdr->bad & kBadSort) return;
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t lo = b0 > kKarrasHalo ? b0 - kKarrasHalo : 0;
  const int64_t hi = b0 + kBuildBlock + kKarrasHalo < n ? b0 + kBuildBlock + kKarrasHalo : n;
  for (int64_t p = lo + threadIdx.x; p < hi; p += blockDim.x) s_keys[p - lo] = keys[p];
  __syncthreads();
  const KeyWindow<K> w{keys, s_keys, lo, hi};
  const int64_t i = b0 + threadIdx.x;
  if (i >= n - 1) return;
  const K ki = w.at(i);
  const int d = delta(w, n, i, ki, i + 1) - delta(w, n, i, ki, i - 1) >= 0 ? 1 : -1;
  const int dmin = delta(w, n, i, ki, i - d);
  int64_t lmax = 2;
  while (delta(w, n, i, ki, i + lmax * d) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(w, n, i, ki, i + (l + t) * d) > dmin) l += t;
  const int64_t j = i + l * d;
  const int dnode = delta(w, n, i, ki, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(w, n, i, ki, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
  const int64_t first = i < j ? i : j, last = i < j ? j : i;
  const bool left_leaf = first == gamma, right_leaf = last == gamma + 1;
  const uint64_t pl = parent_word(i, 0, j), pr = parent_word(i, 1, j);
  if (left_leaf) pw_leaf[gamma] = pl; else pw_int[gamma] = pl;
  if (right_leaf) pw_leaf[gamma + 1] = pr; else pw_int[gamma + 1] = pr;
  other_end[i] = (int32_t)j;
  flags[i] = 0;
}

// ------------------------------------------------------------ FP32 child slots
__device__ __forceinline__ void store_child(NodeF32 *node, int side, const float b[6], int h) {
  float *f = reinterpret_cast<float *>(node);
  const int o = side * 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) f[o + k] = b[k];
  reinterpret_cast<int *>(node)[14 + side] = h;
}

__device__ __forceinline__ void load_child(const NodeF32 *node, int side, float b[6], int &h) {
  const float *f = reinterpret_cast<const float *>(node);
  const int o = side * 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) b[k] = f[o + k];
  h = reinterpret_cast<const int *>(node)[14 + side];
}

// Chunking of the agglomerative build's bottom-up pass (below).
constexpr int kRefitThreads = 1024;
constexpr int kRefitPerThread = 8;
constexpr int kRefitChunk = kRefitThreads * kRefitPerThread;
constexpr int kRefitMaxSteps = 256;  // > any tree height; only bounds the loops
// its middle pass: one workgroup per kMidChunks chunks
constexpr int kMidChunks = 64;
constexpr int64_t kMidLeaves = (int64_t)kRefitChunk * kMidChunks;
// A crossing node inside a super-chunk is an ancestor of the split at one of
// its kMidChunks - 1 inner chunk boundaries, so there are at most
// (kMidChunks - 1) * (tree height, < 96 for 63-bit keys augmented by 31-bit
// positions) of them, each with at most two entries.
constexpr int kMidListCap = 2 * kMidChunks * 96;

// ------------------------------------------------- agglomerative build
// Hierarchy and refit in one bottom-up pass (Apetrei 2014, the single-pass
// construction the paper intends to adopt, section 2.1).  Internal node p is
// the split between sorted positions p and p+1.  A node covering [l, r]
// joins the neighbour it shares the longer augmented-code prefix with: its
// parent is split r (it is the left child) when delta(r, r+1) >
// delta(l-1, l), else split l-1 (right child); the two can never tie.  The
// tree is the same binary radix tree as the Karras build, numbered by split.
//
// Phase 1 (one workgroup per chunk of kRefitChunk leaves): a leaf's thread
// climbs while the parent's split lies strictly inside the chunk (both of
// its children then hold a leaf of the chunk, so any arrival in this phase
// comes from this workgroup): it writes its box, reference, height and range
// end into the parent, then counts its arrival in LDS (workgroup scope); the
// second arrival reads the sibling back and climbs on.  An arrival at a
// split between two chunks is appended to the frontier instead.  At the
// end, each split of the chunk hands its count to the top pass (1 if exactly
// one child arrived, else 0).
// Phase 2 (one workgroup, after the kernel boundary): climbs from every
// frontier entry with global counters, again at workgroup scope.
template <typename K, int KIND, bool kQ16>
__global__ __launch_bounds__(kRefitThreads) void k_agglo_local(
    const K *__restrict__ keys, const float *__restrict__ prims, const int32_t *__restrict__ perm,
    int64_t n, NodeF32 *nodes, int32_t *range_lo, int32_t *range_hi, uint32_t *__restrict__ flags,
    TreeHeader *hdr, void *q16_leaves, int32_t *__restrict__ frontier,
    uint32_t *__restrict__ frontier_count, uint32_t frontier_cap) {
  if (hdr->bad & kBadSort) return;  // as in k_refit_local
  __shared__ uint32_t s_cnt[kRefitChunk];
  for (int i = threadIdx.x; i < kRefitChunk; i += kRefitThreads) s_cnt[i] = 0;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kRefitChunk;
  const int64_t c1 = c0 + kRefitChunk < n ? c0 + kRefitChunk : n;
  for (int rr = 0; rr < kRefitPerThread; ++rr) {
    const int64_t p0 = c0 + (int64_t)rr * kRefitThreads + threadIdx.x;
    if (p0 >= c1) break;
    const int32_t orig = perm[p0];
    float b[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = KIND == ABX_PRIM_POINTS ? prims[3 * (int64_t)orig + a] : prims[6 * (int64_t)orig + a];
      b[3 + a] = KIND == ABX_PRIM_POINTS ? b[a] : prims[6 * (int64_t)orig + 3 + a];
    }
    if (kQ16 && KIND == ABX_PRIM_BOXES) {
      float4 *o = reinterpret_cast<float4 *>(q16_leaves) + 2 * (int64_t)orig;
      o[0] = make_float4(b[0], b[1], b[2], b[3]);
      o[1] = make_float4(b[4], b[5], __int_as_float((int32_t)p0), 0.0f);
    }
    if (n == 1) break;
    int64_t l = p0, r = p0;
    int32_t ref = ~orig;
    int h = 0;
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const bool left = l == 0 || (r != n - 1 && delta(keys, n, r, keys[r], r + 1) >
                                                     delta(keys, n, l - 1, keys[l - 1], l));
      const int64_t p = left ? r : l - 1;
      const int side = left ? 0 : 1;
      store_child(nodes + p, side, b, h);
      reinterpret_cast<int32_t *>(nodes + p)[12 + side] = ref;
      if (left) range_lo[p] = (int32_t)l;
      else range_hi[p] = (int32_t)r;
      if (p < c0 || p > c1 - 2) {
        const uint32_t e = atomicAdd(frontier_count, 1u);
        if (e < frontier_cap) frontier[e] = (int32_t)p;
        else atomicOr(&hdr->bad, 4);
        break;
      }
      const uint32_t old = __hip_atomic_fetch_add(&s_cnt[p - c0], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float sb[6];
      int sh;
      load_child(nodes + p, side ^ 1, sb, sh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      if (left) r = range_hi[p];
      else l = range_lo[p];
      ref = (int32_t)p;
      if (l == 0 && r == n - 1) {
        hdr->root = (int32_t)p;
        hdr->height = h;
        break;
      }
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
  __syncthreads();
  for (int64_t p = c0 + threadIdx.x; p < c1 && p < n - 1; p += kRefitThreads)
    flags[p] = s_cnt[p - c0] == 1 ? 1u : 0u;
}

template <typename K>
__global__ __launch_bounds__(kRefitThreads) void k_agglo_top(const K *__restrict__ keys, int64_t n,
                                                             NodeF32 *nodes, int32_t *range_lo,
                                                             int32_t *range_hi, uint32_t *flags,
                                                             TreeHeader *hdr,
                                                             const int32_t *__restrict__ frontier,
                                                             const uint32_t *__restrict__ frontier_count,
                                                             uint32_t frontier_cap) {
  const uint32_t cnt = min(*frontier_count, frontier_cap);
  for (uint32_t e = threadIdx.x; e < cnt; e += kRefitThreads) {
    int64_t p = frontier[e];
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const uint32_t old = __hip_atomic_fetch_add(flags + p, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float b[6], sb[6];
      int h, sh;
      load_child(nodes + p, 0, b, h);
      load_child(nodes + p, 1, sb, sh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      const int64_t l = range_lo[p], r = range_hi[p];
      if (l == 0 && r == n - 1) {
        hdr->root = (int32_t)p;
        hdr->height = h;
        break;
      }
      const bool left = l == 0 || (r != n - 1 && delta(keys, n, r, keys[r], r + 1) >
                                                     delta(keys, n, l - 1, keys[l - 1], l));
      const int64_t q = left ? r : l - 1;
      const int side = left ? 0 : 1;
      store_child(nodes + q, side, b, h);
      reinterpret_cast<int32_t *>(nodes + q)[12 + side] = (int32_t)p;
      if (left) range_lo[q] = (int32_t)l;
      else range_hi[q] = (int32_t)r;
      p = q;
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

// at most two arrivals per split between chunks
size_t agglo_frontier_cap(int64_t n) {
  return (size_t)(2 * ((n + kRefitChunk - 1) / kRefitChunk) + 64);  // per list (two lists)
}


// ------------------------------------------------------------ Q16 nodes
// The 16-bit code of a box's lower (upper) face: the largest (smallest) q
// whose dequantised value fmaf(q, s, o) is <= x (>= x), so the decoded box
// contains the exact one and is the tightest such box.  Dequantisation is
// monotone in q, so any nearby start reaches that q through the two loops:
// the float estimate (x - o) * (1/s) is within a small fraction of a step
// for x inside the scene box, and the loops take a step or two at most.
__device__ __forceinline__ uint32_t q_clamp(float e) {
  return e <= 0.0f ? 0u : (e >= (float)kQ16Max ? (uint32_t)kQ16Max : (uint32_t)e);
}

__device__ __forceinline__ uint32_t q_lo(float x, float o, float s, float inv) {
  if (s == 0.0f) return 0;
  uint32_t q = q_clamp(floorf((x - o) * inv));
  while (q > 0 && deq(q, s, o) > x) --q;
  while (q < (uint32_t)kQ16Max && deq(q + 1, s, o) <= x) ++q;
  return q;
}

__device__ __forceinline__ uint32_t q_hi(float x, float o, float s, float inv) {
  if (s == 0.0f) return 0;
  uint32_t q = q_clamp(ceilf((x - o) * inv));
  while (q < (uint32_t)kQ16Max && deq(q, s, o) < x) ++q;
  while (q > 0 && deq(q - 1, s, o) >= x) --q;
  return q;
}

// Q16 node from the FP32 one.  Internal children get outward-rounded 16-bit
// boxes; in a point tree a leaf child's 12-byte slot holds the point's
// float32 x, y, z instead (the traversal tells the two apart by the sign of
// the reference), so point leaves need no second memory access.
template <int KIND>
__global__ __launch_bounds__(kBuildBlock) void k_quantise(const NodeF32 *__restrict__ src,
                                                          int64_t ni, TreeHeader *__restrict__ hdr,
                                                          const int32_t *__restrict__ pre,
                                                          NodeQ16 *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  // with `pre` (depth-first index, -1 if unknown), node i goes to slot
  // pre[i] and internal child references are renumbered the same way
  int64_t slot = i;
  if (pre) {
    slot = pre[i];
    if (slot < 0 || slot >= ni) {
      atomicOr(&hdr->bad, 8);
      return;
    }
  }
  const float *f = reinterpret_cast<const float *>(src + i);
  const int4 d = src[i].d;
  float o[3], sc[3], inv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = hdr->q_origin[a];
    sc[a] = hdr->q_scale[a];
    inv[a] = sc[a] != 0.0f ? 1.0f / sc[a] : 0.0f;
  }
  uint32_t w[6];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const bool leaf = (c == 0 ? d.x : d.y) < 0;
    if (KIND == ABX_PRIM_POINTS && leaf) {
#pragma unroll
      for (int a = 0; a < 3; ++a) w[3 * c + a] = __float_as_uint(f[6 * c + a]);
    } else {
      uint32_t q[6];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        q[a] = q_lo(f[6 * c + a], o[a], sc[a], inv[a]);
        q[3 + a] = q_hi(f[6 * c + 3 + a], o[a], sc[a], inv[a]);
      }
#pragma unroll
      for (int h = 0; h < 3; ++h) w[3 * c + h] = q[2 * h] | (q[2 * h + 1] << 16);
    }
  }
  int32_t ref[2] = {d.x, d.y};
  if (pre) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
      if (ref[c] >= 0) {
        const int32_t r = ref[c] < ni ? pre[ref[c]] : -1;
        if (r < 0 || r >= ni) atomicOr(&hdr->bad, 8);
        ref[c] = r;
      }
  }
  NodeQ16 out;
  out.a = make_uint4(w[0], w[1], w[2], w[3]);
  out.b = make_uint4(w[4], w[5], (uint32_t)ref[0], (uint32_t)ref[1]);
  dst[slot] = out;
}

// ------------------------------------------------------------ bottom-up refit
// Internal boxes from the leaves up (section 2.1).  One thread per leaf
// climbs from its leaf; at each parent the first arrival leaves its child
// record (exact box, reference, height) and stops, the second takes both and
// climbs on with their union.  Nodes are written whole in their final form:
// FP32, or Q16 -- outward-rounded child boxes, a point leaf's slot holding
// the float32 point -- at the depth-first slot with renumbered references.
// The rounding needs the exact child boxes, so it happens here rather than in
// a pass over a staged FP32 tree, but not inside the climb itself: a
// wavefront pays for every instruction any of its lanes runs, and the climbs
// are divergent, so finished nodes are emitted afterwards by a pass with one
// thread per node.
//
// Phase 1 (k_fit_chunk): a workgroup owns kFitChunk consecutive leaves, two
// per thread (the LDS records of 2048 leaves fill one CU's 160 KB; larger
// chunks leave fewer nodes to the slower later phases).  A
// Karras node's leaf range contains its own index, so a node whose range lies
// inside the chunk is numbered inside it: the workgroup loads those nodes'
// parent words and output slots into LDS, the climb inside the chunk reads
// nothing else from global memory, and child records meet in LDS, the
// arrivals counted by an LDS atomic at workgroup scope whose value carries
// the first arrival's height.  After a barrier each thread emits its nodes of
// the chunk whose two children arrived.  A climb reaching a node whose range
// leaves the chunk stores its record in the node's staging slot (the FP32
// node layout; for FP32 trees the node itself) and lists (node, side): in its
// group's list when the range stays inside the group of kFitGroup chunks,
// else in the top list.
// Phase 2 (k_fit_climb, one workgroup per group) climbs from the group's list
// through nodes inside the group; every arrival at such a node comes from this
// workgroup, so counters in global memory at workgroup scope order the
// hand-offs.  Phase 3 (one workgroup) climbs the top list to the root.  The
// staged records of a node both of whose children have arrived form the FP32
// node; for Q16 trees such nodes are listed and k_fit_emit quantises them.
// Each phase starts after a kernel boundary has made the previous one's stores
// visible; no step needs agent-scope fences (which write back and invalidate
// the XCDs' L2s).
constexpr int kFitThreads = 1024;
constexpr int kFitPerThread = 2;        // leaves (and nodes) per thread
constexpr int kFitChunk = kFitThreads * kFitPerThread;
constexpr int kFitWaves = 4;            // per SIMD: one workgroup per CU (LDS)
constexpr int kFitGroup = 64;           // chunks per group of phase 2
constexpr int64_t kFitGroupLeaves = (int64_t)kFitChunk * kFitGroup;
// Bound on the nodes of any root path: the augmented codes' common-prefix
// lengths grow strictly along a path and are below 63 + 32.
constexpr int kFitMaxPath = 96;
// A node whose range crosses an inner chunk boundary of a group holds the two
// leaves beside that boundary, so it lies on their common ancestors' path:
// at most (kFitGroup - 1) * kFitMaxPath nodes, two entries each.
constexpr uint32_t kFitGroupCap = 2 * (kFitGroup - 1) * kFitMaxPath;
constexpr int kFitMaxSteps = 256;       // > any tree height; only bounds the loops
constexpr uint32_t kFitDone = 1u << 31;  // LDS counter: both children arrived

int64_t fit_groups(int64_t n) { return (n + kFitGroupLeaves - 1) / kFitGroupLeaves; }

// the top list: nodes crossing a group boundary, likewise
uint32_t fit_top_cap(int64_t n) { return (uint32_t)(2 * kFitMaxPath * fit_groups(n) + 64); }

// Nodes finished by phases 2 and 3: no more than the entries the lists can
// hold.  Among the nodes whose range crosses a chunk, one with a single
// crossing child takes one entry and one with none takes two; one whose two
// children both cross takes none, but in the binary forest they form there
// are fewer of those than of nodes with no crossing child.
uint32_t fit_emit_cap(int64_t n) {
  return fit_top_cap(n) + (uint32_t)fit_groups(n) * kFitGroupCap;
}

// counters (top list, one per group, emit list), the top list, the group
// lists, the emit list
size_t fit_lists_bytes(int64_t n) {
  const size_t g = (size_t)fit_groups(n);
  return align_up((2 + g) * 4, 256) + align_up((size_t)fit_top_cap(n) * 4, 256) +
         align_up(g * kFitGroupCap * 4, 256) + (size_t)fit_emit_cap(n) * 4;
}

struct FitLists {
  uint32_t *count;  // [0]: top list, [1 + g]: group g, [1 + groups]: emit list
  int32_t *top;
  int32_t *group;   // kFitGroupCap entries per group
  int32_t *emit;
  uint32_t *emit_count;
  uint32_t top_cap, emit_cap;
};

FitLists fit_lists(void *mem, int64_t n) {
  const size_t g = (size_t)fit_groups(n);
  char *p = static_cast<char *>(mem);
  FitLists L;
  L.count = reinterpret_cast<uint32_t *>(p);
  L.emit_count = L.count + 1 + g;
  p += align_up((2 + g) * 4, 256);
  L.top = reinterpret_cast<int32_t *>(p);
  L.top_cap = fit_top_cap(n);
  p += align_up((size_t)L.top_cap * 4, 256);
  L.group = reinterpret_cast<int32_t *>(p);
  p += align_up(g * kFitGroupCap * 4, 256);
  L.emit = reinterpret_cast<int32_t *>(p);
  L.emit_cap = fit_emit_cap(n);
  return L;
}

// child record in the staging node (the FP32 node layout: box at floats
// 6 * side, reference at word 12 + side, height at 14 + side)
__device__ __forceinline__ void put_rec(NodeF32 *node, int side, const float b[6], int32_t ref,
                                        int h) {
  store_child(node, side, b, h);
  reinterpret_cast<int32_t *>(node)[12 + side] = ref;
}

__device__ __forceinline__ void get_rec(const NodeF32 *node, int side, float b[6], int32_t &ref,
                                        int &h) {
  load_child(node, side, b, h);
  ref = reinterpret_cast<const int32_t *>(node)[12 + side];
}

struct QGrid {
  float o[3], s[3], inv[3];
};

__device__ __forceinline__ QGrid load_grid(const TreeHeader *hdr) {
  QGrid g;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g.o[a] = hdr->q_origin[a];
    g.s[a] = hdr->q_scale[a];
    g.inv[a] = g.s[a] != 0.0f ? 1.0f / g.s[a] : 0.0f;
  }
  return g;
}

// the three Q16 words of one child slot (a point leaf keeps its float32 point)
template <int KIND>
__device__ __forceinline__ void q16_slot(const float b[6], int32_t ref, const QGrid &g,
                                         uint32_t w[3]) {
  if (KIND == ABX_PRIM_POINTS && ref < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = __float_as_uint(b[a]);
    return;
  }
  uint32_t q[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q[a] = q_lo(b[a], g.o[a], g.s[a], g.inv[a]);
    q[3 + a] = q_hi(b[3 + a], g.o[a], g.s[a], g.inv[a]);
  }
#pragma unroll
  for (int h = 0; h < 3; ++h) w[h] = q[2 * h] | (q[2 * h + 1] << 16);
}

// a finished node, children in side order, written whole at its slot
template <int KIND, bool kQ16>
__device__ __forceinline__ void put_node(void *out, int32_t slot, const float *b0, const float *b1,
                                         int32_t r0, int32_t r1, int h0, int h1, const QGrid &g) {
  if (kQ16) {
    uint32_t w0[3], w1[3];
    q16_slot<KIND>(b0, r0, g, w0);
    q16_slot<KIND>(b1, r1, g, w1);
    NodeQ16 *o = static_cast<NodeQ16 *>(out) + slot;
    o->a = make_uint4(w0[0], w0[1], w0[2], w1[0]);
    o->b = make_uint4(w1[1], w1[2], (uint32_t)r0, (uint32_t)r1);
  } else {
    float4 *o = reinterpret_cast<float4 *>(static_cast<NodeF32 *>(out) + slot);
    o[0] = make_float4(b0[0], b0[1], b0[2], b0[3]);
    o[1] = make_float4(b0[4], b0[5], b1[0], b1[1]);
    o[2] = make_float4(b1[2], b1[3], b1[4], b1[5]);
    o[3] = make_float4(__int_as_float(r0), __int_as_float(r1), __int_as_float(h0),
                       __int_as_float(h1));
  }
}

__device__ __forceinline__ void unite(float b[6], const float sb[6]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    b[a] = fminf(b[a], sb[a]);
    b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
  }
}

__device__ __forceinline__ void fit_push(const FitLists &L, int64_t f, int64_t l, int32_t pp,
                                         TreeHeader *hdr) {
  const int64_t g = f / kFitGroupLeaves;
  if (l < (g + 1) * kFitGroupLeaves) {
    const uint32_t e = atomicAdd(L.count + 1 + g, 1u);
    if (e < kFitGroupCap) L.group[g * kFitGroupCap + e] = pp;
    else atomicOr(&hdr->bad, 4);
  } else {
    const uint32_t e = atomicAdd(L.count, 1u);
    if (e < L.top_cap) L.top[e] = pp;
    else atomicOr(&hdr->bad, 4);
  }
}

// output slot of node x: its depth-first index when renumbering, else x
__device__ __forceinline__ int32_t fit_slot(const int32_t *__restrict__ pre, int64_t x, int64_t ni,
                                            TreeHeader *hdr) {
  if (!pre) return (int32_t)x;
  const int32_t s = pre[x];
  if (s < 0 || s >= ni) {
    atomicOr(&hdr->bad, 8);
    return -1;
  }
  return s;
}

// Phase 1.  The climbs only move records (cheap, but divergent: a wavefront
// keeps looping for its longest climb); the nodes they finish are written
// after a barrier, one thread per node.
template <int KIND, bool kQ16>
__global__ __launch_bounds__(kFitThreads) __attribute__((amdgpu_waves_per_eu(kFitWaves))) void k_fit_chunk(
    const float *__restrict__ prims, const int32_t *__restrict__ perm, int64_t n,
    const uint64_t *__restrict__ pw_leaf, const uint64_t *__restrict__ pw_int,
    const int32_t *__restrict__ pre, void *out, NodeF32 *stage, TreeHeader *hdr, void *box_rec,
    FitLists lists) {
  // after a failed sort the permutation and hierarchy are not valid (the
  // whole workgroup leaves: no barrier is skipped by part of it)
  if (hdr->bad & kBadSort) return;
  __shared__ uint64_t s_pw[kFitChunk];
  __shared__ int32_t s_slot[kFitChunk];
  __shared__ uint32_t s_cnt[kFitChunk];
  __shared__ int32_t s_ref[2 * kFitChunk];
  __shared__ float s_box[2 * kFitChunk * 6];
  // node and leaf indices fit in 31 bits (the parent words hold them)
  const int32_t c0 = (int32_t)blockIdx.x * kFitChunk, ni = (int32_t)(n - 1);
  // leaf and node r * kFitThreads + threadIdx.x of the chunk, for each r
  float b[kFitPerThread][6];
  int32_t ref[kFitPerThread];
  uint64_t pw[kFitPerThread];
#pragma unroll
  for (int r = 0; r < kFitPerThread; ++r) {
    const int t = r * kFitThreads + (int)threadIdx.x;
    const int32_t x = c0 + t;
    if (x < ni) {
      s_pw[t] = pw_int[x];
      s_slot[t] = fit_slot(pre, x, ni, hdr);
    }
    s_cnt[t] = 0;
    ref[r] = 0;
    pw[r] = 0;
    if (x < n) {
      const int32_t orig = perm[x];
      if (n > 1) pw[r] = pw_leaf[x];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[r][a] = KIND == ABX_PRIM_POINTS ? prims[3 * (int64_t)orig + a] : prims[6 * (int64_t)orig + a];
        b[r][3 + a] = KIND == ABX_PRIM_POINTS ? b[r][a] : prims[6 * (int64_t)orig + 3 + a];
      }
      if (KIND == ABX_PRIM_BOXES && box_rec) {
        // exact box record of a Q16 box tree, addressed by primitive index
        float4 *o = static_cast<float4 *>(box_rec) + 2 * (int64_t)orig;
        o[0] = make_float4(b[r][0], b[r][1], b[r][2], b[r][3]);
        o[1] = make_float4(b[r][4], b[r][5], __int_as_float(x), 0.0f);
      }
      ref[r] = ~orig;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kFitPerThread; ++r) {
    const int32_t x = c0 + r * kFitThreads + (int)threadIdx.x;
    if (x >= n || n == 1) break;
    float *bb = b[r];
    int32_t rf = ref[r];
    uint64_t w = pw[r];
    int h = 0;
    for (int step = 0; step < kFitMaxSteps; ++step) {
      // parent << 1 | side in the low word (unsigned: parents reach 2^31 - 2)
      const uint32_t pp = (uint32_t)w;
      const int32_t parent = (int32_t)(pp >> 1), j = (int32_t)(uint32_t)(w >> 32);
      const int side = (int)(pp & 1u);
      const int u = parent - c0;
      // the parent's range [min(parent, j), max(parent, j)] inside the chunk
      if ((uint32_t)u >= (uint32_t)kFitChunk || (uint32_t)(j - c0) >= (uint32_t)kFitChunk) {
        put_rec(stage + parent, side, bb, rf, h);
        fit_push(lists, parent < j ? parent : j, parent < j ? j : parent, (int32_t)pp, hdr);
        break;
      }
      const int mine = 2 * u + side, other = mine ^ 1;
#pragma unroll
      for (int a = 0; a < 6; ++a) s_box[6 * mine + a] = bb[a];
      s_ref[mine] = rf;
      // the first arrival leaves height + 1 (never 0); the second reads it
      // back, then leaves both heights and the done mark for the emit below
      const uint32_t old = __hip_atomic_fetch_max(&s_cnt[u], (uint32_t)h + 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      const uint32_t sh = old - 1u;
      s_cnt[u] = kFitDone | (side == 0 ? (uint32_t)h << 8 | sh : sh << 8 | (uint32_t)h);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bb[a] = fminf(bb[a], s_box[6 * other + a]);
        bb[3 + a] = fmaxf(bb[3 + a], s_box[6 * other + 3 + a]);
      }
      h = (h > (int)sh ? h : (int)sh) + 1;
      rf = s_slot[u];
      w = s_pw[u];
      if (parent == 0) {
        hdr->height = h;
        break;
      }
      if (step + 1 == kFitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
  __syncthreads();
  // emit: this thread's nodes that were finished inside the chunk
  QGrid g{};
  if (kQ16) g = load_grid(hdr);
#pragma unroll
  for (int r = 0; r < kFitPerThread; ++r) {
    const int t = r * kFitThreads + (int)threadIdx.x;
    if (c0 + t >= ni) break;
    const uint32_t c = s_cnt[t];
    const int32_t slot = s_slot[t];
    if ((c & kFitDone) && slot >= 0) {
      float b0[6], b1[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        b0[a] = s_box[12 * t + a];
        b1[a] = s_box[12 * t + 6 + a];
      }
      put_node<KIND, kQ16>(out, slot, b0, b1, s_ref[2 * t], s_ref[2 * t + 1], (int)((c >> 8) & 0xff),
                           (int)(c & 0xff), g);
    }
  }
}

// Phases 2 and 3: climbs from listed (node, side) entries whose records are
// staged.  kGroup: stop at nodes leaving group blockIdx.x and list them for
// the top pass.
//
// The climbs first run in LDS: the nodes they reach (a group's nodes whose
// range crosses one of its inner chunk edges, and the first node above the
// group on each path that leaves it) go into an open-addressing table keyed
// by node index that holds a node's arrival count and both child records, and
// arrivals are counted by LDS atomics at workgroup scope.  A step then waits
// on no global memory but the node's parent word and output slot (read-only),
// where the climb through global memory also waits for its record store, its
// arrival atomic and its sibling's record.  Nothing but the header's height
// is written to global memory until every climb of the workgroup has ended;
// the finished nodes and the exits are then written from the table.  A group
// whose nodes do not fit the table (1 520 top-pass nodes and at most 886 per
// group for 1e7 shell points; a pathological tree can reach
// 2 x 63 x 96 per group) climbs through global memory instead, from the same
// untouched lists and records.
constexpr int kFitHashLog2 = 11;
constexpr int kFitHash = 1 << kFitHashLog2;
constexpr uint32_t kFitExit = 1u << 30;  // table count of a node above the group (| side)

// probes of the table per node before a pass gives up on it
// (abx_set_refit_table_probes; 0 sends every pass through global memory)
std::atomic<uint32_t> g_fit_table_probes{kFitHash};

// slot of node x in the table (inserted if absent), -1 after `probes`
// occupied slots (the whole table by default)
__device__ __forceinline__ int fit_table_slot(int32_t *h_key, int32_t x, uint32_t probes) {
  const uint32_t h0 = ((uint32_t)x * 2654435761u) >> (32 - kFitHashLog2);
  for (uint32_t i = 0; i < probes; ++i) {
    const int s = (int)((h0 + (uint32_t)i) & (kFitHash - 1));
    const int32_t k = atomicCAS(&h_key[s], -1, x);
    if (k == -1 || k == x) return s;
  }
  return -1;
}

// the climbs of one workgroup through global memory (counters in `flags`,
// cleared by the hierarchy kernel; records in the staging nodes)
template <bool kQ16, bool kGroup>
__device__ void fit_climb_global(int64_t n, const uint64_t *__restrict__ pw_int,
                                 const int32_t *__restrict__ pre, NodeF32 *stage, uint32_t *flags,
                                 TreeHeader *hdr, const FitLists &lists, const int32_t *list,
                                 uint32_t cnt, int64_t g0, int64_t g1) {
  const int64_t ni = n - 1;
  for (uint32_t e = threadIdx.x; e < cnt; e += kFitThreads) {
    int32_t pp = list[e];
    int64_t parent = (int64_t)((uint32_t)pp >> 1);
    int side = pp & 1;
    float b[6];
    int32_t ref;
    int h;
    get_rec(stage + parent, side, b, ref, h);
    for (int step = 0; step < kFitMaxSteps; ++step) {
      // read-only: fetched ahead of the hand-off
      const uint64_t up = parent != 0 ? pw_int[parent] : 0;
      const int32_t slot = fit_slot(pre, parent, ni, hdr);
      const uint32_t old = __hip_atomic_fetch_add(flags + parent, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      // both records staged: the FP32 node is complete, a Q16 one is listed
      if (kQ16) {
        const uint32_t e2 = atomicAdd(lists.emit_count, 1u);
        if (e2 < lists.emit_cap) lists.emit[e2] = (int32_t)parent;
        else atomicOr(&hdr->bad, 4);
      }
      float sb[6];
      int32_t sref;
      int sh;
      get_rec(stage + parent, side ^ 1, sb, sref, sh);
      unite(b, sb);
      h = (h > sh ? h : sh) + 1;
      ref = slot;
      if (parent == 0) {
        hdr->height = h;
        break;
      }
      pp = (int32_t)(uint32_t)up;
      parent = (int64_t)((uint32_t)pp >> 1);
      side = pp & 1;
      put_rec(stage + parent, side, b, ref, h);
      if (kGroup) {
        const int64_t j = (int64_t)(uint32_t)(up >> 32);
        const int64_t f = parent < j ? parent : j, l = parent < j ? j : parent;
        if (f < g0 || l >= g1) {
          const uint32_t e2 = atomicAdd(lists.count, 1u);
          if (e2 < lists.top_cap) lists.top[e2] = pp;
          else atomicOr(&hdr->bad, 4);
          break;
        }
      }
      if (step + 1 == kFitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

template <bool kQ16, bool kGroup>
__global__ __launch_bounds__(kFitThreads) void k_fit_climb(
    int64_t n, const uint64_t *__restrict__ pw_int, const int32_t *__restrict__ pre,
    NodeF32 *stage, uint32_t *flags, TreeHeader *hdr, FitLists lists, uint32_t probes) {
  __shared__ int32_t h_key[kFitHash];
  __shared__ uint32_t h_cnt[kFitHash];
  __shared__ int32_t h_ref[2 * kFitHash];
  __shared__ int32_t h_ht[2 * kFitHash];
  __shared__ float h_box[12 * kFitHash];
  __shared__ uint32_t s_full;
  const int64_t ni = n - 1;
  const int64_t g0 = kGroup ? (int64_t)blockIdx.x * kFitGroupLeaves : 0;
  const int64_t g1 = g0 + kFitGroupLeaves;
  const int32_t *list = kGroup ? lists.group + (int64_t)blockIdx.x * kFitGroupCap : lists.top;
  const uint32_t cnt =
      min(lists.count[kGroup ? 1 + blockIdx.x : 0], kGroup ? kFitGroupCap : lists.top_cap);
  // A pass with E entries reaches at most E nodes (every node inside the
  // group takes two arrivals, entries or climbs from finished nodes, and an
  // exit one), so up to kFitHash entries always fit; far more than that
  // seldom do and go to global memory at once.
  if (cnt > 2u * kFitHash) {
    fit_climb_global<kQ16, kGroup>(n, pw_int, pre, stage, flags, hdr, lists, list, cnt, g0, g1);
    return;
  }
  for (int i = threadIdx.x; i < kFitHash; i += kFitThreads) {
    h_key[i] = -1;
    h_cnt[i] = 0;
  }
  if (threadIdx.x == 0) s_full = 0;
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < cnt; e += kFitThreads) {
    const int32_t pp0 = list[e];
    int32_t x = (int32_t)((uint32_t)pp0 >> 1);
    int side = pp0 & 1;
    float b[6];
    int32_t ref;
    int h;
    get_rec(stage + x, side, b, ref, h);
    for (int step = 0; step < kFitMaxSteps; ++step) {
      // read-only: fetched ahead of the hand-off
      const uint64_t up = x != 0 ? pw_int[x] : 0;
      const int32_t slot = fit_slot(pre, x, ni, hdr);
      const int sl = fit_table_slot(h_key, x, probes);
      if (sl < 0) {
        s_full = 1;
        break;
      }
      const int mine = 2 * sl + side, other = mine ^ 1;
#pragma unroll
      for (int a = 0; a < 6; ++a) h_box[6 * mine + a] = b[a];
      h_ref[mine] = ref;
      h_ht[mine] = h;
      const uint32_t old = __hip_atomic_fetch_add(&h_cnt[sl], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], h_box[6 * other + a]);
        b[3 + a] = fmaxf(b[3 + a], h_box[6 * other + 3 + a]);
      }
      const int sh = h_ht[other];
      h = (h > sh ? h : sh) + 1;
      ref = slot;
      if (x == 0) {
        hdr->height = h;
        break;
      }
      const int32_t pp = (int32_t)(uint32_t)up;
      x = (int32_t)((uint32_t)pp >> 1);
      side = pp & 1;
      if (kGroup) {
        const int64_t j = (int64_t)(uint32_t)(up >> 32);
        const int64_t f = x < j ? x : j, l = x < j ? j : x;
        if (f < g0 || l >= g1) {
          // the node above the group gets this one arrival from the group
          // (a node with both children inside the group lies inside it)
          const int se = fit_table_slot(h_key, x, probes);
          if (se < 0) {
            s_full = 1;
            break;
          }
          const int m2 = 2 * se + side;
#pragma unroll
          for (int a = 0; a < 6; ++a) h_box[6 * m2 + a] = b[a];
          h_ref[m2] = ref;
          h_ht[m2] = h;
          h_cnt[se] = kFitExit | (uint32_t)side;
          break;
        }
      }
      if (step + 1 == kFitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
  __syncthreads();
  if (s_full != 0) {
    fit_climb_global<kQ16, kGroup>(n, pw_int, pre, stage, flags, hdr, lists, list, cnt, g0, g1);
    return;
  }
  // write out: finished nodes whole, exits as staged records listed for the
  // top pass
  for (int sl = threadIdx.x; sl < kFitHash; sl += kFitThreads) {
    const int32_t x = h_key[sl];
    if (x < 0) continue;
    const uint32_t c = h_cnt[sl];
    if (c & kFitExit) {
      const int side = (int)(c & 1u);
      put_rec(stage + x, side, &h_box[12 * sl + 6 * side], h_ref[2 * sl + side], h_ht[2 * sl + side]);
      const uint32_t e2 = atomicAdd(lists.count, 1u);
      if (e2 < lists.top_cap) lists.top[e2] = (int32_t)(((uint32_t)x << 1) | (uint32_t)side);
      else atomicOr(&hdr->bad, 4);
    } else if (c == 2) {
      put_rec(stage + x, 0, &h_box[12 * sl], h_ref[2 * sl], h_ht[2 * sl]);
      put_rec(stage + x, 1, &h_box[12 * sl + 6], h_ref[2 * sl + 1], h_ht[2 * sl + 1]);
      if (kQ16) {
        const uint32_t e2 = atomicAdd(lists.emit_count, 1u);
        if (e2 < lists.emit_cap) lists.emit[e2] = x;
        else atomicOr(&hdr->bad, 4);
      }
    } else {
      // one arrival at a node inside the group: the lists did not form a tree
      atomicOr(&hdr->bad, 4);
    }
  }
}

// Q16 nodes finished by phases 2 and 3, quantised from their staged records
// (one thread per listed node)
template <int KIND>
__global__ __launch_bounds__(kBuildBlock) void k_fit_emit(int64_t n, const int32_t *__restrict__ pre,
                                                          const NodeF32 *__restrict__ stage,
                                                          void *out, TreeHeader *hdr,
                                                          FitLists lists) {
  const uint32_t cnt = min(*lists.emit_count, lists.emit_cap);
  const QGrid g = load_grid(hdr);
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
    const int64_t x = lists.emit[e];
    const int32_t slot = fit_slot(pre, x, n - 1, hdr);
    if (slot < 0) continue;
    float b0[6], b1[6];
    int32_t r0, r1;
    int h0, h1;
    get_rec(stage + x, 0, b0, r0, h0);
    get_rec(stage + x, 1, b1, r1, h1);
    put_node<KIND, true>(out, slot, b0, b1, r0, r1, h0, h1, g);
  }
}

// ------------------------------------------------------ depth-first order
// Nodes of a Karras tree renumbered in depth-first (pre-)order, left child
// first: the root is 0 and a node's left child follows it, so a walk going
// down touches consecutive nodes (C3 nearest walk 172 -> 166 ms).  The
// preorder index of a node with leaf range [l, r] is l + the number of its
// ancestors whose left subtree holds it: the internal nodes before it are its
// ancestors plus those of the subtrees left of l, which hold l leaves in as
// many subtrees as there are right turns on its path.  The count is a sum
// along the path to the root, taken by pointer jumping: every round adds the
// ancestor's partial sum and jumps twice as far (7 rounds cover paths of up
// to 128 edges; trees are at most ~95 deep).
constexpr int kPreRounds = 7;

// one 64-bit word per node: two counts summed along the path so far in the
// high half -- left turns (bits 0-15) and edges, i.e. the depth (bits 16-31;
// both stay below 128, so neither carries into the other) -- and the
// ancestor to add next (low half, -1 when the root has been passed), so a
// round gathers one word per node
__global__ __launch_bounds__(kBuildBlock) void k_pre_init(const uint64_t *__restrict__ pw_int,
                                                          int64_t ni, uint64_t *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const uint32_t pp = i == 0 ? 0u : (uint32_t)pw_int[i];  // parent << 1 | side
  const uint32_t left = i != 0 && (pp & 1u) == 0 ? 1u : 0u;  // a left child
  const uint32_t val = i != 0 ? left | (1u << 16) : 0u;
  const int32_t anc = i != 0 ? (int32_t)(pp >> 1) : -1;
  w[i] = ((uint64_t)val << 32) | (uint32_t)anc;
}

__global__ __launch_bounds__(kBuildBlock) void k_pre_jump(const uint64_t *__restrict__ in, int64_t ni,
                                                          uint64_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const uint64_t x = in[i];
  const int32_t a = (int32_t)(uint32_t)x;
  if (a >= 0 && a < ni) {
    const uint64_t y = in[a];
    out[i] = (((x >> 32) + (y >> 32)) << 32) | (uint32_t)y;
  } else {
    out[i] = (x & 0xffffffff00000000ull) | 0xffffffffu;
  }
}

// the last round: the finished count gives the index, first leaf of the
// node's range + left turns (-1 if the path was longer than the rounds), and
// the depth when asked for
__global__ __launch_bounds__(kBuildBlock) void k_pre_last(const uint64_t *__restrict__ in, int64_t ni,
                                                          const int32_t *__restrict__ other_end,
                                                          int32_t *__restrict__ pre,
                                                          int32_t *__restrict__ depth) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const uint64_t x = in[i];
  const int32_t a = (int32_t)(uint32_t)x;
  uint64_t v = x >> 32;
  int32_t rest = -1;
  if (a >= 0 && a < ni) {
    const uint64_t y = in[a];
    v += y >> 32;
    rest = (int32_t)(uint32_t)y;
  }
  const int64_t j = other_end[i];
  pre[i] = rest >= 0 ? -1 : (int32_t)((i < j ? i : j) + (int64_t)(v & 0xffffu));
  if (depth) depth[i] = rest >= 0 ? -1 : (int32_t)((v >> 16) & 0xffffu);
}

// scratch: 2 * ni words + ni int32 for the result (and ni for the depths)
abx_status launch_preorder(const uint64_t *pw_int, const int32_t *other_end, int64_t ni,
                           uint64_t *work, int32_t *pre, int32_t *depth, hipStream_t s) {
  if (ni <= 0) return ABX_OK;
  const unsigned g = grid_for(ni, kBuildBlock);
  uint64_t *buf[2] = {work, work + ni};
  ABX_TRY(launch("preorder", s, [&] { k_pre_init<<<g, kBuildBlock, 0, s>>>(pw_int, ni, buf[0]); }));
  for (int r = 0; r + 1 < kPreRounds; ++r) {
    const int a = r & 1, b = a ^ 1;
    ABX_TRY(launch("preorder", s, [&] { k_pre_jump<<<g, kBuildBlock, 0, s>>>(buf[a], ni, buf[b]); }));
  }
  const int f = (kPreRounds - 1) & 1;
  return launch("preorder", s, [&] {
    k_pre_last<<<g, kBuildBlock, 0, s>>>(buf[f], ni, other_end, pre, depth);
  });
}

// ------------------------------------------------------ 4-wide Q16 nodes
// Which binary nodes become 4-wide nodes: those at even depth, flagged at
// their depth-first position.  A scan of the flags then numbers the 4-wide
// nodes in depth-first order of the 4-wide tree (a binary node's left
// subtree precedes its right one, so the even-depth nodes keep that order).
__global__ __launch_bounds__(kBuildBlock) void k_wide_flags(const int32_t *__restrict__ pre,
                                                            const int32_t *__restrict__ depth,
                                                            int64_t ni, int32_t *__restrict__ flag,
                                                            TreeHeader *__restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni || (hdr->bad & kBadSort)) return;
  const int32_t p = pre[i], d = depth[i];
  if (p < 0 || p >= ni || d < 0) {
    atomicOr(&hdr->bad, 8);
    return;
  }
  flag[p] = (d & 1) == 0 ? 1 : 0;
}

// One thread per binary node at even depth: gather its grandchildren (a leaf
// child is kept as it is), quantise their boxes outward on the scene grid as
// k_quantise does (point leaves keep their float32 coordinates) and write the
// 4-wide node to its depth-first slot widx = rank[pre[i]].
template <int KIND>
__global__ __launch_bounds__(kBuildBlock) void k_wide_emit(const NodeF32 *__restrict__ src, int64_t ni,
                                                           const int32_t *__restrict__ pre,
                                                           const int32_t *__restrict__ depth,
                                                           const int32_t *__restrict__ rank,
                                                           TreeHeader *__restrict__ hdr,
                                                           NodeW *__restrict__ dst, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni || (hdr->bad & (4 | 8 | kBadSort))) return;
  if (i == 0) {
    const int32_t total = rank[ni];
    hdr->node_count = total;
    if (total < 1 || total > cap) atomicOr(&hdr->bad, 8);
  }
  if (depth[i] & 1) return;  // odd depth: folded into its parent
  const int64_t w = rank[pre[i]];
  if (w < 0 || w >= cap) {
    atomicOr(&hdr->bad, 8);
    return;
  }
  float o[3], sc[3], inv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = hdr->q_origin[a];
    sc[a] = hdr->q_scale[a];
    inv[a] = sc[a] != 0.0f ? 1.0f / sc[a] : 0.0f;
  }
  // Slots, without run-time indexing: a binary child that is a leaf gives
  // one slot (its own box), an internal one its two children.  With A0 A1
  // from the left child and B0 B1 from the right (A1, B1 only when that
  // child is internal) the slots are A0, then A1 if present, then B0, B1.
  const int4 d = src[i].d;
  const float *f = reinterpret_cast<const float *>(src + i);
  const bool ai = d.x >= 0, bi = d.y >= 0;
  if ((ai && d.x >= ni) || (bi && d.y >= ni)) {
    atomicOr(&hdr->bad, 8);
    return;
  }
  const float *ga = ai ? reinterpret_cast<const float *>(src + d.x) : f;
  const float *gb = bi ? reinterpret_cast<const float *>(src + d.y) : f;
  const int4 da = ai ? src[d.x].d : make_int4(0, 0, 0, 0);
  const int4 db = bi ? src[d.y].d : make_int4(0, 0, 0, 0);
  // 4-wide numbers of internal grandchildren
  auto wide_ref = [&](int32_t g, bool &ok) -> int32_t {
    if (g < 0) return g;
    if (g >= ni || pre[g] < 0 || pre[g] >= ni) {
      ok = false;
      return kEmptyRef;
    }
    return rank[pre[g]];
  };
  bool ok = true;
  const int32_t ra0 = ai ? wide_ref(da.x, ok) : d.x, ra1 = ai ? wide_ref(da.y, ok) : kEmptyRef;
  const int32_t rb0 = bi ? wide_ref(db.x, ok) : d.y, rb1 = bi ? wide_ref(db.y, ok) : kEmptyRef;
  if (!ok) {
    atomicOr(&hdr->bad, 8);
    return;
  }
  // A0 = left leaf or its first child, A1 its second child; B0, B1 the same
  // on the right
  const float *pa0 = ai ? ga : f, *pa1 = ga + 6, *pb0 = bi ? gb : f + 6, *pb1 = gb + 6;
  // the slots, by selects only: A0, then A1 if present, then B0, then B1
  // if present
  const float *ps[4] = {pa0, ai ? pa1 : pb0, ai ? pb0 : pb1, pb1};
  const int32_t rs[4] = {ra0, ai ? ra1 : rb0, ai ? rb0 : (bi ? rb1 : kEmptyRef), ai && bi ? rb1 : kEmptyRef};
  const bool used[4] = {true, true, ai || bi, ai && bi};
  float box[4][6];
  int32_t ref[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int e = 0; e < 6; ++e) box[c][e] = used[c] ? ps[c][e] : 0.0f;
    ref[c] = rs[c];
  }
  uint32_t wd[12];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (!used[c]) {
      wd[3 * c] = wd[3 * c + 1] = wd[3 * c + 2] = 0u;
    } else if (KIND == ABX_PRIM_POINTS && ref[c] < 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) wd[3 * c + a] = __float_as_uint(box[c][a]);
    } else {
      uint32_t q[6];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        q[a] = q_lo(box[c][a], o[a], sc[a], inv[a]);
        q[3 + a] = q_hi(box[c][3 + a], o[a], sc[a], inv[a]);
      }
#pragma unroll
      for (int h = 0; h < 3; ++h) wd[3 * c + h] = q[2 * h] | (q[2 * h + 1] << 16);
    }
  }
  NodeW out;
  out.a = make_uint4(wd[0], wd[1], wd[2], wd[3]);
  out.b = make_uint4(wd[4], wd[5], wd[6], wd[7]);
  out.c = make_uint4(wd[8], wd[9], wd[10], wd[11]);
  out.d = make_uint4((uint32_t)ref[0], (uint32_t)ref[1], (uint32_t)ref[2], (uint32_t)ref[3]);
  dst[w] = out;
}

// flags [ni], rank [ni + 1] (exclusive scan of the flags), scan scratch
abx_status launch_wide(int kind, const NodeF32 *src, int64_t ni, const int32_t *pre,
                       const int32_t *depth, int32_t *flag, int32_t *rank, int64_t *d_total,
                       void *scan_scratch, size_t scan_bytes, TreeHeader *hdr, NodeW *dst,
                       hipStream_t s) {
  if (ni <= 0) return ABX_OK;
  const unsigned g = grid_for(ni, kBuildBlock);
  ABX_TRY(launch("wide_flags", s, [&] {
    k_wide_flags<<<g, kBuildBlock, 0, s>>>(pre, depth, ni, flag, hdr);
  }));
  ABX_TRY(exclusive_scan(flag, ni, rank, d_total, scan_scratch, scan_bytes, s));
  const int64_t cap = wide_node_cap(ni);
  if (kind == ABX_PRIM_POINTS)
    return launch("wide_emit", s, [&] {
      k_wide_emit<ABX_PRIM_POINTS><<<g, kBuildBlock, 0, s>>>(src, ni, pre, depth, rank, hdr, dst, cap);
    });
  return launch("wide_emit", s, [&] {
    k_wide_emit<ABX_PRIM_BOXES><<<g, kBuildBlock, 0, s>>>(src, ni, pre, depth, rank, hdr, dst, cap);
  });
}

// ------------------------------------------------------------ host launchers
abx_status launch_scene(int kind, const float *prims, int64_t n, float *partial, int blocks,
                        TreeHeader *hdr, hipStream_t s) {
  ABX_TRY(launch("header_init", s, [&] { k_header_init<<<1, 64, 0, s>>>(hdr); }));
  if (kind == ABX_PRIM_POINTS)
    ABX_TRY(launch("scene_partial", s, [&] {
      k_scene_partial<ABX_PRIM_POINTS><<<blocks, kBuildBlock, 0, s>>>(prims, n, partial);
    }));
  else
    ABX_TRY(launch("scene_partial", s, [&] {
      k_scene_partial<ABX_PRIM_BOXES><<<blocks, kBuildBlock, 0, s>>>(prims, n, partial);
    }));
  return launch("scene_final", s, [&] { k_scene_final<<<1, kSceneFinalThreads, 0, s>>>(partial, blocks, hdr); });
}

int scene_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kScenePartials, (n + 4095) / 4096));
}

abx_status launch_morton(int kind, const float *prims, int64_t n, const float *scene, int bits,
                         void *codes, bool wide, hipStream_t s) {
  if (n == 0) return ABX_OK;
  const unsigned g = grid_for(n, kBuildBlock);
  if (!wide) {
    uint32_t *c = static_cast<uint32_t *>(codes);
    if (kind == ABX_PRIM_POINTS)
      return launch("morton", s, [&] {
        k_morton<ABX_PRIM_POINTS, uint32_t><<<g, kBuildBlock, 0, s>>>(prims, n, scene, bits, c);
      });
    return launch("morton", s, [&] {
      k_morton<ABX_PRIM_BOXES, uint32_t><<<g, kBuildBlock, 0, s>>>(prims, n, scene, bits, c);
    });
  }
  uint64_t *c = static_cast<uint64_t *>(codes);
  if (kind == ABX_PRIM_POINTS)
    return launch("morton", s, [&] {
      k_morton<ABX_PRIM_POINTS, uint64_t><<<g, kBuildBlock, 0, s>>>(prims, n, scene, bits, c);
    });
  return launch("morton", s, [&] {
    k_morton<ABX_PRIM_BOXES, uint64_t><<<g, kBuildBlock, 0, s>>>(prims, n, scene, bits, c);
  });
}

abx_status launch_karras(bool wide, const void *keys, int64_t n, uint64_t *pw_leaf, uint64_t *pw_int,
                         int32_t *other_end, uint32_t *flags, const TreeHeader *hdr, hipStream_t s) {
  if (n < 2) return ABX_OK;
  const unsigned g = grid_for(n - 1, kBuildBlock);
  if (wide)
    return launch("karras", s, [&] {
      k_karras<uint64_t><<<g, kBuildBlock, 0, s>>>(static_cast<const uint64_t *>(keys), n, pw_leaf,
                                                   pw_int, other_end, flags, hdr);
    });
  return launch("karras", s, [&] {
    k_karras<uint32_t><<<g, kBuildBlock, 0, s>>>(static_cast<const uint32_t *>(keys), n, pw_leaf,
                                                 pw_int, other_end, flags, hdr);
  });
}

// lists of the refit (and of the agglomerative build, which shares the region)
size_t refit_lists_bytes(int64_t n) {
  const size_t agglo = 256 + 2 * agglo_frontier_cap(n) * 4;
  const size_t fit = fit_lists_bytes(n);
  return fit > agglo ? fit : agglo;
}

abx_status launch_refit(int kind, bool q16, const float *prims, const int32_t *perm, int64_t n,
                        const uint64_t *pw_leaf, const uint64_t *pw_int, const int32_t *pre,
                        void *out, NodeF32 *stage, uint32_t *flags, TreeHeader *hdr, void *box_rec,
                        void *lists_mem, hipStream_t s) {
  if (n == 0) return ABX_OK;
  const FitLists L = fit_lists(lists_mem, n);
  const int64_t groups = fit_groups(n);
  ABX_TRY(fill_u32(L.count, 0, (size_t)(2 + groups), s));
  const unsigned g = grid_for(n, kFitChunk);
#define ABX_FIT(KD, QQ)                                                                        \
  ABX_TRY(launch("refit", s, [&] {                                                             \
    k_fit_chunk<KD, QQ><<<g, kFitThreads, 0, s>>>(prims, perm, n, pw_leaf, pw_int, pre, out,   \
                                                  stage, hdr, box_rec, L);                     \
  }))
  if (kind == ABX_PRIM_POINTS) {
    if (q16) ABX_FIT(ABX_PRIM_POINTS, true);
    else ABX_FIT(ABX_PRIM_POINTS, false);
  } else {
    if (q16) ABX_FIT(ABX_PRIM_BOXES, true);
    else ABX_FIT(ABX_PRIM_BOXES, false);
  }
#undef ABX_FIT
  if (n <= kFitChunk) return ABX_OK;
  const uint32_t probes = std::min<uint32_t>(g_fit_table_probes.load(std::memory_order_relaxed), kFitHash);
  ABX_TRY(launch("refit_mid", s, [&] {
    if (q16)
      k_fit_climb<true, true><<<(unsigned)groups, kFitThreads, 0, s>>>(n, pw_int, pre, stage, flags,
                                                                       hdr, L, probes);
    else
      k_fit_climb<false, true><<<(unsigned)groups, kFitThreads, 0, s>>>(n, pw_int, pre, stage,
                                                                        flags, hdr, L, probes);
  }));
  if (n > kFitGroupLeaves)
    ABX_TRY(launch("refit_top", s, [&] {
      if (q16)
        k_fit_climb<true, false><<<1, kFitThreads, 0, s>>>(n, pw_int, pre, stage, flags, hdr, L,
                                                           probes);
      else
        k_fit_climb<false, false><<<1, kFitThreads, 0, s>>>(n, pw_int, pre, stage, flags, hdr, L,
                                                            probes);
    }));
  if (!q16) return ABX_OK;
  const unsigned ge = (unsigned)std::min<int64_t>(grid_for(L.emit_cap, kBuildBlock), 1024);
  return launch("refit_emit", s, [&] {
    if (kind == ABX_PRIM_POINTS)
      k_fit_emit<ABX_PRIM_POINTS><<<ge, kBuildBlock, 0, s>>>(n, pre, stage, out, hdr, L);
    else
      k_fit_emit<ABX_PRIM_BOXES><<<ge, kBuildBlock, 0, s>>>(n, pre, stage, out, hdr, L);
  });
}

abx_status launch_quantise(int kind, const NodeF32 *src, int64_t ni, TreeHeader *hdr,
                           const int32_t *pre, NodeQ16 *dst, hipStream_t s) {
  if (ni <= 0) return ABX_OK;
  const unsigned g = grid_for(ni, kBuildBlock);
  if (kind == ABX_PRIM_POINTS)
    return launch("quantise", s, [&] {
      k_quantise<ABX_PRIM_POINTS><<<g, kBuildBlock, 0, s>>>(src, ni, hdr, pre, dst);
    });
  return launch("quantise", s, [&] {
    k_quantise<ABX_PRIM_BOXES><<<g, kBuildBlock, 0, s>>>(src, ni, hdr, pre, dst);
  });
}

// Middle pass of the agglomerative build (one workgroup per group of
// kMidChunks chunks): climbs from the frontier entries whose split lies
// strictly inside the group (both of its leaves in the group), through
// splits inside the group only.  Every node it completes has all its splits
// in the group, so every arrival it counts comes from this workgroup; a
// split on or beyond the group's edge goes to the last pass's list
// uncounted, as the chunk pass does at chunk edges.
template <typename K>
__global__ __launch_bounds__(kRefitThreads) void k_agglo_mid(const K *__restrict__ keys, int64_t n,
                                                             NodeF32 *nodes, int32_t *range_lo,
                                                             int32_t *range_hi, uint32_t *flags,
                                                             TreeHeader *hdr,
                                                             const int32_t *__restrict__ fa,
                                                             const uint32_t *__restrict__ fa_count,
                                                             int32_t *__restrict__ fb,
                                                             uint32_t *__restrict__ fb_count,
                                                             uint32_t cap) {
  __shared__ int32_t s_list[kMidListCap];
  __shared__ uint32_t s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const uint32_t cnt = min(*fa_count, cap);
  const int64_t s0 = (int64_t)blockIdx.x * kMidLeaves, s1 = s0 + kMidLeaves;
  const int64_t last = (s1 < n ? s1 : n) - 2;  // last split inside the group
  for (uint32_t e = threadIdx.x; e < cnt; e += kRefitThreads) {
    const int64_t p = fa[e];
    if (p < s0 || p >= s1) continue;  // another group's entry
    if (p > last) {
      const uint32_t i = atomicAdd(fb_count, 1u);
      if (i < cap) fb[i] = (int32_t)p;
      else atomicOr(&hdr->bad, 4);
    } else {
      const uint32_t i = atomicAdd(&s_n, 1u);
      if (i < (uint32_t)kMidListCap) s_list[i] = (int32_t)p;
    }
  }
  __syncthreads();
  const uint32_t own = min(s_n, (uint32_t)kMidListCap);
  if (threadIdx.x == 0 && s_n > (uint32_t)kMidListCap) atomicOr(&hdr->bad, 4);
  for (uint32_t e = threadIdx.x; e < own; e += kRefitThreads) {
    int64_t p = s_list[e];
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const uint32_t old = __hip_atomic_fetch_add(flags + p, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float b[6], sb[6];
      int h, sh;
      load_child(nodes + p, 0, b, h);
      load_child(nodes + p, 1, sb, sh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      const int64_t l = range_lo[p], r = range_hi[p];
      if (l == 0 && r == n - 1) {
        hdr->root = (int32_t)p;
        hdr->height = h;
        break;
      }
      const bool left = l == 0 || (r != n - 1 && delta(keys, n, r, keys[r], r + 1) >
                                                     delta(keys, n, l - 1, keys[l - 1], l));
      const int64_t q = left ? r : l - 1;
      const int side = left ? 0 : 1;
      store_child(nodes + q, side, b, h);
      reinterpret_cast<int32_t *>(nodes + q)[12 + side] = (int32_t)p;
      if (left) range_lo[q] = (int32_t)l;
      else range_hi[q] = (int32_t)r;
      if (q < s0 || q > last) {
        const uint32_t i = atomicAdd(fb_count, 1u);
        if (i < cap) fb[i] = (int32_t)q;
        else atomicOr(&hdr->bad, 4);
        break;
      }
      p = q;
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

abx_status launch_agglo(bool wide, int kind, bool q16, const void *keys, const float *prims,
                        const int32_t *perm, int64_t n, NodeF32 *nodes, int32_t *range_lo,
                        int32_t *range_hi, uint32_t *flags, TreeHeader *hdr, void *q16_leaves,
                        int32_t *frontier, uint32_t *frontier_count, hipStream_t s) {
  if (n == 0) return ABX_OK;
  const unsigned g = grid_for(n, kRefitChunk);
  const uint32_t cap = (uint32_t)agglo_frontier_cap(n);
  ABX_TRY(fill_u32(frontier_count, 0, 2, s));
#define ABX_AGG(KT, KD, QQ)                                                                       \
  ABX_TRY(launch("agglo", s, [&] {                                                               \
    k_agglo_local<KT, KD, QQ><<<g, kRefitThreads, 0, s>>>(static_cast<const KT *>(keys), prims,  \
                                                          perm, n, nodes, range_lo, range_hi,    \
                                                          flags, hdr, q16_leaves, frontier,      \
                                                          frontier_count, cap);                  \
  }))
#define ABX_AGG_KIND(KT)                                                 \
  if (kind == ABX_PRIM_POINTS) {                                         \
    if (q16) ABX_AGG(KT, ABX_PRIM_POINTS, true);                         \
    else ABX_AGG(KT, ABX_PRIM_POINTS, false);                            \
  } else {                                                               \
    if (q16) ABX_AGG(KT, ABX_PRIM_BOXES, true);                          \
    else ABX_AGG(KT, ABX_PRIM_BOXES, false);                             \
  }
  if (wide) {
    ABX_AGG_KIND(uint64_t)
  } else {
    ABX_AGG_KIND(uint32_t)
  }
#undef ABX_AGG_KIND
#undef ABX_AGG
  if (n <= kRefitChunk) return ABX_OK;
  int32_t *frontier2 = frontier + cap;
  const unsigned g2 = (unsigned)((n + kMidLeaves - 1) / kMidLeaves);
  if (wide) {
    const uint64_t *k64 = static_cast<const uint64_t *>(keys);
    ABX_TRY(launch("agglo_mid", s, [&] {
      k_agglo_mid<uint64_t><<<g2, kRefitThreads, 0, s>>>(k64, n, nodes, range_lo, range_hi, flags,
                                                         hdr, frontier, frontier_count, frontier2,
                                                         frontier_count + 1, cap);
    }));
    if (n <= kMidLeaves) return ABX_OK;
    return launch("agglo_top", s, [&] {
      k_agglo_top<uint64_t><<<1, kRefitThreads, 0, s>>>(k64, n, nodes, range_lo, range_hi, flags,
                                                        hdr, frontier2, frontier_count + 1, cap);
    });
  }
  const uint32_t *k32 = static_cast<const uint32_t *>(keys);
  ABX_TRY(launch("agglo_mid", s, [&] {
    k_agglo_mid<uint32_t><<<g2, kRefitThreads, 0, s>>>(k32, n, nodes, range_lo, range_hi, flags,
                                                       hdr, frontier, frontier_count, frontier2,
                                                       frontier_count + 1, cap);
  }));
  if (n <= kMidLeaves) return ABX_OK;
  return launch("agglo_top", s, [&] {
    k_agglo_top<uint32_t><<<1, kRefitThreads, 0, s>>>(k32, n, nodes, range_lo, range_hi, flags, hdr,
                                                      frontier2, frontier_count + 1, cap);
  });
}

}  // namespace abx
