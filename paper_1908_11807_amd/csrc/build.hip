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

// One thread per internal node i: direction from the neighbours, range end
// by exponential then binary search, split by binary search on the prefix,
// children at gamma / gamma+1 (leaf when the child range has one element).
// Writes the two child references, the parents (parent<<1 | side), the far
// end j of the node's range [min(i,j), max(i,j)] and clears the node's
// arrival counter.
template <typename K>
__global__ __launch_bounds__(kBuildBlock) void k_karras(const K *__restrict__ keys, int64_t n,
                                                        NodeF32 *__restrict__ nodes,
                                                        int32_t *__restrict__ parent_leaf,
                                                        int32_t *__restrict__ parent_int,
                                                        int32_t *__restrict__ other_end,
                                                        uint32_t *__restrict__ flags,
                                                        const TreeHeader *__restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the searches stay inside [i, j] only over sorted keys: after a failed
  // sort nothing is built (the refit skips as well)
  if (i >= n - 1 || (hdr->bad & kBadSort)) return;
  const K ki = keys[i];
  const int d = delta(keys, n, i, ki, i + 1) - delta(keys, n, i, ki, i - 1) >= 0 ? 1 : -1;
  const int dmin = delta(keys, n, i, ki, i - d);
  int64_t lmax = 2;
  while (delta(keys, n, i, ki, i + lmax * d) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(keys, n, i, ki, i + (l + t) * d) > dmin) l += t;
  const int64_t j = i + l * d;
  const int dnode = delta(keys, n, i, ki, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(keys, n, i, ki, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
  const int64_t first = i < j ? i : j, last = i < j ? j : i;
  const bool left_leaf = first == gamma, right_leaf = last == gamma + 1;
  const int32_t lref = left_leaf ? ~(int32_t)gamma : (int32_t)gamma;
  const int32_t rref = right_leaf ? ~(int32_t)(gamma + 1) : (int32_t)(gamma + 1);
  nodes[i].d = make_int4(lref, rref, 0, 0);
  const int32_t pl = (int32_t)(i << 1), pr = (int32_t)((i << 1) | 1);
  if (left_leaf) parent_leaf[gamma] = pl; else parent_int[gamma] = pl;
  if (right_leaf) parent_leaf[gamma + 1] = pr; else parent_int[gamma + 1] = pr;
  other_end[i] = (int32_t)j;
  flags[i] = 0;
}

// ------------------------------------------------------------ bottom-up refit
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

// Bottom-up refit in two launches.  One thread per leaf climbs from its
// leaf: at each parent it writes its box into its child slot, then counts
// its arrival; the first arrival stops, the second unions both children and
// climbs on.  The leaf's thread also rewrites its parent's reference to the
// leaf from the sorted position to ~(primitive index), and for Q16 box trees
// writes the exact box record.
//
// Phase 1: each workgroup owns a chunk of kRefitChunk consecutive leaves (in
// sorted order).  An internal node whose leaf range lies inside the chunk has
// both children climbed by threads of the same workgroup, so the hand-off is
// synchronised at workgroup scope (arrival counter in LDS; the sibling's box
// is read back from the node in global memory, ordered by the counter's
// acquire-release).  A thread that reaches a node whose range crosses the
// chunk boundary stops there and appends (node, side) to the frontier list.
// Phase 2 (one workgroup per 64 chunks) climbs the crossing nodes inside its
// 64 chunks; phase 3 (one workgroup) the few that cross those groups.  Each
// phase starts after a kernel boundary has made the previous one's stores
// visible and synchronises at workgroup scope.  No step needs agent-scope
// fences (which would write back and invalidate the XCDs' L2s).
constexpr int kRefitThreads = 1024;
constexpr int kRefitPerThread = 8;
constexpr int kRefitChunk = kRefitThreads * kRefitPerThread;
constexpr int kRefitMaxSteps = 256;  // > any tree height; only bounds the loops

template <int KIND, bool kQ16>
__global__ __launch_bounds__(kRefitThreads) void k_refit_local(
    const float *__restrict__ prims, const int32_t *__restrict__ perm, int64_t n,
    const int32_t *__restrict__ parent_leaf, const int32_t *__restrict__ parent_int,
    const int32_t *__restrict__ other_end, NodeF32 *nodes, TreeHeader *hdr, void *q16_leaves,
    int32_t *__restrict__ frontier, uint32_t *__restrict__ frontier_count, uint32_t frontier_cap) {
  // after a failed sort the permutation and hierarchy are not valid: the
  // whole grid exits (the frontier stays empty, so the later phases do too)
  if (hdr->bad & kBadSort) return;
  __shared__ uint32_t s_cnt[kRefitChunk];
  for (int i = threadIdx.x; i < kRefitChunk; i += kRefitThreads) s_cnt[i] = 0;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kRefitChunk;
  for (int r = 0; r < kRefitPerThread; ++r) {
    const int64_t p = c0 + (int64_t)r * kRefitThreads + threadIdx.x;
    if (p >= n) return;
    const int32_t orig = perm[p];
    float b[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = KIND == ABX_PRIM_POINTS ? prims[3 * (int64_t)orig + a] : prims[6 * (int64_t)orig + a];
      b[3 + a] = KIND == ABX_PRIM_POINTS ? b[a] : prims[6 * (int64_t)orig + 3 + a];
    }
    if (kQ16 && KIND == ABX_PRIM_BOXES) {
      // exact box record of a Q16 box tree, addressed by primitive index
      float4 *o = reinterpret_cast<float4 *>(q16_leaves) + 2 * (int64_t)orig;
      o[0] = make_float4(b[0], b[1], b[2], b[3]);
      o[1] = make_float4(b[4], b[5], __int_as_float((int32_t)p), 0.0f);
    }
    if (n == 1) return;
    int h = 0;
    int32_t pp = parent_leaf[p];
    // the parent's reference to this leaf names the primitive itself
    reinterpret_cast<int32_t *>(nodes + (pp >> 1))[12 + (pp & 1)] = ~orig;
    int64_t j = other_end[pp >> 1];
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const int32_t parent = pp >> 1, side = pp & 1;
      // The climb is a chain of dependent reads.  The hierarchy arrays are
      // read-only here, so the next parent is fetched before this level's
      // hand-off and the next range end while the sibling's box is read:
      // one exposed memory latency per level instead of three.
      const int32_t up = parent_int[parent];
      store_child(nodes + parent, side, b, h);
      const int64_t f = parent < j ? parent : j, l = parent < j ? j : parent;
      if (f < c0 || l >= c0 + kRefitChunk) {
        const uint32_t e = atomicAdd(frontier_count, 1u);
        if (e < frontier_cap) frontier[e] = pp;
        else atomicOr(&hdr->bad, 4);
        break;
      }
      const uint32_t old = __hip_atomic_fetch_add(&s_cnt[parent - c0], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float sb[6];
      int sh;
      load_child(nodes + parent, side ^ 1, sb, sh);
      const int64_t jn = parent != 0 ? other_end[up >> 1] : 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      if (parent == 0) {
        hdr->height = h;
        break;
      }
      pp = up;
      j = jn;
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

// Phase 2: one workgroup per super-chunk of kMidChunks chunks climbs the
// chunk-crossing nodes whose leaf range lies inside its super-chunk.  All
// arrivals at such a node come from that workgroup (from its own entries or
// its own climbs), so workgroup-scope counters in global memory suffice.  A
// climb that reaches a node crossing a super-chunk boundary stores its box
// there and hands (node, side) to the last phase.  Entries are routed by the
// super-chunk holding the first leaf of the node's range; each workgroup
// reads the whole list in unrolled batches, so the reads overlap.
constexpr int kMidChunks = 64;
constexpr int64_t kMidLeaves = (int64_t)kRefitChunk * kMidChunks;
// A crossing node inside a super-chunk is an ancestor of the split at one of
// its kMidChunks - 1 inner chunk boundaries, so there are at most
// (kMidChunks - 1) * (tree height, < 96 for 63-bit keys augmented by 31-bit
// positions) of them, each with at most two entries.
constexpr int kMidListCap = 2 * kMidChunks * 96;

__global__ __launch_bounds__(kRefitThreads) void k_refit_mid(
    const int32_t *__restrict__ parent_int, const int32_t *__restrict__ other_end, NodeF32 *nodes,
    uint32_t *flags, TreeHeader *hdr, const int32_t *__restrict__ fa,
    const uint32_t *__restrict__ fa_count, int32_t *__restrict__ fb, uint32_t *__restrict__ fb_count,
    uint32_t cap) {
  __shared__ int32_t s_list[kMidListCap];
  __shared__ uint32_t s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const uint32_t cnt = min(*fa_count, cap);
  const int64_t s0 = (int64_t)blockIdx.x * kMidLeaves, s1 = s0 + kMidLeaves;
  constexpr int kBatch = 8;
  for (uint32_t e0 = threadIdx.x; e0 < cnt; e0 += kBatch * kRefitThreads) {
    int32_t pp[kBatch], j[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t e = e0 + (uint32_t)u * kRefitThreads;
      pp[u] = e < cnt ? fa[e] : -1;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) j[u] = pp[u] >= 0 ? other_end[pp[u] >> 1] : 0;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (pp[u] < 0) continue;
      const int64_t p = pp[u] >> 1;
      const int64_t f = p < j[u] ? p : j[u], l = p < j[u] ? j[u] : p;
      if (f < s0 || f >= s1) continue;  // another super-chunk's entry
      if (l >= s1) {
        const uint32_t e = atomicAdd(fb_count, 1u);
        if (e < cap) fb[e] = pp[u];
        else atomicOr(&hdr->bad, 4);
      } else {
        const uint32_t e = atomicAdd(&s_n, 1u);
        if (e < (uint32_t)kMidListCap) s_list[e] = pp[u];
      }
    }
  }
  __syncthreads();
  const uint32_t own = min(s_n, (uint32_t)kMidListCap);
  if (threadIdx.x == 0 && s_n > (uint32_t)kMidListCap) atomicOr(&hdr->bad, 4);
  for (uint32_t e = threadIdx.x; e < own; e += kRefitThreads) {
    int32_t pp = s_list[e];
    int32_t parent = pp >> 1, side = pp & 1;
    float b[6];
    int h;
    load_child(nodes + parent, side, b, h);
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const int32_t up = parent_int[parent];  // read-only: overlaps the hand-off
      const uint32_t old = __hip_atomic_fetch_add(flags + parent, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float sb[6];
      int sh;
      load_child(nodes + parent, side ^ 1, sb, sh);
      const int64_t jn = parent != 0 ? other_end[up >> 1] : 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      if (parent == 0) {
        hdr->height = h;
        break;
      }
      pp = up;
      parent = pp >> 1;
      side = pp & 1;
      store_child(nodes + parent, side, b, h);
      const int64_t f = parent < jn ? parent : jn, l = parent < jn ? jn : parent;
      if (f < s0 || l >= s1) {
        const uint32_t e2 = atomicAdd(fb_count, 1u);
        if (e2 < cap) fb[e2] = pp;
        else atomicOr(&hdr->bad, 4);
        break;
      }
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

// Phase 3: one workgroup climbs the nodes that cross super-chunk boundaries.
// The arrival counters are the global `flags` (cleared by the hierarchy
// kernel); every hand-off is between threads of this one workgroup.
__global__ __launch_bounds__(kRefitThreads) void k_refit_top(const int32_t *__restrict__ parent_int,
                                                             NodeF32 *nodes, uint32_t *flags,
                                                             TreeHeader *hdr,
                                                             const int32_t *__restrict__ frontier,
                                                             const uint32_t *__restrict__ frontier_count,
                                                             uint32_t frontier_cap) {
  const uint32_t cnt = min(*frontier_count, frontier_cap);
  for (uint32_t e = threadIdx.x; e < cnt; e += kRefitThreads) {
    int32_t pp = frontier[e];
    int32_t parent = pp >> 1, side = pp & 1;
    float b[6];
    int h;
    load_child(nodes + parent, side, b, h);
    for (int step = 0; step < kRefitMaxSteps; ++step) {
      const int32_t up = parent_int[parent];  // read-only: overlaps the hand-off
      const uint32_t old = __hip_atomic_fetch_add(flags + parent, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      float sb[6];
      int sh;
      load_child(nodes + parent, side ^ 1, sb, sh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], sb[a]);
        b[3 + a] = fmaxf(b[3 + a], sb[3 + a]);
      }
      h = (h > sh ? h : sh) + 1;
      if (parent == 0) {
        hdr->height = h;
        break;
      }
      pp = up;
      parent = pp >> 1;
      side = pp & 1;
      store_child(nodes + parent, side, b, h);
      if (step + 1 == kRefitMaxSteps) atomicOr(&hdr->bad, 4);
    }
  }
}

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

// frontier entries: a crossing node has at most two, and every crossing node
// lies on the root path of some chunk boundary
size_t refit_frontier_cap(int64_t n) {
  const int64_t chunks = (n + kRefitChunk - 1) / kRefitChunk;
  return 2 * (size_t)(2 * 128 * chunks + 64);  // two lists: chunk and super-chunk crossings
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
__global__ __launch_bounds__(kBuildBlock) void k_pre_init(const int32_t *__restrict__ parent_int,
                                                          int64_t ni, uint64_t *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const int32_t pp = i == 0 ? -1 : parent_int[i];
  const uint32_t left = pp >= 0 && (pp & 1) == 0 ? 1u : 0u;  // a left child
  const uint32_t val = pp >= 0 ? left | (1u << 16) : 0u;
  const int32_t anc = pp >= 0 ? pp >> 1 : -1;
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
abx_status launch_preorder(const int32_t *parent_int, const int32_t *other_end, int64_t ni,
                           uint64_t *work, int32_t *pre, int32_t *depth, hipStream_t s) {
  if (ni <= 0) return ABX_OK;
  const unsigned g = grid_for(ni, kBuildBlock);
  uint64_t *buf[2] = {work, work + ni};
  ABX_TRY(launch("preorder", s, [&] { k_pre_init<<<g, kBuildBlock, 0, s>>>(parent_int, ni, buf[0]); }));
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

abx_status launch_karras(bool wide, const void *keys, int64_t n, NodeF32 *nodes,
                         int32_t *parent_leaf, int32_t *parent_int, int32_t *other_end,
                         uint32_t *flags, const TreeHeader *hdr, hipStream_t s) {
  if (n < 2) return ABX_OK;
  const unsigned g = grid_for(n - 1, kBuildBlock);
  if (wide)
    return launch("karras", s, [&] {
      k_karras<uint64_t><<<g, kBuildBlock, 0, s>>>(static_cast<const uint64_t *>(keys), n, nodes,
                                                   parent_leaf, parent_int, other_end, flags, hdr);
    });
  return launch("karras", s, [&] {
    k_karras<uint32_t><<<g, kBuildBlock, 0, s>>>(static_cast<const uint32_t *>(keys), n, nodes,
                                                 parent_leaf, parent_int, other_end, flags, hdr);
  });
}

abx_status launch_refit(int kind, bool q16, const float *prims, const int32_t *perm, int64_t n,
                        const int32_t *parent_leaf, const int32_t *parent_int,
                        const int32_t *other_end, NodeF32 *nodes, uint32_t *flags,
                        TreeHeader *hdr, void *q16_leaves, int32_t *frontier,
                        uint32_t *frontier_count, hipStream_t s) {
  if (n == 0) return ABX_OK;
  const unsigned g = grid_for(n, kRefitChunk);
  const uint32_t cap = (uint32_t)(refit_frontier_cap(n) / 2);  // per list
  ABX_TRY(fill_u32(frontier_count, 0, 2, s));
#define ABX_REFIT(KD, QQ)                                                                        \
  ABX_TRY(launch("refit", s, [&] {                                                              \
    k_refit_local<KD, QQ><<<g, kRefitThreads, 0, s>>>(prims, perm, n, parent_leaf, parent_int, \
                                                       other_end, nodes, hdr, q16_leaves,       \
                                                       frontier, frontier_count, cap);          \
  }))
  if (kind == ABX_PRIM_POINTS) {
    if (q16) ABX_REFIT(ABX_PRIM_POINTS, true);
    else ABX_REFIT(ABX_PRIM_POINTS, false);
  } else {
    if (q16) ABX_REFIT(ABX_PRIM_BOXES, true);
    else ABX_REFIT(ABX_PRIM_BOXES, false);
  }
#undef ABX_REFIT
  if (n <= kRefitChunk) return ABX_OK;
  int32_t *frontier2 = frontier + cap;
  const unsigned g2 = (unsigned)((n + kMidLeaves - 1) / kMidLeaves);
  ABX_TRY(launch("refit_mid", s, [&] {
    k_refit_mid<<<g2, kRefitThreads, 0, s>>>(parent_int, other_end, nodes, flags, hdr, frontier,
                                             frontier_count, frontier2, frontier_count + 1, cap);
  }));
  if (n <= kMidLeaves) return ABX_OK;
  return launch("refit_top", s, [&] {
    k_refit_top<<<1, kRefitThreads, 0, s>>>(parent_int, nodes, flags, hdr, frontier2,
                                            frontier_count + 1, cap);
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
