// Batched forest: many independent point sets ("trees") built and queried
// together (batched mode of the ArborX paper, section 2.2, applied across
// trees as well as across queries).
//
// Construction runs once over all trees: every point gets the composite key
// (tree id << 54) | (18-bit-per-axis Morton code against its own tree's
// scene box), one radix sort orders all points by tree then Morton code, and
// one Karras hierarchy + refit is built over the whole array.  Because the
// tree id forms the top bits of the key, the points of each tree are a
// contiguous run of the sorted order and the hierarchy holds a node whose
// range is exactly that run: the root of the tree (found from the range end
// the hierarchy kernel records).  The nodes above the roots join trees and
// are never visited by a query.
//
// Queries of all trees are ordered by (tree, Morton code) with one sort and
// answered by one persistent launch in which each wavefront pulls tiles of
// 64 sorted queries from an atomic queue; queries that exceed the visit
// budget go to the cooperative pass of the plain path.  No step reads back
// to the host, so a build plus a query can be captured in one HIP graph.
#include <algorithm>

#include "traverse_common.h"

namespace abx {

constexpr int kForestBlock = 256;
constexpr int kForestRun = 256;   // consecutive points per thread in the box reduction
constexpr int kForestMaxTrees = 512;
constexpr int kForestKeyShift = 54;
constexpr int kForestBits = 18;
constexpr int kForestQueryBits = 10;

__device__ __forceinline__ int tree_of(const int64_t *__restrict__ off, int T, int64_t i) {
  int lo = 0, hi = T;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// order-preserving map of floats onto int32 (for atomic min/max)
__device__ __forceinline__ int32_t f2o(float f) {
  const int32_t i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float o2f(int32_t i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

__global__ void k_forest_box_init(int32_t *tbox, int T, TreeHeader *hdr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) {
    for (int a = 0; a < 3; ++a) {
      tbox[6 * t + a] = f2o(INFINITY);
      tbox[6 * t + 3 + a] = f2o(-INFINITY);
    }
  }
  if (t == 0) {
    hdr->bad = 0;
    hdr->height = 0;
  }
}

// Per-tree scene boxes (section 2.1 "Calculate the scene bounding box", once
// per tree): each thread reduces a run of consecutive points, flushing its
// partial box with atomics whenever the run crosses into the next tree.
__global__ __launch_bounds__(kForestBlock) void k_forest_boxes(const float *__restrict__ p, int64_t N,
                                                               const int64_t *__restrict__ off, int T,
                                                               int32_t *tbox, TreeHeader *hdr) {
  const int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kForestRun;
  if (r0 >= N) return;
  const int64_t r1 = r0 + kForestRun < N ? r0 + kForestRun : N;
  int t = tree_of(off, T, r0);
  int64_t tend = off[t + 1];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  auto flush = [&]() {
    if (lo[0] <= hi[0]) {
      for (int a = 0; a < 3; ++a) {
        atomicMin(tbox + 6 * t + a, f2o(lo[a]));
        atomicMax(tbox + 6 * t + 3 + a, f2o(hi[a]));
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
      }
    }
  };
  for (int64_t i = r0; i < r1; ++i) {
    while (i >= tend && t + 1 < T) {
      flush();
      ++t;
      tend = off[t + 1];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float x = p[3 * i + a];
      bad |= !__builtin_isfinite(x);
      lo[a] = fminf(lo[a], x);
      hi[a] = fmaxf(hi[a], x);
    }
  }
  flush();
  if (bad) atomicOr(&hdr->bad, 1);
}

// One workgroup: decode the tree boxes, the scene box of the whole forest
// (the Q16 grid) and a copy of the offsets into tree memory.
__global__ __launch_bounds__(kForestMaxTrees) void k_forest_boxes_final(
    const int32_t *__restrict__ tbox, int T, const int64_t *__restrict__ off_in,
    float *__restrict__ tscene, int64_t *__restrict__ off_out, TreeHeader *hdr) {
  __shared__ float s[6][kForestMaxTrees];
  const int t = threadIdx.x;
  for (int a = 0; a < 6; ++a) {
    float v = a < 3 ? INFINITY : -INFINITY;
    if (t < T) {
      v = o2f(tbox[6 * t + a]);
      tscene[6 * t + a] = v;
    }
    s[a][t] = v;
  }
  for (int i = t; i <= T; i += blockDim.x) off_out[i] = off_in[i];
  __syncthreads();
  if (t < 3) {
    float lo = INFINITY, hi = -INFINITY;
    for (int u = 0; u < T; ++u) {
      lo = fminf(lo, s[t][u]);
      hi = fmaxf(hi, s[3 + t][u]);
    }
    hdr->scene[t] = lo;
    hdr->scene[3 + t] = hi;
    const float ext = hi - lo;
    hdr->inv_ext[t] = ext > 0.0f ? 1.0f / ext : 0.0f;
    float sc = 0.0f;
    if (ext > 0.0f) {
      if (!__builtin_isfinite(ext)) {
        atomicOr(&hdr->bad, 2);
      } else {
        sc = ext / (float)kQ16Max;
        while (__fmaf_rn((float)kQ16Max, sc, lo) < hi) sc = nextafterf(sc, INFINITY);
      }
    }
    hdr->q_origin[t] = lo;
    hdr->q_scale[t] = sc;
  }
}

__device__ __forceinline__ uint64_t spread18(uint64_t x) {
  x &= 0x3ffffull;
  x = (x | (x << 32)) & 0x003f00000000ffffull;
  x = (x | (x << 16)) & 0x003f0000ff0000ffull;
  x = (x | (x << 8)) & 0x300f00f00f00f00full;
  x = (x | (x << 4)) & 0x30c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x9249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t quant(float c, float lo, float hi, int bits) {
  const float ext = hi - lo;
  const float inv = ext > 0.0f ? 1.0f / ext : 0.0f;
  float u = (c - lo) * inv;
  u = u > 0.0f ? u : 0.0f;
  u = u < 1.0f ? u : 1.0f;
  const uint32_t q = (uint32_t)(u * (float)(1u << bits));
  const uint32_t qmax = (1u << bits) - 1u;
  return q > qmax ? qmax : q;
}

// composite key of each point: tree id above its tree-local Morton code
__global__ __launch_bounds__(kForestBlock) void k_forest_keys(const float *__restrict__ p, int64_t N,
                                                              const int64_t *__restrict__ off, int T,
                                                              const float *__restrict__ tscene,
                                                              uint64_t *__restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int t = tree_of(off, T, i);
  const float *b = tscene + 6 * t;
  uint64_t code = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    code |= spread18(quant(p[3 * i + a], b[a], b[3 + a], kForestBits)) << (2 - a);
  keys[i] = ((uint64_t)t << kForestKeyShift) | code;
}

// root of each tree: the hierarchy node whose range is the tree's run, or
// ~(primitive index) for a one-point tree
__global__ void k_forest_roots(const int64_t *__restrict__ off, int T,
                               const int32_t *__restrict__ other_end,
                               const int32_t *__restrict__ perm, int32_t *__restrict__ roots) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int64_t f = off[t], l = off[t + 1] - 1;
  int32_t r;
  if (l < f) r = INT32_MIN;        // empty tree
  else if (l == f) r = ~perm[f];   // one leaf
  else r = other_end[f] == l ? (int32_t)f : (int32_t)l;
  roots[t] = r;
}

// ---------------------------------------------------------------- queries
__global__ __launch_bounds__(kForestBlock) void k_forest_qkeys(const float *__restrict__ q, int64_t M,
                                                               const int64_t *__restrict__ qoff, int T,
                                                               const float *__restrict__ tscene,
                                                               uint64_t *__restrict__ keys,
                                                               int32_t *__restrict__ qtree) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int t = tree_of(qoff, T, i);
  const float *b = tscene + 6 * t;
  uint64_t code = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    code |= (uint64_t)spread18(quant(q[3 * i + a], b[a], b[3 + a], kForestQueryBits)) << (2 - a);
  keys[i] = ((uint64_t)t << (3 * kForestQueryBits)) | code;
  qtree[i] = t;
}

// row lengths min(k, n_t) and the CSR offsets of all rows (caller's order)
__global__ __launch_bounds__(kForestMaxTrees) void k_forest_row_base(const int64_t *__restrict__ poff,
                                                                     const int64_t *__restrict__ qoff,
                                                                     int T, int k,
                                                                     int64_t *__restrict__ base) {
  if (threadIdx.x != 0) return;
  int64_t acc = 0;
  for (int t = 0; t < T; ++t) {
    base[t] = acc;
    const int64_t nt = poff[t + 1] - poff[t];
    acc += (qoff[t + 1] - qoff[t]) * (nt < k ? nt : k);
  }
  base[T] = acc;
}

__global__ __launch_bounds__(kForestBlock) void k_forest_row_offsets(
    const int64_t *__restrict__ poff, const int64_t *__restrict__ qoff, const int32_t *__restrict__ qtree,
    const int64_t *__restrict__ base, int64_t M, int T, int k, int32_t *__restrict__ offsets) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > M) return;
  if (i == M) {
    offsets[M] = (int32_t)base[T];
    return;
  }
  const int t = qtree[i];
  const int64_t nt = poff[t + 1] - poff[t];
  offsets[i] = (int32_t)(base[t] + (i - qoff[t]) * (nt < k ? nt : k));
}

struct ForestMap {
  const int64_t *poff;
  const int32_t *qtree;
  const int32_t *roots;
  const float *tscene;
  const int32_t *offsets;
  int k;
  __device__ __forceinline__ QInfo info(int64_t qi, const TreeArgs &) const {
    const int t = qtree[qi];
    const int64_t nt = poff[t + 1] - poff[t];
    QInfo r;
    r.root = roots[t];
    r.kk = (int)(nt < k ? nt : k);
    r.out = offsets[qi];
    r.base = (int32_t)poff[t];
    r.lbox = tscene + 6 * t;
    return r;
  }
};

// occupancy target: the persistent loop keeps a few more values live than
// the plain pass
constexpr int forest_waves_per_eu(int K) { return K > 16 ? 2 : (K > 10 ? 4 : (K > 4 ? 5 : 8)); }

// Persistent pass 1 over every tree's queries: each wavefront takes
// `grab` tiles of 64 Morton-ordered queries at a time from the queue.
template <int KIND, int FMT, int K>
__global__ __launch_bounds__(kForestBlock)
__attribute__((amdgpu_waves_per_eu(forest_waves_per_eu(K)))) void k_forest_nearest(TreeArgs t, ForestMap map,
                                                                 const float *__restrict__ pts,
                                                                 int64_t M, const int32_t *__restrict__ order,
                                                                 int32_t *__restrict__ indices,
                                                                 float *__restrict__ dist,
                                                                 int64_t budget, HeavyList heavy,
                                                                 uint32_t *__restrict__ queue, int grab) {
  constexpr int W = lane_window(forest_waves_per_eu(K));  // the same window in both forest walks
  __shared__ int32_t s_node[W * kForestBlock];
  __shared__ uint16_t s_dist[W * kForestBlock];
  if (tree_unusable(t)) return;  // abx_forest_check reports why; rows stay unwritten
  resolve_qframe(t);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tiles = (M + kWave - 1) / kWave;
  ABX_LDS int32_t *ln = (ABX_LDS int32_t *)(s_node) + threadIdx.x;
  ABX_LDS uint16_t *ld = (ABX_LDS uint16_t *)(s_dist) + threadIdx.x;
  for (int64_t round = 0; round <= tiles; ++round) {
    uint32_t first = 0;
    if (lane == 0) first = atomicAdd(queue, (uint32_t)grab);
    first = __shfl(first, 0, kWave);
    if ((int64_t)first >= tiles) break;
    for (int g = 0; g < grab; ++g) {
      const int64_t tq = ((int64_t)first + g) * kWave + lane;
      if (tq < M)
        nearest_lane<KIND, FMT, K, false, kForestBlock, W>(t, map, pts, order[tq], ln, ld, indices,
                                                        dist, nullptr, budget, heavy);
    }
  }
}

// Counting walk of every tree's queries (node visits and leaf records read,
// one lane per query throughout, no results): the algorithmic bytes of a
// forest query.
template <int KIND, int FMT, int K>
__global__ __launch_bounds__(kForestBlock) void k_forest_nearest_stats(TreeArgs t, ForestMap map,
                                                                      const float *__restrict__ pts,
                                                                      int64_t M,
                                                                      const int32_t *__restrict__ order,
                                                                      int32_t *__restrict__ stats) {
  constexpr int W = lane_window(forest_waves_per_eu(K));  // the same window in both forest walks
  __shared__ int32_t s_node[W * kForestBlock];
  __shared__ uint16_t s_dist[W * kForestBlock];
  if (tree_unusable(t)) return;
  resolve_qframe(t);
  const int64_t tq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tq >= M) return;
  ABX_LDS int32_t *ln = (ABX_LDS int32_t *)(s_node) + threadIdx.x;
  ABX_LDS uint16_t *ld = (ABX_LDS uint16_t *)(s_dist) + threadIdx.x;
  nearest_lane<KIND, FMT, K, true, kForestBlock, W>(t, map, pts, order[tq], ln, ld, nullptr, nullptr, stats,
                                                 INT64_MAX, HeavyList{});
}

// ---------------------------------------------------------------- host side
size_t forest_tree_extra(int T) {
  return align_up((size_t)T * 4, 256) + align_up((size_t)T * 24, 256) + align_up((size_t)(T + 1) * 8, 256);
}

abx_status forest_launch_build(const float *pts, int64_t N, const int64_t *off_dev, int T,
                               int32_t *tbox, float *tscene, int64_t *off_copy, TreeHeader *hdr,
                               uint64_t *keys, hipStream_t s) {
  ABX_TRY(launch("forest_box_init", s, [&] {
    k_forest_box_init<<<grid_for(T, 256), 256, 0, s>>>(tbox, T, hdr);
  }));
  if (N > 0)
    ABX_TRY(launch("forest_boxes", s, [&] {
      k_forest_boxes<<<grid_for((N + kForestRun - 1) / kForestRun, kForestBlock), kForestBlock, 0, s>>>(
          pts, N, off_dev, T, tbox, hdr);
    }));
  ABX_TRY(launch("forest_boxes_final", s, [&] {
    k_forest_boxes_final<<<1, kForestMaxTrees, 0, s>>>(tbox, T, off_dev, tscene, off_copy, hdr);
  }));
  if (N == 0) return ABX_OK;
  return launch("forest_keys", s, [&] {
    k_forest_keys<<<grid_for(N, kForestBlock), kForestBlock, 0, s>>>(pts, N, off_copy, T, tscene, keys);
  });
}

abx_status forest_launch_roots(const int64_t *off, int T, const int32_t *other_end, const int32_t *perm,
                               int32_t *roots, hipStream_t s) {
  return launch("forest_roots", s, [&] {
    k_forest_roots<<<grid_for(T, 256), 256, 0, s>>>(off, T, other_end, perm, roots);
  });
}

abx_status forest_launch_qkeys(const float *q, int64_t M, const int64_t *qoff, int T, const float *tscene,
                               uint64_t *keys, int32_t *qtree, hipStream_t s) {
  if (M == 0) return ABX_OK;
  return launch("forest_qkeys", s, [&] {
    k_forest_qkeys<<<grid_for(M, kForestBlock), kForestBlock, 0, s>>>(q, M, qoff, T, tscene, keys, qtree);
  });
}

abx_status forest_launch_rows(const int64_t *poff, const int64_t *qoff, const int32_t *qtree, int64_t M,
                              int T, int k, int64_t *base, int32_t *offsets, hipStream_t s) {
  ABX_TRY(launch("forest_row_base", s, [&] {
    k_forest_row_base<<<1, 64, 0, s>>>(poff, qoff, T, k, base);
  }));
  return launch("forest_row_offsets", s, [&] {
    k_forest_row_offsets<<<grid_for(M + 1, kForestBlock), kForestBlock, 0, s>>>(poff, qoff, qtree, base,
                                                                                M, T, k, offsets);
  });
}

int coop_grid(int waves);
int device_cus();

template <int KIND, int FMT, int K>
abx_status forest_nearest_k(const TreeArgs &t, const ForestMap &map, const float *pts, int64_t M,
                            const int32_t *order, int32_t *idx, float *dist, const HeavyList &heavy,
                            uint32_t *queue, int blocks_per_cu, int grab, int64_t budget, hipStream_t s) {
  const unsigned g = (unsigned)std::max(1, device_cus() * blocks_per_cu);
  ABX_TRY(launch("forest_nearest", s, [&] {
    k_forest_nearest<KIND, FMT, K><<<g, kForestBlock, 0, s>>>(t, map, pts, M, order, idx, dist, budget,
                                                             heavy, queue, grab);
  }));
  return launch("forest_nearest_coop", s, [&] {
    k_nearest_coop<KIND, FMT, K, ForestMap, coop_waves(K)>
        <<<(unsigned)coop_grid(coop_waves(K)), CoopShape<coop_waves(K)>::kThreads, 0, s>>>(
            t, map, pts, idx, dist, heavy);
  });
}

template <int FMT>
abx_status forest_nearest_fmt(const TreeArgs &t, const ForestMap &map, const float *pts, int64_t M,
                              const int32_t *order, int k, int32_t *idx, float *dist,
                              const HeavyList &heavy, uint32_t *queue, int bpc, int grab,
                              int64_t budget, hipStream_t s) {
#define ABX_FK(KK) \
  return forest_nearest_k<ABX_PRIM_POINTS, FMT, KK>(t, map, pts, M, order, idx, dist, heavy, queue, bpc, grab, budget, s)
  if (k <= 1) ABX_FK(1);
  if (k <= 2) ABX_FK(2);
  if (k <= 4) ABX_FK(4);
  if (k <= 8) ABX_FK(8);
  if (k <= 10) ABX_FK(10);
  if (k <= 16) ABX_FK(16);
  if (k <= 32) ABX_FK(32);
  if (k <= 48) ABX_FK(48);
  ABX_FK(kMaxRegK);
#undef ABX_FK
}

abx_status forest_launch_nearest(const TreeArgs &t, int format, const int64_t *poff, const int32_t *qtree,
                                 const int32_t *roots, const float *tscene, const int32_t *offsets,
                                 const float *pts, int64_t M, const int32_t *order, int k, int32_t *idx,
                                 float *dist, int32_t *heavy_q, float *heavy_bound, uint32_t *counters,
                                 int blocks_per_cu, int grab, int64_t budget, hipStream_t s) {
  if (M == 0 || k == 0) return ABX_OK;
  if (k > kMaxRegK) return ABX_ERR_UNSUPPORTED;
  const ForestMap map{poff, qtree, roots, tscene, offsets, k};
  const HeavyList heavy{heavy_q, heavy_bound, counters};
  ABX_TRY(fill_u32(counters, 0, 3, s));  // heavy count, next heavy, tile queue
  if (format == ABX_NODES_FP32)
    return forest_nearest_fmt<ABX_NODES_FP32>(t, map, pts, M, order, k, idx, dist, heavy, counters + 2,
                                              blocks_per_cu, grab, budget, s);
  return forest_nearest_fmt<ABX_NODES_Q16>(t, map, pts, M, order, k, idx, dist, heavy, counters + 2,
                                           blocks_per_cu, grab, budget, s);
}

template <int FMT>
abx_status forest_stats_fmt(const TreeArgs &t, const ForestMap &map, const float *pts, int64_t M,
                            const int32_t *order, int k, int32_t *stats, hipStream_t s) {
  const unsigned g = grid_for(M, kForestBlock);
#define ABX_FS(KK)                                                                                 \
  return launch("forest_nearest_stats", s, [&] {                                                  \
    k_forest_nearest_stats<ABX_PRIM_POINTS, FMT, KK><<<g, kForestBlock, 0, s>>>(t, map, pts, M, order, \
                                                                               stats);              \
  })
  if (k <= 1) ABX_FS(1);
  if (k <= 2) ABX_FS(2);
  if (k <= 4) ABX_FS(4);
  if (k <= 8) ABX_FS(8);
  if (k <= 10) ABX_FS(10);
  if (k <= 16) ABX_FS(16);
  if (k <= 32) ABX_FS(32);
  if (k <= 48) ABX_FS(48);
  ABX_FS(kMaxRegK);
#undef ABX_FS
}

abx_status forest_launch_nearest_stats(const TreeArgs &t, int format, const int64_t *poff,
                                       const int32_t *qtree, const int32_t *roots, const float *tscene,
                                       const int32_t *offsets, const float *pts, int64_t M,
                                       const int32_t *order, int k, int32_t *stats, hipStream_t s) {
  if (M == 0) return ABX_OK;
  if (k == 0) return fill_u32(stats, 0, 2 * (size_t)M, s);
  if (k > kMaxRegK) return ABX_ERR_UNSUPPORTED;
  const ForestMap map{poff, qtree, roots, tscene, offsets, k};
  if (format == ABX_NODES_FP32)
    return forest_stats_fmt<ABX_NODES_FP32>(t, map, pts, M, order, k, stats, s);
  return forest_stats_fmt<ABX_NODES_Q16>(t, map, pts, M, order, k, stats, s);
}

int forest_max_trees() { return kForestMaxTrees; }

}  // namespace abx
