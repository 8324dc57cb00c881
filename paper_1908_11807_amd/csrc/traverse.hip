// Tree traversal kernels (ArborX paper, section 2.2).
//
// Batched mode: one lane per query, queries in Morton order so that the 64
// lanes of a wavefront walk nearly the same nodes (section 2.2 "Query
// ordering"); the blockIdx -> query-tile map keeps consecutive tiles on one
// XCD so that they share that XCD's L2.
//
// Spatial (section 2.2 "Traversal for spatial queries"): iterative, with a
// stack of deferred nodes.  A visited node holds both children's boxes; each
// child passing the predicate is emitted (leaf) or descended into (internal,
// the second one deferred on the stack).  Count pass and fill pass (2P).
//
// Nearest (section 2.2 "Traversal for nearest queries"): the same stack walk
// where one child is visited first and the other deferred with its box
// distance (the paper puts the nearer box first; here the child whose box
// centre is nearer goes first, which fills the list sooner); a node is
// pruned when its box is strictly farther than the
// current k-th candidate, which is how the walk stops once the remaining
// candidates cannot improve the result.  The k best candidates are kept
// sorted in registers by (squared distance, index).
//
// Stack: the top entries of each lane live in a circular LDS window (column
// per lane, so a wavefront's pushes hit distinct banks); deeper entries go to
// the lane's private memory.  Trees deeper than kMaxDepth are refused on the
// host.
#include <algorithm>

#include "traverse_common.h"

namespace abx {

// ------------------------------------------------------------------ spatial
template <int PRED>
struct SpatialQuery {
  float a[3], b[3];  // WITHIN: a = point, b[0] = r^2 ; INTERSECTS: a = lo, b = hi
  __device__ __forceinline__ bool test(const float *x) const {
    if (PRED == ABX_PRED_WITHIN)
      return box_dist2(x[0], x[1], x[2], x[3], x[4], x[5], a[0], a[1], a[2]) <= b[0];
    return box_overlap(x[0], x[1], x[2], x[3], x[4], x[5], a[0], a[1], a[2], b[0], b[1], b[2]);
  }
};

template <int KIND, int PRED, int FMT, int MODE>
__global__ __launch_bounds__(kTravBlock) void k_spatial(TreeArgs t, QueryArgs qa,
                                                        int32_t *__restrict__ out_counts,
                                                        const int32_t *__restrict__ offsets,
                                                        int32_t *__restrict__ indices) {
  __shared__ int32_t s_stack[kLdsDepthSpatial * kTravBlock];
  const int64_t tq = xcd_tile(blockIdx.x, gridDim.x) * kTravBlock + threadIdx.x;
  if (tq >= qa.m) return;
  // the fill pass of the one-pass scheme runs only after an overflow, and
  // only when the caller's index buffer holds every hit
  if (MODE == MODE_FILL && qa.flag && (qa.flag[0] == 0 || *qa.total > qa.capacity)) return;
  const int64_t qi = qa.order ? qa.order[tq] : tq;
  SpatialQuery<PRED> q;
  if (PRED == ABX_PRED_WITHIN) {
    const float *p = qa.data + 3 * qi;
    q.a[0] = p[0]; q.a[1] = p[1]; q.a[2] = p[2];
    const float r = qa.radii ? qa.radii[qi] : qa.radius;
    q.b[0] = r >= 0.0f ? r * r : -1.0f;
    q.b[1] = q.b[2] = 0.0f;
  } else {
    const float *p = qa.data + 6 * qi;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      q.a[a] = p[a];
      q.b[a] = p[3 + a];
    }
  }
  int32_t *out = MODE == MODE_FILL    ? indices + offsets[qi]
                 : MODE == MODE_STORE ? qa.buf + tq * qa.bufsize
                                      : nullptr;
  const int32_t row_len = MODE == MODE_FILL    ? offsets[qi + 1] - offsets[qi]
                          : MODE == MODE_STORE ? qa.bufsize
                                               : 0;
  int32_t cnt = 0, visited = 0, leaf_reads = 0;

  // a leaf child (primitive idx) whose node-stored box passed: confirm where
  // the slot is quantised, and emit
  auto leaf = [&](int32_t idx) {
    if (!exact_leaf_slots<KIND, FMT>()) {
      float b[6];
      load_leaf_box(t, idx, b);
      if (MODE == MODE_STATS) ++leaf_reads;
      if (!q.test(b)) return;
    }
    if ((MODE == MODE_FILL || MODE == MODE_STORE) && cnt < row_len) out[cnt] = idx;
    ++cnt;
  };

  if (t.n == 1) {
    // the scene box of a one-primitive tree is that primitive's box
    if (q.test(t.scene)) leaf(0);
  } else {
    int32_t ovf[kMaxDepth];
    ABX_LDS int32_t *lds = (ABX_LDS int32_t *)(s_stack) + threadIdx.x;
    int sp = 0, nl = 0;
    int32_t node = t.root;
    // a tree has n-1 internal nodes, each visited at most once: the bound
    // only guarantees termination
    for (int64_t it = 0; it < t.n; ++it) {
      if constexpr (FMT == ABX_NODES_Q16W) {
        // 4-wide node: emit the leaf children that pass, descend into the
        // first internal one, defer the others
        Kids4 k;
        load_kids4<KIND>(t, node, k);
        if (MODE == MODE_STATS) ++visited;
        int32_t next = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k.ref[j] == kEmptyRef || !q.test(k.b[j])) continue;
          if (k.ref[j] < 0) leaf(~k.ref[j]);
          else if (next < 0) next = k.ref[j];
          else if (sp < kMaxDepth) stack_push<int32_t, kLdsDepthSpatial, kTravBlock>(lds, ovf, sp, nl, k.ref[j]);
        }
        if (next >= 0) {
          node = next;
        } else {
          if (sp == 0) break;
          node = stack_pop<int32_t, kLdsDepthSpatial, kTravBlock>(lds, ovf, sp, nl);
        }
        continue;
      }
      Kids k;
      load_kids<KIND, FMT>(t, node, k);
      if (MODE == MODE_STATS) ++visited;
      const bool hl = q.test(k.l), hr = q.test(k.r);
      const bool ll = k.lref < 0, lr = k.rref < 0;
      if (hl && ll) leaf(~k.lref);
      if (hr && lr) leaf(~k.rref);
      const bool gl = hl && !ll, gr = hr && !lr;
      if (gl) {
        if (gr && sp < kMaxDepth)
          stack_push<int32_t, kLdsDepthSpatial, kTravBlock>(lds, ovf, sp, nl, k.rref);
        node = k.lref;
      } else if (gr) {
        node = k.rref;
      } else {
        if (sp == 0) break;
        node = stack_pop<int32_t, kLdsDepthSpatial, kTravBlock>(lds, ovf, sp, nl);
      }
    }
  }
  if (MODE == MODE_COUNT || MODE == MODE_STORE) out_counts[qi] = cnt;
  if (MODE == MODE_STORE && cnt > qa.bufsize) atomicOr(qa.flag, 1u);
  if (MODE == MODE_STATS) {
    out_counts[2 * qi] = visited;
    out_counts[2 * qi + 1] = leaf_reads;
  }
}

// ------------------------------------------------------------------ nearest
// Pass 1 over one tree: one lane per query, queries in Morton order.
template <int KIND, int FMT, int K, bool STATS>
__global__ __launch_bounds__(kTravBlock)
__attribute__((amdgpu_waves_per_eu(nearest_waves_per_eu(K, FMT)))) void k_nearest(TreeArgs t, PlainMap map,
                                                        const float *__restrict__ pts, int64_t m,
                                                        const int32_t *__restrict__ order,
                                                        int32_t *__restrict__ indices,
                                                        float *__restrict__ dist,
                                                        int32_t *__restrict__ stats, int64_t budget,
                                                        HeavyList heavy) {
  constexpr int W = lane_window(nearest_waves_per_eu(K, FMT));
  __shared__ int32_t s_node[W * kTravBlock];
  __shared__ uint16_t s_dist[W * kTravBlock];
  const int64_t tq = xcd_tile(blockIdx.x, gridDim.x) * kTravBlock + threadIdx.x;
  if (tq >= m) return;
  const int64_t qi = order ? order[tq] : tq;
  nearest_lane<KIND, FMT, K, STATS, kTravBlock, W>(
      t, map, pts, qi, (ABX_LDS int32_t *)(s_node) + threadIdx.x,
      (ABX_LDS uint16_t *)(s_dist) + threadIdx.x, indices, dist, stats, budget, heavy);
}

// ------------------------------------------------------------ large k
// k = 65..128 (register lists serve k <= 64: 64 keys take 128 registers, the
// most that leaves two wavefronts per SIMD): each lane keeps its candidates
// in an LDS max-heap (root = the
// current k-th candidate; the heap is the paper's bounded priority list,
// section 2.2), one wavefront per workgroup, entry e of lane l at e * 64 + l
// so that a wavefront's accesses fall in distinct banks.  The walk is the
// one of pass 1 (child with the nearer box centre first, strict pruning by
// the root once the heap is full) with no visit budget.  At the end a heap
// sort leaves the row ascending in place.
constexpr int kHeapLanes = kWave;

__device__ __forceinline__ void heap_push(ABX_LDS int64_t *h, int &size, int64_t x) {
  int i = size++;
  while (i > 0) {
    const int p = (i - 1) >> 1;
    const int64_t vp = h[p * kHeapLanes];
    if (vp >= x) break;
    h[i * kHeapLanes] = vp;
    i = p;
  }
  h[i * kHeapLanes] = x;
}

// x replaces the root of heap [0, size) and sinks to its place
__device__ __forceinline__ void heap_sink(ABX_LDS int64_t *h, int size, int64_t x) {
  int i = 0;
  for (;;) {
    int c = 2 * i + 1;
    if (c >= size) break;
    int64_t vc = h[c * kHeapLanes];
    if (c + 1 < size) {
      const int64_t v2 = h[(c + 1) * kHeapLanes];
      if (v2 > vc) {
        ++c;
        vc = v2;
      }
    }
    if (vc <= x) break;
    h[i * kHeapLanes] = vc;
    i = c;
  }
  h[i * kHeapLanes] = x;
}

// The heap takes 8k bytes of LDS per lane (dynamic, sized to k), which is
// what bounds residency: registers are capped to match (4 waves per SIMD).
template <int KIND, int FMT, bool STATS>
__global__ __launch_bounds__(kHeapLanes) __attribute__((amdgpu_waves_per_eu(4))) void k_nearest_heap(TreeArgs t,
                                                             const float *__restrict__ pts,
                                                             int64_t m,
                                                             const int32_t *__restrict__ order,
                                                             int k, int32_t *__restrict__ indices,
                                                             float *__restrict__ dist,
                                                             int32_t *__restrict__ stats) {
  extern __shared__ int64_t s_heap[];  // k keys per lane, lane-interleaved
  __shared__ int32_t s_node[kLdsDepthNearest * kHeapLanes];
  __shared__ float s_dist[kLdsDepthNearest * kHeapLanes];
  const int64_t tq = xcd_tile(blockIdx.x, gridDim.x) * kHeapLanes + threadIdx.x;
  if (tq >= m) return;
  const int64_t qi = order ? order[tq] : tq;
  const KnnQuery q{pts[3 * qi], pts[3 * qi + 1], pts[3 * qi + 2]};
  ABX_LDS int64_t *h = (ABX_LDS int64_t *)(s_heap) + threadIdx.x;
  ABX_LDS int32_t *lds_n = (ABX_LDS int32_t *)(s_node) + threadIdx.x;
  ABX_LDS float *lds_d = (ABX_LDS float *)(s_dist) + threadIdx.x;
  int size = 0;
  int32_t visited = 0, reads = 0;
  auto kth = [&]() { return size < k ? INFINITY : key_dist(h[0]); };
  auto offer = [&](int64_t x) {
    if (size < k) heap_push(h, size, x);
    else if (x < h[0]) heap_sink(h, k, x);
  };
  // a leaf child whose node-stored box is at squared distance dbox
  auto leaf = [&](int32_t idx, float dbox) {
    if (!(dbox <= kth())) return;
    if (exact_leaf_slots<KIND, FMT>()) {
      offer(knn_key(dbox, idx));
    } else {
      ++reads;
      float b[6];
      load_leaf_box(t, idx, b);
      const float d = box_dist2(b[0], b[1], b[2], b[3], b[4], b[5], q.x, q.y, q.z);
      if (d <= kth()) offer(knn_key(d, idx));
    }
  };
  if (t.n == 1) {
    const float *b = t.scene;
    leaf(0, box_dist2(b[0], b[1], b[2], b[3], b[4], b[5], q.x, q.y, q.z));
  } else {
    int32_t ovf_n[kMaxDepth];
    float ovf_d[kMaxDepth];
    int sp = 0, nl = 0;
    int32_t node = t.root;
    for (int64_t it = 0; it < 2 * t.n; ++it) {
      if (STATS) ++visited;
      if constexpr (FMT == ABX_NODES_Q16W) {
        // 4-wide node, as knn_visit_w: leaves offered, the qualifying
        // internal children visited nearest box centre first
        Kids4 c;
        load_kids4<KIND>(t, node, c);
        float d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          d[j] = c.ref[j] == kEmptyRef ? INFINITY
                                       : box_dist2(c.b[j][0], c.b[j][1], c.b[j][2], c.b[j][3],
                                                   c.b[j][4], c.b[j][5], q.x, q.y, q.z);
          if (c.ref[j] < 0 && c.ref[j] != kEmptyRef) leaf(~c.ref[j], d[j]);
        }
        const float thr = kth();
        float key[4];
        int32_t r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool g = c.ref[j] >= 0 && d[j] <= thr;
          float cc = 0.0f;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float qa = a == 0 ? q.x : (a == 1 ? q.y : q.z);
            const float mm = (c.b[j][a] - qa) - (qa - c.b[j][3 + a]);
            cc = __fmaf_rn(mm, mm, cc);
          }
          key[j] = g ? cc : INFINITY;
          r[j] = g ? c.ref[j] : -1;
        }
        auto cx = [&](int i, int j) {
          if (key[j] < key[i] || (r[i] < 0 && r[j] >= 0)) {
            const float tk = key[i];
            key[i] = key[j];
            key[j] = tk;
            const int32_t tr = r[i];
            r[i] = r[j];
            r[j] = tr;
            const float td = d[i];
            d[i] = d[j];
            d[j] = td;
          }
        };
        cx(0, 1);
        cx(2, 3);
        cx(0, 2);
        cx(1, 3);
        cx(1, 2);
#pragma unroll
        for (int j = 3; j >= 1; --j)
          if (r[j] >= 0 && sp < kMaxDepth)
            stack_push2<kLdsDepthNearest, kHeapLanes>(lds_n, lds_d, ovf_n, ovf_d, sp, nl, r[j], d[j]);
        node = r[0];
        if (node < 0) node = knn_pop<kHeapLanes>(kth(), lds_n, lds_d, ovf_n, ovf_d, sp, nl);
        if (node < 0) break;
        continue;
      }
      Kids c;
      load_kids<KIND, FMT>(t, node, c);
      const float dl = box_dist2(c.l[0], c.l[1], c.l[2], c.l[3], c.l[4], c.l[5], q.x, q.y, q.z);
      const float dr = box_dist2(c.r[0], c.r[1], c.r[2], c.r[3], c.r[4], c.r[5], q.x, q.y, q.z);
      const bool ll = c.lref < 0, lr = c.rref < 0;
      if (ll) leaf(~c.lref, dl);
      if (lr) leaf(~c.rref, dr);
      const float thr = kth();
      const bool gl = !ll && dl <= thr, gr = !lr && dr <= thr;
      node = -1;
      if (gl && gr) {
        float cl = 0.0f, cr = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float qa = a == 0 ? q.x : (a == 1 ? q.y : q.z);
          const float ml = (c.l[a] - qa) - (qa - c.l[3 + a]);
          const float mr = (c.r[a] - qa) - (qa - c.r[3 + a]);
          cl = __fmaf_rn(ml, ml, cl);
          cr = __fmaf_rn(mr, mr, cr);
        }
        const bool left_first = cl <= cr;
        if (sp < kMaxDepth)
          stack_push2<kLdsDepthNearest, kHeapLanes>(lds_n, lds_d, ovf_n, ovf_d, sp, nl,
                                                    left_first ? c.rref : c.lref,
                                                    left_first ? dr : dl);
        node = left_first ? c.lref : c.rref;
      } else if (gl) {
        node = c.lref;
      } else if (gr) {
        node = c.rref;
      }
      if (node < 0) node = knn_pop<kHeapLanes>(kth(), lds_n, lds_d, ovf_n, ovf_d, sp, nl);
      if (node < 0) break;
    }
  }
  if (STATS) {
    stats[2 * qi] = visited;
    stats[2 * qi + 1] = reads;
    return;
  }
  // heap sort: the largest goes to the back, the rest sinks again
  for (int e = size - 1; e > 0; --e) {
    const int64_t top = h[0];
    const int64_t last = h[e * kHeapLanes];
    h[e * kHeapLanes] = top;
    heap_sink(h, e, last);
  }
  int32_t *oi = indices + qi * k;
  float *od = dist + qi * k;
  for (int j = 0; j < size; ++j) {
    const int64_t x = h[j * kHeapLanes];
    oi[j] = key_index(x);
    od[j] = sqrtf(key_dist(x));
  }
}


// ------------------------------------------------------------ query codes
// 30-bit Morton code of each query's centroid against the tree's scene box
// (clamped), for the query ordering of section 2.2.
__device__ __forceinline__ uint32_t spread10q(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

template <int W>
__global__ __launch_bounds__(kTravBlock) void k_query_codes(const float *__restrict__ q, int64_t m,
                                                            TreeArgs t, uint32_t *__restrict__ codes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = W == 3 ? q[3 * i + a] : 0.5f * (q[6 * i + a] + q[6 * i + 3 + a]);
    const float lo = t.scene[a], ext = t.scene[3 + a] - lo;
    const float inv = ext > 0.0f ? 1.0f / ext : 0.0f;
    float u = (x - lo) * inv;
    u = u > 0.0f ? u : 0.0f;
    u = u < 1.0f ? u : 1.0f;
    const uint32_t v = (uint32_t)(u * 1024.0f);
    c[a] = v > 1023u ? 1023u : v;
  }
  codes[i] = (spread10q(c[0]) << 2) | (spread10q(c[1]) << 1) | spread10q(c[2]);
}

// ------------------------------------------------------------ host launchers
TreeArgs tree_args(const abx_bvh *b) {
  TreeArgs t;
  t.nodes = b->nodes();
  t.leaves = b->leaves();
  t.n = b->n;
  t.root = b->root;
  for (int a = 0; a < 6; ++a) t.scene[a] = b->scene[a];
  for (int a = 0; a < 3; ++a) {
    t.qo[a] = b->q_origin[a];
    t.qs[a] = b->q_scale[a];
  }
  t.scene_dev = b->hdr()->scene;
  t.qframe = nullptr;
  t.guard = nullptr;  // the build checked the header before making the handle
  t.nint = b->nint;
  return t;
}

abx_status launch_query_codes(const abx_bvh *b, const float *q, int64_t m, int width,
                              uint32_t *codes, hipStream_t s) {
  if (m == 0) return ABX_OK;
  const TreeArgs t = tree_args(b);
  const unsigned g = grid_for(m, kTravBlock);
  if (width == 3)
    return launch("query_codes", s, [&] { k_query_codes<3><<<g, kTravBlock, 0, s>>>(q, m, t, codes); });
  return launch("query_codes", s, [&] { k_query_codes<6><<<g, kTravBlock, 0, s>>>(q, m, t, codes); });
}

template <int KIND, int PRED, int FMT>
abx_status spatial_fmt(const abx_bvh *b, const QueryArgs &qa, int mode, int32_t *counts,
                       const int32_t *offsets, int32_t *indices, hipStream_t s) {
  const TreeArgs t = tree_args(b);
  const unsigned g = grid_for(qa.m, kTravBlock);
  const char *name = mode == MODE_COUNT  ? "spatial_count"
                     : mode == MODE_FILL  ? "spatial_fill"
                     : mode == MODE_STORE ? "spatial_store"
                                          : "spatial_stats";
  return launch(name, s, [&] {
    if (mode == MODE_COUNT)
      k_spatial<KIND, PRED, FMT, MODE_COUNT><<<g, kTravBlock, 0, s>>>(t, qa, counts, offsets, indices);
    else if (mode == MODE_STORE)
      k_spatial<KIND, PRED, FMT, MODE_STORE><<<g, kTravBlock, 0, s>>>(t, qa, counts, offsets, indices);
    else if (mode == MODE_FILL)
      k_spatial<KIND, PRED, FMT, MODE_FILL><<<g, kTravBlock, 0, s>>>(t, qa, counts, offsets, indices);
    else
      k_spatial<KIND, PRED, FMT, MODE_STATS><<<g, kTravBlock, 0, s>>>(t, qa, counts, offsets, indices);
  });
}

template <int KIND, int PRED>
abx_status spatial_pred(const abx_bvh *b, const QueryArgs &qa, int mode, int32_t *counts,
                        const int32_t *offsets, int32_t *indices, hipStream_t s) {
  if (b->format == ABX_NODES_FP32)
    return spatial_fmt<KIND, PRED, ABX_NODES_FP32>(b, qa, mode, counts, offsets, indices, s);
  if (b->format == ABX_NODES_Q16W)
    return spatial_fmt<KIND, PRED, ABX_NODES_Q16W>(b, qa, mode, counts, offsets, indices, s);
  return spatial_fmt<KIND, PRED, ABX_NODES_Q16>(b, qa, mode, counts, offsets, indices, s);
}

abx_status launch_spatial(const abx_bvh *b, int pred, const float *data, int64_t m,
                          const float *radii, float radius, const int32_t *order, int mode,
                          int32_t *counts, const int32_t *offsets, int32_t *indices, hipStream_t s,
                          const OnePass *op) {
  if (m == 0) return ABX_OK;
  QueryArgs qa{data, m, radii, radius, order, nullptr, 0, nullptr, nullptr, 0};
  if (op) {
    qa.buf = op->buf;
    qa.bufsize = op->bufsize;
    qa.flag = op->flag;
    qa.total = op->total;
    qa.capacity = op->capacity;
  }
  if (b->kind == ABX_PRIM_POINTS) {
    if (pred == ABX_PRED_WITHIN)
      return spatial_pred<ABX_PRIM_POINTS, ABX_PRED_WITHIN>(b, qa, mode, counts, offsets, indices, s);
    return spatial_pred<ABX_PRIM_POINTS, ABX_PRED_INTERSECTS_BOX>(b, qa, mode, counts, offsets, indices, s);
  }
  if (pred == ABX_PRED_WITHIN)
    return spatial_pred<ABX_PRIM_BOXES, ABX_PRED_WITHIN>(b, qa, mode, counts, offsets, indices, s);
  return spatial_pred<ABX_PRIM_BOXES, ABX_PRED_INTERSECTS_BOX>(b, qa, mode, counts, offsets, indices, s);
}

// ------------------------------------------------------------ 1P compaction
// After a storing pass with no overflow: the row stored for sorted position
// tq (its first count[q] slots) goes to indices[offsets[q] ...].  A group of
// G lanes (8 or 16) copies one query's hits, G consecutive entries per step:
// reads and writes stay coalesced within the row, and the cost follows the
// results rather than the m * buffer_size slots (a buffer sized for the
// longest row is mostly empty when rows are uneven: hollow case, 2.7 hits
// per row against 259 slots).
__global__ __launch_bounds__(kTravBlock) void k_spatial_compact(const int32_t *__restrict__ buf,
                                                                int32_t bufsize, int64_t m,
                                                                int group_log2,
                                                                const int32_t *__restrict__ order,
                                                                const int32_t *__restrict__ counts,
                                                                const int32_t *__restrict__ offsets,
                                                                int32_t *__restrict__ indices,
                                                                const uint32_t *__restrict__ flag,
                                                                const int64_t *__restrict__ total,
                                                                int64_t capacity) {
  if (flag[0] != 0 || *total > capacity) return;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tq = id >> group_log2;
  if (tq >= m) return;
  const int32_t g = 1 << group_log2, j0 = (int32_t)(id & (g - 1));
  const int64_t qi = order ? order[tq] : tq;
  const int32_t c = counts[qi];  // <= bufsize: no row overflowed
  const int32_t *row = buf + tq * (int64_t)bufsize;
  int32_t *out = indices + offsets[qi];
  for (int32_t j = j0; j < c; j += g) out[j] = row[j];
}

// info[0] = status, info[1] = traversals made
__global__ void k_spatial_1p_info(const uint32_t *__restrict__ flag, const int64_t *__restrict__ total,
                                  int64_t capacity, int64_t max_count, int32_t *__restrict__ info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t t = *total;
  const bool fits = t <= capacity;
  info[0] = t >= max_count ? ABX_ERR_OVERFLOW : (fits ? ABX_OK : ABX_ERR_CAPACITY);
  info[1] = flag[0] != 0 && fits ? 2 : 1;
}

abx_status launch_spatial_compact(const OnePass &op, int64_t m, const int32_t *order,
                                  const int32_t *counts, const int32_t *offsets, int32_t *indices,
                                  int32_t *info, int64_t max_count, hipStream_t s) {
  if (m > 0) {
    const int glog = op.bufsize <= 8 ? 3 : 4;  // 8 or 16 lanes per query
    const unsigned g = grid_for(m << glog, kTravBlock);
    ABX_TRY(launch("spatial_compact", s, [&] {
      k_spatial_compact<<<g, kTravBlock, 0, s>>>(op.buf, op.bufsize, m, glog, order, counts,
                                                 offsets, indices, op.flag, op.total, op.capacity);
    }));
  }
  return launch("spatial_1p_info", s, [&] {
    k_spatial_1p_info<<<1, 64, 0, s>>>(op.flag, op.total, op.capacity, max_count, info);
  });
}

struct NearestScratch {
  int32_t *heavy_q;
  float *heavy_bound;
  uint32_t *counters;  // [0] heavy count, [1] next heavy query
  int64_t budget;
  int32_t *heavy_state;  // saved walks (kHeavyStateWords each), or null
  uint32_t state_cap;
};

int device_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

// persistent grid of the cooperative pass: as many workgroups as fit at once
// (LDS bound: a W-wavefront workgroup takes 8 KB per wavefront)
int coop_grid(int waves) { return device_cus() * std::max(1, 16 / waves); }

template <int KIND, int FMT, int K>
abx_status nearest_k(const abx_bvh *b, const float *pts, int64_t m, const int32_t *order, int k,
                     int32_t *idx, float *dist, int32_t *stats, const NearestScratch &ns,
                     hipStream_t s) {
  const TreeArgs t = tree_args(b);
  const PlainMap map{k};
  const HeavyList heavy{ns.heavy_q, ns.heavy_bound, ns.counters, ns.heavy_state, ns.state_cap};
  const unsigned g = grid_for(m, kTravBlock);
  if (stats)
    return launch("nearest_stats", s, [&] {
      k_nearest<KIND, FMT, K, true><<<g, kTravBlock, 0, s>>>(t, map, pts, m, order, idx, dist,
                                                             stats, INT64_MAX, heavy);
    });
  ABX_TRY(fill_u32(ns.counters, 0, 2, s));
  ABX_TRY(launch("nearest", s, [&] {
    k_nearest<KIND, FMT, K, false><<<g, kTravBlock, 0, s>>>(t, map, pts, m, order, idx, dist,
                                                            stats, ns.budget, heavy);
  }));
  constexpr int W = coop_waves(K);
  const unsigned g2 = (unsigned)coop_grid(W);
  return launch("nearest_coop", s, [&] {
    k_nearest_coop<KIND, FMT, K, PlainMap, W>
        <<<g2, CoopShape<W>::kThreads, 0, s>>>(t, map, pts, idx, dist, heavy);
  });
}

template <int KIND, int FMT, bool STATS>
abx_status launch_heap(const TreeArgs &t, const float *pts, int64_t m, const int32_t *order, int k,
                       int32_t *idx, float *dist, int32_t *stats, hipStream_t s) {
  const size_t heap_bytes = (size_t)k * kHeapLanes * sizeof(int64_t);
  // above 64 KB a kernel must be allowed the larger dynamic LDS explicitly
  // (on the current device; cheap, so done at every launch)
  const hipError_t allowed = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&k_nearest_heap<KIND, FMT, STATS>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)heap_bytes);
  if (allowed != hipSuccess) return hip_fail(allowed);
  const unsigned g = grid_for(m, kHeapLanes);
  return launch(STATS ? "nearest_stats" : "nearest", s, [&] {
    k_nearest_heap<KIND, FMT, STATS><<<g, kHeapLanes, heap_bytes, s>>>(t, pts, m, order, k, idx, dist,
                                                                      stats);
  });
}

template <int KIND, int FMT>
abx_status nearest_heap(const abx_bvh *b, const float *pts, int64_t m, const int32_t *order, int k,
                        int32_t *idx, float *dist, int32_t *stats, hipStream_t s) {
  const TreeArgs t = tree_args(b);
  if (stats) return launch_heap<KIND, FMT, true>(t, pts, m, order, k, idx, dist, stats, s);
  return launch_heap<KIND, FMT, false>(t, pts, m, order, k, idx, dist, stats, s);
}

template <int KIND, int FMT>
abx_status nearest_fmt(const abx_bvh *b, const float *pts, int64_t m, const int32_t *order, int k,
                       int32_t *idx, float *dist, int32_t *stats, const NearestScratch &ns,
                       hipStream_t s) {
  if (k <= 1) return nearest_k<KIND, FMT, 1>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 2) return nearest_k<KIND, FMT, 2>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 4) return nearest_k<KIND, FMT, 4>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 8) return nearest_k<KIND, FMT, 8>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 10) return nearest_k<KIND, FMT, 10>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 16) return nearest_k<KIND, FMT, 16>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 32) return nearest_k<KIND, FMT, 32>(b, pts, m, order, k, idx, dist, stats, ns, s);
  if (k <= 48) return nearest_k<KIND, FMT, 48>(b, pts, m, order, k, idx, dist, stats, ns, s);
  return nearest_k<KIND, FMT, kMaxRegK>(b, pts, m, order, k, idx, dist, stats, ns, s);
}

// Small batches leave most of the GPU idle, so their heavy queries are
// better served early by whole workgroups: the one-lane budget shrinks with
// the batch (never below 512 visits, never above the configured budget).
// m / 24 measured best at 1e5 queries on a 1e7-point shell (k = 8: 9.2 ms
// against 11.5 with m / 16); at 1e4 anything from 512 to 4096 ties.
int64_t effective_budget(int64_t budget, int64_t m) {
  const int64_t b = std::max<int64_t>(512, m / 24);
  return std::min(budget, b);
}

abx_status launch_nearest(const abx_bvh *b, const float *pts, int64_t m, const int32_t *order,
                          int k, int32_t *idx, float *dist, int32_t *stats, int32_t *heavy_q,
                          float *heavy_bound, uint32_t *counters, int32_t *heavy_state,
                          int64_t state_cap, int64_t budget, hipStream_t s) {
  if (m == 0 || k == 0) return ABX_OK;
  if (k > kMaxHeapK) return ABX_ERR_UNSUPPORTED;
#define ABX_BY_FORMAT(CALL, KD)                                      \
  do {                                                               \
    if (b->format == ABX_NODES_FP32) return CALL(KD, ABX_NODES_FP32); \
    if (b->format == ABX_NODES_Q16W) return CALL(KD, ABX_NODES_Q16W); \
    return CALL(KD, ABX_NODES_Q16);                                  \
  } while (0)
  if (k > kMaxRegK) {
#define ABX_HEAP(KD, FM) nearest_heap<KD, FM>(b, pts, m, order, k, idx, dist, stats, s)
    if (b->kind == ABX_PRIM_POINTS) ABX_BY_FORMAT(ABX_HEAP, ABX_PRIM_POINTS);
    ABX_BY_FORMAT(ABX_HEAP, ABX_PRIM_BOXES);
#undef ABX_HEAP
  }
  // a 4-wide walk makes about half as many node visits as a binary one
  const int64_t b_eff = b->format == ABX_NODES_Q16W ? std::max<int64_t>(1, budget / 2) : budget;
  const NearestScratch ns{heavy_q, heavy_bound, counters, effective_budget(b_eff, m), heavy_state,
                          (uint32_t)std::min<int64_t>(state_cap, kMaxSavedHeavy)};
#define ABX_FMT(KD, FM) nearest_fmt<KD, FM>(b, pts, m, order, k, idx, dist, stats, ns, s)
  if (b->kind == ABX_PRIM_POINTS) ABX_BY_FORMAT(ABX_FMT, ABX_PRIM_POINTS);
  ABX_BY_FORMAT(ABX_FMT, ABX_PRIM_BOXES);
#undef ABX_FMT
#undef ABX_BY_FORMAT
}

int max_tree_depth() { return kMaxDepth; }

}  // namespace abx
