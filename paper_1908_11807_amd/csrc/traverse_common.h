// Device code shared by the traversal kernels (plain trees and forests):
// tree views, node decoding, per-lane stacks and the nearest-neighbour walk.
// See traverse.hip for the method (ArborX paper, section 2.2).
#pragma once

#include <climits>

#include "abx_internal.h"

namespace abx {

constexpr int kTravBlock = 256;
constexpr int kMaxDepth = 128;
constexpr int kLdsDepthSpatial = 16;
constexpr int kLdsDepthNearest = 16;

struct TreeArgs {
  const void *nodes;
  const void *leaves;
  int64_t n;
  float scene[6];
  float qo[3], qs[3];
  const float *scene_dev;  // the same scene box in device memory
  const float *qframe;     // if set: Q16 origin[3], scale[3] in device memory (read at
                           // kernel start; used where the host has not read them back)
};

__device__ __forceinline__ void resolve_qframe(TreeArgs &t) {
  if (t.qframe) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t.qo[a] = t.qframe[a];
      t.qs[a] = t.qframe[3 + a];
    }
  }
}

struct QueryArgs {
  const float *data;
  int64_t m;
  const float *radii;
  float radius;
  const int32_t *order;  // sorted position -> caller's query index (or null)
};

// hardware dispatches workgroup b to XCD b % 8; hand XCD x a contiguous
// range of tiles so neighbouring (Morton-adjacent) tiles share an L2
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t x = b & 7, k = b >> 3, q = nb >> 3, rem = nb & 7;
  return x * q + (x < rem ? x : rem) + k;
}

struct Kids {
  float l[6], r[6];
  int32_t lref, rref;
};

template <int FMT>
__device__ __forceinline__ void load_kids(const TreeArgs &t, int32_t node, Kids &k) {
  if (FMT == ABX_NODES_FP32) {
    const float4 *p = reinterpret_cast<const float4 *>(t.nodes) + 4 * (int64_t)node;
    const float4 a = p[0], b = p[1], c = p[2];
    const int4 d = reinterpret_cast<const int4 *>(p)[3];
    k.l[0] = a.x; k.l[1] = a.y; k.l[2] = a.z; k.l[3] = a.w; k.l[4] = b.x; k.l[5] = b.y;
    k.r[0] = b.z; k.r[1] = b.w; k.r[2] = c.x; k.r[3] = c.y; k.r[4] = c.z; k.r[5] = c.w;
    k.lref = d.x;
    k.rref = d.y;
  } else {
    const uint4 *p = reinterpret_cast<const uint4 *>(t.nodes) + 2 * (int64_t)node;
    const uint4 a = p[0], b = p[1];
    const uint32_t w[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t q = (w[j / 2] >> (16 * (j & 1))) & 0xffffu;
      const int ax = j % 3;
      k.l[j] = deq(q, t.qs[ax], t.qo[ax]);
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t q = (w[3 + j / 2] >> (16 * (j & 1))) & 0xffffu;
      const int ax = j % 3;
      k.r[j] = deq(q, t.qs[ax], t.qo[ax]);
    }
    k.lref = (int32_t)b.z;
    k.rref = (int32_t)b.w;
  }
}

// exact box of the leaf at sorted position `leaf` (Q16 leaf record) and its
// primitive's index
template <int KIND>
__device__ __forceinline__ int32_t load_leaf_q16(const TreeArgs &t, int32_t leaf, float b[6]) {
  if (KIND == ABX_PRIM_POINTS) {
    const float4 v = reinterpret_cast<const float4 *>(t.leaves)[leaf];
    b[0] = b[3] = v.x;
    b[1] = b[4] = v.y;
    b[2] = b[5] = v.z;
    return __float_as_int(v.w);
  } else {
    const float4 *p = reinterpret_cast<const float4 *>(t.leaves) + 2 * (int64_t)leaf;
    const float4 u = p[0], v = p[1];
    b[0] = u.x; b[1] = u.y; b[2] = u.z; b[3] = u.w; b[4] = v.x; b[5] = v.y;
    return __float_as_int(v.z);
  }
}

// Per-lane stack: entry e of lane t lives at lds[e * kTravBlock + t] for
// e < S, else at ovf[e - S] in the lane's private memory.  The LDS part is
// addressed through an explicit LDS (address space 3) pointer so that the
// two paths stay separate instructions (the compiler would otherwise merge
// them into one generic flat access, slower on the common LDS path).
#define ABX_LDS __attribute__((address_space(3)))

template <typename T, int S, int B>
__device__ __forceinline__ void stack_push(ABX_LDS T *lds, T *ovf, int &sp, T x) {
  if (sp < S) {
    lds[sp * B] = x;
  } else {
    ovf[sp - S] = x;
  }
  ++sp;
}

template <typename T, int S, int B>
__device__ __forceinline__ T stack_pop(ABX_LDS T *lds, const T *ovf, int &sp) {
  --sp;
  T v;
  if (sp < S) {
    v = lds[sp * B];
  } else {
    v = ovf[sp - S];
  }
  return v;
}

// the nearest traversal's stack holds (node, box distance) pairs
template <int S, int B>
__device__ __forceinline__ void stack_push2(ABX_LDS int32_t *ln, ABX_LDS float *ld, int32_t *on,
                                            float *od, int &sp, int32_t n, float d) {
  if (sp < S) {
    ln[sp * B] = n;
    ld[sp * B] = d;
  } else {
    on[sp - S] = n;
    od[sp - S] = d;
  }
  ++sp;
}

template <int S, int B>
__device__ __forceinline__ void stack_pop2(ABX_LDS int32_t *ln, ABX_LDS float *ld, const int32_t *on,
                                           const float *od, int &sp, int32_t &n, float &d) {
  --sp;
  if (sp < S) {
    n = ln[sp * B];
    d = ld[sp * B];
  } else {
    n = on[sp - S];
    d = od[sp - S];
  }
}

enum { MODE_COUNT = 0, MODE_FILL = 1, MODE_STATS = 2 };

// ------------------------------------------------------------------ nearest
// (d, i) precedes (e, j) in (distance, index) order
__device__ __forceinline__ bool precedes(float d, int32_t i, float e, int32_t j) {
  return d < e || (d == e && i < j);
}

// Insert (d, idx) -- known to precede the last entry -- into the ascending
// register list, dropping the last entry.  Fully unrolled: constant register
// indices only.
template <int K>
__device__ __forceinline__ void knn_insert(float (&bd)[K], int32_t (&bi)[K], float d, int32_t idx) {
  bool after_prev = true;  // x precedes a[j] (true for j = K-1)
#pragma unroll
  for (int j = K - 1; j > 0; --j) {
    const bool lt_prev = precedes(d, idx, bd[j - 1], bi[j - 1]);
    const float nd = lt_prev ? bd[j - 1] : (after_prev ? d : bd[j]);
    const int32_t ni = lt_prev ? bi[j - 1] : (after_prev ? idx : bi[j]);
    bd[j] = nd;
    bi[j] = ni;
    after_prev = lt_prev;
  }
  if (after_prev) {
    bd[0] = d;
    bi[0] = idx;
  }
}

// The k best candidates of one lane, ascending by (squared distance, index).
// Slots [0, K-k) hold sentinels that precede everything and never move; the
// k live slots start empty (+inf).
template <int K>
struct KnnList {
  float bd[K];
  int32_t bi[K];
  __device__ __forceinline__ void init(int k) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const bool dummy = j < K - k;
      bd[j] = dummy ? -1.0f : INFINITY;
      bi[j] = dummy ? -1 : INT_MAX;
    }
  }
  __device__ __forceinline__ float kth() const { return bd[K - 1]; }
  __device__ __forceinline__ void offer(float d, int32_t idx) {
    if (precedes(d, idx, bd[K - 1], bi[K - 1])) knn_insert<K>(bd, bi, d, idx);
  }
  // drop the front entry (sentinel or taken), pad the back with +inf
  __device__ __forceinline__ void shift() {
#pragma unroll
    for (int j = 0; j + 1 < K; ++j) {
      bd[j] = bd[j + 1];
      bi[j] = bi[j + 1];
    }
    bd[K - 1] = INFINITY;
    bi[K - 1] = INT_MAX;
  }
};

struct KnnQuery {
  float x, y, z;
};

// A leaf child whose node-stored box is at squared distance dbox: confirm
// with the exact leaf box (Q16) and offer it to the list.  Candidates beyond
// `thr` (an upper bound of the final k-th distance) cannot be in the result.
template <int KIND, int FMT, int K>
__device__ __forceinline__ void knn_leaf(const TreeArgs &t, const KnnQuery &q, int32_t pos,
                                         float dbox, float thr, KnnList<K> &L, int32_t &reads) {
  if (!(dbox <= thr)) return;
  ++reads;
  if (FMT == ABX_NODES_FP32) {
    // the node box of a leaf child is the primitive's exact box
    L.offer(dbox, reinterpret_cast<const int32_t *>(t.leaves)[pos]);
  } else {
    float b[6];
    const int32_t idx = load_leaf_q16<KIND>(t, pos, b);
    const float d = box_dist2(b[0], b[1], b[2], b[3], b[4], b[5], q.x, q.y, q.z);
    if (d <= thr) L.offer(d, idx);
  }
}

// One step of the nearest walk: visit `node`, offer its leaf children, and
// return the nearer qualifying internal child (the farther one is pushed),
// or -1 when neither qualifies.  `bound` is an external upper bound of the
// final k-th distance (+inf when there is none).
template <int KIND, int FMT, int K, int B>
__device__ __forceinline__ int32_t knn_visit(const TreeArgs &t, const KnnQuery &q, int32_t node,
                                             float bound, KnnList<K> &L, ABX_LDS int32_t *lds_n,
                                             ABX_LDS float *lds_d, int32_t *ovf_n, float *ovf_d,
                                             int &sp, int32_t &reads) {
  Kids c;
  load_kids<FMT>(t, node, c);
  const float dl = box_dist2(c.l[0], c.l[1], c.l[2], c.l[3], c.l[4], c.l[5], q.x, q.y, q.z);
  const float dr = box_dist2(c.r[0], c.r[1], c.r[2], c.r[3], c.r[4], c.r[5], q.x, q.y, q.z);
  const bool ll = c.lref < 0, lr = c.rref < 0;
  if (ll) knn_leaf<KIND, FMT, K>(t, q, ~c.lref, dl, fminf(L.kth(), bound), L, reads);
  if (lr) knn_leaf<KIND, FMT, K>(t, q, ~c.rref, dr, fminf(L.kth(), bound), L, reads);
  const float thr = fminf(L.kth(), bound);
  const bool gl = !ll && dl <= thr, gr = !lr && dr <= thr;
  if (gl && gr) {
    const bool left_first = dl <= dr;
    if (sp < kMaxDepth)
      stack_push2<kLdsDepthNearest, B>(lds_n, lds_d, ovf_n, ovf_d, sp,
                                       left_first ? c.rref : c.lref, left_first ? dr : dl);
    return left_first ? c.lref : c.rref;
  }
  if (gl) return c.lref;
  if (gr) return c.rref;
  return -1;
}

// pop deferred nodes until one still qualifies; -1 when the stack runs dry
template <int B>
__device__ __forceinline__ int32_t knn_pop(float thr, ABX_LDS int32_t *lds_n, ABX_LDS float *lds_d,
                                           const int32_t *ovf_n, const float *ovf_d, int &sp) {
  while (sp > 0) {
    int32_t en;
    float ed;
    stack_pop2<kLdsDepthNearest, B>(lds_n, lds_d, ovf_n, ovf_d, sp, en, ed);
    if (ed <= thr) return en;
  }
  return -1;
}

// Where each query's walk starts and where its row goes.
struct QInfo {
  int32_t root;        // internal node to start from, or ~leaf for a one-leaf tree
  int kk;              // row length min(k, n of the query's tree)
  int64_t out;         // first output slot of the row
  int32_t base;        // subtracted from primitive indices (tree-local rows)
  const float *lbox;   // exact box of the leaf when root < 0
};

// One tree, every row of length k.
struct PlainMap {
  int k;
  __device__ __forceinline__ QInfo info(int64_t qi, const TreeArgs &t) const {
    QInfo r;
    r.root = t.n == 1 ? ~0 : 0;
    r.kk = k;
    r.out = qi * k;
    r.base = 0;
    r.lbox = t.scene_dev;
    return r;
  }
};

template <int K>
__device__ __forceinline__ void knn_write(const KnnList<K> &L, int k, int32_t base, int32_t *oi,
                                          float *od) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j >= K - k) {
      oi[j - (K - k)] = L.bi[j] - base;
      od[j - (K - k)] = sqrtf(L.bd[j]);
    }
  }
}

struct HeavyList {
  int32_t *q;          // caller's query index
  float *bound;        // k-th distance reached before the hand-off
  uint32_t *count;     // [0] entries, [1] next entry to serve
};

// Pass 1 for one query (one lane).  A walk that exceeds `budget` node
// visits stops and hands the query to the cooperative pass with the k-th
// distance it has found so far (an upper bound of the final one).
template <int KIND, int FMT, int K, bool STATS, int B, class Map>
__device__ __forceinline__ void nearest_lane(const TreeArgs &t, const Map &map,
                                             const float *__restrict__ pts, int64_t qi,
                                             ABX_LDS int32_t *lds_n, ABX_LDS float *lds_d,
                                             int32_t *__restrict__ indices, float *__restrict__ dist,
                                             int32_t *__restrict__ stats, int64_t budget,
                                             const HeavyList &heavy) {
  const QInfo info = map.info(qi, t);
  if (info.kk == 0) {
    if (STATS) stats[2 * qi] = stats[2 * qi + 1] = 0;
    return;
  }
  const KnnQuery q{pts[3 * qi], pts[3 * qi + 1], pts[3 * qi + 2]};
  KnnList<K> L;
  L.init(info.kk);
  int32_t visited = 0, reads = 0;
  bool done = true;
  if (info.root < 0) {
    const float *b = info.lbox;
    const float d = box_dist2(b[0], b[1], b[2], b[3], b[4], b[5], q.x, q.y, q.z);
    knn_leaf<KIND, FMT, K>(t, q, ~info.root, d, INFINITY, L, reads);
  } else {
    int32_t ovf_n[kMaxDepth - kLdsDepthNearest];
    float ovf_d[kMaxDepth - kLdsDepthNearest];
    int sp = 0;
    int32_t node = info.root;
    const int64_t limit = budget < t.n ? budget : t.n;
    done = false;
    for (int64_t it = 0; it < limit; ++it) {
      if (STATS) ++visited;
      node = knn_visit<KIND, FMT, K, B>(t, q, node, INFINITY, L, lds_n, lds_d, ovf_n, ovf_d, sp,
                                        reads);
      if (node < 0) node = knn_pop<B>(L.kth(), lds_n, lds_d, ovf_n, ovf_d, sp);
      if (node < 0) {
        done = true;
        break;
      }
    }
  }
  if (STATS) {
    stats[2 * qi] = visited;
    stats[2 * qi + 1] = reads;
    return;
  }
  if (!done) {
    const uint32_t h = atomicAdd(heavy.count, 1u);
    heavy.q[h] = (int32_t)qi;
    heavy.bound[h] = L.kth();
    return;
  }
  knn_write<K>(L, info.kk, info.base, indices + info.out, dist + info.out);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return v;
}

constexpr int kCoopFront = 256;      // frontier size at which the lanes split up
constexpr int kCoopFrontCap = 1024;  // > 2 * (kCoopFront - 1)
constexpr int kCoopBlocksPerCU = 6;

// Pass 2: one wavefront per heavy query (several lanes per query).  The wave
// expands the tree breadth-first until the frontier holds kCoopFront nodes,
// then lane l walks frontier entries l, l+64, ... depth-first with its own
// stack and candidate list.  Every step the lanes share the smallest of
// their k-th distances (each is the k-th distance of k real primitives, so
// it bounds the final k-th distance from above) and prune with it.  Every
// primitive of the final result lives in the list of the lane that met it,
// so the k best of the 64 lists, taken in (distance, index) order, are the
// exact answer.  Runs as a persistent grid draining the heavy list.
template <int KIND, int FMT, int K, class Map>
__global__ __launch_bounds__(kWave) void k_nearest_coop(TreeArgs t, Map map,
                                                        const float *__restrict__ pts,
                                                        int32_t *__restrict__ indices,
                                                        float *__restrict__ dist, HeavyList heavy) {
  __shared__ int32_t s_fn[2][kCoopFrontCap];
  __shared__ float s_fd[2][kCoopFrontCap];
  __shared__ int32_t s_node[kLdsDepthNearest * kWave];
  __shared__ float s_dist[kLdsDepthNearest * kWave];
  __shared__ uint32_t s_h;
  const int lane = threadIdx.x;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t total = heavy.count[0];
  resolve_qframe(t);
  int32_t reads = 0;
  while (true) {
    if (lane == 0) s_h = atomicAdd(heavy.count + 1, 1u);
    __syncthreads();
    const uint32_t h = s_h;
    __syncthreads();
    if (h >= total) break;
    const int32_t qi = heavy.q[h];
    const QInfo info = map.info(qi, t);
    const int k = info.kk;
    const KnnQuery q{pts[3 * (int64_t)qi], pts[3 * (int64_t)qi + 1], pts[3 * (int64_t)qi + 2]};
    float bound = heavy.bound[h];
    KnnList<K> L;
    L.init(k);

    // breadth-first expansion of the frontier
    int cur = 0, fsize = 1;
    if (lane == 0) {
      s_fn[0][0] = info.root;
      s_fd[0][0] = 0.0f;
    }
    __syncthreads();
    while (fsize > 0 && fsize < kCoopFront) {
      int nsize = 0;
      for (int base = 0; base < fsize; base += kWave) {
        const int e = base + lane;
        bool el = false, er = false;
        int32_t lref = 0, rref = 0;
        float dl = 0.0f, dr = 0.0f;
        if (e < fsize && s_fd[cur][e] <= fminf(L.kth(), bound)) {
          Kids c;
          load_kids<FMT>(t, s_fn[cur][e], c);
          dl = box_dist2(c.l[0], c.l[1], c.l[2], c.l[3], c.l[4], c.l[5], q.x, q.y, q.z);
          dr = box_dist2(c.r[0], c.r[1], c.r[2], c.r[3], c.r[4], c.r[5], q.x, q.y, q.z);
          if (c.lref < 0) knn_leaf<KIND, FMT, K>(t, q, ~c.lref, dl, fminf(L.kth(), bound), L, reads);
          if (c.rref < 0) knn_leaf<KIND, FMT, K>(t, q, ~c.rref, dr, fminf(L.kth(), bound), L, reads);
          const float thr = fminf(L.kth(), bound);
          el = c.lref >= 0 && dl <= thr;
          er = c.rref >= 0 && dr <= thr;
          lref = c.lref;
          rref = c.rref;
        }
        const uint64_t bl = __ballot(el), br = __ballot(er);
        const int cl = __popcll(bl);
        if (el) {
          const int o = nsize + __popcll(bl & lt);
          s_fn[cur ^ 1][o] = lref;
          s_fd[cur ^ 1][o] = dl;
        }
        if (er) {
          const int o = nsize + cl + __popcll(br & lt);
          s_fn[cur ^ 1][o] = rref;
          s_fd[cur ^ 1][o] = dr;
        }
        nsize += cl + __popcll(br);
        bound = wave_min(fminf(bound, L.kth()));
      }
      __syncthreads();
      cur ^= 1;
      fsize = nsize;
    }

    // depth-first walks of the lane's share of the frontier
    int32_t ovf_n[kMaxDepth - kLdsDepthNearest];
    float ovf_d[kMaxDepth - kLdsDepthNearest];
    ABX_LDS int32_t *lds_n = (ABX_LDS int32_t *)(s_node) + lane;
    ABX_LDS float *lds_d = (ABX_LDS float *)(s_dist) + lane;
    int sp = 0;
    const int mine = fsize > lane ? (fsize - 1 - lane) / kWave + 1 : 0;
    for (int a = mine - 1; a >= 0; --a)
      stack_push2<kLdsDepthNearest, kWave>(lds_n, lds_d, ovf_n, ovf_d, sp,
                                           s_fn[cur][lane + kWave * a], s_fd[cur][lane + kWave * a]);
    __syncthreads();
    bool active = true;
    int32_t node = -1;
    for (int64_t it = 0; it < 4 * t.n + 64; ++it) {
      bound = wave_min(fminf(bound, L.kth()));
      if (!__any(active)) break;
      if (active) {
        if (node < 0) node = knn_pop<kWave>(fminf(L.kth(), bound), lds_n, lds_d, ovf_n, ovf_d, sp);
        if (node < 0) {
          active = false;
        } else {
          node = knn_visit<KIND, FMT, K, kWave>(t, q, node, bound, L, lds_n, lds_d, ovf_n, ovf_d,
                                                sp, reads);
        }
      }
    }

    // merge: k rounds of a wave-wide (distance, index) minimum over the
    // lanes' list fronts
    for (int s = 0; s < K - k; ++s) L.shift();
    float out_d = 0.0f;
    int32_t out_i = 0;
    for (int j = 0; j < k; ++j) {
      float d = L.bd[0];
      int32_t i = L.bi[0];
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const float d2 = __shfl_xor(d, o, kWave);
        const int32_t i2 = __shfl_xor(i, o, kWave);
        if (precedes(d2, i2, d, i)) {
          d = d2;
          i = i2;
        }
      }
      if (L.bi[0] == i && L.bd[0] == d) L.shift();
      if (lane == j) {
        out_d = d;
        out_i = i;
      }
    }
    if (lane < k) {
      indices[info.out + lane] = out_i - info.base;
      dist[info.out + lane] = sqrtf(out_d);
    }
  }
  (void)reads;
}

}  // namespace abx
