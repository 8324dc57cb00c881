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
constexpr int kLdsDepthNearest = 8;
// LDS stack window of the one-lane nearest pass (16-bit stack distances,
// six-byte entries) for an occupancy target of `waves` per SIMD: 16 entries
// take 24 KB per 256-lane workgroup (six workgroups per CU), 32 take 48 KB
// (three).  The 16 entries also cap the k <= 4 walks, whose target is eight
// waves, at six: at k = 1 on the C3 shell that ran 9 % faster than 8 entries
// at eight waves.
constexpr int lane_window(int waves) { return waves > 3 ? 16 : 32; }
constexpr int kMaxRegK = 64;    // largest k kept in registers (lists of 1..64 keys)
constexpr int kMaxHeapK = 128;  // largest k (the LDS-heap kernel serves 65..128)

// Occupancy target of the one-lane nearest pass (waves per SIMD).  Six beat
// eight at k = 10 on the C3 shell (fewer walks competing for L2, no spills);
// the k = 32 list alone takes 64 registers.
// 4-wide walks hold four slots' distances and keys: at the binary targets
// they spilled (66 registers at k = 10); these targets leave them unspilled.
constexpr int nearest_waves_per_eu(int K, int FMT = 0) {
  return FMT == ABX_NODES_Q16W ? (K > 16 ? 2 : (K > 10 ? 3 : (K > 4 ? 5 : 6)))
                               : (K > 48 ? 2 : (K > 16 ? 3 : (K > 10 ? 4 : (K > 4 ? 6 : 8))));
}

struct TreeArgs {
  const void *nodes;
  const void *leaves;
  int64_t n;
  int64_t nint;            // internal nodes stored (n - 1; fewer for 4-wide nodes)
  int32_t root;            // internal node at the root (n >= 2)
  float scene[6];
  float qo[3], qs[3];
  const float *scene_dev;  // the same scene box in device memory
  const float *qframe;     // if set: Q16 origin[3], scale[3] in device memory (read at
                           // kernel start; used where the host has not read them back)
  const TreeHeader *guard; // if set: the construction's header, read at kernel start
                           // (forests, whose build the host does not wait for)
};

// A tree whose construction reported a problem (any flag, or a height the
// stacks cannot hold) is not walked: its nodes may not form a tree.
__device__ __forceinline__ bool tree_unusable(const TreeArgs &t) {
  return t.guard && (t.guard->bad != 0 || t.guard->height + 8 >= kMaxDepth);
}

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
  // one-pass (1P) scheme only
  int32_t *buf;          // [m * bufsize] stored hits, one row per sorted position
  int32_t bufsize;
  uint32_t *flag;        // [0] != 0: some query found more than bufsize hits
  const int64_t *total;  // device total of the scanned counts
  int64_t capacity;      // entries the caller's index buffer holds
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

// Child references: r >= 0 is internal node r; r < 0 is a leaf holding
// primitive ~r.  Whether a node's child slot already holds a leaf's exact
// box: always for FP32 nodes (the slot is the primitive's box), and for Q16
// point trees (the slot holds the point's float32 coordinates).  Q16 box
// trees keep a quantised box in the slot and the exact box in a record
// addressed by primitive index.
template <int KIND, int FMT>
constexpr bool exact_leaf_slots() {
  return FMT == ABX_NODES_FP32 || KIND == ABX_PRIM_POINTS;
}

template <int KIND, int FMT>
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
    k.lref = (int32_t)b.z;
    k.rref = (int32_t)b.w;
    const bool pl = KIND == ABX_PRIM_POINTS && k.lref < 0;
    const bool pr = KIND == ABX_PRIM_POINTS && k.rref < 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t q = (w[j / 2] >> (16 * (j & 1))) & 0xffffu;
      const int ax = j % 3;
      const float v = deq(q, t.qs[ax], t.qo[ax]);
      k.l[j] = pl ? __uint_as_float(w[ax]) : v;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t q = (w[3 + j / 2] >> (16 * (j & 1))) & 0xffffu;
      const int ax = j % 3;
      const float v = deq(q, t.qs[ax], t.qo[ax]);
      k.r[j] = pr ? __uint_as_float(w[3 + ax]) : v;
    }
  }
}

// The four children of a 4-wide node (FMT == ABX_NODES_Q16W).  An unused
// slot has reference kEmptyRef and is never taken.
struct Kids4 {
  float b[4][6];
  int32_t ref[4];
};

template <int KIND>
__device__ __forceinline__ void load_kids4(const TreeArgs &t, int32_t node, Kids4 &k) {
  const uint4 *p = reinterpret_cast<const uint4 *>(t.nodes) + 4 * (int64_t)node;
  const uint4 a = p[0], b = p[1], c = p[2], d = p[3];
  const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
  k.ref[0] = (int32_t)d.x;
  k.ref[1] = (int32_t)d.y;
  k.ref[2] = (int32_t)d.z;
  k.ref[3] = (int32_t)d.w;
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
    const bool pt = KIND == ABX_PRIM_POINTS && k.ref[c4] < 0;  // a point leaf (or unused)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t q = (w[3 * c4 + j / 2] >> (16 * (j & 1))) & 0xffffu;
      const int ax = j % 3;
      const float v = deq(q, t.qs[ax], t.qo[ax]);
      k.b[c4][j] = pt ? __uint_as_float(w[3 * c4 + ax]) : v;
    }
  }
}

// exact box of primitive `idx` of a Q16 box tree (its leaf record)
__device__ __forceinline__ void load_leaf_box(const TreeArgs &t, int32_t idx, float b[6]) {
  const float4 *p = reinterpret_cast<const float4 *>(t.leaves) + 2 * (int64_t)idx;
  const float4 u = p[0], v = p[1];
  b[0] = u.x; b[1] = u.y; b[2] = u.z; b[3] = u.w; b[4] = v.x; b[5] = v.y;
}

// Per-lane stack with its top in LDS.  Positions [sp - nl, sp) (at most S
// entries) live in a circular LDS window, slot (position mod S) of the
// lane's column (stride B lanes); deeper positions live in the lane's
// private memory at ovf[position].  A push into a full window first moves
// the window's bottom entry to private memory; a pop from an empty window
// reads private memory directly.  A walk that pushes and pops near the top
// (a depth-first traversal oscillating around some depth) therefore stays in
// LDS, and private memory is touched only when the depth drifts by more than
// S.  The LDS part is addressed through an explicit LDS (address space 3)
// pointer so the two paths stay separate instructions.
#define ABX_LDS __attribute__((address_space(3)))

template <typename T, int S, int B>
__device__ __forceinline__ void stack_push(ABX_LDS T *lds, T *ovf, int &sp, int &nl, T x) {
  static_assert((S & (S - 1)) == 0, "window size is a power of two");
  const int slot = (sp & (S - 1)) * B;
  if (nl == S) ovf[sp - S] = lds[slot];
  else ++nl;
  lds[slot] = x;
  ++sp;
}

template <typename T, int S, int B>
__device__ __forceinline__ T stack_pop(ABX_LDS T *lds, const T *ovf, int &sp, int &nl) {
  --sp;
  T v;
  if (nl > 0) {
    --nl;
    v = lds[(sp & (S - 1)) * B];
  } else {
    v = ovf[sp];
  }
  return v;
}

// The nearest traversal's stack holds (node, box distance) pairs.  The
// distance is stored as a float, or as its upper 16 bits (DT = uint16_t):
// truncating a non-negative float rounds it down, so the stored value is a
// lower bound of the box distance, and a node that the exact value would
// have pruned when popped is visited instead, its children (boxes inside
// its box, no nearer) then pruned: the same results, 6-byte entries.
__device__ __forceinline__ float stk_enc(float d, float) { return d; }
__device__ __forceinline__ uint16_t stk_enc(float d, uint16_t) {
  return (uint16_t)(__float_as_uint(d) >> 16);
}
__device__ __forceinline__ float stk_dec(float d) { return d; }
__device__ __forceinline__ float stk_dec(uint16_t d) { return __uint_as_float((uint32_t)d << 16); }

template <int S, int B, typename DT>
__device__ __forceinline__ void stack_push2(ABX_LDS int32_t *ln, ABX_LDS DT *ld, int32_t *on,
                                            DT *od, int &sp, int &nl, int32_t n, float d) {
  static_assert((S & (S - 1)) == 0, "window size is a power of two");
  const int slot = (sp & (S - 1)) * B;
  if (nl == S) {
    on[sp - S] = ln[slot];
    od[sp - S] = ld[slot];
  } else {
    ++nl;
  }
  ln[slot] = n;
  ld[slot] = stk_enc(d, DT());
  ++sp;
}

template <int S, int B, typename DT>
__device__ __forceinline__ void stack_pop2(ABX_LDS int32_t *ln, ABX_LDS DT *ld, const int32_t *on,
                                           const DT *od, int &sp, int &nl, int32_t &n, float &d) {
  --sp;
  if (nl > 0) {
    --nl;
    const int slot = (sp & (S - 1)) * B;
    n = ln[slot];
    d = stk_dec(ld[slot]);
  } else {
    n = on[sp];
    d = stk_dec(od[sp]);
  }
}

enum { MODE_COUNT = 0, MODE_FILL = 1, MODE_STATS = 2, MODE_STORE = 3 };

// ------------------------------------------------------------------ nearest
// A candidate (squared distance d, primitive index i) packed into one
// signed 64-bit key: the float bits of d (d >= 0, so its bit pattern orders
// like the value) in the high word, i in the low word.  Key order is then
// exactly the (distance, index) order, and one 64-bit compare replaces the
// two-field comparison.  NaN distances pack above +inf and are never taken.
__device__ __forceinline__ int64_t knn_key(float d, int32_t i) {
  return (int64_t)(((uint64_t)__float_as_uint(d) << 32) | (uint32_t)i);
}
__device__ __forceinline__ float key_dist(int64_t key) {
  return __uint_as_float((uint32_t)((uint64_t)key >> 32));
}
__device__ __forceinline__ int32_t key_index(int64_t key) { return (int32_t)(uint32_t)key; }

constexpr int64_t kKeySentinel = -1;  // precedes every candidate
// an empty slot: (+inf, INT_MAX), preceded by every finite candidate
constexpr int64_t kKeyEmpty = (int64_t)(((uint64_t)0x7f800000u << 32) | 0x7fffffffu);

// The k best candidates of one lane, ascending keys.  Slots [0, K-k) hold
// sentinels that precede everything and never move; the k live slots start
// empty.
template <int K>
struct KnnList {
  int64_t key[K];
  __device__ __forceinline__ void init(int k) {
#pragma unroll
    for (int j = 0; j < K; ++j) key[j] = j < K - k ? kKeySentinel : kKeyEmpty;
  }
  __device__ __forceinline__ float kth() const { return key_dist(key[K - 1]); }
  // Insert x if it precedes the last entry, dropping the last entry.  With
  // c_j = (x < key[j]) (false up to the insertion point, true after it), slot
  // j keeps its entry, takes x, or takes its predecessor's entry.  Fully
  // unrolled: constant register indices only.
  __device__ __forceinline__ void offer_key(int64_t x) {
    if (x < key[K - 1]) {
      bool c_prev = x < key[0];
      int64_t prev = key[0];
      if (c_prev) key[0] = x;
#pragma unroll
      for (int j = 1; j < K; ++j) {
        const bool c = x < key[j];
        const int64_t cur = key[j];
        key[j] = c ? (c_prev ? prev : x) : cur;
        prev = cur;
        c_prev = c;
      }
    }
  }
  __device__ __forceinline__ void offer(float d, int32_t idx) { offer_key(knn_key(d, idx)); }
  // drop the front entry (sentinel or taken), pad the back with an empty slot
  __device__ __forceinline__ void shift() {
#pragma unroll
    for (int j = 0; j + 1 < K; ++j) key[j] = key[j + 1];
    key[K - 1] = kKeyEmpty;
  }
};

// Candidates waiting to enter a lane's list.  Inserting one costs ~70 VALU
// operations for k = 10, and a wavefront pays them whenever any of its lanes
// inserts; a lane meets a qualifying leaf in a few percent of its steps, so
// nearly every step paid for one lane.  Lanes therefore park up to two
// candidates and the wavefront inserts them together once kDeferLanes lanes
// have one waiting (a third candidate goes in at once).  Pruning meanwhile
// uses the list's k-th distance without the parked candidates: an upper
// bound of the final one, so nothing the exact walk needs is pruned.
constexpr int kDeferLanes = 4;

// An empty parking slot.  Parked keys are never negative (a parked distance
// passed a <= test, so it is a non-negative number, and indices are
// non-negative), so -1 marks an empty slot; as an inline constant it costs
// one move to set, where a wider constant can end up reloaded from private
// memory inside the walk loop.
constexpr int64_t kPendNone = -1;

struct KnnPending {
  int64_t a, b;
  __device__ __forceinline__ void init() { a = b = kPendNone; }
  template <int K>
  __device__ __forceinline__ void park(KnnList<K> &L, int64_t x) {
    if (a == kPendNone) a = x;
    else if (b == kPendNone) b = x;
    else L.offer_key(x);
  }
  // called by every active lane of the wavefront
  template <int K>
  __device__ __forceinline__ void flush_some(KnnList<K> &L) {
    if (__popcll(__ballot(a != kPendNone)) >= kDeferLanes && a != kPendNone) {
      L.offer_key(a);
      a = b;
      b = kPendNone;
    }
  }
  template <int K>
  __device__ __forceinline__ void flush_all(KnnList<K> &L) {
    if (a != kPendNone) L.offer_key(a);
    if (b != kPendNone) L.offer_key(b);
    a = b = kPendNone;
  }
};

struct KnnQuery {
  float x, y, z;
};

// A leaf child (primitive idx) whose node-stored box is at squared distance
// dbox: confirm with the exact box where the slot is quantised, and offer
// it to the list.  Candidates beyond `thr` (an upper bound of the final k-th
// distance) cannot be in the result.
template <int KIND, int FMT, int K>
__device__ __forceinline__ void knn_leaf(const TreeArgs &t, const KnnQuery &q, int32_t idx,
                                         float dbox, float thr, KnnList<K> &L, int32_t &reads) {
  if (!(dbox <= thr)) return;
  if (exact_leaf_slots<KIND, FMT>()) {
    L.offer(dbox, idx);
  } else {
    ++reads;
    float b[6];
    load_leaf_box(t, idx, b);
    const float d = box_dist2(b[0], b[1], b[2], b[3], b[4], b[5], q.x, q.y, q.z);
    if (d <= thr) L.offer(d, idx);
  }
}

// One step of the nearest walk: visit `node`, offer its leaf children, and
// return the nearer qualifying internal child (the farther one is pushed),
// or -1 when neither qualifies.  `bound` is an external upper bound of the
// final k-th distance (+inf when there is none).
template <int KIND, int FMT, int K, int B, int S = kLdsDepthNearest, bool DEFER = false, typename DT>
__device__ __forceinline__ int32_t knn_visit2(const TreeArgs &t, const KnnQuery &q, int32_t node,
                                              float bound, KnnList<K> &L, ABX_LDS int32_t *lds_n,
                                              ABX_LDS DT *lds_d, int32_t *ovf_n, DT *ovf_d,
                                              int &sp, int &nl, int32_t &reads,
                                              KnnPending *pend = nullptr) {
  Kids c;
  load_kids<KIND, FMT>(t, node, c);
  const float dl = box_dist2(c.l[0], c.l[1], c.l[2], c.l[3], c.l[4], c.l[5], q.x, q.y, q.z);
  const float dr = box_dist2(c.r[0], c.r[1], c.r[2], c.r[3], c.r[4], c.r[5], q.x, q.y, q.z);
  const bool ll = c.lref < 0, lr = c.rref < 0;
  if (DEFER && exact_leaf_slots<KIND, FMT>()) {
    const float thr0 = fminf(L.kth(), bound);
    const bool ol = ll && dl <= thr0, orr = lr && dr <= thr0;
    if (ol || orr) {
      pend->park(L, ol ? knn_key(dl, ~c.lref) : knn_key(dr, ~c.rref));
      if (ol && orr) pend->park(L, knn_key(dr, ~c.rref));
    }
    pend->flush_some(L);
  } else {
    if (ll) knn_leaf<KIND, FMT, K>(t, q, ~c.lref, dl, fminf(L.kth(), bound), L, reads);
    if (lr) knn_leaf<KIND, FMT, K>(t, q, ~c.rref, dr, fminf(L.kth(), bound), L, reads);
  }
  const float thr = fminf(L.kth(), bound);
  const bool gl = !ll && dl <= thr, gr = !lr && dr <= thr;
  if (gl && gr) {
    // Visit order only (pruning uses the box distances): the child whose box
    // centre is nearer goes first.  Box distances of the large boxes near
    // the root say little about where the nearest primitives are (a box
    // around a curved or slanted patch reaches far in front of it); the
    // centre tracks the primitives better, so the list fills with near
    // candidates sooner and prunes more (C3: 16 % fewer visits).
    // (lo - q) - (q - hi) = 2 (centre - q), from the differences the box
    // distances already formed
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
      stack_push2<S, B>(lds_n, lds_d, ovf_n, ovf_d, sp, nl, left_first ? c.rref : c.lref,
                        left_first ? dr : dl);
    return left_first ? c.lref : c.rref;
  }
  if (gl) return c.lref;
  if (gr) return c.rref;
  return -1;
}

// One 4-wide node decoded for a walk: per slot the squared box distance to
// q (+inf for an unused slot), the squared distance to the box centre
// (times 4; visit order only) and the reference.
template <int KIND>
__device__ __forceinline__ void wide_slots(const TreeArgs &t, int32_t node, const KnnQuery &q,
                                           float d[4], float key[4], int32_t r[4]) {
  const uint4 *p = reinterpret_cast<const uint4 *>(t.nodes) + 4 * (int64_t)node;
  const uint4 a = p[0], b = p[1], c = p[2], e = p[3];
  const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
  r[0] = (int32_t)e.x;
  r[1] = (int32_t)e.y;
  r[2] = (int32_t)e.z;
  r[3] = (int32_t)e.w;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool pt = KIND == ABX_PRIM_POINTS && r[j] < 0;  // a point leaf (or unused)
    float lo[3], hi[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const uint32_t ql = (w[3 * j + ax / 2] >> (16 * (ax & 1))) & 0xffffu;
      const uint32_t qh = (w[3 * j + (ax + 3) / 2] >> (16 * ((ax + 3) & 1))) & 0xffffu;
      const float pv = __uint_as_float(w[3 * j + ax]);
      lo[ax] = pt ? pv : deq(ql, t.qs[ax], t.qo[ax]);
      hi[ax] = pt ? pv : deq(qh, t.qs[ax], t.qo[ax]);
    }
    d[j] = r[j] == kEmptyRef ? INFINITY
                             : box_dist2(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], q.x, q.y, q.z);
    const float qv[3] = {q.x, q.y, q.z};
    float cc = 0.0f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float m = (lo[ax] - qv[ax]) - (qv[ax] - hi[ax]);
      cc = __fmaf_rn(m, m, cc);
    }
    key[j] = cc;
  }
}

// The same step over a 4-wide node: leaf children are offered as above;
// the qualifying internal children are visited nearest box centre first:
// the nearest is returned and the others are pushed farthest first, so they
// come off the stack in the same order.
template <int KIND, int K, int B, int S = kLdsDepthNearest, bool DEFER = false, typename DT>
__device__ __forceinline__ int32_t knn_visit_w(const TreeArgs &t, const KnnQuery &q, int32_t node,
                                               float bound, KnnList<K> &L, ABX_LDS int32_t *lds_n,
                                               ABX_LDS DT *lds_d, int32_t *ovf_n, DT *ovf_d,
                                               int &sp, int &nl, int32_t &reads,
                                               KnnPending *pend = nullptr) {
  // each slot is decoded straight into its box distance and centre key, so
  // the 24 coordinates are never live together (they made the walk spill)
  float d[4], key[4];
  int32_t r[4];
  wide_slots<KIND>(t, node, q, d, key, r);
  if (DEFER && exact_leaf_slots<KIND, ABX_NODES_Q16W>()) {
    const float thr0 = fminf(L.kth(), bound);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (r[j] < 0 && r[j] != kEmptyRef && d[j] <= thr0) pend->park(L, knn_key(d[j], ~r[j]));
    pend->flush_some(L);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (r[j] < 0 && r[j] != kEmptyRef)
        knn_leaf<KIND, ABX_NODES_Q16W, K>(t, q, ~r[j], d[j], fminf(L.kth(), bound), L, reads);
  }
  const float thr = fminf(L.kth(), bound);
  // the qualifying internal children keep their key; the others sort last
  // with reference -1
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool g = r[j] >= 0 && d[j] <= thr;
    key[j] = g ? key[j] : INFINITY;
    r[j] = g ? r[j] : -1;
  }
  // sorting network on four (key, reference, distance) triples; a NaN key
  // only changes the order, never drops a child
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
    if (r[j] >= 0 && sp < kMaxDepth) stack_push2<S, B>(lds_n, lds_d, ovf_n, ovf_d, sp, nl, r[j], d[j]);
  return r[0];
}

template <int KIND, int FMT, int K, int B, int S = kLdsDepthNearest, bool DEFER = false, typename DT>
__device__ __forceinline__ int32_t knn_visit(const TreeArgs &t, const KnnQuery &q, int32_t node,
                                             float bound, KnnList<K> &L, ABX_LDS int32_t *lds_n,
                                             ABX_LDS DT *lds_d, int32_t *ovf_n, DT *ovf_d,
                                             int &sp, int &nl, int32_t &reads,
                                             KnnPending *pend = nullptr) {
  if constexpr (FMT == ABX_NODES_Q16W)
    return knn_visit_w<KIND, K, B, S, DEFER>(t, q, node, bound, L, lds_n, lds_d, ovf_n, ovf_d, sp,
                                             nl, reads, pend);
  else
    return knn_visit2<KIND, FMT, K, B, S, DEFER>(t, q, node, bound, L, lds_n, lds_d, ovf_n, ovf_d,
                                                 sp, nl, reads, pend);
}

// pop deferred nodes until one still qualifies; -1 when the stack runs dry
template <int B, int S = kLdsDepthNearest, typename DT>
__device__ __forceinline__ int32_t knn_pop(float thr, ABX_LDS int32_t *lds_n, ABX_LDS DT *lds_d,
                                           const int32_t *ovf_n, const DT *ovf_d, int &sp, int &nl) {
  while (sp > 0) {
    int32_t en;
    float ed;
    stack_pop2<S, B>(lds_n, lds_d, ovf_n, ovf_d, sp, nl, en, ed);
    if (ed <= thr) return en;
  }
  return -1;
}

// Where each query's walk starts and where its row goes.
struct QInfo {
  int32_t root;        // internal node to start from, or ~primitive for a one-leaf tree
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
    r.root = t.n == 1 ? ~0 : t.root;
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
      oi[j - (K - k)] = key_index(L.key[j]) - base;
      od[j - (K - k)] = sqrtf(key_dist(L.key[j]));
    }
  }
}

struct HeavyList {
  int32_t *q;          // caller's query index
  float *bound;        // k-th distance reached before the hand-off
  uint32_t *count;     // [0] entries, [1] next entry to serve
  int32_t *state = nullptr;  // saved walks, kHeavyStateWords words each (optional)
  uint32_t state_cap = 0;    // entries below this keep their walk
};
static_assert(kHeavyStateWords == 2 + 2 * kHeavyStateEntries + 2 * kMaxRegK, "saved walk layout");

// Pass 1 for one query (one lane).  A walk that exceeds `budget` node
// visits stops and hands the query to the cooperative pass with the k-th
// distance it has found so far (an upper bound of the final one).
template <int KIND, int FMT, int K, bool STATS, int B, int W, class Map, typename DT>
__device__ __forceinline__ void nearest_lane(const TreeArgs &t, const Map &map,
                                             const float *__restrict__ pts, int64_t qi,
                                             ABX_LDS int32_t *lds_n, ABX_LDS DT *lds_d,
                                             int32_t *__restrict__ indices, float *__restrict__ dist,
                                             int32_t *__restrict__ stats, int64_t budget,
                                             const HeavyList &heavy) {
  constexpr int kWin = W;  // LDS window entries per lane (lds_n, lds_d: stride B)
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
    int32_t ovf_n[kMaxDepth];
    DT ovf_d[kMaxDepth];
    int sp = 0, nl = 0;
    int32_t node = info.root;
    const int64_t limit = budget < t.n ? budget : t.n;
    KnnPending pend;
    pend.init();
    done = false;
    for (int64_t it = 0; it < limit; ++it) {
      if (STATS) ++visited;
      node = knn_visit<KIND, FMT, K, B, kWin, true>(
          t, q, node, INFINITY, L, lds_n, lds_d, ovf_n, ovf_d, sp, nl, reads, &pend);
      if (node < 0) node = knn_pop<B, kWin>(L.kth(), lds_n, lds_d, ovf_n, ovf_d, sp, nl);
      if (node < 0) {
        done = true;
        break;
      }
    }
    pend.flush_all(L);
    if (!STATS && !done) {
      const uint32_t h = atomicAdd(heavy.count, 1u);
      heavy.q[h] = (int32_t)qi;
      heavy.bound[h] = L.kth();
      // the walk so far: the next node (not yet visited), the unexplored
      // subtrees on the stack, the candidates; the workgroup resumes it.
      // Lists of more than 32 keys restart instead: the save code's
      // registers made their walk spill (48 keys: 9 -> 525 spill accesses).
      if (K <= 32 && heavy.state && h < heavy.state_cap) {
        int32_t *st = heavy.state + (int64_t)h * kHeavyStateWords;
        if (sp + 1 > kHeavyStateEntries) {
          st[0] = -1;  // too deep to save: the workgroup restarts from the root
        } else {
          st[2] = node;
          st[3] = __float_as_int(0.0f);
          int c = 1;
          while (sp > 0) {
            int32_t en;
            float ed;
            stack_pop2<kWin, B>(lds_n, lds_d, ovf_n, ovf_d, sp, nl, en, ed);
            st[2 + 2 * c] = en;
            st[3 + 2 * c] = __float_as_int(ed);
            ++c;
          }
          st[0] = c;
          int64_t *keys = reinterpret_cast<int64_t *>(st + 2 + 2 * kHeavyStateEntries);
#pragma unroll
          for (int j = 0; j < K; ++j) keys[j] = L.key[j];
        }
      }
      return;
    }
  }
  if (STATS) {
    stats[2 * qi] = visited;
    stats[2 * qi + 1] = reads;
    return;
  }
  knn_write<K>(L, info.kk, info.base, indices + info.out, dist + info.out);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return v;
}

// wavefronts per heavy query: 16 (the heaviest query of a batch bounds the
// launch, so its walk is split 1024 ways); 8 for k > 16, whose lists need
// more registers than a 1024-thread workgroup leaves per lane
constexpr int coop_waves(int K) { return K > 16 ? 8 : 16; }

// the depth-first phase shares the workgroup's bound every 2^kCoopShareLog2
// steps: a fresher bound prunes more, sharing costs a wave-wide minimum and
// an LDS atomic per wave
constexpr int kCoopShareLog2 = 3;

// Pass 2: a workgroup of W wavefronts per heavy query.  The launch lasts as
// long as its heaviest query, whose walk is split W*64 ways.  The workgroup
// expands the tree breadth-first until the frontier holds 256*W nodes, then
// thread i walks frontier entries i, i + 64W, ... depth-first with its own
// stack and candidate list.  The threads share the smallest of their k-th
// distances through LDS (each is the k-th distance of k real primitives, so
// it bounds the final k-th distance from above) and prune with it.  Every
// primitive of the final result lives in the list of the thread that met it,
// so the k best of all lists, taken in (distance, index) order, are the
// exact answer: each wavefront merges its 64 lists, then the first merges
// the W results.  Runs as a persistent grid draining the heavy list.
template <int W, int A = 2>
struct CoopShape {
  static constexpr int kThreads = W * kWave;
  static constexpr int kCap = 512 * W;       // entries of a frontier buffer
  static constexpr int kFront = kCap / A;    // frontier size at which the threads split up:
                                             // one expansion of A-ary nodes stays below kCap
  static constexpr int kWindow = kCap / kThreads;  // LDS stack entries per thread
};

// LDS float minimum through the unsigned bit pattern (values are >= 0)
__device__ __forceinline__ void lds_min(uint32_t *p, float v) {
  atomicMin(p, __float_as_uint(v));
}

template <int KIND, int FMT, int K, class Map, int W>
__global__ __launch_bounds__(CoopShape<W>::kThreads) void k_nearest_coop(
    TreeArgs t, Map map, const float *__restrict__ pts, int32_t *__restrict__ indices,
    float *__restrict__ dist, HeavyList heavy) {
  using S = CoopShape<W, FMT == ABX_NODES_Q16W ? 4 : 2>;
  static_assert(kHeavyStateEntries < S::kFront, "a saved walk fits the first frontier");
  // two frontier buffers; during the depth-first phase the one not holding
  // the final frontier is the threads' stack window
  __shared__ int32_t s_fn[2][S::kCap];
  __shared__ float s_fd[2][S::kCap];
  __shared__ int64_t s_best[W][K];
  __shared__ uint32_t s_size[2], s_bound, s_h;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t total = heavy.count[0];
  resolve_qframe(t);
  int32_t reads = 0;
  while (true) {
    __syncthreads();  // the previous query's buffers are free again
    if (tid == 0) s_h = atomicAdd(heavy.count + 1, 1u);
    __syncthreads();
    const uint32_t h = s_h;
    if (h >= total) break;
    const int32_t qi = heavy.q[h];
    const QInfo info = map.info(qi, t);
    const int k = info.kk;
    const KnnQuery q{pts[3 * (int64_t)qi], pts[3 * (int64_t)qi + 1], pts[3 * (int64_t)qi + 2]};
    KnnList<K> L;
    L.init(k);
    // start from the walk the lane saved (its unexplored subtrees, and its
    // candidates in thread 0's list), else from the root
    int fsize = 1;
    // (lists of more than 32 keys never save their walk)
    const int32_t *st = K <= 32 && heavy.state && h < heavy.state_cap
                            ? heavy.state + (int64_t)h * kHeavyStateWords
                            : nullptr;
    int c = st ? min(st[0], kHeavyStateEntries) : -1;
    {
      // every saved node must be an internal node, else restart from the root
      bool bad = false;
      for (int e = tid; e < c; e += S::kThreads) {
        const int32_t nd = st[2 + 2 * e];
        bad |= nd < 0 || nd >= t.nint;
      }
      if (__syncthreads_or(bad)) c = -1;
    }
    if (c >= 1) {
      for (int e = tid; e < c; e += S::kThreads) {
        s_fn[0][e] = st[2 + 2 * e];
        s_fd[0][e] = __int_as_float(st[3 + 2 * e]);
      }
      fsize = c;
      if (tid == 0) {
        const int64_t *keys = reinterpret_cast<const int64_t *>(st + 2 + 2 * kHeavyStateEntries);
#pragma unroll
        for (int j = 0; j < K; ++j) L.key[j] = keys[j];
      }
    } else if (tid == 0) {
      s_fn[0][0] = info.root;
      s_fd[0][0] = 0.0f;
    }
    if (tid == 0) s_bound = __float_as_uint(heavy.bound[h]);
    __syncthreads();

    // breadth-first expansion of the frontier
    int cur = 0;
    while (fsize > 0 && fsize < S::kFront) {
      // the size of the next frontier counts into s_size[cur ^ 1], last read
      // before the previous level's closing barrier
      if (tid == 0) s_size[cur ^ 1] = 0;
      __syncthreads();
      const float bnd = __uint_as_float(s_bound);
      for (int base = 0; base < fsize; base += S::kThreads) {
        const int e = base + tid;
        if constexpr (FMT == ABX_NODES_Q16W) {
          bool ek[4] = {false, false, false, false};
          int32_t rk[4] = {0, 0, 0, 0};
          float dk[4] = {0.0f, 0.0f, 0.0f, 0.0f};
          if (e < fsize && s_fd[cur][e] <= fminf(L.kth(), bnd)) {
            Kids4 c;
            load_kids4<KIND>(t, s_fn[cur][e], c);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              dk[j] = c.ref[j] == kEmptyRef ? INFINITY
                                            : box_dist2(c.b[j][0], c.b[j][1], c.b[j][2], c.b[j][3],
                                                        c.b[j][4], c.b[j][5], q.x, q.y, q.z);
              if (c.ref[j] < 0 && c.ref[j] != kEmptyRef)
                knn_leaf<KIND, FMT, K>(t, q, ~c.ref[j], dk[j], fminf(L.kth(), bnd), L, reads);
            }
            const float thr = fminf(L.kth(), bnd);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              ek[j] = c.ref[j] >= 0 && dk[j] <= thr;
              rk[j] = c.ref[j];
            }
          }
          uint64_t bk[4];
          int cnt = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            bk[j] = __ballot(ek[j]);
            cnt += __popcll(bk[j]);
          }
          uint32_t o = 0;
          if (lane == 0 && cnt > 0) o = atomicAdd(&s_size[cur ^ 1], (uint32_t)cnt);
          int at0 = (int)__shfl(o, 0, kWave);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (ek[j]) {
              const int at = at0 + __popcll(bk[j] & lt);
              s_fn[cur ^ 1][at] = rk[j];
              s_fd[cur ^ 1][at] = dk[j];
            }
            at0 += __popcll(bk[j]);
          }
          continue;
        }
        bool el = false, er = false;
        int32_t lref = 0, rref = 0;
        float dl = 0.0f, dr = 0.0f;
        if (e < fsize && s_fd[cur][e] <= fminf(L.kth(), bnd)) {
          Kids c;
          load_kids<KIND, FMT>(t, s_fn[cur][e], c);
          dl = box_dist2(c.l[0], c.l[1], c.l[2], c.l[3], c.l[4], c.l[5], q.x, q.y, q.z);
          dr = box_dist2(c.r[0], c.r[1], c.r[2], c.r[3], c.r[4], c.r[5], q.x, q.y, q.z);
          if (c.lref < 0) knn_leaf<KIND, FMT, K>(t, q, ~c.lref, dl, fminf(L.kth(), bnd), L, reads);
          if (c.rref < 0) knn_leaf<KIND, FMT, K>(t, q, ~c.rref, dr, fminf(L.kth(), bnd), L, reads);
          const float thr = fminf(L.kth(), bnd);
          el = c.lref >= 0 && dl <= thr;
          er = c.rref >= 0 && dr <= thr;
          lref = c.lref;
          rref = c.rref;
        }
        // wave-level compaction, one LDS reservation per wave
        const uint64_t bl = __ballot(el), br = __ballot(er);
        const int cl = __popcll(bl), cnt = cl + __popcll(br);
        uint32_t o = 0;
        if (lane == 0 && cnt > 0) o = atomicAdd(&s_size[cur ^ 1], (uint32_t)cnt);
        o = __shfl(o, 0, kWave);
        if (el) {
          const int at = (int)o + __popcll(bl & lt);
          s_fn[cur ^ 1][at] = lref;
          s_fd[cur ^ 1][at] = dl;
        }
        if (er) {
          const int at = (int)o + cl + __popcll(br & lt);
          s_fn[cur ^ 1][at] = rref;
          s_fd[cur ^ 1][at] = dr;
        }
      }
      const float wm = wave_min(L.kth());
      if (lane == 0) lds_min(&s_bound, wm);
      __syncthreads();
      cur ^= 1;
      fsize = (int)s_size[cur];
    }

    // depth-first walks of the thread's share of the frontier
    int32_t ovf_n[kMaxDepth];
    float ovf_d[kMaxDepth];
    ABX_LDS int32_t *lds_n = (ABX_LDS int32_t *)(s_fn[cur ^ 1]) + tid;
    ABX_LDS float *lds_d = (ABX_LDS float *)(s_fd[cur ^ 1]) + tid;
    int sp = 0, nl = 0;
    const int mine = fsize > tid ? (fsize - 1 - tid) / S::kThreads + 1 : 0;
    for (int a = mine - 1; a >= 0; --a)
      stack_push2<S::kWindow, S::kThreads>(lds_n, lds_d, ovf_n, ovf_d, sp, nl,
                                           s_fn[cur][tid + S::kThreads * a],
                                           s_fd[cur][tid + S::kThreads * a]);
    __syncthreads();
    bool active = true;
    int32_t node = -1;
    float bound = __uint_as_float(s_bound);
    KnnPending pend;
    pend.init();
    for (int64_t it = 0; it < 4 * t.n + 64; ++it) {
      // share the workgroup's bound (each lane also prunes with its own list)
      if ((it & ((1 << kCoopShareLog2) - 1)) == 0) {
        const float wm = wave_min(fminf(bound, L.kth()));
        if (lane == 0) lds_min(&s_bound, wm);
        bound = fminf(wm, __uint_as_float(s_bound));
      }
      if (!__any(active)) break;
      if (active) {
        if (node < 0)
          node = knn_pop<S::kThreads, S::kWindow>(fminf(L.kth(), bound), lds_n, lds_d, ovf_n,
                                                  ovf_d, sp, nl);
        if (node < 0) {
          active = false;
        } else {
          node = knn_visit<KIND, FMT, K, S::kThreads, S::kWindow, true>(
              t, q, node, bound, L, lds_n, lds_d, ovf_n, ovf_d, sp, nl, reads, &pend);
        }
      }
    }

    pend.flush_all(L);

    // merge: each wave takes the k best of its 64 lists (k rounds of a
    // wave-wide minimum over the list fronts), then wave 0 the k best of the
    // W wave results
    for (int s2 = 0; s2 < K - k; ++s2) L.shift();
    for (int j = 0; j < k; ++j) {
      int64_t m = L.key[0];
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const int64_t m2 = __shfl_xor(m, o, kWave);
        m = m2 < m ? m2 : m;
      }
      // keys are unique (one entry per primitive), so exactly one lane
      // holds the minimum
      if (L.key[0] == m) L.shift();
      if (lane == 0) s_best[wv][j] = m;
    }
    __syncthreads();
    if (wv == 0) {
      // candidates c = lane, lane + 64, ... of the W*k wave results
      constexpr int kPer = (W * K + kWave - 1) / kWave;
      int64_t mine_c[kPer];
#pragma unroll
      for (int a = 0; a < kPer; ++a) {
        const int c = lane + kWave * a;
        mine_c[a] = c < W * k ? s_best[c / k][c % k] : kKeyEmpty;
      }
      int64_t out = 0;
      for (int j = 0; j < k; ++j) {
        int64_t lo = mine_c[0];
        int at = 0;
#pragma unroll
        for (int a = 1; a < kPer; ++a)
          if (mine_c[a] < lo) {
            lo = mine_c[a];
            at = a;
          }
        int64_t m = lo;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
          const int64_t m2 = __shfl_xor(m, o, kWave);
          m = m2 < m ? m2 : m;
        }
        if (lo == m) {
#pragma unroll
          for (int a = 0; a < kPer; ++a)
            if (a == at) mine_c[a] = kKeyEmpty;
        }
        if (lane == j) out = m;
      }
      if (lane < k) {
        indices[info.out + lane] = key_index(out) - info.base;
        dist[info.out + lane] = sqrtf(key_dist(out));
      }
    }
  }
  (void)reads;
}

}  // namespace abx
