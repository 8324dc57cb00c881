// C-ABI of libabx: argument validation, buffer layout, the launch sequence of
// each entry point and the diagnostics.  No device memory is allocated here.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "abx_internal.h"

namespace abx {

// build.hip
abx_status launch_scene(int kind, const float *prims, int64_t n, float *partial, int blocks,
                        TreeHeader *hdr, hipStream_t s);
int scene_blocks(int64_t n);
abx_status launch_morton(int kind, const float *prims, int64_t n, const float *scene, int bits,
                         void *codes, bool wide, hipStream_t s);
abx_status launch_karras(bool wide, const void *keys, int64_t n, uint64_t *pw_leaf, uint64_t *pw_int,
                         int32_t *other_end, uint32_t *flags, const TreeHeader *hdr, hipStream_t s);
abx_status launch_refit(int kind, bool q16, const float *prims, const int32_t *perm, int64_t n,
                        const uint64_t *pw_leaf, const uint64_t *pw_int, const int32_t *pre,
                        void *out, NodeF32 *stage, uint32_t *flags, TreeHeader *hdr, void *box_rec,
                        void *lists_mem, hipStream_t s);
size_t refit_lists_bytes(int64_t n);
abx_status launch_agglo(bool wide, int kind, bool q16, const void *keys, const float *prims,
                        const int32_t *perm, int64_t n, NodeF32 *nodes, int32_t *range_lo,
                        int32_t *range_hi, uint32_t *flags, TreeHeader *hdr, void *q16_leaves,
                        int32_t *frontier, uint32_t *frontier_count, hipStream_t s);
abx_status launch_quantise(int kind, const NodeF32 *src, int64_t ni, TreeHeader *hdr,
                           const int32_t *pre, NodeQ16 *dst, hipStream_t s);
abx_status launch_preorder(const uint64_t *pw_int, const int32_t *other_end, int64_t ni,
                           uint64_t *work, int32_t *pre, int32_t *depth, hipStream_t s);
abx_status launch_wide(int kind, const NodeF32 *src, int64_t ni, const int32_t *pre,
                       const int32_t *depth, int32_t *flag, int32_t *rank, int64_t *d_total,
                       void *scan_scratch, size_t scan_bytes, TreeHeader *hdr, NodeW *dst,
                       hipStream_t s);
// traverse.hip
abx_status launch_query_codes(const abx_bvh *b, const float *q, int64_t m, int width,
                              uint32_t *codes, hipStream_t s);
abx_status launch_spatial(const abx_bvh *b, int pred, const float *data, int64_t m,
                          const float *radii, float radius, const int32_t *order, int mode,
                          int32_t *counts, const int32_t *offsets, int32_t *indices, hipStream_t s,
                          const OnePass *op = nullptr);
abx_status launch_spatial_compact(const OnePass &op, int64_t m, const int32_t *order,
                                  const int32_t *counts, const int32_t *offsets, int32_t *indices,
                                  int32_t *info, int64_t max_count, hipStream_t s);
abx_status launch_nearest(const abx_bvh *b, const float *pts, int64_t m, const int32_t *order,
                          int k, int32_t *idx, float *dist, int32_t *stats, int32_t *heavy_q,
                          float *heavy_bound, uint32_t *counters, int32_t *heavy_state,
                          int64_t state_cap, int64_t budget, hipStream_t s);
int max_tree_depth();

// node visits after which a nearest query leaves the one-lane pass for the
// cooperative pass (abx_set_nearest_budget)
std::atomic<int64_t> g_nearest_budget{22528};
extern std::atomic<uint32_t> g_sort_spin_limit;  // sort.hip
extern std::atomic<uint32_t> g_fit_table_probes;  // build.hip
int64_t nearest_budget() { return g_nearest_budget.load(std::memory_order_relaxed); }

namespace {

thread_local int g_last_hip = 0;

struct Pending {
  std::string name;
  hipEvent_t a, b;
};
std::atomic<bool> g_timing{false};
std::mutex g_timing_mu;  // launches may come from the server's scheduler thread
std::vector<Pending> g_pending;
std::map<std::string, std::pair<double, int64_t>> g_acc;

constexpr int64_t kMaxCount = INT32_MAX;
constexpr int64_t kMaxNearestK = 128;  // register lists up to 32, LDS heaps up to 128

__global__ void k_row_offsets(int32_t *off, int64_t m, int32_t k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= m) off[i] = (int32_t)(i * k);
}

abx_status row_offsets(int32_t *off, int64_t m, int32_t k, hipStream_t s) {
  return launch("row_offsets", s, [&] {
    k_row_offsets<<<grid_for(m + 1, 256), 256, 0, s>>>(off, m, k);
  });
}

// ---------------------------------------------------------------- build
struct BuildLayout {
  int64_t n, ni;
  bool wide, q16;
  bool boxrec;  // Q16 box tree: exact box records in the leaf region
  int bits;
  size_t node_bytes, leaf_bytes;
  size_t nodes_off, leaves_off, tree_total;
  // scratch
  bool preorder;  // Q16 Karras tree renumbered depth-first
  bool wnodes;    // 4-wide Q16 nodes (collapsed from the binary tree)
  size_t partial, codes, sorted, perm, parent_leaf, parent_int, other_end, flags, frontier,
      staging, pre, wbuf, sort, scratch_total;
};

// 4-wide trees: a walk pushes up to three children per level of half as many
// levels, so the stacks (kMaxDepth entries, 8 of them for the cooperative
// pass's share of its frontier) bound the binary height at 78
bool height_fits(int64_t height, bool wide, int max_depth) {
  const int64_t need = wide ? 3 * ((height + 1) / 2) : height;
  return need + 8 < max_depth;
}

int resolve_bits(const abx_build_options *o) { return (o == nullptr || o->morton_bits == 0) ? 21 : o->morton_bits; }

abx_status check_build_args(const abx_primitives *p, const abx_build_options *o) {
  if (!p) return ABX_ERR_INVALID_ARG;
  if (p->kind != ABX_PRIM_POINTS && p->kind != ABX_PRIM_BOXES) return ABX_ERR_INVALID_ARG;
  if (p->n < 0) return ABX_ERR_INVALID_ARG;
  if (p->n >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (p->n > 0 && !p->data) return ABX_ERR_INVALID_ARG;
  if (o && o->node_format != ABX_NODES_FP32 && o->node_format != ABX_NODES_Q16 &&
      o->node_format != ABX_NODES_Q16W)
    return ABX_ERR_INVALID_ARG;
  const int bits = resolve_bits(o);
  if (bits != 10 && bits != 21) return ABX_ERR_INVALID_ARG;
  if (o && o->hierarchy != ABX_HIERARCHY_KARRAS && o->hierarchy != ABX_HIERARCHY_AGGLOMERATIVE)
    return ABX_ERR_INVALID_ARG;
  if (o && o->node_order != ABX_ORDER_AUTO && o->node_order != ABX_ORDER_BUILD &&
      o->node_order != ABX_ORDER_DEPTH_FIRST)
    return ABX_ERR_INVALID_ARG;
  if (o && o->node_order == ABX_ORDER_DEPTH_FIRST && o->node_format == ABX_NODES_FP32)
    return ABX_ERR_UNSUPPORTED;
  if (o && o->node_order == ABX_ORDER_DEPTH_FIRST && o->hierarchy == ABX_HIERARCHY_AGGLOMERATIVE)
    return ABX_ERR_UNSUPPORTED;
  // 4-wide nodes: collapsed from the Karras tree, always in depth-first order
  if (o && o->node_format == ABX_NODES_Q16W &&
      (o->hierarchy == ABX_HIERARCHY_AGGLOMERATIVE || o->node_order == ABX_ORDER_BUILD))
    return ABX_ERR_UNSUPPORTED;
  return ABX_OK;
}

// automatic depth-first order from this many primitives: 2^22 points make
// 128 MB of Q16 nodes, half the last-level cache (see abx_node_order)
constexpr int64_t kDepthFirstMinN = int64_t(1) << 22;

BuildLayout build_layout(const abx_primitives *p, const abx_build_options *o) {
  BuildLayout L{};
  L.n = p->n;
  L.ni = p->n > 1 ? p->n - 1 : 0;
  L.bits = resolve_bits(o);
  L.wide = L.bits > 10;
  L.wnodes = o && o->node_format == ABX_NODES_Q16W;
  L.q16 = o && (o->node_format == ABX_NODES_Q16 || L.wnodes);  // quantised (binary or 4-wide)
  L.node_bytes = L.wnodes ? sizeof(NodeW) : (L.q16 ? sizeof(NodeQ16) : sizeof(NodeF32));
  L.boxrec = L.q16 && p->kind == ABX_PRIM_BOXES;
  {
    const bool karras = !(o && o->hierarchy == ABX_HIERARCHY_AGGLOMERATIVE);
    const int order = o ? o->node_order : ABX_ORDER_AUTO;
    L.preorder = L.q16 && !L.wnodes && karras &&
                 (order == ABX_ORDER_DEPTH_FIRST || (order == ABX_ORDER_AUTO && L.n >= kDepthFirstMinN));
  }
  L.leaf_bytes = L.boxrec ? 32 : 4;
  const int64_t node_slots = L.wnodes ? wide_node_cap(L.ni) : L.ni;
  size_t off = sizeof(TreeHeader);
  L.nodes_off = off;
  off = align_up(off + (size_t)node_slots * L.node_bytes, 256);
  L.leaves_off = off;
  off = align_up(off + (size_t)L.n * L.leaf_bytes, 256);
  L.tree_total = off;

  const size_t ksz = L.wide ? 8 : 4;
  const size_t n = (size_t)L.n;
  off = 0;
  L.partial = off;
  off = align_up(off + 1024 * 8 * sizeof(float), 256);
  L.codes = off;
  off = align_up(off + n * ksz, 256);
  L.sorted = off;
  off = align_up(off + n * ksz, 256);
  L.perm = off;
  off = align_up(off + (L.boxrec ? n * 4 : 0), 256);
  L.parent_leaf = off;  // parent words (the agglomerative build: range ends)
  off = align_up(off + n * 8, 256);
  L.parent_int = off;
  off = align_up(off + n * 8, 256);
  L.other_end = off;
  off = align_up(off + n * 4, 256);
  L.flags = off;
  off = align_up(off + n * 4, 256);
  L.frontier = off;
  off = align_up(off + refit_lists_bytes(L.n), 256);
  L.staging = off;
  off = align_up(off + (L.q16 ? (size_t)L.ni * sizeof(NodeF32) : 0), 256);
  L.pre = off;  // depth-first order: two buffers of 64-bit pointer-jumping words, the index
  off = align_up(off + (L.preorder || L.wnodes ? 2 * (size_t)L.ni * 8 + (size_t)L.ni * 4 : 0), 256);
  L.wbuf = off;  // 4-wide nodes: depths, flags, ranks [ni + 1], the scan's total and scratch
  off = align_up(off + (L.wnodes ? align_up(3 * (size_t)L.ni * 4 + 4, 256) + 256 + scan_scratch_bytes(L.ni)
                                 : 0), 256);
  L.sort = off;
  off = align_up(off + radix_sort_scratch_bytes(L.n, 3 * L.bits), 256);
  L.scratch_total = off;
  return L;
}

// ---------------------------------------------------------------- queries
struct QueryLayout {
  size_t codes, sorted, order, counts, total, scan, sort, heavy_q, heavy_bound, heavy_state, bytes;
  int64_t state_cap;
};

// `nearest`: also room for the walks heavy nearest queries hand over
QueryLayout query_layout(int64_t m, bool nearest = false) {
  QueryLayout L{};
  const size_t mm = (size_t)m;
  size_t off = 0;
  L.codes = off;
  off = align_up(off + mm * 4, 256);
  L.sorted = off;
  off = align_up(off + mm * 4, 256);
  L.order = off;
  off = align_up(off + mm * 4, 256);
  L.counts = off;
  off = align_up(off + mm * 4, 256);
  L.total = off;
  off = align_up(off + 8, 256);
  L.scan = off;
  off = align_up(off + scan_scratch_bytes(m), 256);
  L.sort = off;
  off = align_up(off + radix_sort_scratch_bytes(m, 30), 256);
  L.heavy_q = off;
  off = align_up(off + mm * 4, 256);
  L.heavy_bound = off;
  off = align_up(off + mm * 4, 256);
  L.heavy_state = off;
  L.state_cap = nearest ? heavy_state_cap(m) : 0;
  off = align_up(off + (size_t)L.state_cap * kHeavyStateWords * 4, 256);
  L.bytes = off;
  return L;
}

abx_status check_bvh(const abx_bvh *b) { return b ? ABX_OK : ABX_ERR_INVALID_ARG; }

abx_status check_preds(const abx_predicates *p) {
  if (!p) return ABX_ERR_INVALID_ARG;
  if (p->kind != ABX_PRED_WITHIN && p->kind != ABX_PRED_INTERSECTS_BOX) return ABX_ERR_INVALID_ARG;
  if (p->m < 0) return ABX_ERR_INVALID_ARG;
  if (p->m >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (p->m > 0 && !p->data) return ABX_ERR_INVALID_ARG;
  return ABX_OK;
}

// queries in Morton order: order[] = permutation sorted position -> query
abx_status order_queries(const abx_bvh *b, const float *data, int64_t m, int width, char *scratch,
                         const QueryLayout &L, const int32_t **order, hipStream_t s) {
  uint32_t *codes = reinterpret_cast<uint32_t *>(scratch + L.codes);
  int32_t *ord = reinterpret_cast<int32_t *>(scratch + L.order);
  ABX_TRY(launch_query_codes(b, data, m, width, codes, s));
  ABX_TRY(radix_sort(codes, nullptr, m, 30, scratch + L.sorted, ord, scratch + L.sort,
                     radix_sort_scratch_bytes(m, 30), s));
  ABX_TRY(order_guard(radix_sort_err_word(scratch + L.sort, m, 30), ord, m, s));
  *order = ord;
  return ABX_OK;
}

}  // namespace

// ---------------------------------------------------------------- internal enqueue sequences
// Non-blocking pieces of the query entry points, shared with the server.
size_t query_scratch_bytes(int64_t m) { return query_layout(m).bytes; }
size_t nearest_scratch_bytes(int64_t m) { return query_layout(m, true).bytes; }

// Spatial count phase: optional Morton ordering, counting traversal, scan of
// the counts into offsets[0..m]; *d_total receives the device address of the
// int64 total (inside scratch).
abx_status spatial_count_enqueue(const abx_bvh *bvh, const abx_predicates *p, char *sc,
                                 int32_t *offsets, int64_t **d_total, hipStream_t s) {
  const QueryLayout L = query_layout(p->m);
  const int64_t m = p->m;
  int64_t *tot = reinterpret_cast<int64_t *>(sc + L.total);
  *d_total = tot;
  if (bvh->n == 0 || m == 0) {
    ABX_TRY(fill_u32(offsets, 0, (size_t)m + 1, s));
    return fill_u32(tot, 0, 2, s);
  }
  const int width = p->kind == ABX_PRED_WITHIN ? 3 : 6;
  const int32_t *order = nullptr;
  if (p->sort_queries) ABX_TRY(order_queries(bvh, p->data, m, width, sc, L, &order, s));
  int32_t *counts = reinterpret_cast<int32_t *>(sc + L.counts);
  ABX_TRY(launch_spatial(bvh, p->kind, p->data, m, p->radii, p->radius, order, 0 /*count*/, counts,
                         nullptr, nullptr, s));
  return exclusive_scan(counts, m, offsets, tot, sc + L.scan, scan_scratch_bytes(m), s);
}

// Spatial fill phase, after spatial_count_enqueue on the same scratch.
abx_status spatial_fill_enqueue(const abx_bvh *bvh, const abx_predicates *p, char *sc,
                                const int32_t *offsets, int32_t *indices, hipStream_t s) {
  if (bvh->n == 0 || p->m == 0) return ABX_OK;
  const QueryLayout L = query_layout(p->m);
  const int32_t *order = p->sort_queries ? reinterpret_cast<const int32_t *>(sc + L.order) : nullptr;
  return launch_spatial(bvh, p->kind, p->data, p->m, p->radii, p->radius, order, 1 /*fill*/, nullptr,
                        offsets, indices, s);
}

// Nearest queries: rows of min(k, n) entries; offsets optional.
abx_status nearest_enqueue(const abx_bvh *bvh, const float *pts, int64_t m, int32_t k, int sort,
                           char *sc, int32_t *offsets, int32_t *indices, float *dist, hipStream_t s) {
  const QueryLayout L = query_layout(m, true);
  const int64_t kk = k < bvh->n ? k : bvh->n;
  if (offsets) ABX_TRY(row_offsets(offsets, m, (int32_t)kk, s));
  if (m == 0 || kk == 0) return ABX_OK;
  const int32_t *order = nullptr;
  if (sort) ABX_TRY(order_queries(bvh, pts, m, 3, sc, L, &order, s));
  return launch_nearest(bvh, pts, m, order, (int)kk, indices, dist, nullptr,
                        reinterpret_cast<int32_t *>(sc + L.heavy_q),
                        reinterpret_cast<float *>(sc + L.heavy_bound),
                        reinterpret_cast<uint32_t *>(sc + L.total),
                        reinterpret_cast<int32_t *>(sc + L.heavy_state), L.state_cap, nearest_budget(), s);
}

abx_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return ABX_ERR_HIP;
}

// whether work enqueued on `s` is being captured into a graph (the stream's
// own state: captures on other streams or threads do not matter)
bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

thread_local int g_no_events = 0;

namespace {
// per fault kind: -1 off, else the number of events still to let pass
std::atomic<int64_t> g_fault[2] = {{-1}, {-1}};
}  // namespace

bool fault_hit(int kind) {
  if (kind < 0 || kind > 1) return false;
  std::atomic<int64_t> &c = g_fault[kind];
  int64_t v = c.load(std::memory_order_relaxed);
  while (v >= 0) {
    if (c.compare_exchange_weak(v, v - 1, std::memory_order_relaxed)) return v == 0;
  }
  return false;
}

// no events inside a graph capture: timing is for eager launches only
bool timing_on(hipStream_t s) {
  return g_timing.load(std::memory_order_relaxed) && g_no_events == 0 && !stream_capturing(s);
}

void timing_record(const char *name, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_pending.push_back(Pending{name, a, b});
}

}  // namespace abx

using namespace abx;

extern "C" {

const char *abx_version(void) { return "abx 0.1 (gfx950)"; }

const char *abx_status_string(abx_status s) {
  switch (s) {
    case ABX_OK: return "ok";
    case ABX_ERR_INVALID_ARG: return "invalid argument";
    case ABX_ERR_INVALID_INPUT: return "invalid input (NaN/Inf coordinate or inverted box)";
    case ABX_ERR_CAPACITY: return "result buffer too small";
    case ABX_ERR_OVERFLOW: return "size or result count reaches 2^31";
    case ABX_ERR_HIP: return "HIP runtime error";
    case ABX_ERR_UNSUPPORTED: return "unsupported request";
    case ABX_PENDING: return "pending";
    case ABX_ERR_DEVICE: return "a bounded device wait gave up (results not valid)";
  }
  return "unknown status";
}

int abx_last_hip_error(void) { return g_last_hip; }

abx_status abx_inject_fault(int32_t kind, int64_t skip) {
  if (kind != ABX_FAULT_LAUNCH && kind != ABX_FAULT_HOST_ALLOC) return ABX_ERR_INVALID_ARG;
  g_fault[kind].store(skip < 0 ? -1 : skip, std::memory_order_relaxed);
  return ABX_OK;
}

int64_t abx_set_nearest_budget(int64_t visits) {
  return g_nearest_budget.exchange(visits > 0 ? visits : INT64_MAX);
}

void abx_timing_enable(int on) { g_timing.store(on != 0, std::memory_order_relaxed); }

// caller holds g_timing_mu
static void timing_flush_locked() {
  for (auto &p : g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto &acc = g_acc[p.name];
      acc.first += ms;
      acc.second += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}

void abx_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  timing_flush_locked();
  g_acc.clear();
}

abx_status abx_timing_get(const char *kernel, double *ms, int64_t *launches) {
  if (!kernel || !ms || !launches) return ABX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  timing_flush_locked();
  auto it = g_acc.find(kernel);
  *ms = it == g_acc.end() ? 0.0 : it->second.first;
  *launches = it == g_acc.end() ? 0 : it->second.second;
  return ABX_OK;
}

// ---------------------------------------------------------------- build
abx_status abx_bvh_build_sizes(const abx_primitives *prims, const abx_build_options *opts,
                               size_t *tree_bytes, size_t *scratch_bytes) {
  ABX_TRY(check_build_args(prims, opts));
  if (!tree_bytes || !scratch_bytes) return ABX_ERR_INVALID_ARG;
  const BuildLayout L = build_layout(prims, opts);
  *tree_bytes = L.tree_total;
  *scratch_bytes = L.scratch_total;
  return ABX_OK;
}

abx_status abx_bvh_build(const abx_primitives *prims, const abx_build_options *opts,
                         void *tree_mem, size_t tree_bytes, void *scratch, size_t scratch_bytes,
                         abx_stream_t stream, abx_bvh **out) {
  ABX_TRY(check_build_args(prims, opts));
  if (!out || !tree_mem || !scratch) return ABX_ERR_INVALID_ARG;
  *out = nullptr;
  const BuildLayout L = build_layout(prims, opts);
  if (tree_bytes < L.tree_total || scratch_bytes < L.scratch_total) return ABX_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(tree_mem) | reinterpret_cast<uintptr_t>(scratch)) & 255)
    return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *tree = static_cast<char *>(tree_mem);
  char *sc = static_cast<char *>(scratch);
  TreeHeader *hdr = reinterpret_cast<TreeHeader *>(tree);
  const int64_t n = L.n;
  const int kind = prims->kind;
  const bool agglo = opts && opts->hierarchy == ABX_HIERARCHY_AGGLOMERATIVE;

  const int blocks = scene_blocks(n);
  ABX_TRY(launch_scene(kind, prims->data, n, reinterpret_cast<float *>(sc + L.partial), blocks, hdr, s));
  int32_t *perm = L.boxrec ? reinterpret_cast<int32_t *>(sc + L.perm)
                           : reinterpret_cast<int32_t *>(tree + L.leaves_off);
  NodeF32 *fnodes = L.q16 ? reinterpret_cast<NodeF32 *>(sc + L.staging)
                          : reinterpret_cast<NodeF32 *>(tree + L.nodes_off);
  uint64_t *pw_leaf = reinterpret_cast<uint64_t *>(sc + L.parent_leaf);
  uint64_t *pw_int = reinterpret_cast<uint64_t *>(sc + L.parent_int);
  int32_t *other_end = reinterpret_cast<int32_t *>(sc + L.other_end);
  uint32_t *flags = reinterpret_cast<uint32_t *>(sc + L.flags);
  if (n > 0) {
    ABX_TRY(launch_morton(kind, prims->data, n, hdr->scene, L.bits, sc + L.codes, L.wide, s));
    // a look-back that gives up marks the header; the refit then skips
    ABX_TRY(radix_sort(sc + L.codes, nullptr, n, 3 * L.bits, sc + L.sorted, perm, sc + L.sort,
                       radix_sort_scratch_bytes(n, 3 * L.bits), s,
                       reinterpret_cast<uint32_t *>(&hdr->bad), kBadSort));
    void *box_rec = L.boxrec ? tree + L.leaves_off : nullptr;
    if (agglo) {
      uint32_t *fcount = reinterpret_cast<uint32_t *>(sc + L.frontier);
      int32_t *frontier = reinterpret_cast<int32_t *>(sc + L.frontier + 256);
      // range ends of the agglomerative climb reuse the parent-word arrays
      ABX_TRY(launch_agglo(L.wide, kind, L.q16, sc + L.sorted, prims->data, perm, n, fnodes,
                           reinterpret_cast<int32_t *>(pw_leaf), reinterpret_cast<int32_t *>(pw_int),
                           flags, hdr, box_rec, frontier, fcount, s));
      if (L.q16)
        ABX_TRY(launch_quantise(kind, fnodes, L.ni, hdr, nullptr,
                                reinterpret_cast<NodeQ16 *>(tree + L.nodes_off), s));
    } else {
      ABX_TRY(launch_karras(L.wide, sc + L.sorted, n, pw_leaf, pw_int, other_end, flags, hdr, s));
      // depth-first order first: the refit writes each node at its final slot
      int32_t *pre = nullptr, *depth = nullptr;
      if (L.preorder || L.wnodes) {
        uint64_t *work = reinterpret_cast<uint64_t *>(sc + L.pre);
        pre = reinterpret_cast<int32_t *>(work + 2 * L.ni);
        depth = L.wnodes ? reinterpret_cast<int32_t *>(sc + L.wbuf) : nullptr;
        ABX_TRY(launch_preorder(pw_int, other_end, L.ni, work, pre, depth, s));
      }
      if (L.wnodes) {
        // 4-wide nodes are collapsed from the FP32 binary tree in build order
        ABX_TRY(launch_refit(kind, false, prims->data, perm, n, pw_leaf, pw_int, nullptr, fnodes,
                             fnodes, flags, hdr, box_rec, sc + L.frontier, s));
        int32_t *flag = depth + L.ni, *rank = flag + L.ni;
        char *tail = sc + L.wbuf + align_up(3 * (size_t)L.ni * 4 + 4, 256);
        ABX_TRY(launch_wide(kind, fnodes, L.ni, pre, depth, flag, rank,
                            reinterpret_cast<int64_t *>(tail), tail + 256, scan_scratch_bytes(L.ni),
                            hdr, reinterpret_cast<NodeW *>(tree + L.nodes_off), s));
      } else {
        // Q16 nodes are written directly (FP32 records of chunk-crossing
        // nodes wait in the staging area); FP32 nodes stage in place
        ABX_TRY(launch_refit(kind, L.q16, prims->data, perm, n, pw_leaf, pw_int, pre,
                             tree + L.nodes_off, fnodes, flags, hdr, box_rec, sc + L.frontier, s));
      }
    }
  }
  TreeHeader h;
  ABX_HIP(hipMemcpyAsync(&h, hdr, sizeof(h), hipMemcpyDeviceToHost, s));
  ABX_HIP(hipStreamSynchronize(s));
  if (h.bad & kBadSort) return ABX_ERR_DEVICE;
  if (h.bad & 1) return ABX_ERR_INVALID_INPUT;
  if (h.bad & 4) return ABX_ERR_UNSUPPORTED;  // refit bound exceeded (malformed hierarchy)
  if (h.bad & 8) return ABX_ERR_UNSUPPORTED;  // depth-first order out of range (too deep)
  if ((h.bad & 2) && L.q16) return ABX_ERR_UNSUPPORTED;
  // traversal stacks hold at most height + 8 entries (8 = the cooperative
  // pass's share of the initial frontier); 4-wide walks more per level
  if (!height_fits(h.height, L.wnodes, max_tree_depth())) return ABX_ERR_UNSUPPORTED;

  abx_bvh *b = new (std::nothrow) abx_bvh;
  if (!b) return ABX_ERR_INVALID_ARG;
  b->n = n;
  b->kind = kind;
  b->format = L.wnodes ? ABX_NODES_Q16W : (L.q16 ? ABX_NODES_Q16 : ABX_NODES_FP32);
  b->nint = L.wnodes ? (n > 1 ? h.node_count : 0) : L.ni;
  b->morton_bits = L.bits;
  b->height = h.height;
  b->hierarchy = agglo ? ABX_HIERARCHY_AGGLOMERATIVE : ABX_HIERARCHY_KARRAS;
  b->node_order = L.preorder || L.wnodes ? ABX_ORDER_DEPTH_FIRST : ABX_ORDER_BUILD;
  b->root = h.root;
  std::memcpy(b->scene, h.scene, sizeof(b->scene));
  std::memcpy(b->q_origin, h.q_origin, sizeof(b->q_origin));
  std::memcpy(b->q_scale, h.q_scale, sizeof(b->q_scale));
  b->tree = tree;
  b->tree_bytes = tree_bytes;
  b->nodes_off = L.nodes_off;
  b->leaves_off = L.leaves_off;
  b->node_bytes = L.node_bytes;
  b->leaf_bytes = L.leaf_bytes;
  *out = b;
  return ABX_OK;
}

abx_status abx_bvh_destroy(abx_bvh *bvh) {
  delete bvh;
  return ABX_OK;
}

abx_status abx_bvh_get_layout(const abx_bvh *b, abx_bvh_layout *o) {
  if (!b || !o) return ABX_ERR_INVALID_ARG;
  o->n = b->n;
  o->kind = b->kind;
  o->node_format = b->format;
  o->morton_bits = b->morton_bits;
  o->height = b->height;
  o->hierarchy = b->hierarchy;
  o->node_order = b->node_order;
  o->root = b->root;
  std::memcpy(o->scene, b->scene, sizeof(o->scene));
  o->nodes_offset = b->nodes_off;
  o->node_bytes = b->node_bytes;
  o->leaves_offset = b->leaves_off;
  o->leaf_bytes = b->leaf_bytes;
  std::memcpy(o->q16_origin, b->q_origin, sizeof(o->q16_origin));
  std::memcpy(o->q16_scale, b->q_scale, sizeof(o->q16_scale));
  o->node_count = b->nint;
  return ABX_OK;
}

// ---------------------------------------------------------------- spatial
abx_status abx_query_spatial_sizes(const abx_bvh *bvh, const abx_predicates *preds,
                                   size_t *scratch_bytes) {
  ABX_TRY(check_bvh(bvh));
  ABX_TRY(check_preds(preds));
  if (!scratch_bytes) return ABX_ERR_INVALID_ARG;
  *scratch_bytes = query_layout(preds->m).bytes;
  return ABX_OK;
}

static abx_status spatial_prologue(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                                   size_t scratch_bytes, QueryLayout *L) {
  ABX_TRY(check_bvh(bvh));
  ABX_TRY(check_preds(preds));
  *L = query_layout(preds->m);
  if (!scratch || scratch_bytes < L->bytes) return ABX_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return ABX_ERR_INVALID_ARG;
  return ABX_OK;
}

abx_status abx_query_spatial(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                             size_t scratch_bytes, int32_t *offsets, int32_t *indices,
                             int64_t capacity, int64_t *total, abx_stream_t stream) {
  QueryLayout L;
  ABX_TRY(spatial_prologue(bvh, preds, scratch, scratch_bytes, &L));
  if (!offsets || !total || capacity < 0 || (capacity > 0 && !indices)) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  const int64_t m = preds->m;
  const int width = preds->kind == ABX_PRED_WITHIN ? 3 : 6;
  int32_t *counts = reinterpret_cast<int32_t *>(sc + L.counts);
  int64_t *d_total = reinterpret_cast<int64_t *>(sc + L.total);
  *total = 0;
  if (bvh->n == 0 || m == 0) {
    ABX_TRY(fill_u32(offsets, 0, (size_t)m + 1, s));
    return ABX_OK;
  }
  const int32_t *order = nullptr;
  if (preds->sort_queries) ABX_TRY(order_queries(bvh, preds->data, m, width, sc, L, &order, s));
  ABX_TRY(launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                         0 /*count*/, counts, nullptr, nullptr, s));
  ABX_TRY(exclusive_scan(counts, m, offsets, d_total, sc + L.scan, scan_scratch_bytes(m), s));
  int64_t t = 0;
  ABX_HIP(hipMemcpyAsync(&t, d_total, sizeof(t), hipMemcpyDeviceToHost, s));
  ABX_HIP(hipStreamSynchronize(s));
  *total = t;
  if (t >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (t > capacity) return ABX_ERR_CAPACITY;
  if (t == 0) return ABX_OK;
  return launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                        1 /*fill*/, nullptr, offsets, indices, s);
}

abx_status abx_query_spatial_fill(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                                  size_t scratch_bytes, const int32_t *offsets, int32_t *indices,
                                  int64_t capacity, abx_stream_t stream) {
  QueryLayout L;
  ABX_TRY(spatial_prologue(bvh, preds, scratch, scratch_bytes, &L));
  if (!offsets || capacity < 0 || (capacity > 0 && !indices)) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  const int64_t m = preds->m;
  if (bvh->n == 0 || m == 0) return ABX_OK;
  int64_t t = 0;
  ABX_HIP(hipMemcpyAsync(&t, sc + L.total, sizeof(t), hipMemcpyDeviceToHost, s));
  ABX_HIP(hipStreamSynchronize(s));
  if (t > capacity) return ABX_ERR_CAPACITY;
  if (t == 0) return ABX_OK;
  const int32_t *order = preds->sort_queries ? reinterpret_cast<const int32_t *>(sc + L.order) : nullptr;
  return launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                        1 /*fill*/, nullptr, offsets, indices, s);
}

// ---------------------------------------------------------------- spatial, one pass
constexpr int32_t kMaxBufferSize = 1 << 16;

// scratch beyond the query layout: 256 B of flags, then the stored rows
static size_t one_pass_bytes(int64_t m, int32_t bufsize) {
  return 256 + align_up((size_t)m * (size_t)bufsize * 4, 256);
}

abx_status abx_query_spatial_1p_sizes(const abx_bvh *bvh, const abx_predicates *preds,
                                      int32_t buffer_size, size_t *scratch_bytes) {
  ABX_TRY(check_bvh(bvh));
  ABX_TRY(check_preds(preds));
  if (!scratch_bytes || buffer_size < 1 || buffer_size > kMaxBufferSize) return ABX_ERR_INVALID_ARG;
  *scratch_bytes = query_layout(preds->m).bytes + one_pass_bytes(preds->m, buffer_size);
  return ABX_OK;
}

abx_status abx_query_spatial_1p(const abx_bvh *bvh, const abx_predicates *preds, int32_t buffer_size,
                                void *scratch, size_t scratch_bytes, int32_t *offsets,
                                int32_t *indices, int64_t capacity, int32_t *info,
                                abx_stream_t stream) {
  QueryLayout L;
  ABX_TRY(spatial_prologue(bvh, preds, scratch, scratch_bytes, &L));
  if (buffer_size < 1 || buffer_size > kMaxBufferSize) return ABX_ERR_INVALID_ARG;
  const int64_t m = preds->m;
  if (scratch_bytes < L.bytes + one_pass_bytes(m, buffer_size)) return ABX_ERR_INVALID_ARG;
  if (!offsets || !info || capacity < 0 || (capacity > 0 && !indices)) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  int64_t *d_total = reinterpret_cast<int64_t *>(sc + L.total);
  uint32_t *flag = reinterpret_cast<uint32_t *>(sc + L.bytes);
  int32_t *buf = reinterpret_cast<int32_t *>(sc + L.bytes + 256);
  const OnePass op{buf, buffer_size, flag, d_total, std::min<int64_t>(capacity, kMaxCount - 1)};
  ABX_TRY(fill_u32(flag, 0, 4, s));
  if (bvh->n == 0 || m == 0) {
    ABX_TRY(fill_u32(offsets, 0, (size_t)m + 1, s));
    ABX_TRY(fill_u32(d_total, 0, 2, s));
    return fill_u32(info, 0, 2, s);  // ABX_OK, no traversal
  }
  const int width = preds->kind == ABX_PRED_WITHIN ? 3 : 6;
  const int32_t *order = nullptr;
  if (preds->sort_queries) ABX_TRY(order_queries(bvh, preds->data, m, width, sc, L, &order, s));
  int32_t *counts = reinterpret_cast<int32_t *>(sc + L.counts);
  // one traversal counts every hit and stores the first buffer_size of each row
  ABX_TRY(launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                         3 /*store*/, counts, nullptr, nullptr, s, &op));
  ABX_TRY(exclusive_scan(counts, m, offsets, d_total, sc + L.scan, scan_scratch_bytes(m), s));
  // after an overflow: the fill traversal of the two-pass scheme (the
  // kernel returns at once otherwise); without one: compaction
  ABX_TRY(launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                         1 /*fill*/, nullptr, offsets, indices, s, &op));
  return launch_spatial_compact(op, m, order, counts, offsets, indices, info, kMaxCount, s);
}

abx_status abx_query_spatial_stats(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                                   size_t scratch_bytes, int32_t *stats, abx_stream_t stream) {
  QueryLayout L;
  ABX_TRY(spatial_prologue(bvh, preds, scratch, scratch_bytes, &L));
  if (!stats && preds->m > 0) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  const int64_t m = preds->m;
  if (m == 0) return ABX_OK;
  if (bvh->n == 0) return fill_u32(stats, 0, 2 * (size_t)m, s);
  const int width = preds->kind == ABX_PRED_WITHIN ? 3 : 6;
  const int32_t *order = nullptr;
  if (preds->sort_queries) ABX_TRY(order_queries(bvh, preds->data, m, width, sc, L, &order, s));
  return launch_spatial(bvh, preds->kind, preds->data, m, preds->radii, preds->radius, order,
                        2 /*stats*/, stats, nullptr, nullptr, s);
}

// ---------------------------------------------------------------- nearest
abx_status abx_query_nearest_sizes(const abx_bvh *bvh, int64_t m, int32_t k, size_t *scratch_bytes) {
  ABX_TRY(check_bvh(bvh));
  if (m < 0 || k < 0 || !scratch_bytes) return ABX_ERR_INVALID_ARG;
  if (m >= kMaxCount) return ABX_ERR_OVERFLOW;
  *scratch_bytes = query_layout(m, true).bytes;
  return ABX_OK;
}

static abx_status nearest_common(const abx_bvh *bvh, const float *points, int64_t m, int32_t k,
                                 int32_t sort_queries, void *scratch, size_t scratch_bytes,
                                 int32_t *offsets, int32_t *indices, float *distances,
                                 int32_t *stats, abx_stream_t stream) {
  ABX_TRY(check_bvh(bvh));
  if (m < 0 || k < 0) return ABX_ERR_INVALID_ARG;
  if (m >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (m > 0 && !points) return ABX_ERR_INVALID_ARG;
  const QueryLayout L = query_layout(m, true);
  if (!scratch || scratch_bytes < L.bytes || (reinterpret_cast<uintptr_t>(scratch) & 255))
    return ABX_ERR_INVALID_ARG;
  const int64_t kk = k < bvh->n ? k : bvh->n;
  if (m * kk >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (kk > kMaxNearestK) return ABX_ERR_UNSUPPORTED;
  if (!stats && (!offsets || (m * kk > 0 && (!indices || !distances)))) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  if (!stats) ABX_TRY(row_offsets(offsets, m, (int32_t)kk, s));
  if (m == 0) return ABX_OK;
  if (kk == 0) return stats ? fill_u32(stats, 0, 2 * (size_t)m, s) : ABX_OK;
  const int32_t *order = nullptr;
  if (sort_queries) ABX_TRY(order_queries(bvh, points, m, 3, sc, L, &order, s));
  return launch_nearest(bvh, points, m, order, (int)kk, indices, distances, stats,
                        reinterpret_cast<int32_t *>(sc + L.heavy_q),
                        reinterpret_cast<float *>(sc + L.heavy_bound),
                        reinterpret_cast<uint32_t *>(sc + L.total),
                        reinterpret_cast<int32_t *>(sc + L.heavy_state), L.state_cap, nearest_budget(), s);
}

abx_status abx_query_nearest(const abx_bvh *bvh, const float *points, int64_t m, int32_t k,
                             int32_t sort_queries, void *scratch, size_t scratch_bytes,
                             int32_t *offsets, int32_t *indices, float *distances,
                             abx_stream_t stream) {
  return nearest_common(bvh, points, m, k, sort_queries, scratch, scratch_bytes, offsets, indices,
                        distances, nullptr, stream);
}

abx_status abx_query_nearest_stats(const abx_bvh *bvh, const float *points, int64_t m, int32_t k,
                                   int32_t sort_queries, void *scratch, size_t scratch_bytes,
                                   int32_t *stats, abx_stream_t stream) {
  if (!stats && m > 0) return ABX_ERR_INVALID_ARG;
  return nearest_common(bvh, points, m, k, sort_queries, scratch, scratch_bytes, nullptr, nullptr,
                        nullptr, stats, stream);
}

// ---------------------------------------------------------------- building blocks
abx_status abx_morton_codes(abx_prim_kind kind, const float *prims, int64_t n, const float *scene,
                            int32_t bits, uint64_t *codes, abx_stream_t stream) {
  if (kind != ABX_PRIM_POINTS && kind != ABX_PRIM_BOXES) return ABX_ERR_INVALID_ARG;
  if (n < 0 || (bits != 10 && bits != 21)) return ABX_ERR_INVALID_ARG;
  if (n >= kMaxCount) return ABX_ERR_OVERFLOW;
  if (n > 0 && (!prims || !scene || !codes)) return ABX_ERR_INVALID_ARG;
  return launch_morton(kind, prims, n, scene, bits, codes, true, reinterpret_cast<hipStream_t>(stream));
}

abx_status abx_radix_sort_sizes(int64_t n, int32_t key_bits, size_t *scratch_bytes) {
  if (n < 0 || key_bits < 1 || key_bits > 64 || !scratch_bytes) return ABX_ERR_INVALID_ARG;
  if (n >= (int64_t)1 << 30) return ABX_ERR_OVERFLOW;
  *scratch_bytes = radix_sort_scratch_bytes(n, key_bits);
  return ABX_OK;
}

abx_status abx_radix_sort_pairs(const void *keys_in, const int32_t *vals_in, int64_t n,
                                int32_t key_bits, void *keys_out, int32_t *vals_out, void *scratch,
                                size_t scratch_bytes, abx_stream_t stream) {
  return radix_sort(keys_in, vals_in, n, key_bits, keys_out, vals_out, scratch, scratch_bytes,
                    reinterpret_cast<hipStream_t>(stream));
}

abx_status abx_radix_sort_check(const void *scratch, int64_t n, int32_t key_bits,
                                abx_stream_t stream) {
  if (n < 0 || key_bits < 1 || key_bits > 64) return ABX_ERR_INVALID_ARG;
  if (n <= 1) return ABX_OK;
  if (!scratch) return ABX_ERR_INVALID_ARG;
  const uint32_t *w = radix_sort_err_word(const_cast<void *>(scratch), n, key_bits);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint32_t v = 0;
  ABX_HIP(hipMemcpyAsync(&v, w, sizeof(v), hipMemcpyDeviceToHost, s));
  ABX_HIP(hipStreamSynchronize(s));
  return v ? ABX_ERR_DEVICE : ABX_OK;
}

int64_t abx_set_sort_spin_limit(int64_t polls) {
  const uint32_t v = polls < 0 ? (1u << 26) : (uint32_t)std::min<int64_t>(polls, UINT32_MAX);
  return g_sort_spin_limit.exchange(v);
}

int64_t abx_set_refit_table_probes(int64_t probes) {
  const uint32_t v = probes < 0 ? 2048u : (uint32_t)std::min<int64_t>(probes, 2048);
  return g_fit_table_probes.exchange(v);
}

}  // extern "C"
