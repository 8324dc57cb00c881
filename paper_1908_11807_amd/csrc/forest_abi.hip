// C-ABI of the batched forest and the HIP-graph helpers.  Launch sequences
// only; no device memory is allocated and nothing is read back to the host
// (except in abx_forest_check and abx_forest_autotune, which say so).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "traverse_common.h"

namespace abx {

// forest.hip
size_t forest_tree_extra(int T);
abx_status forest_launch_build(const float *pts, int64_t N, const int64_t *off_dev, int T,
                               int32_t *tbox, float *tscene, int64_t *off_copy, TreeHeader *hdr,
                               uint64_t *keys, hipStream_t s);
abx_status forest_launch_roots(const int64_t *off, int T, const int32_t *other_end, const int32_t *perm,
                               int32_t *roots, hipStream_t s);
abx_status forest_launch_qkeys(const float *q, int64_t M, const int64_t *qoff, int T, const float *tscene,
                               uint64_t *keys, int32_t *qtree, hipStream_t s);
abx_status forest_launch_rows(const int64_t *poff, const int64_t *qoff, const int32_t *qtree, int64_t M,
                              int T, int k, int64_t *base, int32_t *offsets, hipStream_t s);
abx_status forest_launch_nearest(const TreeArgs &t, int format, const int64_t *poff, const int32_t *qtree,
                                 const int32_t *roots, const float *tscene, const int32_t *offsets,
                                 const float *pts, int64_t M, const int32_t *order, int k, int32_t *idx,
                                 float *dist, int32_t *heavy_q, float *heavy_bound, uint32_t *counters,
                                 int blocks_per_cu, int grab, int64_t budget, hipStream_t s);
abx_status forest_launch_nearest_stats(const TreeArgs &t, int format, const int64_t *poff,
                                       const int32_t *qtree, const int32_t *roots, const float *tscene,
                                       const int32_t *offsets, const float *pts, int64_t M,
                                       const int32_t *order, int k, int32_t *stats, hipStream_t s);
int forest_max_trees();
// build.hip
abx_status launch_karras(bool wide, const void *keys, int64_t n, uint64_t *pw_leaf, uint64_t *pw_int,
                         int32_t *other_end, uint32_t *flags, const TreeHeader *hdr, hipStream_t s);
abx_status launch_refit(int kind, bool q16, const float *prims, const int32_t *perm, int64_t n,
                        const uint64_t *pw_leaf, const uint64_t *pw_int, const int32_t *pre,
                        void *out, NodeF32 *stage, uint32_t *flags, TreeHeader *hdr, void *box_rec,
                        void *lists_mem, hipStream_t s);
size_t refit_lists_bytes(int64_t n);
int max_tree_depth();

namespace {

constexpr int kForestKeyBits = 63;
constexpr int kForestQueryKeyBits = 39;  // 9-bit tree id above a 30-bit code
constexpr abx_forest_config kDefaultConfig = {4, 1, 16384};

struct ForestLayout {
  int64_t N, ni;
  int T;
  bool q16;
  size_t node_bytes, leaf_bytes;
  size_t nodes, leaves, roots, tscene, offs, tree_total;
  size_t tbox, keys, sorted, parent_leaf, parent_int, other_end, flags, frontier, staging, sort,
      scratch_total;
};

ForestLayout forest_layout(int T, int64_t N, bool q16) {
  ForestLayout L{};
  L.T = T;
  L.N = N;
  L.ni = N > 1 ? N - 1 : 0;
  L.q16 = q16;
  L.node_bytes = q16 ? sizeof(NodeQ16) : sizeof(NodeF32);
  L.leaf_bytes = 4;
  size_t off = sizeof(TreeHeader);
  L.nodes = off;
  off = align_up(off + (size_t)L.ni * L.node_bytes, 256);
  L.leaves = off;
  off = align_up(off + (size_t)N * L.leaf_bytes, 256);
  L.roots = off;
  off = align_up(off + (size_t)T * 4, 256);
  L.tscene = off;
  off = align_up(off + (size_t)T * 24, 256);
  L.offs = off;
  off = align_up(off + (size_t)(T + 1) * 8, 256);
  L.tree_total = off;
  const size_t n = (size_t)N;
  off = 0;
  L.tbox = off;
  off = align_up(off + (size_t)T * 24, 256);
  L.keys = off;
  off = align_up(off + n * 8, 256);
  L.sorted = off;
  off = align_up(off + n * 8, 256);
  L.parent_leaf = off;  // parent words
  off = align_up(off + n * 8, 256);
  L.parent_int = off;
  off = align_up(off + n * 8, 256);
  L.other_end = off;
  off = align_up(off + n * 4, 256);
  L.flags = off;
  off = align_up(off + n * 4, 256);
  L.frontier = off;
  off = align_up(off + refit_lists_bytes(N), 256);
  L.staging = off;
  off = align_up(off + (q16 ? (size_t)L.ni * sizeof(NodeF32) : 0), 256);
  L.sort = off;
  off = align_up(off + radix_sort_scratch_bytes(N, kForestKeyBits), 256);
  L.scratch_total = off;
  return L;
}

struct ForestQueryLayout {
  size_t keys, sorted, order, qtree, base, counters, heavy_q, heavy_bound, sort, bytes;
};

ForestQueryLayout forest_query_layout(int T, int64_t M) {
  ForestQueryLayout L{};
  const size_t m = (size_t)M;
  size_t off = 0;
  L.keys = off;
  off = align_up(off + m * 8, 256);
  L.sorted = off;
  off = align_up(off + m * 8, 256);
  L.order = off;
  off = align_up(off + m * 4, 256);
  L.qtree = off;
  off = align_up(off + m * 4, 256);
  L.base = off;
  off = align_up(off + (size_t)(T + 1) * 8, 256);
  L.counters = off;
  off = align_up(off + 16, 256);
  L.heavy_q = off;
  off = align_up(off + m * 4, 256);
  L.heavy_bound = off;
  off = align_up(off + m * 4, 256);
  L.sort = off;
  off = align_up(off + radix_sort_scratch_bytes(M, kForestQueryKeyBits), 256);
  L.bytes = off;
  return L;
}

abx_status check_offsets(const int64_t *off, int T) {
  if (!off || off[0] != 0) return ABX_ERR_INVALID_ARG;
  for (int t = 0; t < T; ++t)
    if (off[t + 1] < off[t]) return ABX_ERR_INVALID_ARG;
  if (off[T] >= INT32_MAX) return ABX_ERR_OVERFLOW;
  return ABX_OK;
}

abx_status check_forest_prims(const abx_forest_primitives *p) {
  if (!p || p->trees < 1 || p->trees > forest_max_trees()) return ABX_ERR_INVALID_ARG;
  if (p->node_format == ABX_NODES_Q16W) return ABX_ERR_UNSUPPORTED;  // binary nodes only
  if (p->node_format != ABX_NODES_FP32 && p->node_format != ABX_NODES_Q16) return ABX_ERR_INVALID_ARG;
  ABX_TRY(check_offsets(p->offsets_host, p->trees));
  if (!p->offsets_dev || (p->offsets_host[p->trees] > 0 && !p->data)) return ABX_ERR_INVALID_ARG;
  return ABX_OK;
}

bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace
}  // namespace abx

struct abx_forest {
  int32_t T;
  int64_t N;
  int32_t format;
  std::vector<int64_t> off;
  char *tree;
  size_t tree_bytes;
  abx::ForestLayout L;
  abx_forest_config cfg;
};

using namespace abx;

namespace {

TreeArgs forest_tree_args(const abx_forest *f) {
  TreeArgs t;
  std::memset(&t, 0, sizeof(t));
  const TreeHeader *hdr = reinterpret_cast<const TreeHeader *>(f->tree);
  t.nodes = f->tree + f->L.nodes;
  t.leaves = f->tree + f->L.leaves;
  t.n = f->N;
  t.nint = f->N > 1 ? f->N - 1 : 0;
  t.scene_dev = hdr->scene;
  t.qframe = hdr->q_origin;  // q_origin[3] then q_scale[3]
  t.guard = hdr;             // the query exits if the construction failed
  return t;
}

abx_status forest_query_check(const abx_forest *f, const abx_forest_queries *q, int32_t k, int64_t *total) {
  if (!f || !q || k < 0) return ABX_ERR_INVALID_ARG;
  ABX_TRY(check_offsets(q->offsets_host, f->T));
  if (!q->offsets_dev) return ABX_ERR_INVALID_ARG;
  const int64_t M = q->offsets_host[f->T];
  if (M > 0 && !q->data) return ABX_ERR_INVALID_ARG;
  int64_t tot = 0;
  for (int t = 0; t < f->T; ++t) {
    const int64_t nt = f->off[t + 1] - f->off[t];
    tot += (q->offsets_host[t + 1] - q->offsets_host[t]) * std::min<int64_t>(k, nt);
  }
  if (tot >= INT32_MAX) return ABX_ERR_OVERFLOW;
  *total = tot;
  return ABX_OK;
}

}  // namespace

extern "C" {

abx_status abx_forest_build_sizes(const abx_forest_primitives *prims, size_t *tree_bytes,
                                  size_t *scratch_bytes) {
  ABX_TRY(check_forest_prims(prims));
  if (!tree_bytes || !scratch_bytes) return ABX_ERR_INVALID_ARG;
  const ForestLayout L = forest_layout(prims->trees, prims->offsets_host[prims->trees],
                                       prims->node_format == ABX_NODES_Q16);
  *tree_bytes = L.tree_total;
  *scratch_bytes = L.scratch_total;
  return ABX_OK;
}

abx_status abx_forest_build(const abx_forest_primitives *prims, void *tree_mem, size_t tree_bytes,
                            void *scratch, size_t scratch_bytes, abx_stream_t stream, abx_forest **out) {
  ABX_TRY(check_forest_prims(prims));
  if (!out || !tree_mem || !scratch || !aligned256(tree_mem) || !aligned256(scratch))
    return ABX_ERR_INVALID_ARG;
  *out = nullptr;
  const int T = prims->trees;
  const int64_t N = prims->offsets_host[T];
  const bool q16 = prims->node_format == ABX_NODES_Q16;
  const ForestLayout L = forest_layout(T, N, q16);
  if (tree_bytes < L.tree_total || scratch_bytes < L.scratch_total) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *tree = static_cast<char *>(tree_mem);
  char *sc = static_cast<char *>(scratch);
  TreeHeader *hdr = reinterpret_cast<TreeHeader *>(tree);
  int64_t *offs = reinterpret_cast<int64_t *>(tree + L.offs);
  float *tscene = reinterpret_cast<float *>(tree + L.tscene);
  int32_t *roots = reinterpret_cast<int32_t *>(tree + L.roots);
  int32_t *other_end = reinterpret_cast<int32_t *>(sc + L.other_end);

  ABX_TRY(forest_launch_build(prims->data, N, prims->offsets_dev, T, reinterpret_cast<int32_t *>(sc + L.tbox),
                              tscene, offs, hdr, reinterpret_cast<uint64_t *>(sc + L.keys), s));
  if (N > 0) {
    int32_t *perm = reinterpret_cast<int32_t *>(tree + L.leaves);
    NodeF32 *fnodes = q16 ? reinterpret_cast<NodeF32 *>(sc + L.staging)
                          : reinterpret_cast<NodeF32 *>(tree + L.nodes);
    uint64_t *pw_leaf = reinterpret_cast<uint64_t *>(sc + L.parent_leaf);
    uint64_t *pw_int = reinterpret_cast<uint64_t *>(sc + L.parent_int);
    uint32_t *flags = reinterpret_cast<uint32_t *>(sc + L.flags);
    ABX_TRY(radix_sort(sc + L.keys, nullptr, N, kForestKeyBits, sc + L.sorted, perm, sc + L.sort,
                       radix_sort_scratch_bytes(N, kForestKeyBits), s,
                       reinterpret_cast<uint32_t *>(&hdr->bad), kBadSort));
    ABX_TRY(launch_karras(true, sc + L.sorted, N, pw_leaf, pw_int, other_end, flags, hdr, s));
    // nodes written whole by the refit (Q16 directly, build order)
    ABX_TRY(launch_refit(ABX_PRIM_POINTS, q16, prims->data, perm, N, pw_leaf, pw_int, nullptr,
                         tree + L.nodes, fnodes, flags, hdr, nullptr, sc + L.frontier, s));
  }
  ABX_TRY(forest_launch_roots(offs, T, other_end, reinterpret_cast<const int32_t *>(tree + L.leaves),
                              roots, s));

  abx_forest *f = new (std::nothrow) abx_forest;
  if (!f) return ABX_ERR_INVALID_ARG;
  f->T = T;
  f->N = N;
  f->format = prims->node_format;
  f->off.assign(prims->offsets_host, prims->offsets_host + T + 1);
  f->tree = tree;
  f->tree_bytes = tree_bytes;
  f->L = L;
  f->cfg = kDefaultConfig;
  *out = f;
  return ABX_OK;
}

abx_status abx_forest_check(const abx_forest *f, abx_stream_t stream) {
  if (!f) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TreeHeader h;
  ABX_HIP(hipMemcpyAsync(&h, f->tree, sizeof(h), hipMemcpyDeviceToHost, s));
  ABX_HIP(hipStreamSynchronize(s));
  if (h.bad & kBadSort) return ABX_ERR_DEVICE;
  if (h.bad & 1) return ABX_ERR_INVALID_INPUT;
  if (h.bad & 6) return ABX_ERR_UNSUPPORTED;
  if (h.height + 8 >= max_tree_depth()) return ABX_ERR_UNSUPPORTED;
  return ABX_OK;
}

abx_status abx_forest_destroy(abx_forest *f) {
  delete f;
  return ABX_OK;
}

abx_status abx_forest_query_nearest_sizes(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                          size_t *scratch_bytes, int64_t *total) {
  int64_t tot = 0;
  ABX_TRY(forest_query_check(f, q, k, &tot));
  if (!scratch_bytes) return ABX_ERR_INVALID_ARG;
  *scratch_bytes = forest_query_layout(f->T, q->offsets_host[f->T]).bytes;
  if (total) *total = tot;
  return ABX_OK;
}

abx_status abx_forest_query_nearest(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                    const abx_forest_config *cfg, void *scratch, size_t scratch_bytes,
                                    int32_t *offsets, int32_t *indices, float *distances,
                                    abx_stream_t stream) {
  int64_t tot = 0;
  ABX_TRY(forest_query_check(f, q, k, &tot));
  if (k > kMaxRegK) return ABX_ERR_UNSUPPORTED;
  const int T = f->T;
  const int64_t M = q->offsets_host[T];
  const ForestQueryLayout L = forest_query_layout(T, M);
  if (!scratch || scratch_bytes < L.bytes || !aligned256(scratch) || !offsets) return ABX_ERR_INVALID_ARG;
  if (tot > 0 && (!indices || !distances)) return ABX_ERR_INVALID_ARG;
  const abx_forest_config c = cfg ? *cfg : f->cfg;
  if (c.blocks_per_cu < 1 || c.blocks_per_cu > 64 || c.tiles_per_grab < 1 || c.tiles_per_grab > 64)
    return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  const int64_t *poff = reinterpret_cast<const int64_t *>(f->tree + f->L.offs);
  const float *tscene = reinterpret_cast<const float *>(f->tree + f->L.tscene);
  const int32_t *roots = reinterpret_cast<const int32_t *>(f->tree + f->L.roots);
  int32_t *order = reinterpret_cast<int32_t *>(sc + L.order);
  int32_t *qtree = reinterpret_cast<int32_t *>(sc + L.qtree);
  ABX_TRY(forest_launch_qkeys(q->data, M, q->offsets_dev, T, tscene, reinterpret_cast<uint64_t *>(sc + L.keys),
                              qtree, s));
  ABX_TRY(radix_sort(sc + L.keys, nullptr, M, kForestQueryKeyBits, sc + L.sorted, order, sc + L.sort,
                     radix_sort_scratch_bytes(M, kForestQueryKeyBits), s));
  ABX_TRY(order_guard(radix_sort_err_word(sc + L.sort, M, kForestQueryKeyBits), order, M, s));
  ABX_TRY(forest_launch_rows(poff, q->offsets_dev, qtree, M, T, k, reinterpret_cast<int64_t *>(sc + L.base),
                             offsets, s));
  if (M == 0 || k == 0 || f->N == 0) return ABX_OK;
  const TreeArgs t = forest_tree_args(f);
  return forest_launch_nearest(t, f->format, poff, qtree, roots, tscene, offsets, q->data, M, order, k,
                               indices, distances, reinterpret_cast<int32_t *>(sc + L.heavy_q),
                               reinterpret_cast<float *>(sc + L.heavy_bound),
                               reinterpret_cast<uint32_t *>(sc + L.counters), c.blocks_per_cu,
                               c.tiles_per_grab, c.budget > 0 ? c.budget : INT64_MAX, s);
}

abx_status abx_forest_query_nearest_stats(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                          void *scratch, size_t scratch_bytes, int32_t *offsets,
                                          int32_t *stats, abx_stream_t stream) {
  int64_t tot = 0;
  ABX_TRY(forest_query_check(f, q, k, &tot));
  if (k > kMaxRegK) return ABX_ERR_UNSUPPORTED;
  const int T = f->T;
  const int64_t M = q->offsets_host[T];
  const ForestQueryLayout L = forest_query_layout(T, M);
  if (!scratch || scratch_bytes < L.bytes || !aligned256(scratch) || !offsets) return ABX_ERR_INVALID_ARG;
  if (M > 0 && !stats) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *sc = static_cast<char *>(scratch);
  const int64_t *poff = reinterpret_cast<const int64_t *>(f->tree + f->L.offs);
  const float *tscene = reinterpret_cast<const float *>(f->tree + f->L.tscene);
  const int32_t *roots = reinterpret_cast<const int32_t *>(f->tree + f->L.roots);
  int32_t *order = reinterpret_cast<int32_t *>(sc + L.order);
  int32_t *qtree = reinterpret_cast<int32_t *>(sc + L.qtree);
  ABX_TRY(forest_launch_qkeys(q->data, M, q->offsets_dev, T, tscene, reinterpret_cast<uint64_t *>(sc + L.keys),
                              qtree, s));
  ABX_TRY(radix_sort(sc + L.keys, nullptr, M, kForestQueryKeyBits, sc + L.sorted, order, sc + L.sort,
                     radix_sort_scratch_bytes(M, kForestQueryKeyBits), s));
  ABX_TRY(order_guard(radix_sort_err_word(sc + L.sort, M, kForestQueryKeyBits), order, M, s));
  ABX_TRY(forest_launch_rows(poff, q->offsets_dev, qtree, M, T, k, reinterpret_cast<int64_t *>(sc + L.base),
                             offsets, s));
  if (M == 0) return ABX_OK;
  if (f->N == 0) return fill_u32(stats, 0, 2 * (size_t)M, s);
  const TreeArgs t = forest_tree_args(f);
  return forest_launch_nearest_stats(t, f->format, poff, qtree, roots, tscene, offsets, q->data, M, order,
                                     k, stats, s);
}

abx_status abx_forest_autotune(abx_forest *f, const abx_forest_queries *q, int32_t k, void *scratch,
                               size_t scratch_bytes, int32_t *offsets, int32_t *indices, float *distances,
                               abx_stream_t stream, const char *json_path, abx_forest_config *best) {
  if (!f || !best) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return ABX_ERR_INVALID_ARG;  // it times eager launches
  const int bpcs[] = {2, 4, 6, 8};
  const int grabs[] = {1, 4};
  const int64_t budgets[] = {8192, 32768, 131072};
  hipEvent_t a, b;
  ABX_HIP(hipEventCreate(&a));
  ABX_HIP(hipEventCreate(&b));
  std::string log = "{\"k\": " + std::to_string(k) + ", \"trees\": " + std::to_string(f->T) +
                    ", \"candidates\": [";
  float best_ms = 1e30f;
  abx_forest_config chosen = f->cfg;
  bool first = true;
  abx_status st = ABX_OK;
  for (int bpc : bpcs)
    for (int grab : grabs)
      for (int64_t budget : budgets) {
        const abx_forest_config c{bpc, grab, budget};
        st = abx_forest_query_nearest(f, q, k, &c, scratch, scratch_bytes, offsets, indices, distances, stream);
        if (st != ABX_OK) goto done;
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          if (hipEventRecord(a, s) != hipSuccess) { st = ABX_ERR_HIP; goto done; }
          st = abx_forest_query_nearest(f, q, k, &c, scratch, scratch_bytes, offsets, indices, distances, stream);
          if (st != ABX_OK) goto done;
          if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
            st = ABX_ERR_HIP;
            goto done;
          }
          float e = 0.0f;
          (void)hipEventElapsedTime(&e, a, b);
          ms = std::min(ms, e);
        }
        char buf[160];
        std::snprintf(buf, sizeof(buf),
                      "%s{\"blocks_per_cu\": %d, \"tiles_per_grab\": %d, \"budget\": %lld, \"ms\": %.4f}",
                      first ? "" : ", ", bpc, grab, (long long)budget, ms);
        log += buf;
        first = false;
        if (ms < best_ms) {
          best_ms = ms;
          chosen = c;
        }
      }
done:
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != ABX_OK) return st;
  f->cfg = chosen;
  *best = chosen;
  if (json_path) {
    char buf[200];
    std::snprintf(buf, sizeof(buf),
                  "], \"best\": {\"blocks_per_cu\": %d, \"tiles_per_grab\": %d, \"budget\": %lld, \"ms\": %.4f}}\n",
                  chosen.blocks_per_cu, chosen.tiles_per_grab, (long long)chosen.budget, best_ms);
    log += buf;
    FILE *fp = std::fopen(json_path, "a");
    if (fp) {
      std::fputs(log.c_str(), fp);
      std::fclose(fp);
    }
  }
  return ABX_OK;
}

// ---------------------------------------------------------------- graphs
abx_status abx_graph_begin(abx_stream_t stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (s == nullptr) return ABX_ERR_INVALID_ARG;  // the null stream cannot be captured
  ABX_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  return ABX_OK;
}

abx_status abx_graph_end(abx_stream_t stream, void **graph_exec) {
  if (!graph_exec) return ABX_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) return hip_fail(e);
  hipGraphExec_t x = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return hip_fail(e2);
  *graph_exec = x;
  return ABX_OK;
}

abx_status abx_graph_launch(void *graph_exec, abx_stream_t stream) {
  if (!graph_exec) return ABX_ERR_INVALID_ARG;
  ABX_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), reinterpret_cast<hipStream_t>(stream)));
  return ABX_OK;
}

abx_status abx_graph_destroy(void *graph_exec) {
  if (graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
  return ABX_OK;
}

}  // extern "C"
