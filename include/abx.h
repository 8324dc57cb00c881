/*
 * abx.h -- C-ABI of libabx, a linear-BVH geometric search library for the
 * AMD MI355X (gfx950).
 *
 * The method is the one of ArborX (Lebrun-Grandie, Prokopenko, Turcksin,
 * Slattery; arXiv:1908.11807):
 *   - construction (section 2.1): boxes of the primitives, scene box, Morton
 *     codes, sort, Karras hierarchy, bottom-up internal boxes;
 *   - traversal (section 2.2): spatial queries by an iterative stack
 *     traversal with count-then-fill (2P) output, nearest queries by a stack
 *     traversal that visits the nearer child first (nearer by box centre
 *     here) and stops when no remaining candidate can improve, query
 *     ordering by Morton code;
 *   - interface (section 2.3): build from primitives, query with a batch of
 *     predicates, results as CSR offsets + indices.
 *
 * Conventions shared by every entry point:
 *   - Pointers are DEVICE pointers unless the parameter is marked (host).
 *   - The library never allocates or frees device memory.  Every device
 *     buffer is owned by the caller; its size comes from the matching
 *     *_sizes call.  Scratch buffers may be reused between calls once the
 *     stream has passed the call that used them.
 *   - Every call enqueues its kernels on `stream` (0 = the null stream) and
 *     returns after enqueueing, except where a host read is stated.
 *   - Arguments are validated before anything is launched; errors are
 *     return codes, never exceptions.  On ABX_ERR_HIP the failing HIP error
 *     code is available from abx_last_hip_error() (per host thread).
 *   - Indices are int32, 0-based positions in the caller's primitive array.
 *     n, m and every result count must be below 2^31 (ABX_ERR_OVERFLOW).
 *   - Primitive and query coordinates are float32, row-major.
 *   - A handle (abx_bvh) lives in host memory and points into the caller's
 *     tree buffer; it is immutable after a successful build and may be
 *     queried concurrently from several streams, one scratch buffer per
 *     in-flight call.
 */
#ifndef ABX_H
#define ABX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *abx_stream_t; /* a hipStream_t */

typedef enum {
  ABX_OK = 0,
  ABX_ERR_INVALID_ARG = 1,   /* bad pointer, size, kind or option          */
  ABX_ERR_INVALID_INPUT = 2, /* a primitive coordinate is NaN or infinite  */
  ABX_ERR_CAPACITY = 3,      /* result buffer too small; see query_spatial */
  ABX_ERR_OVERFLOW = 4,      /* a size or result count reaches 2^31        */
  ABX_ERR_HIP = 5,           /* a HIP runtime call failed                  */
  ABX_ERR_UNSUPPORTED = 6,   /* valid request the library does not handle  */
  ABX_PENDING = 7,           /* (server) the request has not completed yet */
  ABX_ERR_DEVICE = 8         /* a bounded wait between workgroups gave up
                                (the sort's look-back): results not valid  */
} abx_status;

/* Primitives (section 2.1 "Construct AABBs": a point is a degenerate box). */
typedef enum {
  ABX_PRIM_POINTS = 0, /* float32 [n,3]: x y z                      */
  ABX_PRIM_BOXES = 1   /* float32 [n,6]: lo x y z, hi x y z (lo<=hi) */
} abx_prim_kind;

/* Storage of the internal nodes.
 *   FP32: 64 B per internal node -- both children's float32 boxes and
 *         their references.  A leaf child's box is its primitive's exact
 *         box and its reference names the primitive, so traversal reads
 *         nothing else.
 *   Q16 : 32 B per internal node -- internal children's boxes quantised to
 *         16 bits per coordinate on the scene box's grid, rounded outward
 *         so every quantised box contains the exact one.  In point trees a
 *         leaf child's slot holds the point's float32 coordinates; box
 *         trees keep the exact float32 box in a leaf record.  Results are
 *         identical to FP32.  (The paper names quantised bounds as a way to
 *         cut BVH bandwidth, section 2 literature review.)
 *   Q16W: 64 B per internal node with up to FOUR children -- the binary
 *         tree collapsed at even depths: a node keeps its children's
 *         children, a leaf child stays a leaf child -- quantised as Q16 and
 *         stored in depth-first order.  A walk makes half as many dependent
 *         node loads (the paper leaves the load balance of one thread per
 *         query open, section 2.2; wider nodes shorten each thread's chain of
 *         loads).  Karras hierarchy only; trees of binary height above 78
 *         are refused (the walks' stacks).  Results are identical to FP32. */
typedef enum { ABX_NODES_FP32 = 0, ABX_NODES_Q16 = 1, ABX_NODES_Q16W = 2 } abx_node_format;

typedef struct {
  abx_prim_kind kind;
  const float *data; /* device, [n,3] or [n,6] */
  int64_t n;
} abx_primitives;

/* Construction of the hierarchy (section 2.1).
 *   KARRAS       : one thread per internal node finds its range and split by
 *                  binary searches (Karras 2012), then an atomic bottom-up
 *                  refit; internal node 0 is the root.
 *   AGGLOMERATIVE: hierarchy and refit in one bottom-up pass, each node
 *                  merging with the neighbour of longer common prefix
 *                  (Apetrei 2014, which the paper plans to adopt); internal
 *                  node p is the split between sorted positions p and p+1 and
 *                  the root is reported in the layout.  Same tree, other
 *                  numbering; queries give identical results. */
typedef enum { ABX_HIERARCHY_KARRAS = 0, ABX_HIERARCHY_AGGLOMERATIVE = 1 } abx_hierarchy;

/* Order of the internal nodes in tree memory.  DEPTH_FIRST (Q16 Karras trees
 * only): root 0, a node's left child right after it, its right child after
 * the left subtree, so a walk going down reads consecutive nodes; it pays
 * once the nodes outgrow the last-level cache (C3, 1e7 points: nearest walk
 * -5 ms for +0.4 ms of build) and not below (1e6: +0.1 ms of build, walk
 * unchanged).  AUTO picks DEPTH_FIRST for Q16 Karras trees of at least 2^22
 * primitives, else the hierarchy's own numbering (BUILD).  Queries do not
 * depend on the order. */
typedef enum { ABX_ORDER_AUTO = 0, ABX_ORDER_BUILD = 1, ABX_ORDER_DEPTH_FIRST = 2 } abx_node_order;

typedef struct {
  abx_node_format node_format;
  int32_t morton_bits; /* bits per axis of the Morton code: 10 (30-bit codes)
                          or 21 (63-bit codes, the default when 0) */
  int32_t hierarchy;   /* abx_hierarchy (0: Karras) */
  int32_t node_order;  /* abx_node_order (0: automatic); DEPTH_FIRST with
                          FP32 nodes or the agglomerative hierarchy returns
                          ABX_ERR_UNSUPPORTED, as do Q16W nodes with BUILD
                          order or the agglomerative hierarchy */
} abx_build_options;

/* Spatial predicates (section 2.2, spatial traversal). */
typedef enum {
  ABX_PRED_WITHIN = 0,         /* data [m,3] points; hit iff distance <= r    */
  ABX_PRED_INTERSECTS_BOX = 1  /* data [m,6] boxes; hit iff closed boxes meet */
} abx_pred_kind;

typedef struct {
  abx_pred_kind kind;
  const float *data;   /* device [m,3] or [m,6]                         */
  int64_t m;
  const float *radii;  /* device [m] per-query radius, or NULL          */
  float radius;        /* used when radii == NULL; r < 0 gives no hits  */
  int32_t sort_queries;/* 1: traverse in Morton order of the queries
                          (section 2.2 "Query ordering"); 0: input order */
} abx_predicates;

typedef struct abx_bvh abx_bvh; /* opaque host handle */

/* Layout of a built tree inside the caller's tree buffer (for inspection). */
typedef struct {
  int64_t n;              /* number of primitives (leaves)                  */
  int32_t kind;           /* abx_prim_kind                                  */
  int32_t node_format;    /* abx_node_format                                */
  int32_t morton_bits;
  int32_t height;         /* longest root-to-leaf edge count (0 if n <= 1)  */
  int32_t hierarchy;      /* abx_hierarchy the tree was built with          */
  int32_t root;           /* internal node at the root (n >= 2)             */
  int32_t node_order;     /* ABX_ORDER_BUILD or ABX_ORDER_DEPTH_FIRST       */
  float scene[6];         /* scene box lo xyz, hi xyz (section 2.1)         */
  size_t nodes_offset;    /* byte offset of internal node 0 in tree memory */
  size_t node_bytes;      /* 64 (FP32) or 32 (Q16)                          */
  size_t leaves_offset;   /* byte offset of leaf 0                          */
  size_t leaf_bytes;      /* 4: int32 permutation, sorted position ->
                             primitive index (FP32, and Q16 point trees);
                             32: Q16 box trees, record i = primitive i's
                             float lo xyz, hi xyz, its sorted position, pad */
  float q16_origin[3];    /* Q16 dequantisation: x = fmaf(q, scale, origin) */
  float q16_scale[3];
  int64_t node_count;     /* internal nodes stored: n - 1 (binary), fewer for
                             Q16W (node i at nodes_offset + i * node_bytes) */
} abx_bvh_layout;

/* -- construction (section 2.1) ------------------------------------------
 * abx_bvh_build_sizes: device bytes the tree and the build's scratch need.
 * abx_bvh_build: builds the LBVH of `prims` into `tree_mem`.  Steps, all on
 *   `stream`: scene box reduction with a NaN/Inf check, Morton codes of the
 *   box centroids scaled by the scene box, stable LSD radix sort of (code,
 *   index), Karras (2012) hierarchy over the index-augmented codes, atomic
 *   bottom-up refit of the internal boxes (and quantisation for Q16).
 *   Blocks the host once at the end to read the NaN flag and tree height.
 *   Returns ABX_ERR_INVALID_INPUT for NaN/Inf coordinates (no handle), and
 *   ABX_ERR_DEVICE (no handle) if a tile of the sort stopped waiting for
 *   its predecessors' counts (see abx_set_sort_spin_limit).
 *   `*out` receives a new handle; release it with abx_bvh_destroy.
 * abx_bvh_destroy: frees the host handle only (tree memory is the caller's). */
abx_status abx_bvh_build_sizes(const abx_primitives *prims, const abx_build_options *opts,
                               size_t *tree_bytes /*host*/, size_t *scratch_bytes /*host*/);
abx_status abx_bvh_build(const abx_primitives *prims, const abx_build_options *opts,
                         void *tree_mem, size_t tree_bytes, void *scratch, size_t scratch_bytes,
                         abx_stream_t stream, abx_bvh **out /*host*/);
abx_status abx_bvh_destroy(abx_bvh *bvh);
abx_status abx_bvh_get_layout(const abx_bvh *bvh, abx_bvh_layout *out /*host*/);

/* -- spatial queries (section 2.2 spatial traversal, 2P count-and-fill) ---
 * abx_query_spatial_sizes: scratch bytes for a batch of m predicates.
 * abx_query_spatial: orders the queries (optional), counts the hits of each
 *   query by a stack traversal, scans the counts into offsets[0..m] (rows in
 *   the caller's query order, offsets[0] = 0, offsets[m] = total), and
 *   blocks the host to read the total into *total.  If total <= capacity it
 *   traverses again, writing each row's primitive indices (order within a
 *   row unspecified), and returns ABX_OK.  Otherwise it returns
 *   ABX_ERR_CAPACITY with offsets and *total valid; the caller may then call
 *   abx_query_spatial_fill with a large enough `indices` and the same
 *   scratch (which keeps the query order).  total >= 2^31 gives
 *   ABX_ERR_OVERFLOW.  The user-side estimate `capacity` plays the role of
 *   the paper's buffer_size (section 2.3).
 * abx_query_spatial_fill: the second pass alone, after a call of
 *   abx_query_spatial on the same predicates and scratch. */
abx_status abx_query_spatial_sizes(const abx_bvh *bvh, const abx_predicates *preds,
                                   size_t *scratch_bytes /*host*/);
abx_status abx_query_spatial(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                             size_t scratch_bytes, int32_t *offsets /*[m+1]*/, int32_t *indices,
                             int64_t capacity, int64_t *total /*host*/, abx_stream_t stream);
abx_status abx_query_spatial_fill(const abx_bvh *bvh, const abx_predicates *preds, void *scratch,
                                  size_t scratch_bytes, const int32_t *offsets, int32_t *indices,
                                  int64_t capacity, abx_stream_t stream);

/* -- spatial queries, one pass (section 2.2, the 1P scheme) ---------------
 * abx_query_spatial_1p_sizes: scratch bytes for m predicates with a per-query
 *   estimate buffer_size (1 .. 65536) of the hits: the 2P scratch plus
 *   m * buffer_size int32 slots.
 * abx_query_spatial_1p: orders the queries (optional), then ONE traversal
 *   counts every query's hits and stores the first buffer_size of them in
 *   scratch; the counts are scanned into offsets[0..m] (caller's order,
 *   offsets[m] = total).  If no query found more than buffer_size hits, the
 *   stored rows are compacted into indices: one traversal in all.  Otherwise
 *   the fill traversal of the 2P scheme writes indices (the count is
 *   already known): two traversals, as 2P.  Nothing blocks the host and
 *   nothing is read back, so the call can be captured in a graph.
 *   info (device int32[2]) receives, once the stream has passed the call:
 *   info[0] = ABX_OK, or ABX_ERR_CAPACITY when total > capacity (offsets
 *   valid, indices untouched: call abx_query_spatial_fill with the same
 *   scratch and a large enough buffer), or ABX_ERR_OVERFLOW when total
 *   reaches 2^31; info[1] = traversals made (0 for an empty tree or batch).
 *   Within a row the order is the traversal's, as in 2P. */
abx_status abx_query_spatial_1p_sizes(const abx_bvh *bvh, const abx_predicates *preds,
                                      int32_t buffer_size, size_t *scratch_bytes /*host*/);
abx_status abx_query_spatial_1p(const abx_bvh *bvh, const abx_predicates *preds, int32_t buffer_size,
                                void *scratch, size_t scratch_bytes, int32_t *offsets /*[m+1]*/,
                                int32_t *indices, int64_t capacity, int32_t *info /*device [2]*/,
                                abx_stream_t stream);

/* -- nearest queries (section 2.2 nearest traversal) ----------------------
 * abx_query_nearest: for each of the m query points, the min(k, n) nearest
 *   primitives by (distance, index), ascending (distance ties go to the
 *   smaller index); missing results are purged, so every row has length
 *   k' = min(k, n).  offsets[i] = i * k'; indices and distances are [m, k']
 *   in the caller's query order; distances are float32 Euclidean (point to
 *   box for box primitives).  No host synchronisation.  1 <= k <= 64 keeps
 *   the candidates in registers (one lane per query, heavy queries handed to
 *   whole workgroups); 65 <= k <= 128 keeps them in per-lane LDS max-heaps
 *   (one lane per query throughout); larger k returns ABX_ERR_UNSUPPORTED.
 *   Per axis the gap is max(lo - q, q - hi, 0) with IEEE max, which drops a
 *   NaN operand: a NaN query coordinate contributes no gap on its axis (the
 *   same for radius and box tests).  An infinite coordinate puts every
 *   primitive at +inf: the row is the k' smallest indices (the tie rule),
 *   after a walk of the whole tree. */
abx_status abx_query_nearest_sizes(const abx_bvh *bvh, int64_t m, int32_t k,
                                   size_t *scratch_bytes /*host*/);
abx_status abx_query_nearest(const abx_bvh *bvh, const float *points /*[m,3]*/, int64_t m,
                             int32_t k, int32_t sort_queries, void *scratch, size_t scratch_bytes,
                             int32_t *offsets /*[m+1]*/, int32_t *indices, float *distances,
                             abx_stream_t stream);

/* -- nearest queries without any allocation ------------------------------
 * For callers that cannot allocate memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same query, the
 * same kernels and the same results as abx_query_nearest, but the scratch is
 * a library-owned device array of ABX_STATIC_SCRATCH_BYTES per GPU (set up
 * when the library's code is loaded on that GPU, held until the process
 * ends).  The caller still owns points, offsets, indices and distances.
 * Returns ABX_ERR_CAPACITY, before launching anything, when the scratch that
 * abx_query_nearest_sizes reports for (m, k) exceeds ABX_STATIC_SCRATCH_BYTES
 * (about 400 000 queries).  The call allocates nothing, on the device or the
 * host: no hipMalloc, hipFree or event (timing mode does not apply to it).
 * All calls on one GPU share that GPU's array: calls that overlap in time on
 * one GPU (from different streams or threads) race and their results are
 * undefined; calls ordered on one stream are safe. */
#define ABX_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
abx_status abx_query_nearest_static(const abx_bvh *bvh, const float *points /*[m,3]*/, int64_t m,
                                    int32_t k, int32_t sort_queries, int32_t *offsets /*[m+1]*/,
                                    int32_t *indices, float *distances, abx_stream_t stream);

/* -- load balance of nearest queries ------------------------------------------
 * A nearest query is first walked by one lane (the paper's batched mode).  A
 * walk that exceeds `visits` internal-node visits is abandoned and the query
 * is answered again by a whole workgroup (16 wavefronts, 8 for k > 16, i.e.
 * 1024 or 512 lanes sharing one query: a breadth-first frontier is split among
 * the lanes, their pruning bound is shared, their candidate lists are merged
 * exactly), starting from the bound the lane had reached.  Results do not
 * depend on the value.  (k > 64 is walked by one lane throughout.)
 * abx_set_nearest_budget sets the process-wide budget (<= 0: unlimited, i.e.
 * one lane per query throughout) and returns the previous one.  Default 22528.
 * A batch of m queries uses min(budget, max(512, m / 24)): small batches
 * leave the GPU idle and hand heavy queries to whole workgroups sooner. */
int64_t abx_set_nearest_budget(int64_t visits);

/* -- traversal statistics ---------------------------------------------------
 * Same traversals run in a counting mode: stats[2*i] = internal nodes
 * visited by query i (caller's order), stats[2*i+1] = leaf records read.
 * Used to derive the algorithmic bytes of a batch. */
abx_status abx_query_spatial_stats(const abx_bvh *bvh, const abx_predicates *preds,
                                   void *scratch, size_t scratch_bytes, int32_t *stats /*[2m]*/,
                                   abx_stream_t stream);
abx_status abx_query_nearest_stats(const abx_bvh *bvh, const float *points, int64_t m,
                                   int32_t k, int32_t sort_queries, void *scratch,
                                   size_t scratch_bytes, int32_t *stats /*[2m]*/,
                                   abx_stream_t stream);

/* -- building blocks, exported for kernel-level checks ---------------------
 * abx_morton_codes: codes of n primitives against a device scene box
 *   (float[6]) with `bits` bits per axis (10 or 21): centroid, scaled into
 *   [0,1]^3 in float32 (inverse extent, clamp), quantised, interleaved with
 *   x as the most significant bit of each triple (section 2.1).
 * abx_radix_sort_pairs: stable LSD radix sort of n (key, value) pairs on the
 *   low `key_bits` bits (keys uint32 when key_bits <= 32, else uint64;
 *   values int32, or the identity 0..n-1 when vals_in is NULL).  Each pass
 *   is one launch in which a tile of keys waits for the digit counts of the
 *   tiles before it (section 2.1 "Sort the bounding boxes").  That wait is
 *   bounded: a tile that gives up records it in the scratch buffer and the
 *   sort completes with an invalid (though in-bounds) output.
 * abx_radix_sort_check: blocks the host until the stream has passed a sort
 *   on `scratch` (same n, key_bits) and returns ABX_ERR_DEVICE if one of its
 *   tiles gave up, else ABX_OK.  (The library's own sorts act on it: a
 *   build fails with ABX_ERR_DEVICE; a query ordering falls back to the
 *   caller's order, which gives the same results.)
 * abx_set_sort_spin_limit: polls of a predecessor that has published nothing
 *   before a tile gives up (default 2^26, far above any real wait; < 0
 *   restores it; 0 gives up at the first such poll, so tests can force the
 *   failure path with every kernel still ending normally).  Process-wide;
 *   returns the previous value. */
abx_status abx_morton_codes(abx_prim_kind kind, const float *prims, int64_t n, const float *scene,
                            int32_t bits, uint64_t *codes, abx_stream_t stream);
abx_status abx_radix_sort_sizes(int64_t n, int32_t key_bits, size_t *scratch_bytes /*host*/);
abx_status abx_radix_sort_pairs(const void *keys_in, const int32_t *vals_in, int64_t n,
                                int32_t key_bits, void *keys_out, int32_t *vals_out,
                                void *scratch, size_t scratch_bytes, abx_stream_t stream);
abx_status abx_radix_sort_check(const void *scratch, int64_t n, int32_t key_bits,
                                abx_stream_t stream);
int64_t abx_set_sort_spin_limit(int64_t polls);

/* abx_set_refit_table_probes: the refit's passes above its 2048-leaf chunks
 * (section 2.1, internal node boxes) climb in an LDS table of 2048 nodes; a
 * pass gives up on the table after this many probes for one node (default
 * and maximum 2048, the whole table; < 0 restores it) and climbs through
 * global memory instead.  0 sends every pass to global memory, so tests can
 * compare the two climbs; the tree is the same either way.  Process-wide;
 * returns the previous value. */
int64_t abx_set_refit_table_probes(int64_t probes);

/* -- batched forest --------------------------------------------------------------
 * T independent point sets ("trees", 1 <= T <= 512) of uneven sizes, built
 * and queried together: the batched mode of section 2.2 applied across trees
 * as well as queries.  Points of all trees are concatenated; tree t owns rows
 * [offsets[t], offsets[t+1]) (empty trees allowed).  One construction over
 * composite keys (tree id above an 18-bit-per-axis Morton code against the
 * tree's own scene box) gives every tree its own subtree of one LBVH arena;
 * one persistent launch answers the nearest queries of all trees.  Neither
 * call synchronises the host, so both can be captured in a HIP graph
 * (abx_graph_*); abx_forest_check reads the device status afterwards.
 * The offsets are passed twice: a host copy (sizes and launch shapes) and a
 * device copy (read by kernels); both must hold the same values and stay
 * valid for the duration of the call. */
typedef struct {
  int32_t trees;
  const int64_t *offsets_host; /* host   [T+1], offsets[0] = 0, non-decreasing */
  const int64_t *offsets_dev;  /* device [T+1], same values                    */
  const float *data;           /* device [offsets[T], 3] points                 */
  abx_node_format node_format; /* FP32 or Q16 (Q16W: ABX_ERR_UNSUPPORTED)       */
} abx_forest_primitives;

typedef struct {
  const int64_t *offsets_host; /* host   [T+1]: tree t's queries are rows [o[t], o[t+1]) */
  const int64_t *offsets_dev;  /* device [T+1]                                          */
  const float *data;           /* device [offsets[T], 3] query points                   */
} abx_forest_queries;

/* Launch shape of the persistent forest query: workgroups per CU, tiles of
 * 64 queries taken per queue access, and the node-visit budget before a
 * query moves to the cooperative pass. */
typedef struct {
  int32_t blocks_per_cu;
  int32_t tiles_per_grab;
  int64_t budget;
} abx_forest_config;

typedef struct abx_forest abx_forest;

abx_status abx_forest_build_sizes(const abx_forest_primitives *prims, size_t *tree_bytes /*host*/,
                                  size_t *scratch_bytes /*host*/);
/* Enqueues the construction; no host synchronisation.  The scratch buffer
 * may be reused once the stream has passed the call. */
abx_status abx_forest_build(const abx_forest_primitives *prims, void *tree_mem, size_t tree_bytes,
                            void *scratch, size_t scratch_bytes, abx_stream_t stream,
                            abx_forest **out /*host*/);
/* Waits for the stream and reports the construction status:
 * ABX_ERR_INVALID_INPUT for a NaN/Inf coordinate, ABX_ERR_UNSUPPORTED for a
 * tree deeper than the traversal stacks, ABX_ERR_DEVICE if the sort gave up
 * (abx_radix_sort_check), else ABX_OK.  A forest query over a forest whose
 * construction failed walks nothing and leaves its rows unwritten (its
 * kernels read the status on the device, so graph replays are safe too). */
abx_status abx_forest_check(const abx_forest *f, abx_stream_t stream);
abx_status abx_forest_destroy(abx_forest *f);
/* Scratch bytes of a forest nearest query, and (host) the total number of
 * result entries: sum over trees of (queries of t) * min(k, n_t). */
abx_status abx_forest_query_nearest_sizes(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                          size_t *scratch_bytes /*host*/, int64_t *total /*host*/);
/* k nearest points of each query among its own tree's points, ordered by
 * (distance, index); indices are tree-local (0 .. n_t-1).  Rows follow the
 * caller's query order; row i has min(k, n_t) entries starting at
 * offsets[i]; offsets[M] = total.  `cfg` may be NULL (the tuned shape of
 * abx_forest_autotune if any, else a default).  1 <= k <= 64 (larger k:
 * ABX_ERR_UNSUPPORTED). */
abx_status abx_forest_query_nearest(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                    const abx_forest_config *cfg, void *scratch, size_t scratch_bytes,
                                    int32_t *offsets /*[M+1]*/, int32_t *indices, float *distances,
                                    abx_stream_t stream);
/* The same walks in a counting mode (one lane per query throughout, no
 * results): stats[2*i] = internal nodes visited by query i (caller's
 * order), stats[2*i+1] = leaf records read; offsets as for the query.  Used
 * to derive the algorithmic bytes of a forest query. */
abx_status abx_forest_query_nearest_stats(const abx_forest *f, const abx_forest_queries *q, int32_t k,
                                          void *scratch, size_t scratch_bytes, int32_t *offsets /*[M+1]*/,
                                          int32_t *stats /*[2M]*/, abx_stream_t stream);
/* Times the forest nearest query over a grid of launch shapes (the output
 * buffers are overwritten), keeps the fastest in the handle, writes it to
 * *best and, when json_path is not NULL, appends every timing to that file
 * as one JSON object. */
abx_status abx_forest_autotune(abx_forest *f, const abx_forest_queries *q, int32_t k, void *scratch,
                               size_t scratch_bytes, int32_t *offsets, int32_t *indices,
                               float *distances, abx_stream_t stream, const char *json_path,
                               abx_forest_config *best /*host*/);

/* -- HIP graphs ------------------------------------------------------------------
 * Capture of everything enqueued on `stream` between begin and end (no host
 * synchronisation may happen in between: use the forest entry points, not
 * abx_bvh_build / abx_query_spatial, which read results back).  The
 * instantiated graph is replayed with abx_graph_launch. */
abx_status abx_graph_begin(abx_stream_t stream);
abx_status abx_graph_end(abx_stream_t stream, void **graph_exec /*host*/);
abx_status abx_graph_launch(void *graph_exec, abx_stream_t stream);
abx_status abx_graph_destroy(void *graph_exec);

/* -- serving -------------------------------------------------------------------
 * Continuous batching of query requests against device-resident trees (a
 * tree is built once and queried many times, section 2.2; the batched mode
 * of section 2.2 applied across requests).  A scheduler thread owns `slots`
 * HIP streams.  Queued requests on the same tree with the same predicate
 * (nearest with the same k, or radius with the same r) and of the same size
 * class are MERGED: the first waiting one takes the later ones of its class
 * along, up to merge_queries queries for small requests and merge_large for
 * large ones (which queue beside each other only when the slots are behind),
 * and they run as one launch sequence over their concatenated queries; each
 * request's rows are copied back to its own results.  Admission serves the queue in order within each size class
 * (small / large by small_queries): a batch starts as soon as a slot is free
 * and its device reservation fits in the caller's arena (the HBM budget);
 * a request of one class may pass one of the other that cannot start (no
 * memory, or slots - 1 large batches already running: one slot stays for
 * small requests).  Requests that arrive while others run start as slots
 * and memory free up, and their kernels overlap on the device.  Nearest
 * batches run in one phase; radius batches in two (count, then fill once the
 * exact result space is reserved; while a fill waits, new batches are
 * admitted only if that space stays free).  Results are copied to a pinned
 * host arena the server allocates at creation and stay valid until
 * abx_server_release.  Every row is answered by the same kernels as the
 * plain entry points, and a row depends only on its own query, so a
 * request's result does not depend on what else is in flight or merged with
 * it.  Radius batches, and nearest batches of fewer than 4096 queries, are
 * walked in the caller's order; larger nearest batches are Morton-ordered
 * first (at request sizes the ordering pays only for long nearest walks).
 * Times are seconds on abx_server_now()'s steady clock.  Reservations
 * (bytes, 256-B granules): per batch of M queries 12M + query scratch +
 * nearest 8Mk' | radius offsets 4(M+1), then 4*total for the fill; per
 * request its host results.
 * `simulate` = 1 runs the scheduler without HIP (each phase lasts
 * sim_ns_per_query * m ns, radius requests find 10 results per query): for
 * testing admission and accounting on a machine without a GPU. */
typedef enum { ABX_REQ_RADIUS = 0, ABX_REQ_NEAREST = 1 } abx_request_kind;

typedef struct {
  int32_t slots;          /* concurrent requests on the device, 1..64        */
  void *arena;            /* device buffer for request data (caller-owned)   */
  size_t arena_bytes;     /* its size: the HBM budget of in-flight requests  */
  size_t host_bytes;      /* pinned host result arena allocated by the server */
  int32_t poll_us;        /* scheduler sleep when idle-polling (0: 20 us)    */
  int32_t simulate;
  double sim_ns_per_query;
  int64_t merge_queries;  /* a merged launch holds at most this many queries
                             (0: 65536; < 0: no merging)                     */
  int64_t small_queries;  /* requests of at most this many queries are
                             "small", and the two size classes may pass
                             each other (0: 16384)                          */
  int64_t merge_large;    /* large requests of one class queued together are
                             merged up to this many queries (0: 4 x
                             merge_queries; < 0: not merged)                */
} abx_server_config;

typedef struct {
  int32_t tree;            /* id from abx_server_add_tree                    */
  abx_request_kind kind;
  const float *queries;    /* HOST [m,3]; read while the request runs         */
  int64_t m;
  float radius;            /* radius requests                                */
  int32_t k;               /* nearest requests, 0..128                       */
  double t_arrival;        /* caller's arrival time (abx_server_now clock)   */
} abx_request;

typedef struct {
  abx_status status;
  int64_t m, total;                /* rows and result entries               */
  const int32_t *offsets;          /* HOST [m+1] (pinned arena)             */
  const int32_t *indices;          /* HOST [total]                          */
  const float *distances;          /* HOST [total] (nearest) or NULL        */
  double t_arrival, t_admit, t_done;
  double t_device;                 /* GPU time of the phases of the request's
                                      batch (s): copies and kernels, from
                                      events on its stream; excludes
                                      queueing and the wait for the fill's
                                      memory                                */
} abx_result;

typedef struct {
  int64_t submitted, completed, failed, queries, max_in_flight, in_flight, queued;
  size_t device_high_water, host_high_water;
  int64_t requeued;        /* radius requests sent back to the queue after
                              their count: fills that waited on each other's
                              reservations (the earliest keeps its slot)   */
  int64_t batches;         /* launch sequences: one per admitted batch of
                              merged requests                               */
} abx_server_stats;

typedef struct abx_server abx_server;

abx_status abx_server_create(const abx_server_config *cfg, abx_server **out /*host*/);
abx_status abx_server_add_tree(abx_server *srv, const abx_bvh *tree, int32_t *id /*host*/);
/* Queues a copy of *req; returns at once.  ABX_ERR_CAPACITY is reported in
 * the result of a request whose reservation can never fit: at admission, one
 * larger than an arena; at the fill, one whose result space does not fit
 * while nothing else holds either arena.  A fill that waits for host space
 * held by results not yet released waits for abx_server_release.  Requests
 * can complete before requests submitted ahead of them (batches run on
 * several slots at once, and merged requests finish with their batch), so a
 * caller whose host arena cannot hold the results in flight must release
 * results in the order they complete (poll), not wait for them in submission
 * order. */
abx_status abx_server_submit(abx_server *srv, const abx_request *req, uint64_t *ticket /*host*/);
/* ABX_PENDING until the request has completed (results host-visible). */
abx_status abx_server_poll(abx_server *srv, uint64_t ticket, abx_result *out /*host*/);
abx_status abx_server_wait(abx_server *srv, uint64_t ticket, abx_result *out /*host*/);
abx_status abx_server_release(abx_server *srv, uint64_t ticket);
abx_status abx_server_drain(abx_server *srv);
abx_status abx_server_get_stats(abx_server *srv, abx_server_stats *out /*host*/);
/* Stops the scheduler: requests not yet on the device fail, running ones
 * complete; then frees the streams and the pinned host arena. */
abx_status abx_server_destroy(abx_server *srv);
double abx_server_now(void);

/* -- diagnostics -------------------------------------------------------------
 * abx_timing_enable(1) brackets every kernel launch with HIP events on the
 *   launch stream (not on a stream that is being captured into a graph);
 *   abx_timing_get(name) returns the summed milliseconds and launch count
 *   of the kernels called `name` since the last reset (the host waits on
 *   the events).  The switch and the totals are process-wide and may be
 *   used from any thread; for measurement only. */
/* abx_inject_fault: a test hook for failure handling.  The (skip + 1)-th
 *   next event of `kind` fails as a HIP failure would, once: LAUNCH, a
 *   kernel launch (nothing is launched; the call returns ABX_ERR_HIP) or a
 *   phase of the server's simulated executor; HOST_ALLOC, the pinned host
 *   arena of abx_server_create.  skip < 0 disarms.  Process-wide. */
typedef enum { ABX_FAULT_LAUNCH = 0, ABX_FAULT_HOST_ALLOC = 1 } abx_fault_kind;
abx_status abx_inject_fault(int32_t kind, int64_t skip);
const char *abx_status_string(abx_status s);
int abx_last_hip_error(void);
const char *abx_version(void);
void abx_timing_enable(int on);
void abx_timing_reset(void);
abx_status abx_timing_get(const char *kernel, double *ms /*host*/, int64_t *launches /*host*/);

#ifdef __cplusplus
}
#endif
#endif /* ABX_H */
