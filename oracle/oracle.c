/*
 * oracle.c -- CPU reference for the LBVH geometric search path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP path.
 *
 * Everything here is the plain definition of what the method computes,
 * written for a reader to check by eye against the ArborX paper
 * (arXiv:1908.11807):
 *
 *   - scene box, Morton codes     : section 2.1 "Calculate the scene bounding
 *                                   box", "Assign Morton codes for each AABB"
 *   - hierarchy                   : section 2.1 "Generate the bounding volume
 *                                   hierarchy" -- recursive partition of the
 *                                   sorted (index-augmented) codes at their
 *                                   highest differing bit, nodes numbered as in
 *                                   Karras (2012), which the paper adopts
 *   - internal node boxes         : section 2.1 "Calculate internal nodes
 *                                   bounding boxes" -- each box is the union of
 *                                   its children's boxes
 *   - spatial / nearest queries   : section 2.2 -- "all objects within a certain
 *                                   distance" and "a certain number of closest
 *                                   objects", by brute force in double
 *                                   precision on the exact float inputs
 *
 * Floating point: the Morton normalisation is the only step where float32
 * arithmetic decides an integer; it is written in float and this file is
 * compiled with -ffp-contract=off so that no fused multiply-add changes a
 * rounding.  Distances are double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KIND_POINTS 0 /* [n,3]  x y z                     */
#define KIND_BOXES 1  /* [n,6]  lo x y z, hi x y z          */

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Lower and upper corner of primitive i (a point is a degenerate box:
 * section 2.1 "Construct AABBs"). */
static void prim_box(const float *p, int kind, int64_t i, float lo[3], float hi[3]) {
  for (int a = 0; a < 3; ++a) {
    if (kind == KIND_POINTS) {
      lo[a] = p[3 * i + a];
      hi[a] = p[3 * i + a];
    } else {
      lo[a] = p[6 * i + a];
      hi[a] = p[6 * i + 3 + a];
    }
  }
}

/* ---------------------------------------------------------------------------
 * Scene box: reduction of the corners of all primitive boxes (section 2.1).
 * Returns 1 if any coordinate is NaN or infinite, or a box has lo > hi on
 * some axis (then `out` is unspecified), else 0.  n = 0 gives the empty box
 * lo = +inf, hi = -inf.
 * ------------------------------------------------------------------------- */
int oracle_scene_box(const float *prims, int64_t n, int kind, float out[6]) {
  for (int a = 0; a < 3; ++a) {
    out[a] = INFINITY;
    out[3 + a] = -INFINITY;
  }
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    float lo[3], hi[3];
    prim_box(prims, kind, i, lo, hi);
    for (int a = 0; a < 3; ++a) {
      if (!isfinite(lo[a]) || !isfinite(hi[a]) || lo[a] > hi[a]) bad = 1;
      if (lo[a] < out[a]) out[a] = lo[a];
      if (hi[a] > out[3 + a]) out[3 + a] = hi[a];
    }
  }
  return bad;
}

/* ---------------------------------------------------------------------------
 * Morton code of each primitive (section 2.1 "Assign Morton codes").
 *
 * The centroid (a point itself; for a box, half the sum of its corners) is
 * scaled by the scene box into [0,1]^3, each coordinate is quantised to
 * `bits` bits, and the bits are interleaved from the most significant down,
 * x before y before z within each triple.  The paper fixes neither the number
 * of bits nor the interleave order nor the float steps; the readings used:
 *
 *   inv_a = 1 / (hi_a - lo_a)  in float, or 0 when the extent is 0
 *   u_a   = clamp((c_a - lo_a) * inv_a, 0, 1)  in float
 *   q_a   = min(floor(u_a * 2^bits), 2^bits - 1)
 *
 * bits = 10 gives 30-bit codes, bits = 21 gives 63-bit codes.
 * ------------------------------------------------------------------------- */
void oracle_morton(const float *prims, int64_t n, int kind, const float scene[6], int bits,
                   uint64_t *codes) {
  float lo[3], inv[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = scene[a];
    float ext = scene[3 + a] - scene[a];
    inv[a] = ext > 0.0f ? 1.0f / ext : 0.0f;
  }
  const float scale = (float)(1u << bits); /* exact power of two */
  const uint32_t qmax = (1u << bits) - 1u;
  for (int64_t i = 0; i < n; ++i) {
    float blo[3], bhi[3];
    prim_box(prims, kind, i, blo, bhi);
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      float c = (kind == KIND_POINTS) ? blo[a] : 0.5f * (blo[a] + bhi[a]);
      float d = c - lo[a];
      float u = d * inv[a];
      if (!(u > 0.0f)) u = 0.0f; /* also maps NaN to 0 */
      if (u > 1.0f) u = 1.0f;
      float s = u * scale;
      uint32_t qa = (uint32_t)s; /* truncation toward zero, s >= 0 */
      q[a] = qa > qmax ? qmax : qa;
    }
    uint64_t code = 0;
    for (int b = bits - 1; b >= 0; --b) {
      code = (code << 1) | ((q[0] >> b) & 1u);
      code = (code << 1) | ((q[1] >> b) & 1u);
      code = (code << 1) | ((q[2] >> b) & 1u);
    }
    codes[i] = code;
  }
}

/* ---------------------------------------------------------------------------
 * Hierarchy (section 2.1 "Generate the bounding volume hierarchy").
 *
 * The sorted codes are made unique by appending each one's sorted position
 * (the paper's "augmented with an index").  An internal node owns a range
 * [f, l] of sorted positions; its split g is the last position whose
 * augmented code agrees with position f on the highest bit where f and l
 * differ.  Children cover [f, g] and [g+1, l].  A single-position range is a
 * leaf.  Node numbering follows Karras (2012): the root is internal node 0; a
 * child covering [f, g] is numbered g, a child covering [g+1, l] is numbered
 * g+1 (internal or leaf according to its range length).
 *
 * Output per internal node i (0 <= i < n-1):
 *   child_kind[2i+s]  = 0 leaf, 1 internal   (s = 0 left, 1 right)
 *   child_index[2i+s] = leaf position or internal node number
 *   range[2i], range[2i+1] = f, l
 * ------------------------------------------------------------------------- */

/* bit b (0 = most significant) of the augmented key of position i:
 * `keybits` code bits followed by 32 bits of the position */
static int aug_bit(const uint64_t *codes, int keybits, int64_t i, int b) {
  if (b < keybits) return (int)((codes[i] >> (keybits - 1 - b)) & 1u);
  return (int)(((uint64_t)i >> (31 - (b - keybits))) & 1u);
}

/* number of leading bits on which the augmented keys of i and j agree */
static int aug_common_prefix(const uint64_t *codes, int keybits, int64_t i, int64_t j) {
  int b = 0;
  while (b < keybits + 32 && aug_bit(codes, keybits, i, b) == aug_bit(codes, keybits, j, b)) ++b;
  return b;
}

static void split_range(const uint64_t *codes, int keybits, int64_t f, int64_t l, int64_t node,
                        int8_t *child_kind, int64_t *child_index, int64_t *range) {
  range[2 * node] = f;
  range[2 * node + 1] = l;
  int b = aug_common_prefix(codes, keybits, f, l); /* first differing bit */
  int64_t g = f;
  while (g + 1 <= l && aug_bit(codes, keybits, g + 1, b) == 0) ++g;
  /* left child [f, g] */
  if (g == f) {
    child_kind[2 * node] = 0;
    child_index[2 * node] = g;
  } else {
    child_kind[2 * node] = 1;
    child_index[2 * node] = g;
    split_range(codes, keybits, f, g, g, child_kind, child_index, range);
  }
  /* right child [g+1, l] */
  if (g + 1 == l) {
    child_kind[2 * node + 1] = 0;
    child_index[2 * node + 1] = g + 1;
  } else {
    child_kind[2 * node + 1] = 1;
    child_index[2 * node + 1] = g + 1;
    split_range(codes, keybits, g + 1, l, g + 1, child_kind, child_index, range);
  }
}

void oracle_hierarchy(const uint64_t *sorted_codes, int64_t n, int keybits, int8_t *child_kind,
                      int64_t *child_index, int64_t *range) {
  if (n < 2) return;
  split_range(sorted_codes, keybits, 0, n - 1, 0, child_kind, child_index, range);
}

/* ---------------------------------------------------------------------------
 * Internal node boxes (section 2.1 "Calculate internal nodes bounding boxes"):
 * the box of a node is the union of its children's boxes; a leaf's box is its
 * primitive's box.  `perm[p]` is the original index of the primitive at sorted
 * position p.  Output: boxes[6*i .. 6*i+5] for internal node i.
 * ------------------------------------------------------------------------- */
static void node_box(const float *prims, int kind, const int64_t *perm, const int8_t *child_kind,
                     const int64_t *child_index, int is_internal, int64_t idx, float *boxes,
                     float out[6]) {
  if (!is_internal) {
    prim_box(prims, kind, perm[idx], out, out + 3);
    return;
  }
  float a[6], b[6];
  node_box(prims, kind, perm, child_kind, child_index, child_kind[2 * idx], child_index[2 * idx],
           boxes, a);
  node_box(prims, kind, perm, child_kind, child_index, child_kind[2 * idx + 1],
           child_index[2 * idx + 1], boxes, b);
  for (int k = 0; k < 3; ++k) {
    out[k] = a[k] < b[k] ? a[k] : b[k];
    out[3 + k] = a[3 + k] > b[3 + k] ? a[3 + k] : b[3 + k];
  }
  memcpy(boxes + 6 * idx, out, 6 * sizeof(float));
}

void oracle_refit(const float *prims, int kind, const int64_t *perm, int64_t n,
                  const int8_t *child_kind, const int64_t *child_index, float *boxes) {
  if (n < 2) return;
  float root[6];
  node_box(prims, kind, perm, child_kind, child_index, 1, 0, boxes, root);
}

/* ---------------------------------------------------------------------------
 * Distances (double precision on the exact float inputs).
 * Point primitive: Euclidean distance.  Box primitive: distance from the
 * query point to the nearest point of the box, i.e. the norm of the per-axis
 * gaps max(lo - q, 0, q - hi).
 * ------------------------------------------------------------------------- */
static double dist_to_prim(const float *prims, int kind, int64_t i, const float *q) {
  float lo[3], hi[3];
  prim_box(prims, kind, i, lo, hi);
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double qa = (double)q[a];
    double g = 0.0;
    if ((double)lo[a] - qa > g) g = (double)lo[a] - qa;
    if (qa - (double)hi[a] > g) g = qa - (double)hi[a];
    s += g * g;
  }
  return sqrt(s);
}

/* closed-interval overlap of primitive i with query box qb = lo xyz, hi xyz */
static int overlaps(const float *prims, int kind, int64_t i, const float *qb) {
  float lo[3], hi[3];
  prim_box(prims, kind, i, lo, hi);
  for (int a = 0; a < 3; ++a)
    if (!(lo[a] <= qb[3 + a] && qb[a] <= hi[a])) return 0;
  return 1;
}

/* ---------------------------------------------------------------------------
 * Spatial queries, count then fill (section 2.2, spatial traversal and the
 * CSR output of section 2.3).
 *   pred = 0: within(q, r), q = queries[3j..], r = radii ? radii[j] : radius;
 *             hit iff distance <= r (closed ball)
 *   pred = 1: intersects(box), box = queries[6j..]; closed intervals
 * Rows are written in increasing primitive index.
 * ------------------------------------------------------------------------- */
static int spatial_hit(const float *prims, int kind, int64_t i, int pred, const float *queries,
                       const float *radii, float radius, int64_t j) {
  if (pred == 0) {
    double r = (double)(radii ? radii[j] : radius);
    return dist_to_prim(prims, kind, i, queries + 3 * j) <= r;
  }
  return overlaps(prims, kind, i, queries + 6 * j);
}

void oracle_spatial_count(const float *prims, int64_t n, int kind, int pred, const float *queries,
                          int64_t m, const float *radii, float radius, int64_t *counts) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < m; ++j) {
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) c += spatial_hit(prims, kind, i, pred, queries, radii, radius, j);
    counts[j] = c;
  }
}

void oracle_spatial_fill(const float *prims, int64_t n, int kind, int pred, const float *queries,
                         int64_t m, const float *radii, float radius, const int64_t *offsets,
                         int64_t *indices) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < m; ++j) {
    int64_t o = offsets[j];
    for (int64_t i = 0; i < n; ++i)
      if (spatial_hit(prims, kind, i, pred, queries, radii, radius, j)) indices[o++] = i;
  }
}

/* distance of each primitive in `sel` (or all n when sel == NULL) from query
 * point q; used by tests to recompute distances of returned indices */
void oracle_distances(const float *prims, int kind, const float *q, const int64_t *sel,
                      int64_t cnt, double *out) {
  for (int64_t t = 0; t < cnt; ++t) out[t] = dist_to_prim(prims, kind, sel ? sel[t] : t, q);
}

/* ---------------------------------------------------------------------------
 * Nearest queries (section 2.2, nearest traversal): the min(k, n) primitives
 * closest to each query point, ordered by (distance, index) ascending --
 * distance ties go to the smaller index.  A sorted list of the best entries
 * seen so far is kept; each primitive is inserted if it precedes the list's
 * last entry.  Output rows have stride min(k, n).
 * ------------------------------------------------------------------------- */
void oracle_nearest(const float *prims, int64_t n, int kind, const float *queries, int64_t m,
                    int64_t k, int64_t *out_idx, double *out_dist) {
  int64_t kk = k < n ? k : n;
  if (kk <= 0) return;
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)kk);
    int64_t *bi = (int64_t *)malloc(sizeof(int64_t) * (size_t)kk);
#pragma omp for schedule(dynamic, 4)
    for (int64_t j = 0; j < m; ++j) {
      const float *q = queries + 3 * j;
      int64_t cnt = 0;
      for (int64_t i = 0; i < n; ++i) {
        double d = dist_to_prim(prims, kind, i, q);
        if (cnt == kk && !(d < bd[kk - 1] || (d == bd[kk - 1] && i < bi[kk - 1]))) continue;
        int64_t pos = cnt < kk ? cnt++ : kk - 1; /* slot freed at the end */
        while (pos > 0 && (d < bd[pos - 1] || (d == bd[pos - 1] && i < bi[pos - 1]))) {
          bd[pos] = bd[pos - 1];
          bi[pos] = bi[pos - 1];
          --pos;
        }
        bd[pos] = d;
        bi[pos] = i;
      }
      memcpy(out_dist + j * kk, bd, sizeof(double) * (size_t)kk);
      memcpy(out_idx + j * kk, bi, sizeof(int64_t) * (size_t)kk);
    }
    free(bd);
    free(bi);
  }
}
