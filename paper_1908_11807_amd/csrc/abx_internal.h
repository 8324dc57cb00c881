// Internal declarations of libabx: tree memory layout, device helpers shared
// by the construction and traversal kernels, and the host-side launch helper.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "abx.h"

namespace abx {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Tree memory (caller-owned, one buffer):
//   [0, 256)                 TreeHeader
//   [nodes_off, +(n-1)*NB)   internal nodes, NB = 64 (FP32) or 32 (Q16)
//   [leaves_off, +n*LB)      FP32 and Q16 point trees: int32 permutation,
//                            sorted position -> primitive index (LB=4);
//                            Q16 box trees: record i = primitive i's exact
//                            {lo xyz, hi xyz, sorted position, pad} (LB=32)
// Child references: r >= 0 is internal node r, r < 0 is a leaf holding
// primitive ~r (the hierarchy numbers leaves by sorted position; the refit
// rewrites leaf references to name the primitive, so traversal needs no
// permutation lookup).  Internal node 0 is the root (Karras numbering).
// ---------------------------------------------------------------------------
struct TreeHeader {
  float scene[6];     // scene box lo xyz, hi xyz
  float inv_ext[3];   // Morton normalisation: 1/(hi-lo) or 0
  float q_origin[3];  // Q16 grid: x = fmaf(q, q_scale, q_origin)
  float q_scale[3];
  int32_t bad;        // 1: NaN/inf coordinate or inverted box; 2: Q16 grid overflow; 4: refit
                      // bound or frontier exceeded; 8: depth-first order out of range;
                      // kBadSort: the sort's look-back gave up (hierarchy and refit skipped)
  int32_t height;     // longest root-to-leaf path (edges)
  int32_t root;       // internal node at the root (0 for the Karras numbering)
  int32_t node_count; // internal nodes stored (4-wide trees: fewer than n - 1)
  int32_t pad[45];
};
static_assert(sizeof(TreeHeader) == 256, "header is 256 B");
constexpr int32_t kBadSort = 16;

// FP32 internal node, 64 B: four 16-B words
//   a = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)
//   b = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
//   c = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)
//   d = (left ref, right ref, height(left), height(right))
struct __align__(16) NodeF32 {
  float4 a, b, c;
  int4 d;
};
static_assert(sizeof(NodeF32) == 64, "fp32 node is 64 B");

// Q16 internal node, 32 B: 12 uint16 coordinates then the two references
//   w[0..5] = L.lo.xy | L.lo.z L.hi.x | L.hi.yz | R.lo.xy | R.lo.z R.hi.x | R.hi.yz
//   (low half first), w[6] = left ref, w[7] = right ref.  In a point tree
//   a leaf child's three words hold the point's float32 x, y, z instead.
struct __align__(16) NodeQ16 {
  uint4 a, b;
};
static_assert(sizeof(NodeQ16) == 32, "q16 node is 32 B");

constexpr int kQ16Max = 65535;

// 4-wide Q16 node, 64 B: up to four children, each a 12-byte slot laid out
// like a Q16 child (6 uint16 coordinates, or a point leaf's float32 x y z),
// then the four references (kEmptyRef for an unused slot).  A 4-wide tree is
// the binary tree collapsed at even depths: a node at even depth keeps its
// children's children (a leaf child stays a leaf child), so a walk takes one
// dependent node load where the binary tree takes two.
struct __align__(16) NodeW {
  uint4 a, b, c, d;  // a..c: slots 0-3 (3 words each), d: references 0-3
};
static_assert(sizeof(NodeW) == 64, "4-wide node is 64 B");
constexpr int32_t kEmptyRef = INT32_MIN;  // never ~i for a primitive i < 2^31 - 1
// upper bound of the 4-wide nodes of ni binary internal nodes: every node at
// even depth but the root has a parent at odd depth, which has two children,
// so W - 1 <= 2 (ni - W)
inline int64_t wide_node_cap(int64_t ni) { return ni > 0 ? (2 * ni + 1) / 3 + 1 : 0; }

// Walk state a nearest query takes from the one-lane pass to the cooperative
// pass (int32 words per saved query): entry count (-1: restart from the
// root), pad, up to 64 (node, box distance) pairs (the next node and the
// lane's stack of unexplored subtrees), then the candidate list (64 keys of
// 64 bits).  A batch of m queries keeps the walks of its first
// min(m / 8 + 1, kMaxSavedHeavy) heavy queries; later ones, and walks with a
// deeper stack, restart from the root.
constexpr int kHeavyStateEntries = 64;
constexpr int kHeavyStateWords = 2 + 2 * kHeavyStateEntries + 2 * 64;
constexpr int64_t kMaxSavedHeavy = 65536;
inline int64_t heavy_state_cap(int64_t m) {
  const int64_t c = m / 8 + 1;
  return c < kMaxSavedHeavy ? c : kMaxSavedHeavy;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Device helpers.  One float32 formula for the squared point-to-box distance
// is used for internal-node boxes and leaves alike (fixed contraction: the
// x term is a plain product, y and z are fused), so the box value never
// exceeds the value of any primitive inside the box (rounding is monotone):
// pruning is conservative and the result is exactly the set of leaves that
// pass the float32 leaf test, whatever the node format.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float axis_gap(float lo, float hi, float q) {
  return fmaxf(fmaxf(lo - q, q - hi), 0.0f);
}

__device__ __forceinline__ float box_dist2(float lx, float ly, float lz, float hx, float hy, float hz,
                                           float qx, float qy, float qz) {
  float gx = axis_gap(lx, hx, qx);
  float gy = axis_gap(ly, hy, qy);
  float gz = axis_gap(lz, hz, qz);
  return __fmaf_rn(gz, gz, __fmaf_rn(gy, gy, gx * gx));
}

// closed-interval overlap of two boxes
__device__ __forceinline__ bool box_overlap(float lx, float ly, float lz, float hx, float hy, float hz,
                                            float ax, float ay, float az, float bx, float by, float bz) {
  return lx <= bx && ax <= hx && ly <= by && ay <= hy && lz <= bz && az <= hz;
}

// Q16 dequantisation (the construction guarantees outward containment for
// exactly this expression)
__device__ __forceinline__ float deq(uint32_t q, float scale, float origin) {
  return __fmaf_rn((float)q, scale, origin);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
abx_status hip_fail(hipError_t e);  // records e for abx_last_hip_error
bool stream_capturing(hipStream_t s);
bool timing_on(hipStream_t s);      // event timing enabled, `s` not capturing, events allowed
void timing_record(const char *name, hipEvent_t a, hipEvent_t b);

// Injected faults (abx_inject_fault): true when this event of the kind is
// the one armed to fail
bool fault_hit(int kind);

// While one exists on a thread, launches from that thread create no events
// (entry points that promise to allocate nothing).
extern thread_local int g_no_events;
struct NoEventsScope {
  NoEventsScope() { ++g_no_events; }
  ~NoEventsScope() { --g_no_events; }
  NoEventsScope(const NoEventsScope &) = delete;
  NoEventsScope &operator=(const NoEventsScope &) = delete;
};

#define ABX_TRY(expr)                         \
  do {                                        \
    abx_status _s = (expr);                   \
    if (_s != ABX_OK) return _s;              \
  } while (0)

#define ABX_HIP(expr)                         \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return hip_fail(_e);\
  } while (0)

// Launch `f` (which enqueues one kernel on `s`) and, in timing mode, bracket
// it with events recorded on the same stream.
template <typename F>
abx_status launch(const char *name, hipStream_t s, F &&f) {
  hipEvent_t a = nullptr, b = nullptr;
  const bool timed = timing_on(s);
  if (timed) {
    ABX_HIP(hipEventCreate(&a));
    ABX_HIP(hipEventCreate(&b));
    ABX_HIP(hipEventRecord(a, s));
  }
  if (fault_hit(ABX_FAULT_LAUNCH)) {  // a test's injected failure: nothing is launched
    if (timed) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
    return hip_fail(hipErrorLaunchFailure);
  }
  f();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  if (timed) {
    ABX_HIP(hipEventRecord(b, s));
    timing_record(name, a, b);
  }
  return ABX_OK;
}

inline unsigned grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

// fill kernel (graph-safe replacement for hipMemsetAsync)
abx_status fill_u32(void *p, uint32_t value, size_t count, hipStream_t s);

// radix sort (sort.hip).  A look-back wait that gives up marks a word of the
// sort's own scratch (cleared by every sort, found with radix_sort_err_word,
// which is NULL when n <= 1: nothing waits) and, if err is given, ORs
// err_bit into *err: the output is then not a valid permutation, though
// every store stayed inside the buffers.
size_t radix_sort_scratch_bytes(int64_t n, int key_bits);
abx_status radix_sort(const void *keys_in, const int32_t *vals_in, int64_t n, int key_bits,
                      void *keys_out, int32_t *vals_out, void *scratch, size_t scratch_bytes,
                      hipStream_t s, uint32_t *err = nullptr, uint32_t err_bit = 1);
uint32_t *radix_sort_err_word(void *scratch, int64_t n, int key_bits);
// after a sort into order[0..m): if *err is set, order becomes the identity
// (queries in input order give the same results, only slower)
abx_status order_guard(const uint32_t *err, int32_t *order, int64_t m, hipStream_t s);

// exclusive scan of int32 counts into int32 offsets[0..m] (scan.hip);
// total (int64) is written to *d_total
size_t scan_scratch_bytes(int64_t m);
abx_status exclusive_scan(const int32_t *counts, int64_t m, int32_t *offsets, int64_t *d_total,
                          void *scratch, size_t scratch_bytes, hipStream_t s);

}  // namespace abx

// Opaque handle definition (host memory).
// State of a one-pass (1P) spatial query in the caller's scratch: the stored
// rows, the overflow flag and the scanned total, and the caller's capacity.
struct OnePass {
  int32_t *buf;          // [m * bufsize]
  int32_t bufsize;
  uint32_t *flag;        // [0] overflow seen
  const int64_t *total;
  int64_t capacity;
};

struct abx_bvh {
  int64_t n;
  int32_t kind, format, morton_bits, height;
  int32_t hierarchy, root;  // construction used; internal node at the root
  int32_t node_order;       // abx_node_order: BUILD or DEPTH_FIRST
  int64_t nint;             // internal nodes stored (n - 1, fewer for 4-wide nodes)
  float scene[6];
  float q_origin[3], q_scale[3];
  char *tree;  // device base
  size_t tree_bytes;
  size_t nodes_off, leaves_off, node_bytes, leaf_bytes;
  const abx::TreeHeader *hdr() const { return reinterpret_cast<const abx::TreeHeader *>(tree); }
  const void *nodes() const { return tree + nodes_off; }
  const void *leaves() const { return tree + leaves_off; }
};
