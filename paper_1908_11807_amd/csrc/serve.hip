// Serving loop: continuous batching of query requests against device-resident
// trees (a tree is built once and queried many times, section 2.2).
//
// A scheduler thread owns `slots` HIP streams.  Requests wait in a FIFO; the
// head is admitted as soon as a slot is free AND its device reservation fits
// in the caller's HBM arena (the budget), so requests that arrive while
// others run start as slots and memory free up, and their kernels overlap on
// the device.  A nearest request is one phase (copy in, order, walk, copy
// out).  A radius request is two (section 2.2, count-and-fill): the count
// phase ends with its total in pinned host memory; the scheduler then
// reserves exactly the result space and launches the fill phase.  Results
// land in a pinned host arena the server allocates once; they stay there
// until the caller releases them.  Completion is detected by polling the
// slot's event; timestamps (arrival given by the caller, admission, host-
// visible completion) use one steady clock (abx_server_now).
//
// In simulation mode no HIP call is made: each phase completes after
// `sim_ns_per_query * m` nanoseconds and a radius request finds 10 results
// per query.  The admission, memory and latency bookkeeping is the same code.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "abx_internal.h"

namespace abx {
size_t query_scratch_bytes(int64_t m);
size_t nearest_scratch_bytes(int64_t m);
abx_status spatial_count_enqueue(const abx_bvh *bvh, const abx_predicates *p, char *sc,
                                 int32_t *offsets, int64_t **d_total, hipStream_t s);
abx_status spatial_fill_enqueue(const abx_bvh *bvh, const abx_predicates *p, char *sc,
                                const int32_t *offsets, int32_t *indices, hipStream_t s);
abx_status nearest_enqueue(const abx_bvh *bvh, const float *pts, int64_t m, int32_t k, int sort,
                           char *sc, int32_t *offsets, int32_t *indices, float *dist, hipStream_t s);
}  // namespace abx

using namespace abx;

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

constexpr size_t kGrain = 256;

// first-fit allocator over [0, size) in kGrain units, coalescing on release
class Arena {
 public:
  void reset(size_t size) {
    size_ = size / kGrain * kGrain;
    free_.clear();
    if (size_) free_[0] = size_;
    used_ = high_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(std::max<size_t>(bytes, 1), kGrain);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        high_ = std::max(high_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, 1), kGrain);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t high() const { return high_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0, high_ = 0;
};

struct Block {
  size_t off = 0, bytes = 0;
  bool held = false;
};

enum Phase { P_QUEUED, P_RUN_A, P_WAIT_FILL, P_RUN_B, P_DONE };

struct Batch;

struct Req {
  uint64_t ticket;
  abx_request r;
  Phase phase = P_QUEUED;
  Batch *batch = nullptr;
  int64_t kk = 0, total = 0;
  int64_t base = 0;           // first row of the request in its batch
  int64_t row0 = 0;           // radius: the batch offset at `base` (its first result)
  abx_status status = ABX_OK;
  double t_admit = 0, t_done = 0;
  double t_device = 0;        // summed GPU time of the phases of its batch
  Block host;                 // results, pinned host arena
  int32_t *h_off = nullptr, *h_idx = nullptr;
  float *h_dist = nullptr;
};

// Requests on one tree with the same predicate (kind and k, or radius) run
// as one launch sequence over their concatenated queries.  Each row's result
// depends only on its own query, so a request's rows are the same alone or
// merged (results are copied back per request).
struct Batch {
  std::vector<Req *> reqs;
  int32_t tree = 0;
  abx_request_kind kind = ABX_REQ_NEAREST;
  int32_t k = 0;
  float radius = 0.0f;
  int64_t kk = 0, M = 0, total = 0;
  bool large = false;
  Phase phase = P_RUN_A;
  int slot = -1;
  Block dev_a, dev_b;
  double sim_deadline = 0;
  float *d_q = nullptr;
  char *d_scratch = nullptr;
  int32_t *d_off = nullptr, *d_idx = nullptr;
  float *d_dist = nullptr;
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;        // completion (polled)
  hipEvent_t t0 = nullptr, t1 = nullptr;  // timing: start and end of a phase
  Batch *b = nullptr;
};

}  // namespace

struct abx_server {
  abx_server_config cfg;
  int device = 0;
  // resolved merge limits (0: no merging): small batches, large batches
  int64_t merge_queries = 0, small_queries = 0, merge_large = 0;
  std::vector<const abx_bvh *> trees;
  std::vector<Slot> slots;
  Arena dev, host;
  char *dev_base = nullptr, *host_base = nullptr;
  std::deque<Req *> queue;
  std::unordered_map<uint64_t, Req *> reqs;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::thread th;
  bool stop = false;
  abx_server_stats st{};
  int in_flight = 0;
};

namespace {

constexpr int kMaxBatchRequests = 64;

bool same_class(const Req *a, const Req *b) {
  if (a->r.tree != b->r.tree || a->r.kind != b->r.kind) return false;
  if (a->r.kind == ABX_REQ_NEAREST) return a->kk == b->kk;
  return std::memcmp(&a->r.radius, &b->r.radius, sizeof(float)) == 0;
}

bool is_large(const abx_server *S, const Req *q) { return q->r.m > S->small_queries; }

// Query ordering per batch.  At request sizes (up to ~1e5 queries) the
// ordering's sort costs 60-90 us, measured against 1e7-point trees: radius
// requests never win it back (their walks are short), nearest requests do
// from ~1e4 queries where walks are long (a shell: 3.5 vs 4.4 ms at 1e4
// queries, k = 8), and lose it below.
constexpr int64_t kServeSortMin = 4096;
int sort_batch(const Batch *b) { return b->kind == ABX_REQ_NEAREST && b->M >= kServeSortMin ? 1 : 0; }

size_t batch_scratch_bytes(const Batch *b) {
  return b->kind == ABX_REQ_NEAREST ? nearest_scratch_bytes(b->M) : query_scratch_bytes(b->M);
}

// device reservation of a batch's first phase: queries, query scratch and
// the nearest results or the radius offsets
size_t dev_bytes_a(const Batch *b) {
  const int64_t M = b->M;
  size_t n = align_up((size_t)M * 12, kGrain) + align_up(batch_scratch_bytes(b), kGrain);
  if (b->kind == ABX_REQ_NEAREST) n += 2 * align_up((size_t)(M * b->kk) * 4, kGrain);
  else n += align_up((size_t)(M + 1) * 4, kGrain);
  return n;
}

// host reservation of one request's first phase: offsets (+ nearest results)
size_t host_bytes_a(const Req *q) {
  const int64_t m = q->r.m;
  size_t b = align_up((size_t)(m + 1) * 4, kGrain) + kGrain;
  if (q->r.kind == ABX_REQ_NEAREST) b += 2 * align_up((size_t)(m * q->kk) * 4, kGrain);
  return b;
}

void release_block(Arena &a, Block &b) {
  if (b.held) {
    a.release(b.off, b.bytes);
    b.held = false;
  }
}

bool take(Arena &a, Block &b, size_t bytes) {
  size_t off;
  if (!a.alloc(bytes, &off)) return false;
  b.off = off;
  b.bytes = bytes;
  b.held = true;
  return true;
}

void finish(abx_server *S, Req *q, abx_status status) {
  q->status = status;
  q->phase = P_DONE;
  q->t_done = now_s();
  q->batch = nullptr;
  if (status != ABX_OK) release_block(S->host, q->host);
  S->in_flight--;
  if (status == ABX_OK) {
    S->st.completed++;
    S->st.queries += q->r.m;
  } else {
    S->st.failed++;
  }
  S->cv_done.notify_all();
}

// ends a batch: every member finishes with `status` (OK: its results are
// in place), the batch's memory and slot are released.  After a failure
// part of the batch's work may still be enqueued: the slot's stream is
// drained first, so no copy or kernel touches memory handed to another batch.
void finish_batch(abx_server *S, Batch *b, abx_status status) {
  if (status != ABX_OK && !S->cfg.simulate && b->slot >= 0) (void)hipStreamSynchronize(S->slots[b->slot].s);
  for (Req *q : b->reqs) finish(S, q, status);
  release_block(S->dev, b->dev_a);
  release_block(S->dev, b->dev_b);
  if (b->slot >= 0) S->slots[b->slot].b = nullptr;
  delete b;
}

abx_status launch_a(abx_server *S, Batch *b) {
  const abx_bvh *tree = S->trees[b->tree];
  const int64_t M = b->M;
  char *d = S->dev_base + b->dev_a.off;
  b->d_q = reinterpret_cast<float *>(d);
  d += align_up((size_t)M * 12, kGrain);
  b->d_scratch = d;
  d += align_up(batch_scratch_bytes(b), kGrain);
  if (b->kind == ABX_REQ_NEAREST) {
    b->d_idx = reinterpret_cast<int32_t *>(d);
    d += align_up((size_t)(M * b->kk) * 4, kGrain);
    b->d_dist = reinterpret_cast<float *>(d);
  } else {
    b->d_off = reinterpret_cast<int32_t *>(d);
  }
  for (Req *q : b->reqs) {
    char *h = S->host_base + q->host.off;
    q->h_off = reinterpret_cast<int32_t *>(h);
    h += align_up((size_t)(q->r.m + 1) * 4, kGrain) + kGrain;
    if (b->kind == ABX_REQ_NEAREST) {
      q->h_idx = reinterpret_cast<int32_t *>(h);
      h += align_up((size_t)(q->r.m * q->kk) * 4, kGrain);
      q->h_dist = reinterpret_cast<float *>(h);
    }
  }
  if (S->cfg.simulate) {
    // the simulated executor's stand-in for a failed launch
    if (fault_hit(ABX_FAULT_LAUNCH)) return hip_fail(hipErrorLaunchFailure);
    b->sim_deadline = now_s() + 1e-9 * S->cfg.sim_ns_per_query * (double)(M > 0 ? M : 1);
    return ABX_OK;
  }
  Slot &sl = S->slots[b->slot];
  ABX_HIP(hipEventRecord(sl.t0, sl.s));
  for (Req *q : b->reqs)
    if (q->r.m > 0)
      ABX_HIP(hipMemcpyAsync(b->d_q + 3 * q->base, q->r.queries, (size_t)q->r.m * 12,
                             hipMemcpyHostToDevice, sl.s));
  if (b->kind == ABX_REQ_NEAREST) {
    ABX_TRY(nearest_enqueue(tree, b->d_q, M, b->k, sort_batch(b), b->d_scratch, nullptr, b->d_idx,
                            b->d_dist, sl.s));
    for (Req *q : b->reqs) {
      const size_t ob = (size_t)(q->r.m * b->kk) * 4;
      if (!ob) continue;
      ABX_HIP(hipMemcpyAsync(q->h_idx, b->d_idx + q->base * b->kk, ob, hipMemcpyDeviceToHost, sl.s));
      ABX_HIP(hipMemcpyAsync(q->h_dist, b->d_dist + q->base * b->kk, ob, hipMemcpyDeviceToHost, sl.s));
    }
  } else {
    abx_predicates p{ABX_PRED_WITHIN, b->d_q, M, nullptr, b->radius, sort_batch(b)};
    int64_t *d_total = nullptr;
    ABX_TRY(spatial_count_enqueue(tree, &p, b->d_scratch, b->d_off, &d_total, sl.s));
    // each request's slice of the offsets: its row count and first result
    for (Req *q : b->reqs)
      ABX_HIP(hipMemcpyAsync(q->h_off, b->d_off + q->base, (size_t)(q->r.m + 1) * 4,
                             hipMemcpyDeviceToHost, sl.s));
  }
  ABX_HIP(hipEventRecord(sl.t1, sl.s));
  ABX_HIP(hipEventRecord(sl.ev, sl.s));
  return ABX_OK;
}

// fill phase of a radius batch: reserve the exact result space (device: the
// batch's indices; host: each request's offsets and indices), launch
bool try_launch_b(abx_server *S, Batch *b, abx_status *err) {
  const size_t ib = align_up((size_t)b->total * 4, kGrain);
  if (!take(S->dev, b->dev_b, ib)) return false;
  std::vector<Block> hb(b->reqs.size());
  for (size_t i = 0; i < b->reqs.size(); ++i) {
    const Req *q = b->reqs[i];
    if (!take(S->host, hb[i], align_up((size_t)(q->r.m + 1) * 4, kGrain) + align_up((size_t)q->total * 4, kGrain))) {
      for (size_t j = 0; j < i; ++j) release_block(S->host, hb[j]);
      release_block(S->dev, b->dev_b);
      return false;
    }
  }
  for (size_t i = 0; i < b->reqs.size(); ++i) {
    Req *q = b->reqs[i];
    release_block(S->host, q->host);
    q->host = hb[i];
    char *h = S->host_base + q->host.off;
    q->h_off = reinterpret_cast<int32_t *>(h);
    q->h_idx = reinterpret_cast<int32_t *>(h + align_up((size_t)(q->r.m + 1) * 4, kGrain));
    q->h_dist = nullptr;
    q->phase = P_RUN_B;
  }
  b->d_idx = reinterpret_cast<int32_t *>(S->dev_base + b->dev_b.off);
  b->phase = P_RUN_B;
  if (S->cfg.simulate) {
    b->sim_deadline = now_s() + 1e-9 * S->cfg.sim_ns_per_query * (double)(b->M > 0 ? b->M : 1);
    return true;
  }
  Slot &sl = S->slots[b->slot];
  const abx_bvh *tree = S->trees[b->tree];
  abx_predicates p{ABX_PRED_WITHIN, b->d_q, b->M, nullptr, b->radius, sort_batch(b)};
  *err = ABX_OK;
  if (hipEventRecord(sl.t0, sl.s) != hipSuccess) *err = ABX_ERR_HIP;
  if (*err == ABX_OK) *err = spatial_fill_enqueue(tree, &p, b->d_scratch, b->d_off, b->d_idx, sl.s);
  for (Req *q : b->reqs) {
    if (*err != ABX_OK) break;
    if (hipMemcpyAsync(q->h_off, b->d_off + q->base, (size_t)(q->r.m + 1) * 4, hipMemcpyDeviceToHost,
                       sl.s) != hipSuccess)
      *err = ABX_ERR_HIP;
    if (*err == ABX_OK && q->total > 0 &&
        hipMemcpyAsync(q->h_idx, b->d_idx + q->row0, (size_t)q->total * 4, hipMemcpyDeviceToHost,
                       sl.s) != hipSuccess)
      *err = ABX_ERR_HIP;
  }
  if (*err == ABX_OK && hipEventRecord(sl.t1, sl.s) != hipSuccess) *err = ABX_ERR_HIP;
  if (*err == ABX_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) *err = ABX_ERR_HIP;
  return true;
}

bool phase_done(abx_server *S, const Batch *b) {
  if (S->cfg.simulate) return now_s() >= b->sim_deadline;
  const hipError_t e = hipEventQuery(S->slots[b->slot].ev);
  return e != hipErrorNotReady;
}

// after the count phase: each request's result count from its offset slice
// (simulated: 10 per query), the batch total; false if it overflows
bool count_results(abx_server *S, Batch *b) {
  int64_t T = 0;
  for (Req *q : b->reqs) {
    if (S->cfg.simulate) {
      q->row0 = T;
      q->total = 10 * q->r.m;
    } else {
      q->row0 = q->h_off[0];
      q->total = (int64_t)q->h_off[q->r.m] - q->h_off[0];
    }
    T += q->total;
  }
  b->total = T;
  return T < INT32_MAX;
}

void complete_batch(abx_server *S, Batch *b) {
  if (b->kind == ABX_REQ_NEAREST) {
    for (Req *q : b->reqs)
      for (int64_t i = 0; i <= q->r.m; ++i) q->h_off[i] = (int32_t)(i * q->kk);
  } else if (!S->cfg.simulate) {
    // the offsets of the batch, rebased to each request's first result
    for (Req *q : b->reqs)
      for (int64_t i = 0; i <= q->r.m; ++i) q->h_off[i] -= (int32_t)q->row0;
  }
  finish_batch(S, b, ABX_OK);
}

// The batch a request heads: itself and the later queued requests of its
// class and size class (in queue order) while the batch stays within the
// merge limit of that size class.  Members leave the queue.  Large requests
// find others queued beside them only when the slots are behind, so their
// merging acts under backlog: one launch sequence over more queries fills
// the GPU better than several overlapping ones.
Batch *form_batch(abx_server *S, std::deque<Req *>::iterator head) {
  Req *h = *head;
  Batch *b = new (std::nothrow) Batch;
  if (!b) return nullptr;
  b->tree = h->r.tree;
  b->kind = h->r.kind;
  b->k = h->r.k;
  b->radius = h->r.radius;
  b->kk = h->kk;
  b->large = is_large(S, h);
  b->reqs.push_back(h);
  b->M = h->r.m;
  auto it = S->queue.erase(head);
  const int64_t limit = b->large ? S->merge_large : S->merge_queries;
  if (limit > 0) {
    while (it != S->queue.end() && (int)b->reqs.size() < kMaxBatchRequests) {
      Req *q = *it;
      if (is_large(S, q) == b->large && same_class(h, q) && b->M + q->r.m <= limit) {
        q->base = b->M;
        b->M += q->r.m;
        b->reqs.push_back(q);
        it = S->queue.erase(it);
      } else {
        ++it;
      }
    }
  }
  h->base = 0;
  return b;
}

// the queue in submission order (after requests went back to it)
void sort_queue(abx_server *S) {
  std::sort(S->queue.begin(), S->queue.end(), [](const Req *x, const Req *y) { return x->ticket < y->ticket; });
}

// returns a batch's requests to the queue, at their places by ticket
void requeue_batch(abx_server *S, Batch *b) {
  for (Req *q : b->reqs) {
    release_block(S->host, q->host);
    q->phase = P_QUEUED;
    q->batch = nullptr;
    q->total = 0;
    q->base = 0;
    S->in_flight--;
    S->st.requeued++;
    S->queue.push_back(q);
  }
  sort_queue(S);
  release_block(S->dev, b->dev_a);
  release_block(S->dev, b->dev_b);
  if (b->slot >= 0) S->slots[b->slot].b = nullptr;
  delete b;
}

// admits the batch headed by *head on slot `slot`: reserves its memory,
// launches its first phase; false (nothing changed) if the memory is not
// there
bool admit(abx_server *S, std::deque<Req *>::iterator head, int slot) {
  Req *h = *head;
  // a request that can never fit fails at once
  {
    Batch probe;
    probe.kind = h->r.kind;
    probe.kk = h->kk;
    probe.M = h->r.m;
    if (dev_bytes_a(&probe) > S->dev.size() || host_bytes_a(h) > S->host.size()) {
      S->queue.erase(head);
      S->in_flight++;
      finish(S, h, ABX_ERR_CAPACITY);
      return true;
    }
  }
  Batch *b = form_batch(S, head);
  if (!b) return false;
  // memory for the batch; members whose host space is not there go back
  bool ok = take(S->dev, b->dev_a, dev_bytes_a(b));
  std::vector<Req *> back;
  if (ok) {
    for (size_t i = 0; i < b->reqs.size(); ++i) {
      Req *q = b->reqs[i];
      if (!take(S->host, q->host, host_bytes_a(q))) {
        if (i == 0) ok = false;
        back.assign(b->reqs.begin() + (ptrdiff_t)i, b->reqs.end());
        b->reqs.resize(i);
        break;
      }
    }
  }
  if (!ok) {
    // nothing admitted: the requests return to their places at the front
    release_block(S->dev, b->dev_a);
    for (Req *q : b->reqs) release_block(S->host, q->host);
    for (Req *q : b->reqs) S->queue.push_back(q);
    for (Req *q : back) S->queue.push_back(q);
    sort_queue(S);
    delete b;
    return false;
  }
  if (!back.empty()) {
    // shrink the batch to the members that got host space; the rest requeue
    for (Req *q : back) S->queue.push_back(q);
    sort_queue(S);
    int64_t M = 0;
    for (Req *q : b->reqs) {
      q->base = M;
      M += q->r.m;
    }
    release_block(S->dev, b->dev_a);
    b->M = M;
    if (!take(S->dev, b->dev_a, dev_bytes_a(b))) {  // cannot happen: it shrank
      for (Req *q : b->reqs) {
        release_block(S->host, q->host);
        S->queue.push_back(q);
      }
      sort_queue(S);
      delete b;
      return false;
    }
  }
  const double t = now_s();
  b->slot = slot;
  b->phase = P_RUN_A;
  S->slots[slot].b = b;
  for (Req *q : b->reqs) {
    q->phase = P_RUN_A;
    q->batch = b;
    q->t_admit = t;
    S->in_flight++;
  }
  S->st.max_in_flight = std::max<int64_t>(S->st.max_in_flight, S->in_flight);
  S->st.batches++;
  const abx_status e = launch_a(S, b);
  if (e != ABX_OK) finish_batch(S, b, e);
  return true;
}

// one pass of the scheduler; returns true if anything changed
bool step(abx_server *S) {
  bool changed = false;
  size_t fill_need = 0;  // device bytes a waiting fill needs; admission leaves them free
  // 1. completions
  for (auto &sl : S->slots) {
    Batch *b = sl.b;
    if (!b) continue;
    if (b->phase == P_WAIT_FILL) {
      abx_status err = ABX_OK;
      if (try_launch_b(S, b, &err)) {
        changed = true;
        if (err != ABX_OK) finish_batch(S, b, err);
      } else {
        size_t hold = 0;
        for (Req *q : b->reqs) hold += q->host.bytes;
        if (S->dev.used() == b->dev_a.bytes && S->host.used() == hold) {
          // alone in both arenas and the result space still does not fit
          // (results the caller has not released hold host space: wait)
          finish_batch(S, b, ABX_ERR_CAPACITY);
          changed = true;
        } else {
          fill_need = std::max(fill_need, align_up((size_t)b->total * 4, kGrain));
        }
      }
      continue;
    }
    if (!phase_done(S, b)) continue;
    changed = true;
    if (!S->cfg.simulate && hipEventQuery(sl.ev) != hipSuccess) {
      finish_batch(S, b, ABX_ERR_HIP);
      continue;
    }
    double dt = 0.0;
    if (S->cfg.simulate) {
      dt = 1e-9 * S->cfg.sim_ns_per_query * (double)(b->M > 0 ? b->M : 1);
    } else {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, sl.t0, sl.t1) == hipSuccess) dt = 1e-3 * (double)ms;
    }
    for (Req *q : b->reqs) q->t_device += dt;
    if (b->phase == P_RUN_A && b->kind == ABX_REQ_RADIUS) {
      if (!count_results(S, b)) {
        finish_batch(S, b, ABX_ERR_OVERFLOW);
        continue;
      }
      abx_status err = ABX_OK;
      if (!try_launch_b(S, b, &err)) {
        b->phase = P_WAIT_FILL;
        for (Req *q : b->reqs) q->phase = P_WAIT_FILL;
        fill_need = std::max(fill_need, align_up((size_t)b->total * 4, kGrain));
      } else if (err != ABX_OK) {
        finish_batch(S, b, err);
      }
      continue;
    }
    complete_batch(S, b);
  }
  // 1b. fills that wait on each other: when every occupied slot holds a fill
  // waiting for memory, no running phase will free any, and each may be
  // blocked by the others' reservations.  The earliest batch keeps its slot;
  // the later ones give their reservations back and return to the head of
  // the queue (to be counted again once the earliest has finished).
  if (fill_need > 0) {
    Batch *keep = nullptr;
    bool running = false;
    for (auto &sl : S->slots) {
      if (!sl.b) continue;
      if (sl.b->phase != P_WAIT_FILL) running = true;
      else if (!keep || sl.b->reqs.front()->ticket < keep->reqs.front()->ticket) keep = sl.b;
    }
    if (!running && keep) {
      for (auto &sl : S->slots)
        if (sl.b && sl.b != keep) {
          requeue_batch(S, sl.b);
          changed = true;
        }
    }
  }
  // 2. admission.  The queue is served in order, each size class (small:
  // at most small_queries queries, large: more) first in first out, but a
  // request may pass one of the other class that cannot start: a large
  // request waits when slots - 1 large batches run (a slot stays for small
  // ones) or when its memory is not there, and small requests behind it go
  // ahead; the same the other way round.  While a fill waits for device
  // memory, a batch is admitted only if that memory stays free.
  int large_running = 0;
  for (auto &sl : S->slots)
    if (sl.b && sl.b->large) ++large_running;
  const int max_large = std::max(1, (int)S->slots.size() - 1);
  bool blocked[2] = {false, false};  // [large]
  for (auto it = S->queue.begin(); it != S->queue.end();) {
    int free_slot = -1;
    for (size_t i = 0; i < S->slots.size(); ++i)
      if (!S->slots[i].b) {
        free_slot = (int)i;
        break;
      }
    if (free_slot < 0) break;
    Req *q = *it;
    const bool large = is_large(S, q);
    if (blocked[large] || (large && large_running >= max_large)) {
      blocked[large] = true;
      if (blocked[0] && blocked[1]) break;
      ++it;
      continue;
    }
    if (fill_need > 0) {
      Batch probe;
      probe.kind = q->r.kind;
      probe.kk = q->kk;
      probe.M = q->r.m;
      if (S->dev.used() + dev_bytes_a(&probe) + fill_need > S->dev.size()) {
        blocked[large] = true;
        if (blocked[0] && blocked[1]) break;
        ++it;
        continue;
      }
    }
    // the iterator is invalidated by admission (members leave the queue):
    // restart from the front, where the earlier blocked requests are skipped
    // again by their class flags
    const ptrdiff_t pos = it - S->queue.begin();
    if (admit(S, it, free_slot)) {
      changed = true;
      if (large) ++large_running;
      // members left the queue: rescan from the front (the requests before
      // `pos` are of blocked classes and are skipped again)
      it = S->queue.begin();
    } else {
      // admit() put the requests back in ticket order, the failed head at `pos`
      blocked[large] = true;
      if (blocked[0] && blocked[1]) break;
      it = S->queue.begin() + pos + 1;
    }
  }
  S->st.device_high_water = S->dev.high();
  S->st.host_high_water = S->host.high();
  return changed;
}

// on shutdown: requests not yet on the device (queued, or waiting for fill
// memory the caller may never release) fail; running phases complete
void abandon_waiting(abx_server *S) {
  while (!S->queue.empty()) {
    Req *q = S->queue.front();
    S->queue.pop_front();
    S->in_flight++;
    finish(S, q, ABX_ERR_INVALID_ARG);
  }
  for (auto &sl : S->slots)
    if (sl.b && sl.b->phase == P_WAIT_FILL) finish_batch(S, sl.b, ABX_ERR_INVALID_ARG);
}

void scheduler(abx_server *S) {
  if (!S->cfg.simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    if (S->stop) abandon_waiting(S);
    const bool changed = step(S);
    const bool busy = S->in_flight > 0 || !S->queue.empty();
    if (S->stop && !busy) break;
    if (!busy) {
      S->cv_work.wait(lk);
      continue;
    }
    if (!changed) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(S->cfg.poll_us > 0 ? S->cfg.poll_us : 20));
      lk.lock();
    }
  }
}

void fill_result(const Req *q, abx_result *o) {
  o->status = q->status;
  o->m = q->r.m;
  o->total = q->r.kind == ABX_REQ_NEAREST ? q->r.m * q->kk : q->total;
  o->offsets = q->h_off;
  o->indices = q->h_idx;
  o->distances = q->h_dist;
  o->t_arrival = q->r.t_arrival;
  o->t_admit = q->t_admit;
  o->t_done = q->t_done;
  o->t_device = q->t_device;
}

}  // namespace

extern "C" {

double abx_server_now(void) { return now_s(); }

abx_status abx_server_create(const abx_server_config *cfg, abx_server **out) {
  if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->host_bytes == 0) return ABX_ERR_INVALID_ARG;
  if (!cfg->simulate && (!cfg->arena || (reinterpret_cast<uintptr_t>(cfg->arena) & 255)))
    return ABX_ERR_INVALID_ARG;
  abx_server *S = new (std::nothrow) abx_server;
  if (!S) return ABX_ERR_INVALID_ARG;
  S->cfg = *cfg;
  S->merge_queries = cfg->merge_queries == 0 ? 65536 : std::max<int64_t>(0, cfg->merge_queries);
  S->small_queries = cfg->small_queries > 0 ? cfg->small_queries : 16384;
  S->merge_large = cfg->merge_large == 0 ? 4 * std::min<int64_t>(S->merge_queries, INT64_MAX / 4)
                                          : std::max<int64_t>(0, cfg->merge_large);
  S->dev.reset(cfg->arena_bytes);
  S->host.reset(cfg->host_bytes);
  S->dev_base = static_cast<char *>(cfg->arena);
  if (fault_hit(ABX_FAULT_HOST_ALLOC)) {  // a test's injected allocation failure
    delete S;
    return hip_fail(hipErrorOutOfMemory);
  }
  if (!cfg->simulate) {
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&S->host_base), cfg->host_bytes, hipHostMallocDefault) != hipSuccess) {
      delete S;
      return ABX_ERR_HIP;
    }
    S->slots.resize(cfg->slots);
    for (auto &sl : S->slots) {
      if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
          hipEventCreate(&sl.t0) != hipSuccess || hipEventCreate(&sl.t1) != hipSuccess) {
        for (auto &x : S->slots) {
          if (x.t0) (void)hipEventDestroy(x.t0);
          if (x.t1) (void)hipEventDestroy(x.t1);
          if (x.ev) (void)hipEventDestroy(x.ev);
          if (x.s) (void)hipStreamDestroy(x.s);
        }
        (void)hipHostFree(S->host_base);
        delete S;
        return ABX_ERR_HIP;
      }
    }
  } else {
    S->host_base = static_cast<char *>(::operator new(cfg->host_bytes, std::nothrow));
    if (!S->host_base) {
      delete S;
      return ABX_ERR_HIP;
    }
    S->slots.resize(cfg->slots);
  }
  S->th = std::thread(scheduler, S);
  *out = S;
  return ABX_OK;
}

abx_status abx_server_add_tree(abx_server *S, const abx_bvh *tree, int32_t *id) {
  if (!S || (!tree && !S->cfg.simulate) || !id) return ABX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  S->trees.push_back(tree);
  *id = (int32_t)S->trees.size() - 1;
  return ABX_OK;
}

abx_status abx_server_submit(abx_server *S, const abx_request *r, uint64_t *ticket) {
  if (!S || !r || !ticket || r->m < 0 || (r->m > 0 && !r->queries && !S->cfg.simulate))
    return ABX_ERR_INVALID_ARG;
  if (r->kind != ABX_REQ_RADIUS && r->kind != ABX_REQ_NEAREST) return ABX_ERR_INVALID_ARG;
  if (r->kind == ABX_REQ_NEAREST && (r->k < 0 || r->k > 128)) return ABX_ERR_INVALID_ARG;
  if (r->m >= INT32_MAX) return ABX_ERR_OVERFLOW;
  Req *q = new (std::nothrow) Req;
  if (!q) return ABX_ERR_INVALID_ARG;
  q->r = *r;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->tree < 0 || r->tree >= (int32_t)S->trees.size()) {
      delete q;
      return ABX_ERR_INVALID_ARG;
    }
    const int64_t n = S->cfg.simulate ? INT32_MAX : S->trees[r->tree]->n;
    q->kk = r->kind == ABX_REQ_NEAREST ? std::min<int64_t>(r->k, n) : 0;
    if (r->m * q->kk >= INT32_MAX) {
      delete q;
      return ABX_ERR_OVERFLOW;
    }
    q->ticket = S->next_ticket++;
    S->reqs[q->ticket] = q;
    S->queue.push_back(q);
    S->st.submitted++;
  }
  S->cv_work.notify_one();
  *ticket = q->ticket;
  return ABX_OK;
}

abx_status abx_server_poll(abx_server *S, uint64_t ticket, abx_result *out) {
  if (!S || !out) return ABX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return ABX_ERR_INVALID_ARG;
  if (it->second->phase != P_DONE) return ABX_PENDING;
  fill_result(it->second, out);
  return ABX_OK;
}

abx_status abx_server_wait(abx_server *S, uint64_t ticket, abx_result *out) {
  if (!S || !out) return ABX_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return ABX_ERR_INVALID_ARG;
  Req *q = it->second;
  S->cv_done.wait(lk, [&] { return q->phase == P_DONE; });
  fill_result(q, out);
  return ABX_OK;
}

abx_status abx_server_release(abx_server *S, uint64_t ticket) {
  if (!S) return ABX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end() || it->second->phase != P_DONE) return ABX_ERR_INVALID_ARG;
  release_block(S->host, it->second->host);
  delete it->second;
  S->reqs.erase(it);
  S->cv_work.notify_one();
  return ABX_OK;
}

abx_status abx_server_drain(abx_server *S) {
  if (!S) return ABX_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->queue.empty() && S->in_flight == 0; });
  return ABX_OK;
}

abx_status abx_server_get_stats(abx_server *S, abx_server_stats *out) {
  if (!S || !out) return ABX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->in_flight = S->in_flight;
  out->queued = (int64_t)S->queue.size();
  return ABX_OK;
}

abx_status abx_server_destroy(abx_server *S) {
  if (!S) return ABX_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  for (auto &kv : S->reqs) delete kv.second;
  if (!S->cfg.simulate) {
    for (auto &sl : S->slots) {
      if (sl.t0) (void)hipEventDestroy(sl.t0);
      if (sl.t1) (void)hipEventDestroy(sl.t1);
      if (sl.ev) (void)hipEventDestroy(sl.ev);
      if (sl.s) (void)hipStreamDestroy(sl.s);
    }
    if (S->host_base) (void)hipHostFree(S->host_base);
  } else {
    ::operator delete(S->host_base);
  }
  delete S;
  return ABX_OK;
}

}  // extern "C"
