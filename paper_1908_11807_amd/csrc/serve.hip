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

struct Req {
  uint64_t ticket;
  abx_request r;
  Phase phase = P_QUEUED;
  int slot = -1;
  int64_t kk = 0, total = 0;
  abx_status status = ABX_OK;
  double t_admit = 0, t_done = 0, sim_deadline = 0;
  double t_device = 0;        // summed GPU time of the request's phases
  Block dev_a, dev_b, host;   // device: phase A / fill reservation; host: results
  // carved device pointers
  float *d_q = nullptr;
  char *d_scratch = nullptr;
  int32_t *d_off = nullptr, *d_idx = nullptr;
  float *d_dist = nullptr;
  int64_t *d_total = nullptr;
  // carved host pointers (pinned arena)
  int32_t *h_off = nullptr, *h_idx = nullptr;
  float *h_dist = nullptr;
  int64_t *h_total = nullptr;
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;        // completion (polled)
  hipEvent_t t0 = nullptr, t1 = nullptr;  // timing: start and end of a phase
  Req *r = nullptr;
};

}  // namespace

struct abx_server {
  abx_server_config cfg;
  int device = 0;
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

size_t request_scratch_bytes(const Req *q) {
  return q->r.kind == ABX_REQ_NEAREST ? nearest_scratch_bytes(q->r.m) : query_scratch_bytes(q->r.m);
}

size_t dev_bytes_a(const abx_server *S, const Req *q) {
  const int64_t m = q->r.m;
  size_t b = align_up((size_t)m * 12, kGrain) + align_up(request_scratch_bytes(q), kGrain);
  if (q->r.kind == ABX_REQ_NEAREST) b += 2 * align_up((size_t)(m * q->kk) * 4, kGrain);
  else b += align_up((size_t)(m + 1) * 4, kGrain);
  (void)S;
  return b;
}

size_t host_bytes_a(const Req *q) {
  const int64_t m = q->r.m;
  size_t b = align_up((size_t)(m + 1) * 4, kGrain) + kGrain;  // offsets + total
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
  release_block(S->dev, q->dev_a);
  release_block(S->dev, q->dev_b);
  if (status != ABX_OK) release_block(S->host, q->host);
  if (q->slot >= 0) S->slots[q->slot].r = nullptr;
  q->slot = -1;
  S->in_flight--;
  if (status == ABX_OK) {
    S->st.completed++;
    S->st.queries += q->r.m;
  } else {
    S->st.failed++;
  }
  S->cv_done.notify_all();
}

// Query ordering per request.  At request sizes (up to ~1e5 queries) the
// ordering's sort costs 60-90 us, measured against 1e7-point trees: radius
// requests never win it back (their walks are short), nearest requests do
// from ~1e4 queries where walks are long (a shell: 3.5 vs 4.4 ms at 1e4
// queries, k = 8), and lose it below.
constexpr int64_t kServeSortMin = 4096;
int sort_request(const Req *q) {
  return q->r.kind == ABX_REQ_NEAREST && q->r.m >= kServeSortMin ? 1 : 0;
}

// host-side offsets of a nearest request: row i starts at i * k'
void nearest_offsets(Req *q) {
  if (!q->h_off) return;
  for (int64_t i = 0; i <= q->r.m; ++i) q->h_off[i] = (int32_t)(i * q->kk);
}

abx_status launch_a(abx_server *S, Req *q) {
  const abx_bvh *tree = S->trees[q->r.tree];
  const int64_t m = q->r.m;
  Slot &sl = S->slots[q->slot];
  char *d = S->dev_base + q->dev_a.off;
  char *h = S->host_base + q->host.off;
  q->d_q = reinterpret_cast<float *>(d);
  d += align_up((size_t)m * 12, kGrain);
  q->d_scratch = d;
  d += align_up(request_scratch_bytes(q), kGrain);
  q->h_off = reinterpret_cast<int32_t *>(h);
  h += align_up((size_t)(m + 1) * 4, kGrain);
  q->h_total = reinterpret_cast<int64_t *>(h);
  h += kGrain;
  if (q->r.kind == ABX_REQ_NEAREST) {
    q->d_idx = reinterpret_cast<int32_t *>(d);
    d += align_up((size_t)(m * q->kk) * 4, kGrain);
    q->d_dist = reinterpret_cast<float *>(d);
    q->h_idx = reinterpret_cast<int32_t *>(h);
    h += align_up((size_t)(m * q->kk) * 4, kGrain);
    q->h_dist = reinterpret_cast<float *>(h);
  } else {
    q->d_off = reinterpret_cast<int32_t *>(d);
  }
  if (S->cfg.simulate) {
    q->sim_deadline = now_s() + 1e-9 * S->cfg.sim_ns_per_query * (double)(m > 0 ? m : 1);
    return ABX_OK;
  }
  ABX_HIP(hipEventRecord(sl.t0, sl.s));
  if (m > 0) ABX_HIP(hipMemcpyAsync(q->d_q, q->r.queries, (size_t)m * 12, hipMemcpyHostToDevice, sl.s));
  if (q->r.kind == ABX_REQ_NEAREST) {
    ABX_TRY(nearest_enqueue(tree, q->d_q, m, q->r.k, sort_request(q), q->d_scratch, nullptr, q->d_idx,
                            q->d_dist, sl.s));
    const size_t ob = (size_t)(m * q->kk) * 4;
    if (ob) {
      ABX_HIP(hipMemcpyAsync(q->h_idx, q->d_idx, ob, hipMemcpyDeviceToHost, sl.s));
      ABX_HIP(hipMemcpyAsync(q->h_dist, q->d_dist, ob, hipMemcpyDeviceToHost, sl.s));
    }
  } else {
    abx_predicates p{ABX_PRED_WITHIN, q->d_q, m, nullptr, q->r.radius, sort_request(q)};
    ABX_TRY(spatial_count_enqueue(tree, &p, q->d_scratch, q->d_off, &q->d_total, sl.s));
    ABX_HIP(hipMemcpyAsync(q->h_total, q->d_total, 8, hipMemcpyDeviceToHost, sl.s));
  }
  ABX_HIP(hipEventRecord(sl.t1, sl.s));
  ABX_HIP(hipEventRecord(sl.ev, sl.s));
  return ABX_OK;
}

// fill phase of a radius request: reserve the exact result space, launch
bool try_launch_b(abx_server *S, Req *q, abx_status *err) {
  const int64_t m = q->r.m, t = q->total;
  const size_t ib = align_up((size_t)t * 4, kGrain);
  if (!take(S->dev, q->dev_b, ib)) return false;
  // grow the host block: results (offsets already reserved) + indices
  Block hb;
  if (!take(S->host, hb, align_up((size_t)(m + 1) * 4, kGrain) + ib)) {
    release_block(S->dev, q->dev_b);
    return false;
  }
  release_block(S->host, q->host);
  q->host = hb;
  char *h = S->host_base + hb.off;
  q->h_off = reinterpret_cast<int32_t *>(h);
  q->h_idx = reinterpret_cast<int32_t *>(h + align_up((size_t)(m + 1) * 4, kGrain));
  q->h_dist = nullptr;
  q->d_idx = reinterpret_cast<int32_t *>(S->dev_base + q->dev_b.off);
  q->phase = P_RUN_B;
  if (S->cfg.simulate) {
    q->sim_deadline = now_s() + 1e-9 * S->cfg.sim_ns_per_query * (double)(m > 0 ? m : 1);
    return true;
  }
  Slot &sl = S->slots[q->slot];
  const abx_bvh *tree = S->trees[q->r.tree];
  abx_predicates p{ABX_PRED_WITHIN, q->d_q, m, nullptr, q->r.radius, sort_request(q)};
  if (hipEventRecord(sl.t0, sl.s) != hipSuccess) {
    *err = ABX_ERR_HIP;
    return true;
  }
  *err = spatial_fill_enqueue(tree, &p, q->d_scratch, q->d_off, q->d_idx, sl.s);
  if (*err == ABX_OK && hipMemcpyAsync(q->h_off, q->d_off, (size_t)(m + 1) * 4, hipMemcpyDeviceToHost, sl.s) != hipSuccess)
    *err = ABX_ERR_HIP;
  if (*err == ABX_OK && t > 0 &&
      hipMemcpyAsync(q->h_idx, q->d_idx, (size_t)t * 4, hipMemcpyDeviceToHost, sl.s) != hipSuccess)
    *err = ABX_ERR_HIP;
  if (*err == ABX_OK && hipEventRecord(sl.t1, sl.s) != hipSuccess) *err = ABX_ERR_HIP;
  if (*err == ABX_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) *err = ABX_ERR_HIP;
  return true;
}

bool phase_done(abx_server *S, Req *q) {
  if (S->cfg.simulate) return now_s() >= q->sim_deadline;
  const hipError_t e = hipEventQuery(S->slots[q->slot].ev);
  return e != hipErrorNotReady;
}

// one pass of the scheduler; returns true if anything changed
bool step(abx_server *S) {
  bool changed = false;
  bool fill_waiting = false;
  // 1. completions
  for (auto &sl : S->slots) {
    Req *q = sl.r;
    if (!q) continue;
    if (q->phase == P_WAIT_FILL) {
      abx_status err = ABX_OK;
      if (try_launch_b(S, q, &err)) {
        changed = true;
        if (err != ABX_OK) finish(S, q, err);
      } else if (S->dev.used() == q->dev_a.bytes && S->host.used() == q->host.bytes) {
        // alone in both arenas and the result space still does not fit (results
        // that the caller has not released yet hold host space: wait for them)
        finish(S, q, ABX_ERR_CAPACITY);
        changed = true;
      } else {
        fill_waiting = true;
      }
      continue;
    }
    if (!phase_done(S, q)) continue;
    changed = true;
    if (!S->cfg.simulate && hipEventQuery(sl.ev) != hipSuccess) {
      finish(S, q, ABX_ERR_HIP);
      continue;
    }
    if (S->cfg.simulate) {
      q->t_device += 1e-9 * S->cfg.sim_ns_per_query * (double)(q->r.m > 0 ? q->r.m : 1);
    } else {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, sl.t0, sl.t1) == hipSuccess) q->t_device += 1e-3 * (double)ms;
    }
    if (q->phase == P_RUN_A && q->r.kind == ABX_REQ_RADIUS) {
      q->total = S->cfg.simulate ? 10 * q->r.m : *q->h_total;
      if (q->total >= INT32_MAX) {
        finish(S, q, ABX_ERR_OVERFLOW);
        continue;
      }
      release_block(S->dev, q->dev_b);
      abx_status err = ABX_OK;
      if (!try_launch_b(S, q, &err)) {
        q->phase = P_WAIT_FILL;
        fill_waiting = true;
      } else if (err != ABX_OK) {
        finish(S, q, err);
      }
      continue;
    }
    if (q->r.kind == ABX_REQ_NEAREST) nearest_offsets(q);
    finish(S, q, ABX_OK);
  }
  // 1b. fills that wait on each other: when every occupied slot holds a fill
  // waiting for memory, no running phase will free any, and each may be
  // blocked by the others' reservations.  The earliest request keeps its
  // slot; the later ones give their reservations back and return to the
  // head of the queue (to be counted again once the earliest has finished).
  if (fill_waiting) {
    Req *keep = nullptr;
    bool running = false;
    for (auto &sl : S->slots) {
      if (!sl.r) continue;
      if (sl.r->phase != P_WAIT_FILL) {
        running = true;
      } else if (!keep || sl.r->ticket < keep->ticket) {
        keep = sl.r;
      }
    }
    if (!running && keep) {
      std::vector<Req *> back;
      for (auto &sl : S->slots) {
        Req *q = sl.r;
        if (!q || q == keep) continue;
        release_block(S->dev, q->dev_a);
        release_block(S->dev, q->dev_b);
        release_block(S->host, q->host);
        q->phase = P_QUEUED;
        q->slot = -1;
        q->total = 0;
        sl.r = nullptr;
        S->in_flight--;
        S->st.requeued++;
        back.push_back(q);
      }
      std::sort(back.begin(), back.end(), [](const Req *a, const Req *b) { return a->ticket > b->ticket; });
      for (Req *q : back) S->queue.push_front(q);
      if (!back.empty()) changed = true;
    }
  }
  // 2. admission: FIFO, stop while a fill waits for memory (it drains the device)
  while (!fill_waiting && !S->queue.empty()) {
    int free_slot = -1;
    for (size_t i = 0; i < S->slots.size(); ++i)
      if (!S->slots[i].r) {
        free_slot = (int)i;
        break;
      }
    if (free_slot < 0) break;
    Req *q = S->queue.front();
    const size_t db = dev_bytes_a(S, q), hb = host_bytes_a(q);
    if (db > S->dev.size() || hb > S->host.size()) {  // can never fit
      S->queue.pop_front();
      S->in_flight++;
      finish(S, q, ABX_ERR_CAPACITY);
      changed = true;
      continue;
    }
    if (!take(S->dev, q->dev_a, db)) break;
    if (!take(S->host, q->host, hb)) {
      release_block(S->dev, q->dev_a);
      break;
    }
    S->queue.pop_front();
    q->slot = free_slot;
    q->phase = P_RUN_A;
    q->t_admit = now_s();
    S->slots[free_slot].r = q;
    S->in_flight++;
    S->st.max_in_flight = std::max<int64_t>(S->st.max_in_flight, S->in_flight);
    changed = true;
    const abx_status e = launch_a(S, q);
    if (e != ABX_OK) finish(S, q, e);
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
    if (sl.r && sl.r->phase == P_WAIT_FILL) finish(S, sl.r, ABX_ERR_INVALID_ARG);
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
  S->dev.reset(cfg->arena_bytes);
  S->host.reset(cfg->host_bytes);
  S->dev_base = static_cast<char *>(cfg->arena);
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
