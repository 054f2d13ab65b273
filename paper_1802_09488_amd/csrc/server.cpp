// server.cpp -- a request loop that serves point joins against resident
// indexes (continuous admission of point batches, overlapping on the GPU).
//
// The paper's probe is a streaming operator over a stream of points
// (Section III-E, Section V); a service receives that stream as requests of
// uneven size aimed at different polygon sets. This runtime keeps the
// indexes resident and runs a scheduler thread:
//   * requests wait in FIFO order;
//   * a request is admitted when one of `slots` streams is free and its
//     buffers fit both arenas (device memory for points and results, and
//     pinned host memory for staging) -- memory is the admission budget;
//   * an admitted request is staged into pinned memory, copied to the GPU,
//     joined and copied back on its own stream, so admitted requests
//     overlap on the device; completions are found by polling stream events;
//   * results are copied to the caller's buffer and the request's times are
//     kept (arrival, admission, completion).
// Arenas are allocated once at creation; the hot loop allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/act.h"

namespace {

using clock_type = std::chrono::steady_clock;

double now_s() {
  return std::chrono::duration<double>(clock_type::now().time_since_epoch()).count();
}

// First-fit allocator over a byte range (offsets), 256-byte granules.
class Arena {
 public:
  explicit Arena(int64_t bytes = 0) { reset(bytes); }
  void reset(int64_t bytes) {
    free_.clear();
    if (bytes > 0) free_[0] = bytes;
    size_ = bytes;
  }
  int64_t size() const { return size_; }
  bool alloc(int64_t bytes, int64_t &off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        off = it->first;
        const int64_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return true;
      }
    return false;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
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

 private:
  std::map<int64_t, int64_t> free_;
  int64_t size_ = 0;
};

struct Request {
  uint64_t ticket;
  int32_t index;
  const double *h_points;
  int64_t n;
  int32_t *h_out;
  double arrival, admitted = 0, done = 0;
  int64_t dev_off = -1, pin_off = -1, bytes = 0;
  int slot = -1;
  int status = ACT_OK;
};

}  // namespace

struct act_server {
  std::vector<const act_index *> indexes;
  int device = 0;
  int64_t max_request = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<Request *> running;  // per slot
  char *dev_base = nullptr;
  char *pin_base = nullptr;
  Arena dev_arena, pin_arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  act_server_stats stats{};
  std::string err;
};

namespace {

thread_local std::string g_server_err;

int fail(int code, const std::string &msg) {
  g_server_err = msg;
  return code;
}

// Start an admitted request on its slot's stream (scheduler thread).
int launch(act_server *s, Request *r) {
  const int64_t n = r->n;
  char *pin = s->pin_base + r->pin_off;
  char *dev = s->dev_base + r->dev_off;
  double *pin_pts = (double *)pin;
  int32_t *pin_out = (int32_t *)(pin + 16 * n);
  double *dev_pts = (double *)dev;
  int32_t *dev_out = (int32_t *)(dev + 16 * n);
  hipStream_t st = s->streams[r->slot];
  std::memcpy(pin_pts, r->h_points, 16 * (size_t)n);
  if (hipMemcpyAsync(dev_pts, pin_pts, 16 * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess)
    return ACT_E_HIP;
  int rc = act_join(s->indexes[r->index], dev_pts, n, dev_out, st);
  if (rc) return rc;
  if (hipMemcpyAsync(pin_out, dev_out, 4 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess)
    return ACT_E_HIP;
  if (hipEventRecord(s->events[r->slot], st) != hipSuccess) return ACT_E_HIP;
  return ACT_OK;
}

void finish(act_server *s, Request *r, int status) {
  if (status == ACT_OK && r->n > 0)
    std::memcpy(r->h_out, s->pin_base + r->pin_off + 16 * r->n, 4 * (size_t)r->n);
  r->status = status;
  r->done = now_s();
  if (r->bytes) {
    s->dev_arena.release(r->dev_off, r->bytes);
    s->pin_arena.release(r->pin_off, r->bytes);
  }
  if (r->slot >= 0) s->running[r->slot] = nullptr;
  s->stats.completed++;
  s->stats.points += r->n;
  if (status != ACT_OK) s->stats.failed++;
}

void worker_loop(act_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = false;
    // completions
    for (size_t k = 0; k < s->running.size(); k++) {
      Request *r = s->running[k];
      if (!r) continue;
      const hipError_t q = hipEventQuery(s->events[k]);
      if (q == hipErrorNotReady) continue;
      finish(s, r, q == hipSuccess ? ACT_OK : ACT_E_HIP);
      progress = true;
    }
    if (progress) s->cv_done.notify_all();
    // admissions, in arrival order
    while (!s->queue.empty()) {
      Request *r = s->queue.front();
      int slot = -1;
      for (size_t k = 0; k < s->running.size(); k++)
        if (!s->running[k]) {
          slot = (int)k;
          break;
        }
      if (slot < 0) break;
      r->bytes = 20 * r->n;
      if (r->n > 0) {
        int64_t d, p;
        if (!s->dev_arena.alloc(r->bytes, d)) break;
        if (!s->pin_arena.alloc(r->bytes, p)) {
          s->dev_arena.release(d, r->bytes);
          break;
        }
        r->dev_off = d;
        r->pin_off = p;
      } else {
        r->bytes = 0;
      }
      s->queue.pop_front();
      r->slot = slot;
      r->admitted = now_s();
      s->running[slot] = r;
      s->stats.admitted++;
      const int rc = r->n > 0 ? launch(s, r) : ACT_OK;
      if (rc != ACT_OK || r->n == 0) {
        // whatever was enqueued must finish before the buffers are reused
        if (rc != ACT_OK) (void)hipStreamSynchronize(s->streams[slot]);
        finish(s, r, rc);
        s->cv_done.notify_all();
      }
      progress = true;
    }
    bool busy = false;
    for (Request *r : s->running) busy |= r != nullptr;
    if (s->stop && !busy && s->queue.empty()) break;
    if (!progress) {
      if (busy) {  // poll the in-flight requests' events
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
      }
    }
  }
}

}  // namespace

extern "C" {

void act_server_opts_init(act_server_opts *o) {
  if (!o) return;
  o->slots = 4;
  o->device = 0;
  o->arena_bytes = 0;
  o->max_request_points = 1 << 20;
}

int act_server_create(const act_index *const *indexes, int32_t n_indexes,
                      const act_server_opts *opts, act_server **out) {
  if (!out || !indexes || n_indexes <= 0) return fail(ACT_E_ARG, "bad argument");
  *out = nullptr;
  act_server_opts o;
  act_server_opts_init(&o);
  if (opts) o = *opts;
  if (o.slots < 1 || o.slots > 64) return fail(ACT_E_ARG, "slots must be 1..64");
  if (o.max_request_points < 1) return fail(ACT_E_ARG, "max_request_points must be > 0");
  if (hipSetDevice(o.device) != hipSuccess) return fail(ACT_E_DEVICE, "no such HIP device");
  for (int k = 0; k < n_indexes; k++)
    if (!indexes[k]) return fail(ACT_E_ARG, "index is NULL");
  int64_t arena = o.arena_bytes;
  if (arena <= 0) {  // 90% of the free HBM left after the indexes, capped for the pinned side
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(ACT_E_HIP, "hipMemGetInfo failed");
    arena = std::min<int64_t>((int64_t)(0.9 * (double)fr), 4ll << 30);
  }
  act_server *s = new (std::nothrow) act_server;
  if (!s) return fail(ACT_E_OOM, "out of host memory");
  s->indexes.assign(indexes, indexes + n_indexes);
  s->device = o.device;
  s->max_request = o.max_request_points;
  int rc = ACT_OK;
  if (hipMalloc((void **)&s->dev_base, (size_t)arena) != hipSuccess ||
      hipHostMalloc((void **)&s->pin_base, (size_t)arena, hipHostMallocDefault) != hipSuccess)
    rc = fail(ACT_E_OOM, "cannot allocate the request arenas");
  s->dev_arena.reset(arena);
  s->pin_arena.reset(arena);
  for (int k = 0; k < o.slots && !rc; k++) {
    hipStream_t st;
    hipEvent_t ev;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      rc = fail(ACT_E_HIP, "cannot create streams/events");
      break;
    }
    s->streams.push_back(st);
    s->events.push_back(ev);
    // size every index's exact-mode workspace on this stream now, so that
    // joins on it never allocate
    for (const act_index *x : s->indexes) {
      int r = act_workspace_reserve(x, st, o.max_request_points);
      if (r) {
        rc = fail(r, std::string("workspace reserve: ") + act_last_error());
        break;
      }
    }
  }
  if (rc) {
    act_server_destroy(s);
    return rc;
  }
  s->running.assign(s->streams.size(), nullptr);
  s->stats.arena_bytes = arena;
  s->stats.slots = (int32_t)s->streams.size();
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return ACT_OK;
}

int act_server_submit(act_server *s, int32_t index, const double *h_points, int64_t n,
                      int32_t *h_out, double arrival_s, uint64_t *ticket) {
  if (!s || !ticket || n < 0 || (n > 0 && (!h_points || !h_out)))
    return fail(ACT_E_ARG, "bad argument");
  if (index < 0 || index >= (int32_t)s->indexes.size()) return fail(ACT_E_ARG, "no such index");
  if (20 * n > s->dev_arena.size()) return fail(ACT_E_RANGE, "request larger than the arena");
  Request *r = new (std::nothrow) Request;
  if (!r) return fail(ACT_E_OOM, "out of host memory");
  r->index = index;
  r->h_points = h_points;
  r->n = n;
  r->h_out = h_out;
  r->arrival = arrival_s > 0 ? arrival_s : now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    s->stats.submitted++;
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return ACT_OK;
}

int act_server_wait(act_server *s, uint64_t ticket, act_request_times *t) {
  if (!s) return fail(ACT_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(ACT_E_ARG, "unknown ticket");
  Request *r = it->second;
  s->cv_done.wait(lk, [r] { return r->done > 0; });
  if (t) {
    t->arrival_s = r->arrival;
    t->admitted_s = r->admitted;
    t->done_s = r->done;
    t->n = r->n;
  }
  const int st = r->status;
  s->all.erase(it);
  delete r;
  return st == ACT_OK ? ACT_OK : fail(st, "request failed");
}

int act_server_stats_get(act_server *s, act_server_stats *st) {
  if (!s || !st) return fail(ACT_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  st->queued = (int64_t)s->queue.size();
  return ACT_OK;
}

double act_server_clock(void) { return now_s(); }

void act_server_destroy(act_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->all) delete kv.second;
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
  if (s->dev_base) (void)hipFree(s->dev_base);
  if (s->pin_base) (void)hipHostFree(s->pin_base);
  delete s;
}

const char *act_server_last_error(void) { return g_server_err.c_str(); }

}  // extern "C"
