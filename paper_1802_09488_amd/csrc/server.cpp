// server.cpp -- a request loop that serves point joins against resident
// indexes (continuous admission of point batches, overlapping on the GPU).
//
// The paper's probe is a streaming operator over a stream of points
// (Section III-E, Section V); a service receives that stream as requests of
// uneven size aimed at different polygon sets. This runtime keeps the
// indexes resident and runs a scheduler thread:
//   * requests wait in FIFO order;
//   * when one of `slots` streams is free, the front request is admitted
//     together with the requests for the same index waiting behind it, as
//     one launch group of up to max_request_points points whose buffers fit
//     both arenas (device memory for points and results, and pinned host
//     memory for staging) -- memory is the admission budget, and under load
//     one launch serves many requests (continuous batching);
//   * an admitted group is staged into pinned memory and joined on its
//     slot's stream, straight from pinned memory if it is small, else
//     between a copy to the GPU and a copy back, so admitted groups
//     overlap on the device; completions are found by polling stream events;
//   * results are copied to the callers' buffers and each request's times
//     are kept (arrival, admission, completion).
// Arenas are allocated once at creation; the hot loop allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
  double arrival, admitted = 0, launched = 0, copied = 0, done = 0;
  int64_t offset = 0;  // first point in its launch group
  int status = ACT_OK;
};

// Requests for one index joined in one launch on one slot: their points
// sit back to back in one device and one pinned buffer (20 bytes a point:
// 16 in, 4 out).
struct Group {
  std::vector<Request *> reqs;
  int32_t index = 0;
  int64_t n = 0, dev_off = 0, pin_off = 0, bytes = 0;
  bool busy() const { return !reqs.empty(); }
};

// Host copies shared by the scheduler thread and a few helper threads that
// only copy (every HIP call stays on the scheduler thread). Idle helpers
// sleep; a batch of pieces is split between the caller and them.
class CopyPool {
 public:
  struct Piece {
    void *dst;
    const void *src;
    size_t n;
  };
  explicit CopyPool(int helpers) {
    for (int k = 0; k < helpers; k++) th_.emplace_back([this] { helper(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : th_) t.join();
  }
  // Runs every piece; returns when all are copied.
  void run(const std::vector<Piece> &pieces) {
    if (pieces.empty()) return;
    {
      std::lock_guard<std::mutex> lk(mu_);
      jobs_ = &pieces;
      next_ = 0;
      remaining_ = pieces.size();
      gen_++;
    }
    cv_.notify_all();
    const size_t done = drain(pieces);
    std::unique_lock<std::mutex> lk(mu_);
    remaining_ -= done;
    done_.wait(lk, [this] { return remaining_ == 0 && busy_ == 0; });
    jobs_ = nullptr;
  }

 private:
  size_t drain(const std::vector<Piece> &J) {
    size_t done = 0;
    for (size_t k; (k = next_.fetch_add(1)) < J.size(); done++)
      std::memcpy(J[k].dst, J[k].src, J[k].n);
    return done;
  }
  void helper() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      if (!jobs_) continue;  // that batch has already finished
      const std::vector<Piece> *J = jobs_;
      busy_++;
      lk.unlock();
      const size_t done = drain(*J);
      lk.lock();
      remaining_ -= done;
      busy_--;
      if (remaining_ == 0 && busy_ == 0) done_.notify_all();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  const std::vector<Piece> *jobs_ = nullptr;
  std::atomic<size_t> next_{0};
  size_t remaining_ = 0;  // pieces not yet copied (guarded by mu_)
  int busy_ = 0;          // helpers inside the current batch (guarded by mu_)
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Copies of a group below this many bytes run on the scheduler thread
// alone (waking the helpers costs more); larger ones are cut into pieces.
constexpr size_t kParallelCopyBytes = 1 << 20;
constexpr size_t kCopyPiece = 256 << 10;
constexpr int kCopyHelpers = 3;

// Run the copies (dst, src, bytes) of a group, in pieces on the pool if
// they are large (`pieces` is the caller's scratch list).
void group_copies(CopyPool &pool, const std::vector<CopyPool::Piece> &work,
                  std::vector<CopyPool::Piece> &pieces) {
  size_t total = 0;
  for (const auto &w : work) total += w.n;
  if (total < kParallelCopyBytes) {
    for (const auto &w : work) std::memcpy(w.dst, w.src, w.n);
    return;
  }
  pieces.clear();
  for (const auto &w : work)
    for (size_t o = 0; o < w.n; o += kCopyPiece)
      pieces.push_back({(char *)w.dst + o, (const char *)w.src + o, std::min(kCopyPiece, w.n - o)});
  pool.run(pieces);
}

}  // namespace

// Ownership: the queue, the ticket map, the statistics and the requests'
// status and times are shared and guarded by `mu`. The slots (`running`),
// the arenas and the requests taken from the queue belong to the scheduler
// thread, which stages and launches without holding `mu`.
struct act_server {
  std::vector<const act_index *> indexes;
  int device = 0;
  int64_t max_request = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<Group> running;  // per slot
  char *dev_base = nullptr;
  char *pin_base = nullptr;
  char *pin_dev = nullptr;  // the pinned arena as the device addresses it
  Arena dev_arena, pin_arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  CopyPool copies{kCopyHelpers};
  std::vector<CopyPool::Piece> copy_work, copy_pieces;  // scheduler thread's scratch
  act_server_stats stats{};
  std::string err;
};

namespace {

thread_local std::string g_server_err;

int fail(int code, const std::string &msg) {
  g_server_err = msg;
  return code;
}

// A launch group takes at most this many waiting requests.
constexpr size_t kGroupMax = 1024;
// How far down the queue the scheduler looks for requests of the front
// request's index.
constexpr size_t kGroupScan = 4096;

// Longest durations, kept by the scheduler thread (under `mu`).
void note_max(act_server *s, double act_server_stats::*field, double v) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (v > s->stats.*field) s->stats.*field = v;
}

// Groups of at most this many points are joined straight from the pinned
// arena (the kernels read the points and write the results over PCIe, no
// copy engine); larger ones are copied to device memory and back. Below
// saturation, where groups are small, this halved the p50 latency; the
// copies keep the throughput of the large groups near saturation.
constexpr int64_t kZeroCopyPoints = 1 << 16;

// Stage a group into pinned memory and start its join (and copies) on its
// slot's stream (scheduler thread, `mu` not held).
int launch(act_server *s, int slot, const Group &g) {
  const int64_t n = g.n;
  char *pin = s->pin_base + g.pin_off;
  char *dev = s->dev_base + g.dev_off;
  double *pin_pts = (double *)pin;
  int32_t *pin_out = (int32_t *)(pin + 16 * n);
  double *dev_pts = (double *)dev;
  int32_t *dev_out = (int32_t *)(dev + 16 * n);
  hipStream_t st = s->streams[slot];
  s->copy_work.clear();
  for (const Request *r : g.reqs)
    if (r->n) s->copy_work.push_back({pin_pts + 2 * r->offset, r->h_points, 16 * (size_t)r->n});
  const double t_stage = now_s();
  group_copies(s->copies, s->copy_work, s->copy_pieces);
  note_max(s, &act_server_stats::max_stage_s, now_s() - t_stage);
  if (n <= kZeroCopyPoints) {
    char *pd = s->pin_dev + g.pin_off;
    const int rc = act_join(s->indexes[g.index], (const double *)pd, n, (int32_t *)(pd + 16 * n), st);
    if (rc) return rc;
  } else {
    if (hipMemcpyAsync(dev_pts, pin_pts, 16 * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess)
      return ACT_E_HIP;
    const int rc = act_join(s->indexes[g.index], dev_pts, n, dev_out, st);
    if (rc) return rc;
    if (hipMemcpyAsync(pin_out, dev_out, 4 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess)
      return ACT_E_HIP;
  }
  if (hipEventRecord(s->events[slot], st) != hipSuccess) return ACT_E_HIP;
  const double t = now_s();
  for (Request *r : g.reqs) r->launched = t;  // written before the group is shared
  return ACT_OK;
}

// Copy a finished group's results out, free its buffers and complete its
// requests (scheduler thread, `mu` not held on entry).
void finish(act_server *s, Group &g, int status) {
  const double t_gpu = now_s();  // the group's results are in pinned memory
  if (status == ACT_OK) {
    s->copy_work.clear();
    for (const Request *r : g.reqs)
      if (r->n)
        s->copy_work.push_back(
            {r->h_out, s->pin_base + g.pin_off + 16 * g.n + 4 * r->offset, 4 * (size_t)r->n});
    group_copies(s->copies, s->copy_work, s->copy_pieces);
  }
  if (g.bytes) {
    s->dev_arena.release(g.dev_off, g.bytes);
    s->pin_arena.release(g.pin_off, g.bytes);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = now_s();
    for (Request *r : g.reqs) {
      r->status = status;
      r->copied = t_gpu;
      r->done = t;
      s->stats.completed++;
      s->stats.points += r->n;
      if (status != ACT_OK) s->stats.failed++;
    }
  }
  s->cv_done.notify_all();
  g = Group();
}

// Take the front request and the waiting requests of its index behind it
// (in arrival order, up to max_request points in all, or the front request
// alone if it is longer) whose buffers fit both arenas. `mu` held. False if
// even the front request does not fit yet.
bool take_group(act_server *s, Group &g) {
  Request *r0 = s->queue.front();
  g.index = r0->index;
  g.reqs.assign(1, r0);
  g.n = r0->n;
  std::vector<size_t> picked;
  const size_t scan = std::min(s->queue.size(), kGroupScan);
  for (size_t k = 1; k < scan && g.reqs.size() < kGroupMax; k++) {
    Request *r = s->queue[k];
    if (r->index != g.index || g.n + r->n > s->max_request) continue;
    g.reqs.push_back(r);
    picked.push_back(k);
    g.n += r->n;
  }
  for (int attempt = 0; attempt < 2; attempt++) {
    if (attempt == 1) {  // the group does not fit: try the front request alone
      if (g.reqs.size() == 1) break;
      g.reqs.resize(1);
      picked.clear();
      g.n = r0->n;
    }
    g.bytes = 20 * g.n;
    if (g.n == 0) {
      g.bytes = 0;
    } else {
      if (!s->dev_arena.alloc(g.bytes, g.dev_off)) continue;
      if (!s->pin_arena.alloc(g.bytes, g.pin_off)) {
        s->dev_arena.release(g.dev_off, g.bytes);
        continue;
      }
    }
    // remove the picked requests (back to front), then the front one
    for (auto it = picked.rbegin(); it != picked.rend(); ++it)
      s->queue.erase(s->queue.begin() + (std::ptrdiff_t)*it);
    s->queue.pop_front();
    int64_t off = 0;
    const double t = now_s();
    for (Request *r : g.reqs) {
      r->offset = off;
      off += r->n;
      r->admitted = t;
    }
    s->stats.admitted += (int64_t)g.reqs.size();
    s->stats.launches++;
    return true;
  }
  g = Group();
  return false;
}

void worker_loop(act_server *s) {
  (void)hipSetDevice(s->device);
  double last = now_s();
  for (;;) {
    const double t_pass = now_s();
    if (t_pass - last > s->stats.max_pass_s) note_max(s, &act_server_stats::max_pass_s, t_pass - last);
    last = t_pass;
    bool progress = false;
    // completions
    for (size_t k = 0; k < s->running.size(); k++) {
      Group &g = s->running[k];
      if (!g.busy()) continue;
      const hipError_t q = hipEventQuery(s->events[k]);
      if (q == hipErrorNotReady) continue;
      const double t0 = now_s();
      finish(s, g, q == hipSuccess ? ACT_OK : ACT_E_HIP);
      note_max(s, &act_server_stats::max_finish_s, now_s() - t0);
      progress = true;
    }
    // admissions, front of the queue first: one launch per pass, so that
    // the completions are looked at again between launches (a launch's
    // staging and enqueues can take milliseconds, and groups that finish
    // meanwhile would otherwise wait for all of the pass's launches)
    for (;;) {
      int slot = -1;
      for (size_t k = 0; k < s->running.size(); k++)
        if (!s->running[k].busy()) {
          slot = (int)k;
          break;
        }
      if (slot < 0) break;
      Group g;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->queue.empty() || !take_group(s, g)) break;
      }
      progress = true;
      const double t0 = now_s();
      const int rc = g.n > 0 ? launch(s, slot, g) : ACT_OK;
      note_max(s, &act_server_stats::max_launch_s, now_s() - t0);
      if (rc != ACT_OK || g.n == 0) {
        // whatever was enqueued must finish before the buffers are reused
        if (rc != ACT_OK) (void)hipStreamSynchronize(s->streams[slot]);
        finish(s, g, rc);
        continue;
      }
      s->running[slot] = std::move(g);
      break;
    }
    bool busy = false;
    for (const Group &g : s->running) busy |= g.busy();
    if (!progress) {
      if (busy) {  // poll the in-flight groups' events
        std::this_thread::yield();
      } else {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty()) break;
        s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        last = now_s();  // an idle wait is not a pass
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
  // touch every page of the pinned arena once: the first host writes to
  // its pages otherwise fault them in during staging, which stretched the
  // first requests' staging to milliseconds
  if (!rc) std::memset(s->pin_base, 0, (size_t)arena);
  if (!rc && hipHostGetDevicePointer((void **)&s->pin_dev, s->pin_base, 0) != hipSuccess)
    rc = fail(ACT_E_HIP, "no device address for the pinned arena");
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
  // warm the slots up (per slot: a staging copy, a join with each index
  // and a result copy on its stream, all slots in flight together, twice
  // over): the runtime's first operations on a stream, and its first
  // stretch with that many operations in flight, can take milliseconds, and
  // the first requests would pay them. The groups are request-sized
  // (max_request_points, at most 2^20 points: 16 MiB in, 4 MiB out) and
  // each slot has its own buffers: after a warm-up with one 64-point join
  // per slot in turn, launches in the first second of serving still
  // stalled for several milliseconds. Slot k's buffers start at k * stride,
  // 256-byte aligned like the arena's own allocations.
  const int64_t n_slots = std::max<int64_t>((int64_t)s->streams.size(), 1);
  const int64_t n_warm = std::min<int64_t>({o.max_request_points, 1 << 20, (arena / n_slots - 255) / 20});
  const int64_t stride = (20 * n_warm + 255) / 256 * 256;
  if (!rc && n_warm >= 1) {
    const int64_t n = n_warm;
    for (int round = 0; round < 2 && !rc; round++) {
      for (int64_t k = 0; k < (int64_t)s->streams.size() && !rc; k++) {
        hipStream_t st = s->streams[(size_t)k];
        char *pin = s->pin_base + stride * k;
        char *dev = s->dev_base + stride * k;
        // the pinned arena was zeroed above: n points at (0, 0), valid
        if (hipMemcpyAsync(dev, pin, 16 * (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess)
          rc = fail(ACT_E_HIP, "warm-up copy failed");
        for (const act_index *x : s->indexes)
          if (!rc && act_join(x, (const double *)dev, n, (int32_t *)(dev + 16 * n), st) != ACT_OK)
            rc = fail(ACT_E_HIP, std::string("warm-up join: ") + act_last_error());
        if (!rc && hipMemcpyAsync(pin + 16 * n, dev + 16 * n, 4 * (size_t)n, hipMemcpyDeviceToHost,
                                  st) != hipSuccess)
          rc = fail(ACT_E_HIP, "warm-up failed");
        // and a join straight from the pinned arena, as small groups run
        // (its outputs overwrite the copied-out ones, later on this stream)
        const int64_t nz = std::min<int64_t>(n, kZeroCopyPoints);
        char *pd = s->pin_dev + stride * k;
        for (const act_index *x : s->indexes)
          if (!rc && act_join(x, (const double *)pd, nz, (int32_t *)(pd + 16 * n), st) != ACT_OK)
            rc = fail(ACT_E_HIP, std::string("warm-up join: ") + act_last_error());
        if (!rc && hipEventRecord(s->events[(size_t)k], st) != hipSuccess)
          rc = fail(ACT_E_HIP, "warm-up failed");
      }
    }
    for (size_t k = 0; k < s->streams.size(); k++)
      if (hipStreamSynchronize(s->streams[k]) != hipSuccess && !rc)
        rc = fail(ACT_E_HIP, "warm-up failed");
  }
  if (rc) {
    act_server_destroy(s);
    return rc;
  }
  s->running.resize(s->streams.size());
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
  // (the arenas hand out 256-byte granules: a request whose rounded size
  // exceeds them could never be admitted, and would block the queue)
  if (n > s->dev_arena.size() / 20 || (20 * n + 255) / 256 * 256 > s->dev_arena.size())
    return fail(ACT_E_RANGE, "request larger than the arena");
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
    t->launched_s = r->launched > 0 ? r->launched : r->admitted;
    t->results_s = r->copied;
    t->done_s = r->done;
    t->n = r->n;
  }
  const int st = r->status;
  s->all.erase(it);
  delete r;
  return st == ACT_OK ? ACT_OK : fail(st, "request failed");
}

int act_server_replay(act_server *s, int64_t n, const int32_t *index,
                      const double *const *h_points, const int64_t *n_points,
                      const double *arrival_s, int64_t ring_points, act_request_times *times) {
  if (!s || n < 0 || (n > 0 && (!index || !h_points || !n_points || !arrival_s)) ||
      ring_points < 1)
    return fail(ACT_E_ARG, "bad argument");
  for (int64_t k = 0; k < n; k++)
    if (n_points[k] < 0 || n_points[k] > ring_points)
      return fail(ACT_E_RANGE, "a request is longer than the output ring");
  std::vector<int32_t> ring;
  std::vector<uint64_t> tickets;
  std::vector<int64_t> start;  // each request's place in the ring
  std::vector<int> sub_rc;
  try {
    ring.resize((size_t)ring_points);
    tickets.assign((size_t)n, 0);
    start.assign((size_t)n, 0);
    sub_rc.assign((size_t)n, ACT_OK);
  } catch (...) {
    return fail(ACT_E_OOM, "out of host memory");
  }
  // the ring is used in request order: [tail, head) holds the outputs of
  // requests submitted and not yet waited for
  std::mutex mu;
  std::condition_variable cv;
  int64_t head = 0, tail = 0, used = 0, submitted = 0, waited = 0;
  int first_err = ACT_OK;
  std::string err_msg;
  std::thread waiter([&] {
    for (int64_t k = 0; k < n; k++) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return submitted > k; });
      }
      int rc = sub_rc[k];
      act_request_times t{};
      if (rc == ACT_OK) {
        rc = act_server_wait(s, tickets[k], &t);
      } else {
        t.arrival_s = arrival_s[k];
        t.n = n_points[k];
      }
      if (rc != ACT_OK) t.done_s = t.results_s = t.launched_s = t.admitted_s = -1.0;
      if (times) times[k] = t;
      std::lock_guard<std::mutex> lk(mu);
      if (rc != ACT_OK && first_err == ACT_OK) {
        first_err = rc;
        err_msg = g_server_err;
      }
      // release this request's outputs and any gap before them (the unused
      // end of the ring when its outputs wrapped to the start)
      const int64_t end = start[k] + n_points[k];
      used -= start[k] >= tail ? end - tail : (ring_points - tail) + end;
      tail = end;
      waited = k + 1;
      cv.notify_all();
    }
  });
  for (int64_t k = 0; k < n; k++) {
    const int64_t m = n_points[k];
    {
      // room for m outputs: at head, or from 0 when the end is too short
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        if (waited == submitted) {  // nothing outstanding: restart at 0
          head = tail = used = 0;
          return true;
        }
        // in use: [tail, head), or once wrapped, [tail, the end) (with the
        // end's unused gap) and [0, head); the two cases differ in `used`
        if (used == head - tail) return head + m <= ring_points || m <= tail;
        return head + m <= tail;
      });
      const int64_t at = head + m <= ring_points ? head : 0;
      if (at != head) used += ring_points - head;  // the end's gap
      start[k] = at;
      head = at + m;
      used += m;
    }
    const double due = arrival_s[k];
    while (now_s() < due) {
    }
    uint64_t t = 0;
    const int rc = act_server_submit(s, index[k], h_points[k], m, ring.data() + start[k], due, &t);
    std::lock_guard<std::mutex> lk(mu);
    tickets[k] = t;
    sub_rc[k] = rc;
    submitted = k + 1;
    cv.notify_all();
  }
  waiter.join();
  if (first_err != ACT_OK) return fail(first_err, "replay: " + err_msg);
  return ACT_OK;
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
  // the indexes outlive the server: drop the workspaces its streams hold
  for (hipStream_t st : s->streams)
    for (const act_index *x : s->indexes) (void)act_workspace_release(x, st);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
  if (s->dev_base) (void)hipFree(s->dev_base);
  if (s->pin_base) (void)hipHostFree(s->pin_base);
  delete s;
}

const char *act_server_last_error(void) { return g_server_err.c_str(); }

}  // extern "C"
