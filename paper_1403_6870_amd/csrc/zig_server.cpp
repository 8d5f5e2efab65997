// Serving loop: continuous batching of fill requests.
//
//   submit -> FIFO intake -> scheduler thread (spinning briefly on a work
//   counter before it parks, so a request is taken up in about a
//   microsecond): admission against the output arena (first fit, in
//   arrival order, so a client's requests keep their order), first indices
//   from the client counters in admission order, one batch per free
//   (stream, slot), all on that fill stream -> completion thread: polls the
//   batches' events, stamps the completions, wakes waiters.
//   A batch of one request runs as that request's plain fill; a batch of a
//   few requests passes its descriptors in the kernel arguments of the
//   batch kernel; a larger one copies them to the device first.  The batch
//   kernel's last workgroup raises the device-resident client counters to
//   the batch's ends; a plain fill's raise is owed and made in bulk before
//   the counters are next read.  Optional copies of outputs follow on the
//   same stream.
//
// The host mirror of the client counters decides every first index, at
// admission and in admission order, so batches on different fill streams
// need no ordering among themselves and a request's samples are the same
// whether it ran alone or in any mix.  The device counters are its
// persistent copy: they end at the same values whatever order the batches
// finish in (a max of increasing ends), and they are what a checkpoint
// reads.  A request whose indices would pass 2^64 - 2 is rejected at
// admission.
//
// The host fake backend makes no device call: it writes first_index + k as
// the k-th output into a host arena after an optional delay, and can fail
// every k-th request at admission (such a request uses no index and the
// others are unaffected).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/zig.h"
#include "zig_internal.hpp"
#include "zig_tune.hpp"

namespace zig {
namespace {

constexpr uint32_t kServeMaxBatch = 4096;  // requests per batch
constexpr uint64_t kSchedSpinNs = 200000;  // the scheduler spins this long before parking

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int fail(int code, const std::string& m) {
  set_error(m);
  return code;
}

// Deadline `ns` from now for timed condition waits.  On the system clock,
// whose waits are plain pthread_cond_timedwait calls (a steady-clock wait
// goes through pthread_cond_clockwait, which some thread checkers do not
// follow).
std::chrono::system_clock::time_point wall_deadline(uint64_t ns) {
  return std::chrono::system_clock::now() +
         std::chrono::duration_cast<std::chrono::system_clock::duration>(std::chrono::nanoseconds(ns));
}

// First-fit allocator over the output arena in 256-byte granules.
class Arena {
 public:
  void init(uint64_t cap) {
    free_.clear();
    free_[0] = cap & ~(uint64_t)255;
    used_ = 0;
  }
  static uint64_t round(uint64_t b) { return (b + 255) & ~(uint64_t)255; }
  bool fits(uint64_t bytes) const {
    const uint64_t b = round(bytes);
    for (const auto& kv : free_)
      if (kv.second >= b) return true;
    return false;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    const uint64_t b = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= b) {
        *off = it->first;
        const uint64_t rest = it->second - b, at = it->first + b;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += b;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    const uint64_t b = round(bytes);
    used_ -= b;
    auto next = free_.lower_bound(off);
    uint64_t start = off, size = b;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + b == next->first) {
      size += next->second;
      free_.erase(next);
    }
    free_[start] = size;
  }
  uint64_t used() const { return used_; }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> size of each free range
  uint64_t used_ = 0;
};

enum : int { kQueued = 0, kLaunched = 1, kDone = 2 };

// A trace replay in progress: where its completions go.
struct ReplaySink {
  zig_completion* out;
  uint64_t done = 0;  // requests completed (guarded by the server's mu)
};

struct Ticket {
  zig_completion comp;
  uint64_t off = 0, bytes = 0;  // arena range (bytes = 0: none)
  int state = kQueued;
  bool orphan = false;          // client dropped: release when complete
  ReplaySink* sink = nullptr;   // replay: record the completion here and release at once
  uint64_t sink_index = 0;
  void* copy_to = nullptr;      // replay: copy the output here before release
};

struct Pending {
  uint64_t ticket;
  uint32_t client;
  zig_spec spec;
  double scale, shift;
  uint64_t bytes;
};

struct DevSlot {
  void* desc_host = nullptr;  // pinned: BatchHeader + BatchReq[kServeMaxBatch]
  void* desc_dev = nullptr;
  uint32_t* tile_counters = nullptr;
  hipEvent_t ev_done = nullptr;
  bool busy = false;
};

// One admitted request of a batch.
struct Item {
  uint32_t client, dist, dtype;
  uint64_t n, first;
  double p0, p1;  // as submitted (lambda, or mu and sigma)
  double scale, shift;
  void* out;
  void* copy_to;
};

struct Batch {
  uint64_t id = 0;
  std::vector<uint64_t> tickets;
  std::vector<Item> items;
  std::vector<int> status;  // per request
  int stream = 0, slot = 0;
  int launch_status = ZIG_OK;
  std::atomic<bool> done{false};  // host fake finished, or the launch failed
};

}  // namespace

struct Server {
  zig_server_cfg cfg;
  bool device = true;
  // device backend
  int dev_id = 0;  // the device current at creation; every server thread uses it
  char* arena_dev = nullptr;
  bool own_arena = false;
  uint64_t* counters_dev = nullptr;
  std::vector<hipStream_t> fill_streams;
  const DevTable* tabs = nullptr;
  uint32_t wg = 256, spl = 4, groups = 0, groups_full = 0;  // resident workgroups: lean and staged-table kernels
  // host fake backend
  std::vector<char> arena_host;
  uint64_t fake_seen = 0;
  std::thread fake_worker;
  std::deque<Batch*> fake_q;
  std::mutex fake_mu;
  std::condition_variable fake_cv;
  // scheduling state, guarded by mu
  std::vector<std::vector<DevSlot>> slots;  // [stream][2]; the host fake uses only `busy`
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_inflight;
  std::deque<Pending> intake;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::vector<uint64_t> next_host;  // host mirror of the client counters (decides first indices)
  // Client counter raises owed by requests that ran as plain fills: the
  // device copy catches up in bulk before it is read (raise_dev stages them).
  std::vector<uint64_t> owed;
  bool any_owed = false;
  uint64_t* raise_dev = nullptr;
  Arena arena;
  uint64_t queued_bytes = 0;
  uint64_t next_ticket = 1, next_batch = 1;
  std::vector<std::deque<Batch*>> inflight;  // per fill stream, in launch order
  uint64_t inflight_count = 0;               // formed and not yet completed
  uint32_t launching = 0;                    // batches being launched outside mu
  int next_stream = 0;
  int broken = ZIG_OK;  // a device step failed: the server accepts no more work
  bool replaying_naive = false;
  std::atomic<bool> stop{false};
  // bumped with every change the scheduler may be waiting for (new
  // request, free slot, free arena space); it watches it while it spins
  std::atomic<uint64_t> work_epoch{0};
  bool stop_completers = false;  // set once the scheduler has exited
  std::thread sched;
  std::vector<std::thread> completers;  // one per fill stream
  zig_server_stats stats;
};

// Tells the scheduler (spinning or parked) that something it waits for
// changed; caller holds mu.  Cheap when no thread is parked on cv_sched.
void wake_sched(Server* s) {
  s->work_epoch.fetch_add(1, std::memory_order_release);
  s->cv_sched.notify_all();
}

namespace {

char* arena_base(Server* s) { return s->device ? s->arena_dev : s->arena_host.data(); }

// a free (stream, slot), streams taken round robin
bool free_slot(Server* s, int* stream, int* slot) {
  const int K = (int)s->cfg.streams;
  for (int d = 0; d < K; ++d) {
    const int k = (s->next_stream + d) % K;
    for (int j = 0; j < 2; ++j) {
      if (!s->slots[k][j].busy) {
        *stream = k;
        *slot = j;
        return true;
      }
    }
  }
  return false;
}

// A batch of one request runs as the plain fill of that request (the
// kernel a lone request is fastest with) and its completion event is
// recorded right after it; the raise of its client's device counter is
// owed and made in bulk before the counters are next read.
int launch_single(Server* s, Batch* b) {
  DevSlot& d = s->slots[b->stream][b->slot];
  const Item& it = b->items[0];
  hipStream_t fs = s->fill_streams[b->stream];
  // the slot's own counter pair: a large request takes the counter
  // schedule without waiting on another stream
  int r = fill_own_counters(it.dist, it.dtype, s->cfg.seed_base + it.client, it.first, it.n, it.p0, it.p1, it.out,
                            fs, d.tile_counters);
  if (r != ZIG_OK) return fail(ZIG_EHIP, std::string("serve: fill: ") + zig_last_error());
  hipError_t e = hipSuccess;
  if (it.copy_to) {
    e = hipMemcpyAsync(it.copy_to, it.out, it.n * (it.dtype == ZIG_F64 ? 8 : 4), hipMemcpyDeviceToDevice, fs);
    if (e != hipSuccess) return fail(ZIG_EHIP, std::string("serve: output copy: ") + hipGetErrorString(e));
  }
  e = hipEventRecord(d.ev_done, fs);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("serve: completion record: ") + hipGetErrorString(e));
  return ZIG_OK;
}

// Makes the owed counter raises (caller holds mu, no launch in progress):
// stages the owed ends and raises the device counters to them on fill
// stream 0.
int pay_owed_locked(Server* s) {
  if (!s->any_owed) return ZIG_OK;
  hipError_t e = hipMemcpy(s->raise_dev, s->owed.data(), s->cfg.clients * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("counter raise: ") + hipGetErrorString(e));
  const int le = launch_raise_counters(s->counters_dev, s->raise_dev, s->cfg.clients, s->fill_streams[0]);
  if (le != 0) return fail(ZIG_EHIP, std::string("counter raise: ") + hipGetErrorString((hipError_t)le));
  std::fill(s->owed.begin(), s->owed.end(), 0);
  s->any_owed = false;
  return ZIG_OK;
}

int launch_device(Server* s, Batch* b) {
  if (b->items.size() == 1) return launch_single(s, b);
  DevSlot& d = s->slots[b->stream][b->slot];
  const uint32_t m = (uint32_t)b->items.size();
  const uint32_t tile_blocks = s->wg * s->spl;
  // a batch of a few requests passes its descriptors in the kernel
  // arguments: no copy to the device ahead of the kernel
  const bool inline_desc = m <= kInlineReqs;
  BatchInline inl;
  BatchHeader* h = inline_desc ? &inl.hdr : static_cast<BatchHeader*>(d.desc_host);
  BatchReq* q = reinterpret_cast<BatchReq*>(h + 1);
  uint64_t total = 0;
  for (uint32_t i = 0; i < m; ++i) {
    const Item& it = b->items[i];
    make_descriptor(it.dist, it.dtype, s->cfg.seed_base + it.client, it.first, it.n, it.scale, it.shift, it.out,
                    &q[i]);
    const uint64_t blocks = q[i].blk_last - q[i].blk0 + 1;
    q[i].tiles = (uint32_t)(blocks / tile_blocks + (blocks % tile_blocks != 0));
    q[i].tile_start = (uint32_t)total;
    total += q[i].tiles;
  }
  std::memset(h, 0, sizeof(*h));
  h->count = m;
  h->total_tiles = (uint32_t)total;
  const bool full = batch_full(total, s->groups);
  const uint32_t groups = full ? s->groups_full : s->groups;
  h->chunk = batch_chunk(total, tile_blocks, groups);
  hipStream_t fs = s->fill_streams[b->stream];
  hipError_t e = hipSuccess;
  if (!inline_desc) {
    e = hipMemcpyAsync(d.desc_dev, d.desc_host, sizeof(BatchHeader) + (size_t)m * sizeof(BatchReq),
                       hipMemcpyHostToDevice, fs);
    if (e != hipSuccess) return fail(ZIG_EHIP, std::string("serve: descriptor copy: ") + hipGetErrorString(e));
  }
  BatchArgs ba;
  ba.hdr = static_cast<const BatchHeader*>(d.desc_dev);
  ba.tabs = s->tabs;
  ba.counters = d.tile_counters;
  ba.client_next = s->counters_dev;
  ba.seed_base = s->cfg.seed_base;
  // no more workgroups than counter steps: a small batch then dispatches
  // (and retires) a few workgroups instead of every resident one
  const uint64_t steps = (total + h->chunk - 1) / h->chunk;
  const uint32_t grid = steps < (uint64_t)groups ? (uint32_t)steps : groups;
  const int le = inline_desc ? launch_batch_inline(s->wg, s->spl, full, grid, ba, inl, fs)
                             : launch_batch(s->wg, s->spl, full, grid, ba, fs);
  if (le != 0) return fail(ZIG_EHIP, std::string("serve: batch launch: ") + hipGetErrorString((hipError_t)le));
  for (const Item& it : b->items) {
    if (!it.copy_to) continue;
    e = hipMemcpyAsync(it.copy_to, it.out, it.n * (it.dtype == ZIG_F64 ? 8 : 4), hipMemcpyDeviceToDevice, fs);
    if (e != hipSuccess) return fail(ZIG_EHIP, std::string("serve: output copy: ") + hipGetErrorString(e));
  }
  e = hipEventRecord(d.ev_done, fs);
  if (e != hipSuccess) return fail(ZIG_EHIP, std::string("serve: completion record: ") + hipGetErrorString(e));
  return ZIG_OK;
}

void fake_loop(Server* s) {
  for (;;) {
    Batch* b;
    {
      std::unique_lock<std::mutex> lk(s->fake_mu);
      s->fake_cv.wait(lk, [&] { return s->stop.load() || !s->fake_q.empty(); });
      if (s->fake_q.empty()) return;
      b = s->fake_q.front();
      s->fake_q.pop_front();
    }
    if (s->cfg.fake_latency_us) std::this_thread::sleep_for(std::chrono::microseconds(s->cfg.fake_latency_us));
    for (size_t i = 0; i < b->items.size(); ++i) {
      if (b->status[i] != ZIG_OK) continue;
      const Item& it = b->items[i];
      for (uint64_t k = 0; k < it.n; ++k) {
        if (it.dtype == ZIG_F64)
          static_cast<double*>(it.out)[k] = (double)(it.first + k);
        else
          static_cast<float*>(it.out)[k] = (float)(it.first + k);
      }
      if (it.copy_to) std::memcpy(it.copy_to, it.out, it.n * (it.dtype == ZIG_F64 ? 8 : 4));
    }
    b->done.store(true, std::memory_order_release);
  }
}

// Marks a ticket complete; a replay ticket is recorded in its sink and
// released at once.
void complete_locked(Server* s, uint64_t id, int status, uint64_t t) {
  auto it = s->tickets.find(id);
  Ticket& tk = it->second;
  tk.state = kDone;
  tk.comp.status = status;
  tk.comp.t_done_ns = t;
  if (status != ZIG_OK) tk.comp.out = nullptr;
  if (tk.sink) {
    tk.sink->out[tk.sink_index] = tk.comp;
    tk.sink->done += 1;
  }
  if (tk.sink || tk.orphan) {
    if (tk.bytes) s->arena.release(tk.off, tk.bytes);
    s->tickets.erase(it);
  }
}

void cancel_queued_locked(Server* s, int status) {
  const uint64_t t = now_ns();
  for (Pending& p : s->intake) complete_locked(s, p.ticket, status, t);
  s->intake.clear();
  s->queued_bytes = 0;
  s->cv_done.notify_all();
}

// Forms one batch from the head of the intake on (stream k, slot j), both
// free, and launches it (the HIP calls outside mu).  Called by the
// scheduler thread, holding mu through lk.
void form_and_launch(Server* s, std::unique_lock<std::mutex>& lk, int k, int j) {
  Batch* b = new Batch();
  b->id = s->next_batch++;
  b->stream = k;
  b->slot = j;
  const uint64_t t_admit = now_ns();
  bool rejected = false;
  while (!s->intake.empty() && b->items.size() < s->cfg.max_batch) {
    Pending& p = s->intake.front();
    uint64_t off;
    if (!s->arena.alloc(p.bytes, &off)) break;  // FIFO: later requests wait too
    Ticket& tk = s->tickets[p.ticket];
    uint64_t& next = s->next_host[p.client];
    int st = ZIG_OK;
    if (p.spec.n > UINT64_MAX - next)  // indices up to 2^64 - 2, so a counter never wraps
      st = ZIG_EINVAL;
    else if (!s->device && s->cfg.fake_fail_every && ++s->fake_seen % s->cfg.fake_fail_every == 0)
      st = ZIG_EHIP;
    if (st != ZIG_OK) {  // completes now, uses no index
      s->arena.release(off, p.bytes);
      tk.comp.t_admit_ns = tk.comp.t_launch_ns = t_admit;
      s->stats.failed_requests += 1;
      s->queued_bytes -= Arena::round(p.bytes);
      const uint64_t id = p.ticket;
      s->intake.pop_front();
      complete_locked(s, id, st, t_admit);
      rejected = true;
      continue;
    }
    tk.off = off;
    tk.bytes = p.bytes;
    tk.state = kLaunched;
    tk.comp.t_admit_ns = t_admit;
    tk.comp.out = arena_base(s) + off;
    tk.comp.batch_id = b->id;
    tk.comp.first_index = next;
    Item item;
    item.client = p.client;
    item.dist = p.spec.dist;
    item.dtype = p.spec.dtype;
    item.n = p.spec.n;
    item.first = next;
    item.p0 = p.spec.p0;
    item.p1 = p.spec.p1;
    item.scale = p.scale;
    item.shift = p.shift;
    item.out = tk.comp.out;
    item.copy_to = tk.copy_to;
    next += p.spec.n;
    b->items.push_back(item);
    b->tickets.push_back(p.ticket);
    s->queued_bytes -= Arena::round(p.bytes);
    s->intake.pop_front();
  }
  if (rejected) s->cv_done.notify_all();
  if (b->items.empty()) {
    delete b;
    return;
  }
  b->status.assign(b->items.size(), ZIG_OK);
  s->slots[k][j].busy = true;
  s->next_stream = (k + 1) % (int)s->cfg.streams;
  const uint64_t t_launch = now_ns();
  for (uint64_t tid : b->tickets) {
    Ticket& tk = s->tickets[tid];
    tk.comp.batch_size = (uint32_t)b->items.size();
    tk.comp.t_launch_ns = t_launch;
  }
  s->stats.batches += 1;
  s->stats.requests += b->items.size();
  for (const Item& it : b->items) s->stats.samples += it.n;
  if (s->arena.used() > s->stats.max_bytes_in_use) s->stats.max_bytes_in_use = s->arena.used();
  s->inflight_count += 1;
  if (s->inflight_count > s->stats.max_inflight_batches) s->stats.max_inflight_batches = s->inflight_count;
  if (s->device) {
    // The slot is ours and the indices are fixed: launch without the lock,
    // so submitters and completions are not held up by the HIP calls.
    s->launching += 1;
    lk.unlock();
    const int st = launch_device(s, b);
    lk.lock();
    s->launching -= 1;
    b->launch_status = st;
    if (st == ZIG_OK && b->items.size() == 1) {  // ran as a plain fill: its counter raise is owed
      const Item& it = b->items[0];
      uint64_t& o = s->owed[it.client];
      if (it.first + it.n > o) o = it.first + it.n;
      s->any_owed = true;
    }
    if (st != ZIG_OK) {
      s->broken = st;
      for (int& x : b->status) x = st;
      b->done.store(true);
      cancel_queued_locked(s, ZIG_EHIP);
    }
    s->cv_done.notify_all();
  } else {
    std::lock_guard<std::mutex> fl(s->fake_mu);
    s->fake_q.push_back(b);
    s->fake_cv.notify_one();
  }
  s->inflight[k].push_back(b);
  s->cv_inflight.notify_all();
}

void sched_loop(Server* s) {
  if (s->device) (void)hipSetDevice(s->dev_id);
  std::unique_lock<std::mutex> lk(s->mu);
  const uint64_t window = (uint64_t)s->cfg.window_us * 1000;
  for (;;) {
    int k = 0, j = 0;
    auto ready = [&] {
      return s->stop.load() || (!s->intake.empty() && !s->replaying_naive && s->broken == ZIG_OK &&
                                free_slot(s, &k, &j) && s->arena.fits(s->intake.front().bytes));
    };
    while (!ready()) {
      // spin a little before parking, so that a request arriving now is
      // taken up in about a microsecond rather than after a thread wake-up
      const uint64_t seen = s->work_epoch.load(std::memory_order_acquire);
      lk.unlock();
      const uint64_t until = now_ns() + kSchedSpinNs;
      bool moved = false;
      do {
        std::this_thread::yield();
        moved = s->work_epoch.load(std::memory_order_acquire) != seen || s->stop.load();
      } while (!moved && now_ns() < until);
      lk.lock();
      if (!moved) s->cv_sched.wait(lk, ready);
    }
    if (s->stop.load()) break;
    if (window) {  // gathering window after the oldest queued submission
      const uint64_t deadline = s->tickets[s->intake.front().ticket].comp.t_submit_ns + window;
      while (!s->stop.load() && !s->intake.empty() && s->intake.size() < s->cfg.max_batch) {
        const uint64_t t = now_ns();
        if (t >= deadline) break;
        s->cv_sched.wait_until(lk, wall_deadline(deadline - t));
      }
      if (s->stop.load()) break;
      if (s->intake.empty() || !free_slot(s, &k, &j)) continue;
    }
    form_and_launch(s, lk, k, j);
  }
}

// t: when the batch's completion was observed.
void finish_locked(Server* s, Batch* b, uint64_t t) {
  for (size_t i = 0; i < b->tickets.size(); ++i) {
    if (b->status[i] != ZIG_OK) s->stats.failed_requests += 1;
    complete_locked(s, b->tickets[i], b->status[i], t);
  }
  // after a failed launch the slot may still have work queued: keep it busy
  if (b->launch_status == ZIG_OK) s->slots[b->stream][b->slot].busy = false;
}

// Completion thread of fill stream k: batches on one stream finish in
// launch order, so it waits on the oldest one only, without the lock.
void complete_loop(Server* s, int k) {
  if (s->device) (void)hipSetDevice(s->dev_id);
  std::unique_lock<std::mutex> lk(s->mu);
  std::deque<Batch*>& q = s->inflight[k];
  for (;;) {
    s->cv_inflight.wait(lk, [&] { return s->stop_completers || !q.empty(); });
    if (q.empty()) return;  // stop_completers and nothing left
    Batch* b = q.front();
    const hipEvent_t ev = s->device ? s->slots[b->stream][b->slot].ev_done : nullptr;
    lk.unlock();
    bool failed = false;
    // poll without sleeping: a timed sleep costs tens of microseconds
    while (!b->done.load(std::memory_order_acquire)) {
      if (s->device) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) {
          failed = true;
          break;
        }
      }
      std::this_thread::yield();
    }
    const uint64_t t_seen = now_ns();
    lk.lock();
    if (failed) {
      for (int& x : b->status) x = ZIG_EHIP;
      s->broken = ZIG_EHIP;
    }
    finish_locked(s, b, t_seen);
    q.pop_front();
    s->inflight_count -= 1;
    delete b;
    s->cv_done.notify_all();
    // a slot is free: only queued work needs the scheduler woken
    if (!s->intake.empty() || s->stop.load()) zig::wake_sched(s);
  }
}

void free_device(Server* s) {
  for (auto& row : s->slots)
    for (DevSlot& d : row) {
      if (d.desc_host) (void)hipHostFree(d.desc_host);
      if (d.desc_dev) (void)hipFree(d.desc_dev);
      if (d.tile_counters) (void)hipFree(d.tile_counters);
      if (d.ev_done) (void)hipEventDestroy(d.ev_done);
    }
  s->slots.clear();
  for (hipStream_t st : s->fill_streams)
    if (st) (void)hipStreamDestroy(st);
  s->fill_streams.clear();
  if (s->counters_dev) (void)hipFree(s->counters_dev);
  if (s->raise_dev) (void)hipFree(s->raise_dev);
  if (s->own_arena && s->arena_dev) (void)hipFree(s->arena_dev);
}

#define ZIG_CK(x, what)                                                                  \
  do {                                                                                   \
    const hipError_t ee = (x);                                                           \
    if (ee != hipSuccess)                                                                \
      return fail(ee == hipErrorOutOfMemory ? ZIG_ENOMEM : ZIG_EHIP,                     \
                  std::string(what) + ": " + hipGetErrorString(ee));                     \
  } while (0)

int setup_device(Server* s) {
  ZIG_CK(hipGetDevice(&s->dev_id), "hipGetDevice");
  const int r = device_tables_for(256, &s->tabs);
  if (r != ZIG_OK) return r;
  tuned_batch_shape(&s->wg, &s->spl);
  ZIG_CK((hipError_t)batch_groups(s->wg, s->spl, false, &s->groups), "batch occupancy");
  ZIG_CK((hipError_t)batch_groups(s->wg, s->spl, true, &s->groups_full), "batch occupancy");
  if (s->cfg.arena) {
    s->arena_dev = static_cast<char*>(s->cfg.arena);
  } else {
    ZIG_CK(hipMalloc(&s->arena_dev, s->cfg.cap_bytes), "hipMalloc(arena)");
    s->own_arena = true;
  }
  ZIG_CK(hipMalloc(&s->counters_dev, s->cfg.clients * sizeof(uint64_t)), "hipMalloc(counters)");
  ZIG_CK(hipMemset(s->counters_dev, 0, s->cfg.clients * sizeof(uint64_t)), "hipMemset(counters)");
  ZIG_CK(hipMalloc(&s->raise_dev, s->cfg.clients * sizeof(uint64_t)), "hipMalloc(counter raises)");
  s->fill_streams.assign(s->cfg.streams, nullptr);
  const size_t bbytes = sizeof(BatchHeader) + (size_t)kServeMaxBatch * sizeof(BatchReq);
  for (uint32_t k = 0; k < s->cfg.streams; ++k) {
    ZIG_CK(hipStreamCreateWithFlags(&s->fill_streams[k], hipStreamNonBlocking), "hipStreamCreate");
    for (DevSlot& d : s->slots[k]) {
      ZIG_CK(hipHostMalloc(&d.desc_host, bbytes, hipHostMallocDefault), "hipHostMalloc");
      ZIG_CK(hipMalloc(&d.desc_dev, bbytes), "hipMalloc");
      ZIG_CK(hipMalloc(&d.tile_counters, 2 * sizeof(uint32_t)), "hipMalloc");
      ZIG_CK(hipMemset(d.tile_counters, 0, 2 * sizeof(uint32_t)), "hipMemset");
      ZIG_CK(hipEventCreateWithFlags(&d.ev_done, hipEventDisableTiming), "hipEventCreate");
    }
  }
  return ZIG_OK;
}

// Sleeps until the monotonic time `target` (ns): coarse sleep, then yield.
void sleep_until_ns(uint64_t target) {
  const uint64_t t = now_ns();
  if (t + 200000 < target) std::this_thread::sleep_for(std::chrono::nanoseconds(target - t - 150000));
  while (now_ns() < target) std::this_thread::yield();
}

int submit_impl(Server* s, uint32_t client, const zig_spec& spec, uint32_t flags, uint64_t* ticket,
                ReplaySink* sink, uint64_t sink_index, void* copy_to) {
  if (client >= s->cfg.clients) return fail(ZIG_EINVAL, "client out of range");
  if (spec.dist > 1 || spec.dtype > 1) return fail(ZIG_EINVAL, "unknown distribution or dtype");
  double scale = 0.0, shift = 0.0;
  const int r = params_for(spec.dist, spec.p0, spec.p1, &scale, &shift);
  if (r != ZIG_OK) return r;
  const uint64_t esize = spec.dtype == ZIG_F64 ? 8 : 4;
  if (spec.n > (s->cfg.cap_bytes & ~(uint64_t)255) / esize)
    return fail(ZIG_EINVAL, "request larger than the admission cap");
  const uint64_t bytes = spec.n * esize;
  const uint64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop.load()) return fail(ZIG_ESTATE, "server is shutting down");
  if (s->broken != ZIG_OK) return fail(s->broken, "server stopped after a failed device step");
  if ((flags & ZIG_SUBMIT_NONBLOCK) && s->arena.used() + s->queued_bytes + Arena::round(bytes) > s->cfg.cap_bytes)
    return fail(ZIG_EBUSY, "admission would exceed the output cap");
  const uint64_t id = s->next_ticket++;
  Ticket& tk = s->tickets[id];
  std::memset(&tk.comp, 0, sizeof(tk.comp));
  tk.comp.status = ZIG_OK;
  tk.comp.seed = s->cfg.seed_base + client;
  tk.comp.n = spec.n;
  tk.comp.client = client;
  tk.comp.dist = spec.dist;
  tk.comp.dtype = spec.dtype;
  tk.comp.t_submit_ns = t;
  tk.comp.t_arrival_ns = spec.t_arrival_ns ? spec.t_arrival_ns : t;
  tk.sink = sink;
  tk.sink_index = sink_index;
  tk.copy_to = copy_to;
  *ticket = id;
  if (spec.n == 0) {  // nothing to generate: complete at once, no index used
    tk.comp.t_admit_ns = tk.comp.t_launch_ns = t;
    complete_locked(s, id, ZIG_OK, t);
    s->cv_done.notify_all();
    return ZIG_OK;
  }
  Pending p;
  p.ticket = id;
  p.client = client;
  p.spec = spec;
  p.scale = scale;
  p.shift = shift;
  p.bytes = bytes;
  s->intake.push_back(p);
  s->queued_bytes += Arena::round(bytes);
  zig::wake_sched(s);
  return ZIG_OK;
}

int replay_batched(Server* s, const zig_trace_item* items, uint64_t count, zig_completion* out);
int replay_naive(Server* s, const zig_trace_item* items, uint64_t count, zig_completion* out);

}  // namespace
}  // namespace zig

using zig::Server;

extern "C" {

uint64_t zig_server_now_ns(void) { return zig::now_ns(); }

int zig_server_create(const zig_server_cfg* cfg, zig_server** out) {
  zig::clear_error();
  if (!cfg || !out) return zig::fail(ZIG_EINVAL, "cfg and out must not be null");
  zig_server_cfg c = *cfg;
  if (c.streams == 0) c.streams = 4;
  if (c.max_batch == 0) c.max_batch = 1024;
  if (c.clients == 0) c.clients = 64;
  if (c.cap_bytes < 256) return zig::fail(ZIG_EINVAL, "cap_bytes must be at least 256");
  if (c.streams > 8) return zig::fail(ZIG_EINVAL, "at most 8 streams");
  if (c.max_batch > zig::kServeMaxBatch) return zig::fail(ZIG_EINVAL, "max_batch must be <= 4096");
  if (c.clients > (1u << 20)) return zig::fail(ZIG_EINVAL, "at most 2^20 clients");
  if (c.backend != ZIG_BACKEND_DEVICE && c.backend != ZIG_BACKEND_HOST_FAKE)
    return zig::fail(ZIG_EINVAL, "unknown backend");
  if (c.backend == ZIG_BACKEND_HOST_FAKE && c.arena)
    return zig::fail(ZIG_EINVAL, "the host fake backend allocates its own arena");
  if (c.backend == ZIG_BACKEND_DEVICE && c.arena && ((uintptr_t)c.arena & 255u))
    return zig::fail(ZIG_EINVAL, "a supplied arena must be 256-byte aligned");
  std::unique_ptr<Server> s(new Server());
  s->cfg = c;
  std::memset(&s->stats, 0, sizeof(s->stats));
  s->device = c.backend == ZIG_BACKEND_DEVICE;
  s->arena.init(c.cap_bytes);
  s->next_host.assign(c.clients, 0);
  s->owed.assign(c.clients, 0);
  s->slots.assign(c.streams, std::vector<zig::DevSlot>(2));
  s->inflight.assign(c.streams, std::deque<zig::Batch*>());
  if (s->device) {
    const int r = zig::setup_device(s.get());
    if (r != ZIG_OK) {
      zig::free_device(s.get());
      return r;
    }
  } else {
    try {
      s->arena_host.assign(c.cap_bytes, 0);
    } catch (...) {
      return zig::fail(ZIG_ENOMEM, "host fake arena");
    }
    s->fake_worker = std::thread(zig::fake_loop, s.get());
  }
  s->sched = std::thread(zig::sched_loop, s.get());
  for (uint32_t k = 0; k < c.streams; ++k) s->completers.emplace_back(zig::complete_loop, s.get(), (int)k);
  *out = reinterpret_cast<zig_server*>(s.release());
  return ZIG_OK;
}

int zig_server_submit(zig_server* srv, uint32_t client, const zig_spec* spec, uint32_t flags, uint64_t* ticket) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !spec || !ticket) return zig::fail(ZIG_EINVAL, "null argument");
  if (flags & ~(uint32_t)ZIG_SUBMIT_NONBLOCK) return zig::fail(ZIG_EINVAL, "unknown flags");
  return zig::submit_impl(s, client, *spec, flags, ticket, nullptr, 0, nullptr);
}

int zig_server_wait(zig_server* srv, uint64_t ticket, int64_t timeout_us, zig_completion* out) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return zig::fail(ZIG_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->tickets.find(ticket) == s->tickets.end()) return zig::fail(ZIG_ESTATE, "unknown ticket");
  auto ready = [&] {
    auto jt = s->tickets.find(ticket);
    return jt == s->tickets.end() || jt->second.state == zig::kDone;
  };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_until(lk, zig::wall_deadline((uint64_t)timeout_us * 1000), ready)) {
    return zig::fail(ZIG_EBUSY, "timed out");
  }
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return zig::fail(ZIG_ESTATE, "ticket released while waiting");
  if (out) *out = it->second.comp;
  const int st = it->second.comp.status;
  return st == ZIG_OK ? ZIG_OK : zig::fail(st, st == ZIG_ESTATE ? "request cancelled" : "request failed");
}

int zig_server_release(zig_server* srv, uint64_t ticket) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return zig::fail(ZIG_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return zig::fail(ZIG_ESTATE, "unknown ticket");
  if (it->second.state != zig::kDone) return zig::fail(ZIG_ESTATE, "request not complete");
  if (it->second.bytes) s->arena.release(it->second.off, it->second.bytes);
  s->tickets.erase(it);
  zig::wake_sched(s);
  return ZIG_OK;
}

int zig_server_drop_client(zig_server* srv, uint32_t client, uint64_t* reclaimed) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return zig::fail(ZIG_EINVAL, "null server");
  if (client >= s->cfg.clients) return zig::fail(ZIG_EINVAL, "client out of range");
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t n = 0;
  const uint64_t t = zig::now_ns();
  for (auto it = s->intake.begin(); it != s->intake.end();) {
    if (it->client == client) {
      s->queued_bytes -= zig::Arena::round(it->bytes);
      s->tickets[it->ticket].orphan = true;
      zig::complete_locked(s, it->ticket, ZIG_ESTATE, t);  // cancelled: forgotten at once
      it = s->intake.erase(it);
      ++n;
    } else {
      ++it;
    }
  }
  for (auto it = s->tickets.begin(); it != s->tickets.end();) {
    zig::Ticket& tk = it->second;
    if (tk.comp.client != client) {
      ++it;
      continue;
    }
    ++n;
    if (tk.state == zig::kDone) {
      if (tk.bytes) s->arena.release(tk.off, tk.bytes);
      it = s->tickets.erase(it);
    } else {
      tk.orphan = true;
      ++it;
    }
  }
  if (reclaimed) *reclaimed = n;
  s->cv_done.notify_all();
  zig::wake_sched(s);
  return ZIG_OK;
}

int zig_server_counters(zig_server* srv, uint64_t* next_index, uint32_t count) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !next_index) return zig::fail(ZIG_EINVAL, "null argument");
  if (count > s->cfg.clients) return zig::fail(ZIG_EINVAL, "count exceeds the number of clients");
  std::unique_lock<std::mutex> lk(s->mu);  // no batch can be formed meanwhile
  s->cv_done.wait(lk, [&] { return s->launching == 0; });
  if (s->device) {
    const int r = zig::pay_owed_locked(s);
    if (r != ZIG_OK) return r;
    hipError_t e = hipSuccess;
    for (hipStream_t st : s->fill_streams)
      if (e == hipSuccess) e = hipStreamSynchronize(st);  // every launched batch has raised its counters
    if (e == hipSuccess)
      e = hipMemcpy(next_index, s->counters_dev, count * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return zig::fail(ZIG_EHIP, std::string("counter snapshot: ") + hipGetErrorString(e));
  } else {
    std::memcpy(next_index, s->next_host.data(), count * sizeof(uint64_t));
  }
  return ZIG_OK;
}

int zig_server_set_counters(zig_server* srv, const uint64_t* next_index, uint32_t count) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !next_index) return zig::fail(ZIG_EINVAL, "null argument");
  if (count > s->cfg.clients) return zig::fail(ZIG_EINVAL, "count exceeds the number of clients");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->intake.empty() || s->inflight_count) return zig::fail(ZIG_ESTATE, "server is not idle");
  if (s->device) {
    const hipError_t e =
        hipMemcpy(s->counters_dev, next_index, count * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return zig::fail(ZIG_EHIP, std::string("counter restore: ") + hipGetErrorString(e));
  }
  std::memcpy(s->next_host.data(), next_index, count * sizeof(uint64_t));
  std::fill(s->owed.begin(), s->owed.end(), 0);  // the restored values replace any owed raise
  s->any_owed = false;
  return ZIG_OK;
}

int zig_server_stats_get(zig_server* srv, zig_server_stats* out) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || !out) return zig::fail(ZIG_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->bytes_in_use = s->arena.used();
  out->queued = s->intake.size();
  out->inflight_batches = s->inflight_count;
  return ZIG_OK;
}

int zig_server_replay(zig_server* srv, const zig_trace_item* items, uint64_t count, uint32_t flags,
                      zig_completion* out) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s || (count && (!items || !out))) return zig::fail(ZIG_EINVAL, "null argument");
  if (flags & ~(uint32_t)ZIG_REPLAY_NAIVE) return zig::fail(ZIG_EINVAL, "unknown flags");
  for (uint64_t i = 0; i < count; ++i) {
    if (items[i].client >= s->cfg.clients)
      return zig::fail(ZIG_EINVAL, "trace item " + std::to_string(i) + ": client out of range");
    if (i && items[i].spec.t_arrival_ns < items[i - 1].spec.t_arrival_ns)
      return zig::fail(ZIG_EINVAL, "trace arrivals must not decrease");
  }
  if (flags & ZIG_REPLAY_NAIVE) return zig::replay_naive(s, items, count, out);
  return zig::replay_batched(s, items, count, out);
}

int zig_server_destroy(zig_server* srv) {
  zig::clear_error();
  Server* s = reinterpret_cast<Server*>(srv);
  if (!s) return ZIG_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop.store(true);
    zig::cancel_queued_locked(s, ZIG_ESTATE);
    zig::wake_sched(s);
    s->cv_inflight.notify_all();
  }
  s->sched.join();
  if (!s->device) {
    {
      std::lock_guard<std::mutex> fl(s->fake_mu);
      s->fake_cv.notify_all();
    }
    s->fake_worker.join();  // drains the queued fake batches first
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop_completers = true;
    s->cv_inflight.notify_all();
  }
  for (std::thread& t : s->completers) t.join();  // each returns once its stream's batches have completed
  if (s->device) zig::free_device(s);
  delete s;
  return ZIG_OK;
}

}  // extern "C"

namespace zig {
namespace {

// Batched replay: this thread keeps the arrival schedule; every request
// records its completion in `out` and returns its arena space as soon as it
// completes (its copy, if any, runs on the batch's stream before that).
int replay_batched(Server* s, const zig_trace_item* items, uint64_t count, zig_completion* out) {
  ReplaySink sink;
  sink.out = out;
  const uint64_t t0 = now_ns();
  int result = ZIG_OK;
  std::string message;
  for (uint64_t i = 0; i < count; ++i) {
    const uint64_t target = t0 + items[i].spec.t_arrival_ns;
    sleep_until_ns(target);
    zig_spec sp = items[i].spec;
    sp.t_arrival_ns = target;
    uint64_t tk = 0;
    const int r = submit_impl(s, items[i].client, sp, 0, &tk, &sink, i, items[i].copy_to);
    if (r != ZIG_OK) {
      if (result == ZIG_OK) {
        result = r;
        message = "trace item " + std::to_string(i) + ": " + zig_last_error();
      }
      std::lock_guard<std::mutex> lk(s->mu);
      std::memset(&out[i], 0, sizeof(out[i]));
      out[i].status = r;
      out[i].client = items[i].client;
      out[i].t_arrival_ns = target;
      sink.done += 1;
    }
  }
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return sink.done == count; });
  }
  if (result != ZIG_OK) set_error(message);
  for (uint64_t i = 0; i < count && result == ZIG_OK; ++i)
    if (out[i].status != ZIG_OK) {
      result = out[i].status;
      set_error("trace item " + std::to_string(i) + " failed");
    }
  return result;
}

// Naive server: every request launched on arrival as its own fill, on the
// fill streams in turn, with an event each; one completion thread per
// stream waits on that stream's oldest event.
int replay_naive(Server* s, const zig_trace_item* items, uint64_t count, zig_completion* out) {
  if (!s->device) return fail(ZIG_EINVAL, "the naive replay needs the device backend");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->intake.empty() || s->inflight_count || s->replaying_naive)
      return fail(ZIG_ESTATE, "server is not idle");
    s->replaying_naive = true;
  }
  const uint32_t K = s->cfg.streams;
  constexpr size_t kEvents = 1024;
  std::vector<hipEvent_t> pool;
  for (size_t i = 0; i < kEvents; ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) break;
    pool.push_back(e);
  }
  struct Out {
    uint64_t i, off, bytes;
    hipEvent_t ev;
  };
  std::mutex qm;
  std::condition_variable qc;  // a queue grew, an event was freed, or the submitter finished
  std::vector<std::deque<Out>> q(K);
  std::vector<hipEvent_t> free_ev = pool;
  bool submit_done = false;
  std::vector<uint64_t> counters(s->cfg.clients, 0);
  int result = ZIG_OK;
  std::string message;
  if (pool.size() != kEvents) {
    result = ZIG_EHIP;
    message = "naive replay: event pool";
  }
  auto complete = [&](uint32_t k) {
    (void)hipSetDevice(s->dev_id);
    std::unique_lock<std::mutex> lk(qm);
    for (;;) {
      qc.wait(lk, [&] { return submit_done || !q[k].empty(); });
      if (q[k].empty()) return;
      const Out d = q[k].front();
      lk.unlock();
      if (out[d.i].status == ZIG_OK) {
        for (;;) {  // poll without sleeping
          const hipError_t e = hipEventQuery(d.ev);
          if (e == hipSuccess) break;
          if (e != hipErrorNotReady) {
            out[d.i].status = ZIG_EHIP;
            break;
          }
          std::this_thread::yield();
        }
      }
      out[d.i].t_done_ns = now_ns();
      if (d.bytes) {
        std::lock_guard<std::mutex> al(s->mu);
        s->arena.release(d.off, d.bytes);
        zig::wake_sched(s);
      }
      lk.lock();
      q[k].pop_front();
      free_ev.push_back(d.ev);
      qc.notify_all();
    }
  };
  std::vector<std::thread> completers;
  for (uint32_t k = 0; k < K; ++k) completers.emplace_back(complete, k);
  const uint64_t t0 = now_ns();
  std::thread submitter([&] {
    (void)hipSetDevice(s->dev_id);
    for (uint64_t i = 0; i < count; ++i) {
      {
        std::lock_guard<std::mutex> lk(qm);
        if (result != ZIG_OK) break;
      }
      const zig_trace_item& it = items[i];
      const uint64_t target = t0 + it.spec.t_arrival_ns;
      sleep_until_ns(target);
      zig_completion& c = out[i];
      std::memset(&c, 0, sizeof(c));
      c.client = it.client;
      c.dist = it.spec.dist;
      c.dtype = it.spec.dtype;
      c.n = it.spec.n;
      c.seed = s->cfg.seed_base + it.client;
      c.t_arrival_ns = target;
      c.t_submit_ns = now_ns();
      const uint64_t esize = it.spec.dtype == ZIG_F64 ? 8 : 4;
      const uint64_t bytes = it.spec.n * esize;
      uint64_t off = 0;
      bool allocated = false;
      int r = ZIG_OK;
      if (it.spec.n > (s->cfg.cap_bytes & ~(uint64_t)255) / esize) {
        r = fail(ZIG_EINVAL, "request larger than the admission cap");
      } else if (bytes) {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_sched.wait(lk, [&] { return s->arena.fits(bytes); });
        allocated = s->arena.alloc(bytes, &off);
      }
      hipEvent_t ev = nullptr;
      {
        std::unique_lock<std::mutex> lk(qm);
        qc.wait(lk, [&] { return !free_ev.empty(); });
        ev = free_ev.back();
        free_ev.pop_back();
      }
      c.t_admit_ns = now_ns();
      c.first_index = counters[it.client];
      c.out = s->arena_dev + off;
      hipStream_t st = s->fill_streams[i % K];
      if (r == ZIG_OK && it.spec.n)
        r = zig_fill(it.spec.dist, it.spec.dtype, c.seed, c.first_index, it.spec.n, it.spec.p0, it.spec.p1, c.out,
                     st, nullptr);
      if (r == ZIG_OK) counters[it.client] += it.spec.n;
      if (r == ZIG_OK && it.copy_to && bytes &&
          hipMemcpyAsync(it.copy_to, c.out, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        r = fail(ZIG_EHIP, "output copy");
      if (r == ZIG_OK && hipEventRecord(ev, st) != hipSuccess) r = fail(ZIG_EHIP, "event record");
      c.t_launch_ns = now_ns();
      c.status = r;
      const std::string err = r == ZIG_OK ? std::string() : std::string(zig_last_error());
      if (r != ZIG_OK) {
        c.out = nullptr;
        if (allocated) {
          std::lock_guard<std::mutex> al(s->mu);
          s->arena.release(off, bytes);
          zig::wake_sched(s);
        }
      }
      std::lock_guard<std::mutex> lk(qm);
      if (r != ZIG_OK && result == ZIG_OK) {
        result = r;
        message = "naive replay item " + std::to_string(i) + ": " + err;
      }
      q[i % K].push_back(Out{i, off, r == ZIG_OK ? bytes : 0, ev});
      qc.notify_all();
    }
    std::lock_guard<std::mutex> lk(qm);
    submit_done = true;
    qc.notify_all();
  });
  submitter.join();
  for (std::thread& t : completers) t.join();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->replaying_naive = false;
    zig::wake_sched(s);
  }
  if (result != ZIG_OK) set_error(message);
  return result;
}

}  // namespace
}  // namespace zig
