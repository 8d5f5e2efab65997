// Host stress program for the scratch-slot ring (zig_ring.hpp) on a
// simulated device: each stream is a worker thread running its queue in
// order, events complete when their stream reaches them, and a "kernel"
// checks that it holds its slot alone and that the slot's counters start
// at zero, as the fill kernel requires, then leaves them at zero.  Many
// host threads launch at once, several of them through the same stream
// object (the way threads share a special handle such as the per-thread
// stream's), over a ring far smaller than the launches in flight.
// Prints "ok" when no kernel ever saw its slot busy or dirty.
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_1403_6870_amd/csrc/zig_ring.hpp"

namespace {

struct FakeStream {
  std::mutex m;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool stop = false;
  std::thread worker;

  FakeStream() {
    worker = std::thread([this] {
      for (;;) {
        std::function<void()> task;
        {
          std::unique_lock<std::mutex> lk(m);
          cv.wait(lk, [this] { return stop || !q.empty(); });
          if (q.empty()) return;
          task = std::move(q.front());
          q.pop_front();
        }
        task();
      }
    });
  }
  void enqueue(std::function<void()> f) {
    std::lock_guard<std::mutex> lk(m);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void finish() {
    {
      std::lock_guard<std::mutex> lk(m);
      stop = true;
      cv.notify_all();
    }
    worker.join();
  }
};

struct FakeEvent {
  std::mutex m;
  std::condition_variable cv;
  uint64_t recorded = 0, done = 0;
};

struct FakeOps {
  using Event = FakeEvent*;
  using Stream = FakeStream*;
  static int wait(FakeStream* s, FakeEvent* e) {
    uint64_t t;
    {
      std::lock_guard<std::mutex> lk(e->m);
      t = e->recorded;
    }
    s->enqueue([e, t] {
      std::unique_lock<std::mutex> lk(e->m);
      e->cv.wait(lk, [e, t] { return e->done >= t; });
    });
    return 0;
  }
  static int record(FakeEvent* e, FakeStream* s) {
    uint64_t t;
    {
      std::lock_guard<std::mutex> lk(e->m);
      t = ++e->recorded;
    }
    s->enqueue([e, t] {
      std::lock_guard<std::mutex> lk(e->m);
      if (e->done < t) e->done = t;
      e->cv.notify_all();
    });
    return 0;
  }
};

// One slot of simulated device scratch: an occupancy flag for the check
// and the counter pair a fill kernel uses.
struct Slot {
  std::atomic<int> busy{0};
  std::atomic<uint32_t> next{0}, done{0};
};

std::atomic<long> g_bad{0}, g_runs{0};

}  // namespace

int main() {
  constexpr int kStreams = 4, kThreads = 8, kLaunches = 3000;
  constexpr uint32_t kSlots = 3;
  std::vector<std::unique_ptr<FakeStream>> streams;
  for (int i = 0; i < kStreams; ++i) streams.emplace_back(new FakeStream());
  std::vector<Slot> slots(kSlots);
  std::vector<std::unique_ptr<FakeEvent>> events;
  zig::SlotRing<FakeOps> ring;
  ring.base = reinterpret_cast<char*>(slots.data());
  ring.slot_bytes = sizeof(Slot);
  ring.slots = kSlots;
  for (uint32_t k = 0; k < kSlots; ++k) {
    events.emplace_back(new FakeEvent());
    ring.ev.push_back(events.back().get());
  }
  ring.recorded.assign(kSlots, 0);

  std::vector<std::thread> hosts;
  for (int h = 0; h < kThreads; ++h) {
    hosts.emplace_back([&, h] {
      std::mt19937 rng(1234 + h);
      for (int i = 0; i < kLaunches; ++i) {
        // threads 0 and 1 share stream 0, the others pick at random
        FakeStream* s = streams[h < 2 ? 0 : rng() % kStreams].get();
        const int work = (int)(rng() % 4);
        const int rc = zig::ring_launch(&ring, s, [&](void* p) {
          Slot* slot = static_cast<Slot*>(p);
          s->enqueue([slot, work] {
            if (slot->busy.exchange(1) != 0) g_bad.fetch_add(1);
            if (slot->next.load() != 0 || slot->done.load() != 0) g_bad.fetch_add(1);
            for (int w = 0; w <= work; ++w) {
              slot->next.fetch_add(1);
              std::this_thread::yield();
            }
            slot->done.fetch_add(1);
            // the last workgroup leaves the pair at zero for the next user
            slot->next.store(0);
            slot->done.store(0);
            slot->busy.store(0);
            g_runs.fetch_add(1);
          });
          return 0;
        });
        if (rc != 0) g_bad.fetch_add(1);
      }
    });
  }
  for (auto& t : hosts) t.join();
  for (auto& s : streams) s->finish();
  const long runs = g_runs.load(), bad = g_bad.load();
  std::printf("launches %ld, violations %ld\n", runs, bad);
  if (runs != (long)kThreads * kLaunches || bad != 0) return 1;
  std::printf("ok\n");
  return 0;
}
