// Host stress of the serving scheduler on the host fake backend (no device
// calls), built with sanitizers by test_host_sanitizers.py: concurrent
// submitters, a client that disconnects with work queued, an open-loop
// replay, counter snapshots and statistics while work is in flight,
// injected failures, and shutdown with requests still queued.  Exits 0 and
// prints "ok" when every per-client index sequence is contiguous.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../include/zig.h"

static void check(int r, const char* what) {
  if (r != ZIG_OK) {
    std::printf("FAIL %s: %d %s\n", what, r, zig_last_error());
    std::exit(1);
  }
}

int main() {
  for (int round = 0; round < 3; ++round) {
    zig_server_cfg cfg = {};
    cfg.backend = ZIG_BACKEND_HOST_FAKE;
    cfg.streams = 3;
    cfg.max_batch = 8;
    cfg.clients = 8;
    cfg.cap_bytes = 1 << 16;
    cfg.fake_latency_us = 50;
    cfg.fake_fail_every = 7;
    cfg.window_us = round == 1 ? 30 : 0;
    zig_server* s = nullptr;
    check(zig_server_create(&cfg, &s), "create");
    std::vector<std::thread> th;
    std::vector<int> bad(6, 0);
    for (int c = 0; c < 6; ++c)
      th.emplace_back([&, c] {
        std::vector<uint64_t> t;
        for (int i = 0; i < 200; ++i) {
          zig_spec sp = {};
          sp.dist = i & 1;
          sp.dtype = (i >> 1) & 1;
          sp.n = 1 + (i * 37 + c) % 300;
          sp.p0 = 1.0;
          sp.p1 = 1.0;
          uint64_t tk = 0;
          check(zig_server_submit(s, c, &sp, 0, &tk), "submit");
          t.push_back(tk);
        }
        uint64_t next = 0;
        for (uint64_t tk : t) {
          zig_completion cc;
          if (zig_server_wait(s, tk, -1, &cc) == ZIG_OK) {
            if (cc.first_index != next) bad[c] = 1;
            next += cc.n;
          }
          zig_server_release(s, tk);
        }
      });
    th.emplace_back([&] {  // a client that disconnects with work queued
      for (int i = 0; i < 50; ++i) {
        zig_spec sp = {};
        sp.n = 100;
        sp.p0 = 1.0;
        uint64_t tk = 0;
        zig_server_submit(s, 6, &sp, 0, &tk);
      }
      uint64_t n = 0;
      zig_server_drop_client(s, 6, &n);
    });
    th.emplace_back([&] {  // an open-loop replay on client 7
      std::vector<zig_trace_item> tr(300);
      std::vector<zig_completion> out(300);
      for (int i = 0; i < 300; ++i) {
        tr[i] = zig_trace_item{};
        tr[i].client = 7;
        tr[i].spec.n = 1 + i;
        tr[i].spec.p0 = 2.0;
        tr[i].spec.t_arrival_ns = i * 3000ull;
      }
      zig_server_replay(s, tr.data(), tr.size(), 0, out.data());
    });
    th.emplace_back([&] {  // observers
      zig_server_stats st;
      uint64_t c[8];
      for (int i = 0; i < 100; ++i) {
        zig_server_stats_get(s, &st);
        zig_server_counters(s, c, 8);
        std::this_thread::yield();
      }
    });
    for (auto& t : th) t.join();
    for (int c = 0; c < 6; ++c)
      if (bad[c]) {
        std::printf("FAIL client %d indices not contiguous\n", c);
        return 1;
      }
    for (int i = 0; i < 40; ++i) {  // queued work for the shutdown
      zig_spec sp = {};
      sp.n = 4000;
      sp.p0 = 1.0;
      uint64_t tk = 0;
      zig_server_submit(s, 0, &sp, 0, &tk);
    }
    check(zig_server_destroy(s), "destroy");
  }
  std::printf("ok\n");
  return 0;
}
