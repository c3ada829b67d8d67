// Host stress test of the serving scheduler (server_core.cpp) under ThreadSanitizer
// or AddressSanitizer: several submitter threads, concurrent pollers, a fake
// executor that checks that the arena blocks of running requests are disjoint and
// within the budget, and a destroy while requests are still queued.
//
// Build (done by tests/test_server_cpu.py):
//   g++ -std=c++17 -O1 -g -fsanitize=thread tests/native/server_stress.cpp \
//       paper_1901_00155_amd/csrc/server_core.cpp -o server_stress -lpthread
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../../include/discord.h"

// footprint stand-in for the library's discord_workspace_bytes: 4 bytes per
// (row, window element) plus a fixed part; 0 on invalid sizes
extern "C" size_t discord_workspace_bytes(int64_t m, int32_t n, const discord_opts*) {
  if (n < 1 || m < 2 * (int64_t)n) return 0;
  return (size_t)(m - n + 1) * 4 + 1000;
}

namespace {

constexpr size_t kBudget = 1 << 20;
std::mutex g_mu;
std::map<size_t, size_t> g_live;   // offset -> bytes of running requests
std::atomic<int> g_errors{0};
std::atomic<int> g_running{0};
std::atomic<int> g_peak{0};

void fail(const char* what) {
  std::fprintf(stderr, "FAIL: %s\n", what);
  g_errors.fetch_add(1);
}

int fake_exec(void*, const discord_request* rq, const discord_opts*, discord_result* out,
              char* detail, size_t len) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t used = rq->ws_bytes;
    for (auto& kv : g_live) {
      used += kv.second;
      const bool disjoint = rq->ws_offset + rq->ws_bytes <= kv.first ||
                            kv.first + kv.second <= rq->ws_offset;
      if (!disjoint) fail("overlapping arena blocks");
    }
    if (used > kBudget) fail("budget exceeded");
    if (rq->ws_offset + rq->ws_bytes > kBudget) fail("block beyond the arena");
    if (rq->ws_offset % 256) fail("unaligned block");
    g_live[rq->ws_offset] = rq->ws_bytes;
  }
  const int r = g_running.fetch_add(1) + 1;
  int p = g_peak.load();
  while (r > p && !g_peak.compare_exchange_weak(p, r)) {
  }
  // deterministic "result" from the series only
  double acc = 0.0;
  int64_t arg = 0;
  for (int64_t i = 0; i < rq->m; ++i)
    if (rq->T[i] > rq->T[arg]) arg = i;
  for (int64_t i = 0; i < rq->m; ++i) acc += rq->T[i];
  std::this_thread::sleep_for(std::chrono::microseconds(50 + (rq->tag % 7) * 30));
  g_running.fetch_sub(1);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_live.erase(rq->ws_offset);
  }
  if (rq->tag % 97 == 13) {
    std::snprintf(detail, len, "planted failure %llu", (unsigned long long)rq->tag);
    return DISCORD_ECONST;
  }
  out->index = arg;
  out->d2 = acc;
  return DISCORD_OK;
}

}  // namespace

int main() {
  discord_server_config cfg{};
  cfg.hbm_budget_bytes = kBudget;
  cfg.slots = 6;
  cfg.max_queued = 100000;
  cfg.opts.precision = DISCORD_PREC_FP32;
  cfg.opts.abandon = 1;
  cfg.opts.order = 1;
  cfg.opts.paa_w = 4;
  cfg.opts.alphabet = 4;
  discord_server s = nullptr;
  if (discord_server_create_with_executor(&cfg, fake_exec, nullptr, &s) != DISCORD_OK) {
    std::fprintf(stderr, "create failed\n");
    return 2;
  }
  constexpr int kThreads = 4, kPer = 300;
  std::atomic<int> accepted{0};
  std::vector<std::thread> subs;
  for (int t = 0; t < kThreads; ++t) {
    subs.emplace_back([&, t] {
      std::vector<float> T;
      for (int k = 0; k < kPer; ++k) {
        const uint64_t tag = (uint64_t)t * kPer + k;
        const int64_t m = 256 + (int64_t)((tag * 7919) % 60000);
        T.resize(m);
        for (int64_t i = 0; i < m; ++i) T[i] = (float)((i * 31 + tag) % 1009);
        const int st = discord_server_submit(s, T.data(), m, 16, tag);
        if (st == DISCORD_OK) accepted.fetch_add(1);
        else fail("submit refused a valid request");
      }
      // invalid and oversized requests are refused without disturbing the rest
      if (discord_server_submit(s, T.data(), 10, 16, 999999) != DISCORD_EINVAL) fail("EINVAL");
      std::vector<float> big(kBudget / 2);
      if (discord_server_submit(s, big.data(), (int64_t)big.size(), 16, 999998) != DISCORD_ENOMEM)
        fail("ENOMEM");
    });
  }
  std::set<uint64_t> seen;
  std::mutex seen_mu;
  std::atomic<bool> subs_done{false};
  std::atomic<int> got{0}, failed{0};
  std::vector<std::thread> pollers;
  for (int q = 0; q < 2; ++q) {
    pollers.emplace_back([&] {
      discord_completion buf[16];
      for (;;) {
        int32_t c = 0;
        if (discord_server_poll(s, buf, 16, 5, &c) != DISCORD_OK) fail("poll");
        for (int i = 0; i < c; ++i) {
          std::lock_guard<std::mutex> lk(seen_mu);
          if (!seen.insert(buf[i].tag).second) fail("duplicate completion");
          if (buf[i].status != DISCORD_OK) {
            failed.fetch_add(1);
            if (buf[i].tag % 97 != 13) fail("unexpected failure");
          } else if (buf[i].tag % 97 == 13) {
            fail("planted failure lost");
          }
          if (buf[i].t_admit_ms < buf[i].t_submit_ms || buf[i].t_done_ms < buf[i].t_admit_ms)
            fail("clock order");
        }
        got.fetch_add(c);
        if (subs_done.load() && got.load() >= accepted.load()) return;
      }
    });
  }
  for (auto& t : subs) t.join();
  subs_done.store(true);
  for (auto& t : pollers) t.join();

  discord_server_stats st{};
  discord_server_get_stats(s, &st);
  if ((int)st.completed != accepted.load()) fail("completed count");
  if ((int)st.failed != failed.load()) fail("failed count");
  if (st.bytes_in_use != 0 || st.running != 0 || st.queued != 0) fail("leftover state");
  if (st.peak_bytes_in_use > kBudget) fail("peak bytes");
  if (st.rejected != 2 * kThreads) fail("rejected count");

  // destroy with requests still queued: the running ones finish, the rest are dropped
  std::vector<float> T(50000, 1.0f);
  for (int k = 0; k < 200; ++k) T[k] = (float)k, discord_server_submit(s, T.data(), 50000, 16, 500000 + k);
  discord_server_destroy(s);

  std::printf("requests %d failed %d peak_running %d peak_bytes %zu errors %d\n", accepted.load(),
              failed.load(), g_peak.load(), st.peak_bytes_in_use, g_errors.load());
  if (g_errors.load() == 0) std::printf("OK\n");
  return g_errors.load() == 0 ? 0 : 1;
}
