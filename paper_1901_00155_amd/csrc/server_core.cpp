// server_core.cpp -- request scheduler of the serving loop (host C++ only).
//
// Requests are copied at submit and wait in one FIFO queue.  A worker thread per
// slot takes the head of the queue as soon as the head's footprint fits in the
// free part of the arena (strict FIFO: a large request at the head is never
// overtaken, so it cannot starve), runs it through the executor without holding
// the lock, returns its arena block and appends a completion.  Every shared
// field is guarded by one mutex; workers sleep on a condition variable that
// submit and every completion signal.
#include "server_core.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace dd {

struct ArenaAllocator::Impl {
  std::map<size_t, size_t> free_blocks;   // offset -> size, disjoint and non-adjacent
};

ArenaAllocator::ArenaAllocator(size_t capacity)
    : impl_(new Impl), capacity_(capacity / kAlign * kAlign) {
  if (capacity_) impl_->free_blocks.emplace(0, capacity_);
}

ArenaAllocator::~ArenaAllocator() { delete impl_; }

size_t ArenaAllocator::alloc(size_t bytes) {
  const size_t b = std::max(round(bytes), kAlign);
  auto& fb = impl_->free_blocks;
  for (auto it = fb.begin(); it != fb.end(); ++it) {
    if (it->second < b) continue;
    const size_t off = it->first, rest = it->second - b;
    fb.erase(it);
    if (rest) fb.emplace(off + b, rest);
    in_use_ += b;
    return off;
  }
  return kNone;
}

size_t ArenaAllocator::alloc_at(size_t off, size_t bytes) {
  const size_t b = std::max(round(bytes), kAlign);
  if (off % kAlign || off > capacity_ || b > capacity_ - off) return kNone;
  auto& fb = impl_->free_blocks;
  auto it = fb.upper_bound(off);            // first free block starting after off
  if (it == fb.begin()) return kNone;
  --it;                                      // the free block starting at or before off
  const size_t s = it->first, e = it->first + it->second;
  if (off + b > e) return kNone;
  fb.erase(it);
  if (off > s) fb.emplace(s, off - s);
  if (off + b < e) fb.emplace(off + b, e - off - b);
  in_use_ += b;
  return off;
}

void ArenaAllocator::release(size_t offset, size_t bytes) {
  const size_t b = std::max(round(bytes), kAlign);
  auto& fb = impl_->free_blocks;
  auto it = fb.emplace(offset, b).first;
  auto nx = std::next(it);
  if (nx != fb.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    fb.erase(nx);
  }
  if (it != fb.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      fb.erase(it);
    }
  }
  in_use_ -= b;
}

size_t ArenaAllocator::free_blocks() const { return impl_->free_blocks.size(); }

}  // namespace dd

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
  uint64_t tag = 0;
  std::vector<float> T;
  int64_t m = 0;
  int32_t n = 0;
  size_t bytes = 0;
  double t_submit = 0.0;
};

}  // namespace

struct discord_server_s {
  discord_server_config cfg{};
  discord_executor_fn exec = nullptr;
  void* ctx = nullptr;
  char* arena = nullptr;
  void (*fini)(void*) = nullptr;
  Clock::time_point t0 = Clock::now();

  std::mutex mu;
  std::condition_variable cv_work;   // queue grew, a block was freed, or stop
  std::condition_variable cv_done;   // a completion arrived, or stop
  std::deque<Pending> queue;
  std::deque<discord_completion> done;
  dd::ArenaAllocator alloc;
  std::vector<std::thread> workers;
  bool stop = false;

  uint64_t submitted = 0, rejected = 0, completed = 0, failed = 0;
  int32_t running = 0, peak_running = 0;
  size_t peak_bytes = 0;
  double busy_ms = 0.0;

  explicit discord_server_s(size_t budget) : alloc(budget) {}
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
  void worker(int slot);
  void shutdown();
};

void discord_server_s::worker(int slot) {
  std::unique_lock<std::mutex> lk(mu);
  // the block of this slot's previous request: a request of the same footprint
  // gets it back when it is free, so a slot that serves one shape keeps its
  // device addresses (and can replay its captured graph)
  size_t last_off = dd::ArenaAllocator::kNone, last_bytes = 0;
  for (;;) {
    size_t off = dd::ArenaAllocator::kNone;
    while (!stop) {
      if (!queue.empty()) {
        const size_t want = queue.front().bytes;
        if (want == last_bytes) off = alloc.alloc_at(last_off, want);
        if (off == dd::ArenaAllocator::kNone) off = alloc.alloc(want);
        if (off != dd::ArenaAllocator::kNone) break;
      }
      cv_work.wait(lk);
    }
    if (off == dd::ArenaAllocator::kNone) return;   // stopping

    Pending rq = std::move(queue.front());
    queue.pop_front();
    last_off = off;
    last_bytes = rq.bytes;
    ++running;
    peak_running = std::max(peak_running, running);
    peak_bytes = std::max(peak_bytes, alloc.in_use());
    const double t_admit = now_ms();
    lk.unlock();

    discord_request view;
    view.tag = rq.tag;
    view.T = rq.T.data();
    view.m = rq.m;
    view.n = rq.n;
    view.slot = slot;
    view.workspace = arena ? arena + off : nullptr;
    view.ws_offset = off;
    view.ws_bytes = rq.bytes;
    discord_completion c;
    std::memset(&c, 0, sizeof(c));
    int st = exec(ctx, &view, &cfg.opts, &c.result, c.detail, sizeof(c.detail));
    c.detail[sizeof(c.detail) - 1] = 0;
    if (st != DISCORD_OK) std::memset(&c.result, 0, sizeof(c.result));
    std::vector<float>().swap(rq.T);   // the host copy is no longer needed
    c.tag = rq.tag;
    c.status = st;
    c.slot = slot;
    c.ws_offset = off;
    c.ws_bytes = rq.bytes;
    c.t_submit_ms = rq.t_submit;
    c.t_admit_ms = t_admit;

    lk.lock();
    c.t_done_ms = now_ms();
    alloc.release(off, rq.bytes);
    --running;
    ++completed;
    if (st < 0) ++failed;
    busy_ms += c.t_done_ms - t_admit;
    done.push_back(c);
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

void discord_server_s::shutdown() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  cv_done.notify_all();
  for (auto& t : workers)
    if (t.joinable()) t.join();
  workers.clear();
  queue.clear();
  if (fini) fini(ctx);
  fini = nullptr;
}

namespace dd {

int server_create(const discord_server_config* cfg, discord_executor_fn exec, void* ctx,
                  void* arena, void (*fini)(void*), discord_server* out) {
  auto cleanup = [&] {
    if (fini) fini(ctx);
  };
  if (!out) {
    cleanup();
    return DISCORD_EINVAL;
  }
  *out = nullptr;
  if (!cfg || !exec || cfg->slots < 1 || cfg->slots > 64 || cfg->max_queued < 0 ||
      cfg->hbm_budget_bytes < ArenaAllocator::kAlign ||
      discord_workspace_bytes(64, 8, &cfg->opts) == 0) {
    cleanup();
    return DISCORD_EINVAL;
  }
  discord_server s = new (std::nothrow) discord_server_s(cfg->hbm_budget_bytes);
  if (!s) {
    cleanup();
    return DISCORD_ENOMEM;
  }
  s->cfg = *cfg;
  if (s->cfg.max_queued == 0) s->cfg.max_queued = 65536;
  s->exec = exec;
  s->ctx = ctx;
  s->arena = static_cast<char*>(arena);
  s->fini = fini;
  try {
    s->workers.reserve(cfg->slots);
    for (int i = 0; i < cfg->slots; ++i) s->workers.emplace_back([s, i] { s->worker(i); });
  } catch (...) {
    s->shutdown();
    delete s;
    return DISCORD_ENOMEM;
  }
  *out = s;
  return DISCORD_OK;
}

}  // namespace dd

extern "C" {

int discord_server_create_with_executor(const discord_server_config* cfg, discord_executor_fn exec,
                                        void* ctx, discord_server* out) {
  return dd::server_create(cfg, exec, ctx, nullptr, nullptr, out);
}

int discord_server_submit(discord_server s, const float* T, int64_t m, int32_t n, uint64_t tag) {
  if (!s) return DISCORD_EINVAL;
  auto reject = [s](int st) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rejected;
    return st;
  };
  if (!T || n < 1 || m < 2 * (int64_t)n) return reject(DISCORD_EINVAL);
  if (s->cfg.opts.precision == DISCORD_PREC_BF16X3 && n > DISCORD_MIXED_MAX_N)
    return reject(DISCORD_ERANGE);
  const size_t fp = discord_workspace_bytes(m, n, &s->cfg.opts);
  if (fp == 0) return reject(DISCORD_EINVAL);
  const size_t bytes = dd::ArenaAllocator::round(fp);
  if (bytes > s->alloc.capacity()) return reject(DISCORD_ENOMEM);
  Pending p;
  try {
    p.T.assign(T, T + m);
  } catch (...) {
    return reject(DISCORD_ENOMEM);
  }
  p.tag = tag;
  p.m = m;
  p.n = n;
  p.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      ++s->rejected;
      return DISCORD_EBUSY;
    }
    if ((int64_t)s->queue.size() >= s->cfg.max_queued) {
      ++s->rejected;
      return DISCORD_EBUSY;
    }
    p.t_submit = s->now_ms();
    try {
      s->queue.push_back(std::move(p));
    } catch (...) {
      ++s->rejected;
      return DISCORD_ENOMEM;
    }
    ++s->submitted;
  }
  s->cv_work.notify_one();
  return DISCORD_OK;
}

int discord_server_poll(discord_server s, discord_completion* out, int32_t max, int32_t timeout_ms,
                        int32_t* count) {
  if (!s || !count || max < 0 || (max > 0 && !out)) return DISCORD_EINVAL;
  *count = 0;
  const int32_t wait = std::min(std::max(timeout_ms, 0), 60000);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait > 0 && max > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait),
                        [s] { return !s->done.empty() || s->stop; });
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *count = k;
  return DISCORD_OK;
}

int discord_server_get_stats(discord_server s, discord_server_stats* out) {
  if (!s || !out) return DISCORD_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->rejected = s->rejected;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int32_t)s->queue.size();
  out->running = s->running;
  out->peak_running = s->peak_running;
  out->slots = s->cfg.slots;
  out->budget_bytes = s->alloc.capacity();
  out->bytes_in_use = s->alloc.in_use();
  out->peak_bytes_in_use = s->peak_bytes;
  out->busy_ms = s->busy_ms;
  out->elapsed_ms = s->now_ms();
  return DISCORD_OK;
}

void discord_server_destroy(discord_server s) {
  if (!s) return;
  s->shutdown();
  delete s;
}

}  // extern "C"
