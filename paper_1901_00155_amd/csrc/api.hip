// api.hip -- host runtime of libdiscord: the C ABI of include/discord.h.
//
// A plan owns (or borrows) one device arena holding the padded series, the
// preparation structures of PhiDD (Algorithm 2) and the search/certification
// buffers.  Every step of the method runs in this library's kernels; the host
// only orders launches and reads back counts and the final result.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/discord.h"
#include "internal.hpp"

namespace dd {

void sax_breakpoints(int alpha, double* out) {
  // beta_k = Phi^{-1}(k / alpha), k = 1..alpha-1, by Newton's method on
  // Phi(x) = erfc(-x / sqrt(2)) / 2 from x = 0 (Phi is monotone with a
  // positive density, and the targets lie in [1/8, 7/8]).
  const double inv_sqrt2 = 0.70710678118654752440;
  const double inv_sqrt2pi = 0.39894228040143267794;
  for (int k = 1; k < alpha; ++k) {
    const double p = (double)k / (double)alpha;
    double x = 0.0;
    for (int it = 0; it < 100; ++it) {
      const double f = 0.5 * std::erfc(-x * inv_sqrt2) - p;
      const double dens = inv_sqrt2pi * std::exp(-0.5 * x * x);
      const double nx = x - f / dens;
      if (nx == x) break;
      x = nx;
    }
    if (2 * k == alpha) x = 0.0;   // the median is exactly 0
    out[k - 1] = x;
  }
  for (int k = alpha - 1; k < 8; ++k) out[k] = HUGE_VAL;
}

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kRowPad = 64;   // zero rows after N in the FP32 row-statistics arrays

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The small per-search counters, in one block so that one fill clears them and
// one copy reads them back.  The best-so-far, which every scanning wavefront
// polls after each step, and the pair counter, which every wavefront adds to,
// sit on cache lines of their own (sharing one with the other counters made the
// polls wait behind the atomics: the first window of a walk1m search took 2x
// as long).
struct SearchScalars {
  alignas(128) uint64_t pairs;   // pair distances evaluated (the sum of the pair slots)
  alignas(128) uint32_t bsf;     // best-so-far (float bits)
  alignas(128) uint64_t seed;    // packed (distance, ~row) of the certification seed
  uint32_t n_surv;               // survivors of the last window launch
  uint32_t n_aband;              // rows left early
  uint32_t unc_count;            // rows the witnesses could not clear
  uint32_t relerr;               // largest relative error checked (float bits)
  int32_t n_cand_groups;         // items holding Cand rows
};
static_assert(sizeof(SearchScalars) % 4 == 0, "filled as 32-bit words");

// What a plan reads back to the host: the preparation's statistics and
// counts, and the search's counters and certified answer.  The arena holds
// one block with this same layout, so each readback is a single copy (a copy
// into pageable memory waits on the host before the next one can start).
struct HostOut {
  SearchScalars sc;
  Exact ex;
  double stats[8];   // eq. (2): mean, sigma (as laid out on the device) ...
  int32_t bad[4];    // ... followed by the NaN/Inf flag
  int32_t cand[8];   // |Cand| at [0], the longest bucket at [4]
};
static_assert(offsetof(HostOut, sc) == 0, "the search's readback starts at the block");
static_assert(offsetof(HostOut, bad) == offsetof(HostOut, stats) + sizeof(double) * 8 &&
                  offsetof(HostOut, cand) == offsetof(HostOut, bad) + sizeof(int32_t) * 4,
              "the statistics, the flag and the counts are copied as one");
constexpr size_t kPrepareOut = offsetof(HostOut, stats);   // the preparation's part
constexpr size_t kPrepareOutBytes = sizeof(HostOut) - kPrepareOut;
constexpr size_t kSearchOutBytes = offsetof(HostOut, ex) + sizeof(Exact);

struct Layout {
  // out: the block laid out as HostOut; stats (8 doubles of eq. (2)), the
  // NaN/Inf flag (`bad`), cand_count (|Cand| followed by the longest bucket,
  // `max_bucket`), srch and exact are its fields
  size_t T, out, stats, partials, bad, words, hist, minfreq, cand, cand_count, seg, csr_off, csr_mem,
      best, nn_approx, nn_wit, row_state, row_mean, row_cnorm, rows, part_d, part_j, out_d,
      out_j, exact, unc, srch, pair_slots, alive, done, survivors, survivors2, score, rank_hist, gflags,
      cand_groups, bgrp_cnt, bgrp_off, bgrp, max_bucket, mu32, smu32, cn32, r32, row_sigma,
      ctl, wins, lb, lb_range, lb_bmin, lb_bmax, bflags, total;
};

// work descriptors of one search: the Cand and bound launches and one or two
// per round (window, completion); rounds grow the window 2x at least, so a
// sequence of 2^31 entries needs fewer than 40 rounds
constexpr int kMaxWins = 128;

Layout make_layout(int64_t m, int32_t n, int dict, bool mixed, bool znorm) {
  const int64_t N = m - n + 1;
  const int64_t nchunks = (N + kFp64Cols - 1) / kFp64Cols;
  const int64_t seg = std::max<int64_t>(csr_waves(N) * dict, compact_waves(N));
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.T = take(sizeof(float) * (size_t)(kFrontPad + m + kBackPad));
  L.out = take(sizeof(HostOut));
  L.srch = L.out + offsetof(HostOut, sc);
  L.exact = L.out + offsetof(HostOut, ex);
  L.stats = L.out + offsetof(HostOut, stats);
  L.bad = L.out + offsetof(HostOut, bad);
  L.cand_count = L.out + offsetof(HostOut, cand);
  L.max_bucket = L.cand_count + sizeof(int32_t) * 4;
  L.partials = take(sizeof(double) * kStatBlocks);
  L.words = take(sizeof(int32_t) * N);
  L.hist = take(sizeof(int32_t) * kMaxWords);
  L.minfreq = take(sizeof(int32_t) * 4);
  L.cand = take(sizeof(int32_t) * N);
  L.seg = take(sizeof(int32_t) * seg);
  L.csr_off = take(sizeof(int32_t) * (kMaxWords + 1));
  L.csr_mem = take(sizeof(int32_t) * N);
  L.best = take(sizeof(uint64_t) * N);
  L.nn_approx = take(sizeof(float) * N);
  L.nn_wit = take(sizeof(int32_t) * N);
  L.row_state = take(sizeof(int32_t) * N);
  L.row_mean = take(sizeof(double) * N);
  L.row_cnorm = take(sizeof(double) * N);
  L.rows = take(sizeof(int64_t) * kFp64BatchRows);
  L.part_d = take(sizeof(double) * kFp64BatchRows * nchunks);
  L.part_j = take(sizeof(int64_t) * kFp64BatchRows * nchunks);
  L.out_d = take(sizeof(double) * kFp64BatchRows);
  L.out_j = take(sizeof(int64_t) * kFp64BatchRows);
  L.unc = take(sizeof(int64_t) * N);
  const int64_t G = (N + kRowGroup - 1) / kRowGroup;
  L.ctl = take(sizeof(SearchCtl));
  L.wins = take(sizeof(WinDesc) * kMaxWins);
  L.pair_slots = take(sizeof(uint64_t) * kPairSlots * kPairStride);
  L.alive = take(sizeof(uint32_t) * G);
  L.done = take(sizeof(uint32_t) * G);
  L.survivors = take(sizeof(int32_t) * G);
  L.survivors2 = take(sizeof(int32_t) * G);
  L.score = take(sizeof(uint32_t) * G);
  L.rank_hist = take(sizeof(uint32_t) * rank_hist_bins());
  L.gflags = take(sizeof(int32_t) * G);
  L.bflags = take(sizeof(int32_t) * G);
  L.cand_groups = take(sizeof(int32_t) * G);
  L.bgrp_cnt = take(sizeof(int32_t) * kMaxWords);
  L.bgrp_off = take(sizeof(int32_t) * (kMaxWords + 1));
  L.bgrp = take(sizeof(int32_t) * N);
  L.mu32 = take(sizeof(float) * (N + kRowPad));
  L.smu32 = take(sizeof(float) * (N + kRowPad));
  L.cn32 = take(sizeof(float) * (N + kRowPad));
  // per-window normalisation: FP64 row standard deviations, FP32 row scales
  L.r32 = take(znorm ? sizeof(float) * (N + kRowPad) : 0);
  L.row_sigma = take(znorm ? sizeof(double) * N : 0);
  // the mean-gap bound of every row's NN (global normalisation only: under
  // per-window normalisation every window has mean 0)
  L.lb = take(znorm ? 0 : sizeof(float) * N);
  L.lb_range = take(znorm ? 0 : sizeof(uint64_t) * 2);
  L.lb_bmin = take(znorm ? 0 : sizeof(int32_t) * bound_bins());
  L.lb_bmax = take(znorm ? 0 : sizeof(int32_t) * bound_bins());
  L.total = off;
  return L;
}

bool opts_valid(int32_t n, const discord_opts& o) {
  if (o.precision != DISCORD_PREC_FP32 && o.precision != DISCORD_PREC_BF16X3) return false;
  if (o.abandon != 0 && o.abandon != 1) return false;
  if (o.order < 0 || o.order > 2) return false;
  if (o.znorm != 0 && o.znorm != 1) return false;
  (void)n;
  if (o.paa_w < 1 || o.paa_w > 8) return false;
  if (o.alphabet < 2 || o.alphabet > 8) return false;
  int64_t dict = 1;
  for (int k = 0; k < o.paa_w; ++k) dict *= o.alphabet;
  return dict <= kMaxWords;
}

int dict_size(const discord_opts& o) {
  int d = 1;
  for (int k = 0; k < o.paa_w; ++k) d *= o.alphabet;
  return d;
}

}  // namespace
}  // namespace dd

using namespace dd;

struct discord_plan_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* arena = nullptr;
  bool own_arena = false;
  Layout L{};
  int64_t m = 0, N = 0;
  int32_t n = 0;
  discord_opts opts{};
  int dict = 256;
  double mu = 0.0, sigma = 0.0;
  int64_t cand_count = 0;
  int64_t max_bucket = 0;     // longest word bucket, in scan column blocks
  double ms_prepare = 0.0;
  bool searched = false;
  bool timed = true;          // false: no HIP events (the allocation-free entry point)
  // false: the preparation skips Index_Word (eq. (10)), which only the PhiDD
  // order's sequences and the introspection of a kept plan read
  bool index_word = true;
  hipGraphExec_t gexec = nullptr;   // the search captured by discord_search_graph
  int glaunches = 0;                // scan launches in that graph
  void* hout = nullptr;             // pinned block the captured search reads back into
  char err[512] = {0};

  template <class P>
  P* at(size_t off) const {
    return reinterpret_cast<P*>(arena + off);
  }
  float* Tp() const { return at<float>(L.T) + kFrontPad; }
};

namespace {

int fail(discord_plan p, int code, const char* fmt, ...) {
  if (p) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p->err, sizeof(p->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIP_TRY(plan, expr)                                                                  \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(plan, DISCORD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

int check_launch(discord_plan p, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(p, DISCORD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return DISCORD_OK;
}

#define LAUNCH_OK(plan, what)                       \
  do {                                              \
    int st_ = check_launch(plan, what);             \
    if (st_ != DISCORD_OK) return st_;              \
  } while (0)

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// HIP events, reused: each host thread keeps a pool that grows as needed and
// lives until the process ends (a serving worker times every request with the
// same events instead of creating and destroying them per call).  A search or
// preparation synchronises its stream before it returns, so the events are idle
// whenever the next call on the thread takes them.  Pair 0 brackets a whole
// preparation or search and keeps the default system-scope release; the pairs
// around the scan launches only time device work, so they release to the
// device, and their interval holds the kernel rather than a system-scope
// write-back.  Each record is still a packet of its own in the queue, a few us
// between the kernels it separates; untimed searches (graphs, the
// allocation-free entry point) take none.
struct EventPool {
  int device = -1;
  std::vector<hipEvent_t> ev;
  hipEvent_t get(size_t k) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (dev != device) {   // another device: start a new pool (the old events stay valid)
      ev.clear();
      device = dev;
    }
    while (ev.size() <= k) {
      hipEvent_t e = nullptr;
      const unsigned flags = ev.size() >= 2 ? hipEventReleaseToDevice : hipEventDefault;
      if (hipEventCreateWithFlags(&e, flags) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      ev.push_back(e);
    }
    return ev[k];
  }
};
thread_local EventPool g_events;

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float t = 0.f;
  if (!a || !b || hipEventElapsedTime(&t, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return t;
}

// on = false: no events are taken (a plan that must not create runtime
// objects); recording is then a no-op and the time reads 0
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  bool on = true;
  explicit EventPair(size_t slot, bool use = true) : on(use) {
    if (on) {
      a = g_events.get(2 * slot);
      b = g_events.get(2 * slot + 1);
    }
  }
  bool ready() const { return !on || (a && b); }
  hipError_t start(hipStream_t s) const { return on ? hipEventRecord(a, s) : hipSuccess; }
  hipError_t stop(hipStream_t s) const { return on ? hipEventRecord(b, s) : hipSuccess; }
  float ms() const { return on ? elapsed_ms(a, b) : 0.f; }
};

ZStats zstats(discord_plan p) {
  if (!p->opts.znorm) return ZStats{nullptr, nullptr};
  return ZStats{p->at<double>(p->L.row_mean), p->at<double>(p->L.row_sigma)};
}

int rows_nn_batch(discord_plan p, const int64_t* d_rows, int64_t count) {
  launch_rows_nn_fp64(p->Tp(), p->n, p->N, d_rows, count, zstats(p), p->at<double>(p->L.part_d),
                      p->at<int64_t>(p->L.part_j), p->at<double>(p->L.out_d),
                      p->at<int64_t>(p->L.out_j), p->stream);
  LAUNCH_OK(p, "rows_nn_fp64");
  return DISCORD_OK;
}

}  // namespace

extern "C" {

void discord_default_opts(discord_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = DISCORD_PREC_FP32;
  o->abandon = 1;
  o->order = 2;
  o->paa_w = 4;
  o->alphabet = 4;
}

int32_t discord_abi_version(void) { return DISCORD_ABI_VERSION; }

const char* discord_strerror(int status) {
  switch (status) {
    case DISCORD_OK: return "ok";
    case DISCORD_EINVAL: return "invalid argument (NULL series, n < 1, m < 2n, non-finite value or bad option)";
    case DISCORD_ECONST: return "constant series: sigma == 0, z-normalisation undefined";
    case DISCORD_ENOMEM: return "not enough device memory or workspace too small";
    case DISCORD_EDEVICE: return "HIP runtime error";
    case DISCORD_EBUSY: return "busy";
    case DISCORD_ERANGE: return "size beyond a documented limit";
    default: return "unknown status";
  }
}

static thread_local char g_prepare_err[512];

}  // extern "C"

void dd::set_thread_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_prepare_err, sizeof(g_prepare_err), fmt, ap);
  va_end(ap);
}

extern "C" {

const char* discord_plan_error(discord_plan p) { return p ? p->err : g_prepare_err; }

size_t discord_workspace_bytes(int64_t m, int32_t n, const discord_opts* opts) {
  discord_opts o;
  if (opts) o = *opts; else discord_default_opts(&o);
  if (n >= 1 && o.paa_w >= 1 && o.paa_w <= 8 && o.paa_w > n) o.paa_w = n;
  if (n < 1 || m < 2 * (int64_t)n || !opts_valid(n, o)) return 0;
  if (m > (int64_t)INT32_MAX - kBackPad - kFrontPad) return 0;
  if (o.precision == DISCORD_PREC_BF16X3 && n > kMixedMaxN) return 0;
  return make_layout(m, n, dict_size(o), o.precision == DISCORD_PREC_BF16X3, o.znorm != 0).total;
}

}  // extern "C"

namespace {

// Validates the arguments of a preparation; *o receives the options in use.
int check_prepare_args(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                       discord_opts* o) {
  if (opts) *o = *opts; else discord_default_opts(o);
  if (o->paa_w >= 1 && o->paa_w <= 8 && o->paa_w > n) o->paa_w = n;   // eq. (3) needs w <= n
  if (!T || n < 1 || m < 2 * (int64_t)n || !opts_valid(n, *o)) return DISCORD_EINVAL;
  if (m > (int64_t)INT32_MAX - kBackPad - kFrontPad) return DISCORD_ERANGE;
  if (o->precision == DISCORD_PREC_BF16X3 && n > kMixedMaxN) return DISCORD_ERANGE;
  return DISCORD_OK;
}

void init_plan(discord_plan p, int64_t m, int32_t n, const discord_opts& o) {
  p->m = m;
  p->n = n;
  p->N = m - n + 1;
  p->opts = o;
  p->dict = dict_size(o);
  p->L = make_layout(m, n, p->dict, o.precision == DISCORD_PREC_BF16X3, o.znorm != 0);
}


// The preparation kernels on a plan whose arena and stream are set, with no
// host synchronisation: on a series with NaN/Inf or sigma = 0 they run on
// meaningless values (every index they form stays in range), and the search
// loop stops at once (control.hip) -- the error is reported from the readback.
int prepare_enqueue(discord_plan p, const float* T) {
  const int64_t m = p->m;
  const int32_t n = p->n;
  const discord_opts& o = p->opts;
  hipStream_t s = p->stream;
  // padded series: zero pads, then the values
  float* Tbase = p->at<float>(p->L.T);
  {
    const FillOp fills[] = {
        {Tbase, kFrontPad, 0, 0},
        {Tbase + kFrontPad + m, kBackPad, 0, 0},
        {p->at<int32_t>(p->L.bad), 4, 0, 0},
        {p->at<int32_t>(p->L.hist), kMaxWords, 0, 0},
    };
    launch_fill_many(fills, 4, s);
  }
  const hipMemcpyKind kind = is_device_pointer(T) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(p, hipMemcpyAsync(p->Tp(), T, sizeof(float) * m, kind, s));
  // eq. (2)
  launch_stats(p->Tp(), m, p->at<double>(p->L.partials), p->at<double>(p->L.stats),
               p->at<int32_t>(p->L.bad), s);
  LAUNCH_OK(p, "stats");
  // row statistics, the mean-gap bound, PAA -> SAX -> word ids, histogram,
  // Cand, Index_Word
  const bool zn = o.znorm != 0;
  double* row_sigma = zn ? p->at<double>(p->L.row_sigma) : nullptr;
  launch_row_stats(p->Tp(), p->N, n, p->at<double>(p->L.row_mean), p->at<double>(p->L.row_cnorm),
                   row_sigma, s);
  if (!zn)
    launch_row_bound(p->at<double>(p->L.row_mean), p->N, n, p->at<uint64_t>(p->L.lb_range),
                     p->at<int32_t>(p->L.lb_bmin), p->at<int32_t>(p->L.lb_bmax),
                     p->at<float>(p->L.lb), s);
  launch_sax(p->Tp(), p->N, n, o.paa_w, o.alphabet, p->at<double>(p->L.stats),
             zn ? p->at<double>(p->L.row_mean) : nullptr, row_sigma,
             p->at<int32_t>(p->L.words), p->at<int32_t>(p->L.hist), s);
  launch_cand(p->at<int32_t>(p->L.words), p->at<int32_t>(p->L.hist), p->N, p->dict,
              p->at<int32_t>(p->L.minfreq), p->at<int32_t>(p->L.seg), p->at<int32_t>(p->L.cand),
              p->at<int32_t>(p->L.cand_count), s);
  if (p->index_word)
    launch_csr(p->at<int32_t>(p->L.words), p->at<int32_t>(p->L.hist), p->N, p->dict,
               p->at<int32_t>(p->L.seg), p->at<int32_t>(p->L.csr_off),
               p->at<int32_t>(p->L.csr_mem), s);
  const bool mixed = o.precision == DISCORD_PREC_BF16X3;
  // FP32 centres and scales: the split-BF16 operands, and under per-window
  // normalisation also the FP32 scan's
  float* r32 = zn ? p->at<float>(p->L.r32) : nullptr;
  if (mixed || zn)
    launch_row_stats32(p->Tp(), p->N, n, p->N + kRowPad, p->at<double>(p->L.row_mean), row_sigma,
                       p->at<double>(p->L.stats), p->at<float>(p->L.mu32),
                       p->at<float>(p->L.smu32), p->at<float>(p->L.cn32), r32, s);
  // the bucket column blocks serve only the PhiDD order (same-word columns first)
  if (o.order == 1) {
    // (bucket entries are the scan's column blocks: 8 or 128 columns)
    launch_bucket_groups(p->at<int32_t>(p->L.csr_off), p->at<int32_t>(p->L.csr_mem), p->dict,
                         mixed ? 7 : 3,
                         p->at<int32_t>(p->L.bgrp_cnt), p->at<int32_t>(p->L.bgrp_off),
                         p->at<int32_t>(p->L.bgrp), s);
    launch_max_bucket(p->at<int32_t>(p->L.bgrp_off), p->dict, p->at<int32_t>(p->L.max_bucket), s);
  }
  LAUNCH_OK(p, "prepare kernels");
  p->cand_count = -1;   // on the device only, until a readback
  p->max_bucket = -1;
  return DISCORD_OK;
}

// Copies of the preparation's statistics and counts into h.
int prepare_readback(discord_plan p, HostOut* h) {
  HIP_TRY(p, hipMemcpyAsync(reinterpret_cast<char*>(h) + kPrepareOut, p->arena + p->L.out +
                            kPrepareOut, kPrepareOutBytes, hipMemcpyDeviceToHost, p->stream));
  return DISCORD_OK;
}

// After the copies of prepare_readback have landed: the errors of eq. (2) and
// the counts the host uses.
int prepare_check(discord_plan p, const HostOut& h) {
  if (h.bad[0]) return fail(p, DISCORD_EINVAL, "series holds NaN or Inf");
  p->mu = h.stats[0];
  p->sigma = h.stats[1];
  if (!(p->sigma > 0.0)) return fail(p, DISCORD_ECONST, "sigma == 0");
  p->cand_count = h.cand[0];
  p->max_bucket = p->opts.order == 1 ? h.cand[4] : 0;
  return DISCORD_OK;
}

// The preparation of discord_prepare: the kernels and one synchronisation.
int prepare_run(discord_plan p, const float* T) {
  EventPair ev(0, p->timed);
  hipStream_t s = p->stream;
  if (!ev.ready()) return fail(p, DISCORD_EDEVICE, "hipEventCreate failed");
  HIP_TRY(p, ev.start(s));
  int st = prepare_enqueue(p, T);
  if (st != DISCORD_OK) return st;
  HostOut h;
  if ((st = prepare_readback(p, &h)) != DISCORD_OK) return st;
  HIP_TRY(p, ev.stop(s));
  HIP_TRY(p, hipStreamSynchronize(s));
  if ((st = prepare_check(p, h)) != DISCORD_OK) return st;
  p->ms_prepare = ev.ms();
  return DISCORD_OK;
}

}  // namespace

extern "C" {

int discord_prepare(const float* T, int64_t m, int32_t n, const discord_opts* opts, void* workspace,
                    size_t ws_bytes, void* stream, discord_plan* out) {
  if (!out) return DISCORD_EINVAL;
  *out = nullptr;
  g_prepare_err[0] = 0;
  discord_opts o;
  const int bad = check_prepare_args(T, m, n, opts, &o);
  if (bad != DISCORD_OK) return bad;

  discord_plan p = new (std::nothrow) discord_plan_s();
  if (!p) return DISCORD_ENOMEM;
  init_plan(p, m, n, o);
  auto bail = [&](int st) {
    discord_release(p);
    return st;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return bail(DISCORD_EDEVICE);
  if (stream) {
    p->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(DISCORD_EDEVICE);
    p->own_stream = true;
  }
  if (workspace) {
    if (ws_bytes < p->L.total || ((uintptr_t)workspace % kAlign) != 0) return bail(DISCORD_ENOMEM);
    p->arena = (char*)workspace;
  } else {
    if (hipMalloc(&p->arena, p->L.total) != hipSuccess) {
      (void)hipGetLastError();
      p->arena = nullptr;
      return bail(DISCORD_ENOMEM);
    }
    p->own_arena = true;
  }
  const int st = prepare_run(p, T);
  if (st != DISCORD_OK) {
    // keep the message for the caller: copy before release
    std::snprintf(g_prepare_err, sizeof(g_prepare_err), "%s", p->err);
    return bail(st);
  }
  *out = p;
  return DISCORD_OK;
}

}  // extern "C"

namespace {

constexpr int64_t kDevRows = 8;   // uncertain rows rescanned before the readback

// One search in flight.  timed: event pairs taken for ms_scan (0, or 1: pair 1
// spans the scan launches); events are taken only if the plan is timed and the
// search is not being captured into a graph.
struct SearchRun {
  HostOut* h = nullptr;
  bool events = true;
  bool with_prepare = false;   // the readback also carries the preparation's part
  int timed = 0;
  int launches = 0;   // scan launches enqueued
};

// Enqueues the whole search on the plan's stream, up to the copies of its
// counters and answer into run.h; nothing here waits for the device, so the
// sequence can also be captured into a graph.
int search_enqueue(discord_plan p, SearchRun& run) {
  hipStream_t s = p->stream;
  const int64_t N = p->N;
  const int n = p->n;
  int& timed = run.timed;
  HIP_TRY(p, hipSetDevice(p->device));

  const bool mixed = p->opts.precision == DISCORD_PREC_BF16X3;
  // rows per scan group: 8 (FP32 micro-tile) or 32 (one MFMA tile side)
  const int gsz = mixed ? kMixedBlock : kRowGroup;
  const int64_t G = (N + gsz - 1) / gsz;
  // row groups per work item: one wavefront (FP32) or one workgroup (MFMA)
  const int rb = mixed ? kMixedItemBlocks : 1;
  // the unit of the scan's lists: one row group (FP32) or one workgroup's fixed
  // set of rb row blocks (MFMA)
  const int64_t item_rows = (int64_t)gsz * rb;
  int item_shift = 0;
  while ((int64_t{1} << item_shift) < item_rows) ++item_shift;
  const int64_t n_items = (N + item_rows - 1) / item_rows;
  // work items a window launch aims at: about 4 wavefronts per SIMD (split-
  // BF16 workgroups, FP32 under per-window normalisation); FP32 searches under
  // global normalisation, in 256-column steps, gain from more: 10240 below
  // 2^21 rows, 16384 from there (against 6144: 2^20 walk 4.60 -> 4.49 ms,
  // noisy walk 5.69 -> 5.56 ms; 2^22 series 35.7 -> 32.1 ms, 10^7-point walk
  // n = 1024 509 -> 430 ms; per-window normalisation 8.5 -> 8.6 ms at 10240)
  // FP32 early abandon in the near-first order: 256-column steps (most rows
  // meet a neighbour below the best-so-far within their first 256 columns);
  // the PhiDD and matrix orders keep 512 (2^20 walk 164 -> 183 and 718 -> 762
  // ms with 256)
  const bool fine = !mixed && p->opts.abandon && p->opts.order == 2;
  const int64_t target_items =
      mixed ? 1024
            : (p->opts.znorm ? 4096 : (fine ? (N >= (int64_t{1} << 21) ? 16384 : 10240) : 6144));
  // The launch that completes the bound-ranked items holds few items with
  // long sequences, so it is split finer: 16384 work items (FP32), 2048
  // (split-BF16).
  const int64_t seed_items = mixed ? 2048 : 16384;
  const bool abandon = p->opts.abandon != 0;
  const bool order = p->opts.order != 0;          // Cand first (Algorithm 3)
  const bool buckets = p->opts.order == 1;        // same-word columns first
  const bool near_first = p->opts.order == 2;     // columns nearest the row first
  uint64_t* best = p->at<uint64_t>(p->L.best);
  SearchScalars* sc = p->at<SearchScalars>(p->L.srch);
  uint64_t* pairs = p->at<uint64_t>(p->L.pair_slots);
  uint32_t* bsf = &sc->bsf;
  uint32_t* alive = p->at<uint32_t>(p->L.alive);
  uint32_t* n_surv = &sc->n_surv;
  int32_t* gflags = p->at<int32_t>(p->L.gflags);
  {
    // one launch clears the search state (the alive masks follow below)
    const FillOp fills[] = {
        {best, N, kEmptyMin, 1},
        {sc, (int64_t)(sizeof(SearchScalars) / 4), 0, 0},
        {pairs, (int64_t)kPairSlots * kPairStride, 0, 1},
        {p->at<uint32_t>(p->L.done), G, 0, 0},
        {gflags, G, 0, 0},
        {p->at<int32_t>(p->L.bflags), G, 0, 0},
    };
    launch_fill_many(fills, abandon ? 6 : 3, s);
  }
  // ---- approximate scan (Algorithms 3 and 4) ----------------------------------
  ScanJob J{};
  J.Tp = p->Tp();
  J.n = n;
  J.N = N;
  J.best = best;
  J.pairs = pairs;
  J.bsf = bsf;
  J.alive = alive;
  J.done = p->at<uint32_t>(p->L.done);
  J.survivors = p->at<int32_t>(p->L.survivors);
  J.n_survivors = n_surv;
  const bool zn = p->opts.znorm != 0;
  const MixedRows R{p->at<float>(p->L.mu32), p->at<float>(p->L.smu32), p->at<float>(p->L.cn32),
                    zn ? p->at<float>(p->L.r32) : nullptr};
  J.raise_sub = 0.0f;
  if (zn && !mixed) {
    J.zc = p->at<float>(p->L.mu32);
    J.zr = p->at<float>(p->L.r32);
  }
  if (mixed) {
    // The split-BF16 minima carry errors of order 2^-16 |a'||b'|, with no
    // simple relative bound; raising the best-so-far by a 2^-10 margin is a
    // heuristic only -- the FP64 certification below keeps the result exact
    // whatever the best-so-far was.
    J.raise_scale = (float)(1.0 - std::ldexp(1.0, -10));
  } else if (zn) {
    // Normalised FP32 form q_i + q_j - 2 C s_i s_j: C is a sum of n products of
    // centred values, off by at most about (n + 2) 2^-24 n sigma_i sigma_j, and
    // s_i s_j carries two more roundings; the distance is then off by less than
    // 2.2 (n + 4) n 2^-24 + 16 n 2^-24 in absolute terms (the quantities are at
    // most 4n), which completed rows subtract before raising the best-so-far.
    J.raise_scale = 1.0f;
    J.raise_sub = (float)((2.2 * (n + 4.0) * n + 16.0 * n) * std::ldexp(1.0, -24));
  } else {
    // A row whose scan completed has exact NN >= (its FP32 minimum) / (1 + gamma),
    // gamma = (n + 3) 2^-24 bounding the direct-form rounding; raising the
    // best-so-far by that lower bound keeps it <= the discord's NN.
    J.raise_scale = (float)(1.0 - ((n + 3) * std::ldexp(1.0, -24) * 1.01 + std::ldexp(1.0, -22)));
  }
  // The scan launches are timed as one span, from an event before the first
  // to one after the last.  An event record is a packet of its own in the
  // queue and costs a few us between the kernels it separates: a pair per
  // launch cost about 0.1 ms of a search of the 2^20 walk.  The span also
  // holds the small kernels between the scans (the one-thread window
  // decisions, a few us each; the rankings of per-window normalisation).
  EventPair span(1, run.events);
  if (!span.ready()) return fail(p, DISCORD_EDEVICE, "hipEventCreate failed");
  bool span_open = false;
  auto launch = [&](const char* what) -> int {
    ++run.launches;
    if (run.events && !span_open) {
      HIP_TRY(p, span.start(s));
      span_open = true;
    }
    if (mixed) {
      if (!launch_scan_mfma(J, R, s)) return fail(p, DISCORD_ERANGE, "window too long for bf16x3");
    } else {
      launch_scan_fp32(J, s);
    }
    LAUNCH_OK(p, what);
    return DISCORD_OK;
  };
  // Sequence entries are column groups of 8 (FP32) or blocks of 128 (MFMA); a
  // sequence is at most the word bucket plus every column block.
  const int64_t col_w = mixed ? kMixedCols : (fine ? kColBlockSearch : kColBlock);
  const int64_t nq = (N + col_w - 1) / col_w;
  if (buckets && p->max_bucket < 0) return fail(p, DISCORD_EDEVICE, "bucket sizes not read back");
  const int64_t seq_max = nq + (buckets ? p->max_bucket : 0);
  const int64_t gran = 512 / col_w;   // entries per 512 columns
  // entries [begin, end) of every listed item, split into chunks so that the
  // launch holds enough work items to fill the GPU
  auto set_window = [&](int64_t groups, int64_t begin, int64_t end, int64_t target) {
    const int64_t items = std::max<int64_t>(1, groups);
    const int64_t width = std::max<int64_t>(end - begin, 1);
    const int64_t maxc = (width + gran - 1) / gran;
    const int64_t c = std::min<int64_t>(maxc, std::max<int64_t>(1, (target + items - 1) / items));
    J.seq_begin = begin;
    J.seq_chunk = ((width + c - 1) / c + gran - 1) / gran * gran;
    J.chunks = (width + J.seq_chunk - 1) / J.seq_chunk;
  };
  int st = DISCORD_OK;
  if (!abandon) {
    J.abandon = 0;
    J.n_groups = n_items;
    set_window(n_items, 0, nq, target_items);
    if ((st = launch("scan (full)"))) return st;
  } else {
    J.abandon = 1;
    launch_init_alive(alive, G, N, gsz, s);
    J.words = buckets ? p->at<int32_t>(p->L.words) : nullptr;
    J.bgrp_off = p->at<int32_t>(p->L.bgrp_off);
    J.bgrp = p->at<int32_t>(p->L.bgrp);
    J.near_first = near_first;
    // The whole loop is enqueued now and decided on the device (control.hip):
    // for the near-first order first the items with the largest mean-gap
    // bound, then a Cand launch (Algorithm 3), then rounds of Algorithm 4 over
    // every other item -- a window of each listed item's sequence, the items
    // with rows still live continuing in a window `growth` times longer (for
    // the other orders the survivors finish in a second window).  Every launch
    // resumes an item where its previous window ended, and rows already below
    // the best-so-far leave before any work.  The host mirrors the window
    // sizes to know how many rounds the sequences allow; a loop that ends
    // sooner leaves the remaining launches without work.
    SearchCtl* ctl = p->at<SearchCtl>(p->L.ctl);
    WinDesc* wins = p->at<WinDesc>(p->L.wins);
    // Ranked rounds (near-first order under per-window normalisation, where
    // the mean-gap bound is zero): after each window the items still searched
    // are ranked by the largest published minimum of a live row, the
    // best-ranked are completed at once to raise the best-so-far, and the rest
    // continue.  With the bound-ranked items completed first (global
    // normalisation) the best-so-far is already near its final value and these
    // completions only cost time (FP32 2^20 walk 8.0 -> 6.6 ms without them).
    const bool ranked = near_first && zn;
    // first window: 2 steps of 512 columns in the near-first order (4 for
    // split-BF16 in ranked rounds; without them 2 took the 2^20 walk 4.6 ->
    // 4.1 ms)
    const int probe = p->opts.probe_steps > 0 ? p->opts.probe_steps
                                              : (near_first ? ((ranked && mixed) ? 4 : 2) : 16);
    // windows grow 4x, 2x on sequences of 2^20 entries and more (measured
    // with the bound-ranked items completed first: FP32 2^20 walk 6.6 -> 6.2
    // ms with 4x; FP32 10^7-point walk n = 1024 613 -> 559 ms with 2x); in
    // ranked rounds 2x from 2^15 entries
    // (sequence lengths counted in blocks of 8 FP32 or 128 split-BF16 columns)
    const int64_t seq_units = mixed ? seq_max : seq_max * col_w / kColBlock;
    const int64_t growth = seq_units >= (int64_t{1} << (ranked ? 15 : 20)) ? 2 : 4;
    // ranked rounds: items completed after each ranking (split-BF16: 16
    // workgroup items; FP32 groups: more for longer windows)
    const int64_t seeds = mixed ? 16 : (n >= 1024 ? 512 : (n >= 512 ? 256 : 128));
    // shortest chunk of the launches that complete whole sequences, in 512
    // columns: FP32 4 (2^20 walk 5.86 -> 5.60 ms, noisy walk 7.82 -> 7.53 ms,
    // 2^22 series 47.7 -> 47.2 ms: the bound-ranked launch had 2 steps per
    // wavefront); split-BF16 1 (2 and 4 were no better across the workloads);
    // a minimum on the windows or the ranked completions did not help either
    const int64_t min_full = mixed ? 1 : 4;
    const CtlParams P{seq_max, gran, target_items, seed_items, growth, seeds, near_first ? 1 : 0,
                      min_full * gran};
    // A launch whose work is decided on the device gets a grid sized for the
    // most work its descriptor can hold, at most `cap` work items (beyond, its
    // wavefronts or workgroups stride over the work).
    const int64_t cap = mixed ? 16384 : 65536;
    auto grid_work = [&](int64_t items_max, int64_t width_max, int64_t target) {
      const int64_t maxc = (std::max<int64_t>(width_max, 1) + gran - 1) / gran;
      return std::min(cap, std::min(items_max * maxc, items_max + target));
    };
    int nw = 0;
    // |Cand| is known on the host after discord_prepare; in a request run as
    // one sequence (prepare and search together) it exists only on the device
    const bool cand_known = p->cand_count >= 0;
    const bool cand = order && (!cand_known || p->cand_count > 0);
    const int64_t cand_max = cand_known ? std::min<int64_t>(n_items, p->cand_count) : n_items;
    if (cand) {
      // Algorithm 3: the items holding Cand rows, each over its whole sequence
      launch_cand_group_flags(p->at<int32_t>(p->L.cand), p->at<int32_t>(p->L.cand_count),
                              cand_known ? p->cand_count : N, item_shift, gflags, s);
      launch_compact_flags(gflags, n_items, p->at<int32_t>(p->L.seg),
                           p->at<int32_t>(p->L.cand_groups), &sc->n_cand_groups, s);
    }
    const int64_t width0 = (int64_t)probe * gran;
    // split-BF16: 2 items of 128 rows up to n = 512, 8 beyond (time to
    // discord: 2^20 walk n = 128 3.25 ms with 2, 3.35 with 8; 10^7-point walk
    // n = 2048 420 ms with 8, 1290 with 2; n = 1024 109 / 113 ms)
    const int64_t bound_seeds =
        (near_first && !zn) ? std::min<int64_t>(n_items, mixed ? ((n + 15) / 16 > 32 ? 8 : 2) : 16)
                            : 0;
    WinDesc* cand_win = cand ? &wins[nw++] : nullptr;
    WinDesc* bound_win = bound_seeds > 0 ? &wins[nw++] : nullptr;
    launch_ctl_start(ctl, n_items, width0, &sc->n_cand_groups, cand_win, bound_seeds, bound_win,
                     p->at<double>(p->L.stats), p->at<int32_t>(p->L.bad), P, s);
    // survivor lists: round r lists its survivors in lists[r & 1]; the bound
    // ranking goes to lists[1] before the first round
    int32_t* const lists[2] = {p->at<int32_t>(p->L.survivors), p->at<int32_t>(p->L.survivors2)};
    int32_t* const spare = lists[1];
    // Near-first order, global normalisation: first of all, the items whose
    // rows have the largest mean-gap bound of their NN (bound.hip) are
    // completed, which puts the best-so-far near its final value; the Cand
    // rows and every later window then leave early against it.  These items
    // are skipped by the Cand launch and the first window.  16 FP32 groups
    // measured best among 1..64 (time to discord against none: 2^20 walk
    // n = 128 12.3 -> 8.3 ms; 2^20 noisy walk n = 256 22.9 -> 10.3 ms; 2^22
    // series n = 512 277 -> 65 ms, with these items searched after Cand).
    int32_t* bflags = p->at<int32_t>(p->L.bflags);
    if (bound_seeds > 0) {
      launch_item_bound(p->at<float>(p->L.lb), N, item_rows, n_items, p->at<uint32_t>(p->L.score),
                        s);
      launch_rank_scores(nullptr, &ctl->count, n_items, p->at<uint32_t>(p->L.score),
                         p->at<uint32_t>(p->L.rank_hist), spare, s);
      LAUNCH_OK(p, "bound ranking");
      J.win = bound_win;
      J.groups = spare;
      J.max_work = grid_work(bound_seeds, seq_max, seed_items);
      J.skip = nullptr;
      J.precheck = 0;
      if ((st = launch("scan (bound seeds)"))) return st;
      launch_flag_items(spare, bound_seeds, bound_win, gflags, bflags, s);
    }
    if (cand) {
      // Algorithm 3: the items holding Cand rows, each over its whole sequence
      J.win = cand_win;
      J.groups = p->at<int32_t>(p->L.cand_groups);
      J.skip = bound_seeds > 0 ? bflags : nullptr;
      J.precheck = 0;
      J.max_work = grid_work(cand_max, seq_max, target_items);
      if ((st = launch("scan (Cand)"))) return st;
    }
    int64_t covered = 0, width = width0;   // the device's window sizes while its loop runs
    for (int round = 0;; ++round) {
      const int64_t end = std::min<int64_t>(seq_max, covered + width);
      if (nw + 2 > kMaxWins) return fail(p, DISCORD_EDEVICE, "search needs too many rounds");
      WinDesc* w = &wins[nw++];
      // the first window, or the next one after a ranking; else the decision
      // after the previous window and this window's description in one launch
      if (round == 0 || ranked)
        launch_ctl_window(ctl, w, n_surv, P, s);
      else
        launch_ctl_next(ctl, w, n_surv, P, s);
      J.win = w;
      // lists: ranked rounds read the ranked list (`spare`, past its completed
      // head) and always list survivors in lists[0]; otherwise the lists alternate
      J.groups = round == 0 ? nullptr : (ranked ? spare : lists[(round - 1) & 1]);
      J.skip = (round == 0 && (cand || bound_seeds > 0)) ? gflags : nullptr;
      J.precheck = round > 0;
      J.survivors = ranked ? lists[0] : lists[round & 1];
      J.max_work = grid_work(n_items, end - covered, target_items);
      if ((st = launch("scan (window)"))) return st;
      if (end >= seq_max) break;                  // final for every item
      if (ranked) launch_ctl_after(ctl, n_surv, P, s);
      covered = end;
      width = near_first ? width * growth : seq_max;
      if (ranked) {
        launch_rank_groups(lists[0], &ctl->count, n_items, item_rows, gsz, alive, best, N,
                           p->at<uint32_t>(p->L.score), p->at<uint32_t>(p->L.rank_hist), spare, s);
        LAUNCH_OK(p, "rank");
        WinDesc* ws = &wins[nw++];
        launch_ctl_seeds(ctl, ws, P, s);
        J.win = ws;
        J.groups = spare;
        J.skip = nullptr;
        J.precheck = 1;
        J.max_work = grid_work(std::min<int64_t>(seeds, n_items), seq_max - covered, seed_items);
        if ((st = launch("scan (seeds)"))) return st;
        launch_ctl_post(ctl, s);
      }
    }
    J.win = nullptr;
  }
  if (span_open) {
    HIP_TRY(p, span.stop(s));
    timed = 1;
  }

  // ---- certification in FP64 ---------------------------------------------------
  launch_sum_pairs(pairs, &sc->pairs, s);
  float* nn_approx = p->at<float>(p->L.nn_approx);
  int32_t* nn_wit = p->at<int32_t>(p->L.nn_wit);
  int32_t* row_state = p->at<int32_t>(p->L.row_state);
  uint32_t* n_aband = &sc->n_aband;
  launch_unpack_best(best, N, abandon ? alive : nullptr, gsz, nn_approx, nn_wit, row_state, n_aband,
                     s);
  uint64_t* seed = &sc->seed;
  launch_seed_argmax(best, row_state, N, seed, s);
  int64_t* rows = p->at<int64_t>(p->L.rows);
  launch_seed_row(seed, rows, s);
  st = rows_nn_batch(p, rows, 1);
  if (st) return st;
  Exact* ex = p->at<Exact>(p->L.exact);
  launch_exact_from_rows(rows, p->at<double>(p->L.out_d), p->at<int64_t>(p->L.out_j), 1, ex, s);
  uint32_t* unc_count = &sc->unc_count;
  uint32_t* relerr = &sc->relerr;
  int64_t* unc = p->at<int64_t>(p->L.unc);
  launch_verify(p->Tp(), n, N, zstats(p), nn_wit, nn_approx, ex, unc, unc_count, relerr, s);
  LAUNCH_OK(p, "verify");
  // the first rows the witnesses could not clear (usually none) are rescanned
  // before the one readback; more than that continue in host-sized batches
  launch_rows_nn_fp64(p->Tp(), n, N, unc, kDevRows, zstats(p), p->at<double>(p->L.part_d),
                      p->at<int64_t>(p->L.part_j), p->at<double>(p->L.out_d),
                      p->at<int64_t>(p->L.out_j), s, unc_count);
  launch_merge_exact(unc, p->at<double>(p->L.out_d), p->at<int64_t>(p->L.out_j), kDevRows, ex,
                     nn_wit, s, unc_count);
  LAUNCH_OK(p, "rescan");
  // the counters and the answer (HostOut.sc, .ex), with the preparation's
  // statistics and counts behind them when the caller has not read those yet
  HIP_TRY(p, hipMemcpyAsync(run.h, p->arena + p->L.out,
                            run.with_prepare ? sizeof(HostOut) : kSearchOutBytes,
                            hipMemcpyDeviceToHost, s));
  return DISCORD_OK;
}

// After the copies of search_enqueue have landed: the uncertain rows beyond the
// device batch (rare) are rescanned here, then the result is filled in.
// `ev` brackets the search for ms_search (its stop is recorded again after
// the extra rescans).
int search_finish(discord_plan p, SearchRun& run, const EventPair& ev, discord_result* out) {
  hipStream_t s = p->stream;
  const int64_t N = p->N;
  const int n = p->n;
  SearchScalars* sc = p->at<SearchScalars>(p->L.srch);
  Exact* ex = p->at<Exact>(p->L.exact);
  int32_t* nn_wit = p->at<int32_t>(p->L.nn_wit);
  int64_t* unc = p->at<int64_t>(p->L.unc);
  (void)sc;
  (void)N;
  (void)n;
  const HostOut& h = *run.h;
  const uint32_t hunc = h.sc.unc_count, hrel = h.sc.relerr, hab = h.sc.n_aband;
  const uint64_t hpairs = h.sc.pairs;
  Exact hex = h.ex;
  if ((int64_t)hunc > kDevRows) {
    for (int64_t b = kDevRows; b < (int64_t)hunc; b += kFp64BatchRows) {
      const int64_t c = std::min<int64_t>(kFp64BatchRows, (int64_t)hunc - b);
      const int st = rows_nn_batch(p, unc + b, c);
      if (st) return st;
      launch_merge_exact(unc + b, p->at<double>(p->L.out_d), p->at<int64_t>(p->L.out_j), c, ex,
                         nn_wit, s);
      LAUNCH_OK(p, "merge_exact");
    }
    HIP_TRY(p, hipMemcpyAsync(&hex, ex, sizeof(hex), hipMemcpyDeviceToHost, s));
    HIP_TRY(p, ev.stop(s));
    HIP_TRY(p, hipStreamSynchronize(s));
  }
  if (hex.i < 0) return fail(p, DISCORD_EDEVICE, "certification produced no discord");

  discord_result r;
  std::memset(&r, 0, sizeof(r));
  const bool zn = p->opts.znorm != 0;
  r.index = hex.i;
  r.nn_index = hex.j;
  r.d2 = hex.d2;
  r.distance_raw = std::sqrt(hex.d2);
  r.distance = zn ? r.distance_raw : r.distance_raw / p->sigma;
  r.mu = p->mu;
  r.sigma = p->sigma;
  r.max_rel_err = (double)__builtin_bit_cast(float, hrel);
  r.certified = 1;
  r.precision = p->opts.precision;
  r.rows_rescored = 1 + hunc;
  r.rows_abandoned = hab;
  r.pairs_evaluated = hpairs;
  r.cand_rows = (uint64_t)p->cand_count;
  r.ms_prepare = p->ms_prepare;
  r.ms_search = ev.ms();
  for (int k = 0; k < run.timed; ++k) r.ms_scan += EventPair(1 + k).ms();
  r.scan_launches = (uint64_t)run.launches;
  p->searched = true;
  *out = r;
  return DISCORD_OK;
}

}  // namespace

extern "C" {

int discord_search(discord_plan p, discord_result* out) {
  if (!p || !out) return DISCORD_EINVAL;
  EventPair ev(0, p->timed);
  if (!ev.ready()) return fail(p, DISCORD_EDEVICE, "hipEventCreate failed");
  HIP_TRY(p, hipSetDevice(p->device));
  HIP_TRY(p, ev.start(p->stream));
  HostOut h;
  SearchRun run;
  run.h = &h;
  run.events = p->timed;
  int st = search_enqueue(p, run);
  if (st != DISCORD_OK) return st;
  HIP_TRY(p, ev.stop(p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return search_finish(p, run, ev, out);
}

int discord_search_graph(discord_plan p, discord_result* out) {
  if (!p || !out) return DISCORD_EINVAL;
  HIP_TRY(p, hipSetDevice(p->device));
  hipStream_t s = p->stream;
  if (!p->hout) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(HostOut), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(p, DISCORD_ENOMEM, "hipHostMalloc of the graph's readback block failed");
    }
    p->hout = h;
  }
  HostOut* h = static_cast<HostOut*>(p->hout);
  const bool captured = !p->gexec;
  if (!p->gexec) {
    // capture once: the sequence depends only on the plan, and every launch's
    // work is decided on the device, so the same graph serves every search
    SearchRun cap;
    cap.h = h;
    cap.events = false;
    HIP_TRY(p, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int st = search_enqueue(p, cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != DISCORD_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return st != DISCORD_OK ? st
                              : fail(p, DISCORD_EDEVICE, "stream capture failed: %s",
                                     hipGetErrorString(e));
    }
    p->glaunches = cap.launches;
    const hipError_t ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      p->gexec = nullptr;
      (void)hipGetLastError();
      return fail(p, DISCORD_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
  }
  EventPair ev(0, p->timed);
  if (!ev.ready()) return fail(p, DISCORD_EDEVICE, "hipEventCreate failed");
  HIP_TRY(p, ev.start(s));
  HIP_TRY(p, hipGraphLaunch(p->gexec, s));
  HIP_TRY(p, ev.stop(s));
  HIP_TRY(p, hipStreamSynchronize(s));
  SearchRun run;
  run.h = h;
  run.events = false;
  run.launches = p->glaunches;
  const int st = search_finish(p, run, ev, out);
  if (st == DISCORD_OK) out->graph = captured ? 1 : 2;
  return st;
}

void discord_release(discord_plan p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->hout) (void)hipHostFree(p->hout);
  if (p->own_arena && p->arena) (void)hipFree(p->arena);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

int discord_search_series(const float* T, int64_t m, int32_t n, int64_t* index, double* distance) {
  if (!index || !distance) return DISCORD_EINVAL;
  discord_plan p = nullptr;
  int st = discord_prepare(T, m, n, nullptr, nullptr, 0, nullptr, &p);
  if (st != DISCORD_OK) return st;
  discord_result r;
  st = discord_search(p, &r);
  discord_release(p);
  if (st != DISCORD_OK) return st;
  *index = r.index;
  *distance = r.distance;
  return DISCORD_OK;
}

int discord_search_once(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                        void* workspace, size_t ws_bytes, void* stream, discord_result* out) {
  g_prepare_err[0] = 0;
  if (!out) return DISCORD_EINVAL;
  discord_opts o;
  const int bad = check_prepare_args(T, m, n, opts, &o);
  if (bad != DISCORD_OK) return bad;
  const size_t need = discord_workspace_bytes(m, n, &o);
  void* arena = workspace;
  size_t bytes = ws_bytes;
  if (arena) {
    if (ws_bytes < need || ((uintptr_t)arena % kAlign) != 0) {
      std::snprintf(g_prepare_err, sizeof(g_prepare_err),
                    "workspace of %zu bytes at %p: the plan needs %zu, 256-byte aligned", ws_bytes,
                    arena, need);
      return DISCORD_ENOMEM;
    }
  } else {
    if (hipMalloc(&arena, need) != hipSuccess) {
      (void)hipGetLastError();
      return DISCORD_ENOMEM;
    }
    bytes = need;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int st = dd::search_series_in_arena(T, m, n, &o, arena, bytes, s, out, g_prepare_err,
                                            sizeof(g_prepare_err), true);
  if (!workspace) {
    (void)hipStreamSynchronize(s);   // nothing of this call is left in flight on the buffer
    (void)hipFree(arena);
  }
  return st;
}

int64_t discord_plan_count(discord_plan p, int32_t field) {
  if (!p) return DISCORD_EINVAL;
  switch (field) {
    case DISCORD_FIELD_WORDS:
    case DISCORD_FIELD_CSR_MEMBERS:
    case DISCORD_FIELD_NN_APPROX:
    case DISCORD_FIELD_NN_WITNESS:
    case DISCORD_FIELD_ROW_STATE:
    case DISCORD_FIELD_ROW_MEAN:
    case DISCORD_FIELD_ROW_CNORM: return p->N;
    case DISCORD_FIELD_ROW_SIGMA: return p->opts.znorm ? p->N : DISCORD_EINVAL;
    case DISCORD_FIELD_ROW_BOUND: return p->opts.znorm ? DISCORD_EINVAL : p->N;
    case DISCORD_FIELD_HIST: return p->dict;
    case DISCORD_FIELD_CSR_OFFSETS: return p->dict + 1;
    case DISCORD_FIELD_CAND: return p->cand_count;
    default: return DISCORD_EINVAL;
  }
}

int discord_plan_copy(discord_plan p, int32_t field, void* host_dst, size_t bytes) {
  if (!p || !host_dst) return DISCORD_EINVAL;
  const int64_t count = discord_plan_count(p, field);
  if (count < 0) return DISCORD_EINVAL;
  size_t elem = 4, off = 0;
  switch (field) {
    case DISCORD_FIELD_WORDS: off = p->L.words; break;
    case DISCORD_FIELD_HIST: off = p->L.hist; break;
    case DISCORD_FIELD_CAND: off = p->L.cand; break;
    case DISCORD_FIELD_CSR_OFFSETS: off = p->L.csr_off; break;
    case DISCORD_FIELD_CSR_MEMBERS: off = p->L.csr_mem; break;
    case DISCORD_FIELD_NN_APPROX: off = p->L.nn_approx; break;
    case DISCORD_FIELD_NN_WITNESS: off = p->L.nn_wit; break;
    case DISCORD_FIELD_ROW_STATE: off = p->L.row_state; break;
    case DISCORD_FIELD_ROW_MEAN: off = p->L.row_mean; elem = 8; break;
    case DISCORD_FIELD_ROW_CNORM: off = p->L.row_cnorm; elem = 8; break;
    case DISCORD_FIELD_ROW_SIGMA: off = p->L.row_sigma; elem = 8; break;
    case DISCORD_FIELD_ROW_BOUND: off = p->L.lb; break;
    default: return DISCORD_EINVAL;
  }
  if (bytes < elem * (size_t)count) return DISCORD_EINVAL;
  if (count == 0) return DISCORD_OK;
  HIP_TRY(p, hipMemcpyAsync(host_dst, p->arena + off, elem * (size_t)count, hipMemcpyDeviceToHost,
                            p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return DISCORD_OK;
}

int discord_rows_nn_fp64(discord_plan p, const int64_t* rows, int64_t count, double* d2_out,
                         int64_t* j_out) {
  if (!p || count < 0 || (count > 0 && (!rows || !d2_out || !j_out))) return DISCORD_EINVAL;
  for (int64_t k = 0; k < count; ++k)
    if (rows[k] < 0 || rows[k] >= p->N) return DISCORD_EINVAL;
  int64_t* d_rows = p->at<int64_t>(p->L.rows);
  for (int64_t b = 0; b < count; b += kFp64BatchRows) {
    const int64_t c = std::min<int64_t>(kFp64BatchRows, count - b);
    HIP_TRY(p, hipMemcpyAsync(d_rows, rows + b, sizeof(int64_t) * c, hipMemcpyHostToDevice, p->stream));
    int st = rows_nn_batch(p, d_rows, c);
    if (st) return st;
    HIP_TRY(p, hipMemcpyAsync(d2_out + b, p->at<double>(p->L.out_d), sizeof(double) * c,
                              hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipMemcpyAsync(j_out + b, p->at<int64_t>(p->L.out_j), sizeof(int64_t) * c,
                              hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
  }
  return DISCORD_OK;
}

int discord_sax_breakpoints(int32_t alpha, double* out) {
  if (!out || alpha < 2 || alpha > 8) return DISCORD_EINVAL;
  double b[8];
  sax_breakpoints(alpha, b);
  for (int k = 0; k < alpha - 1; ++k) out[k] = b[k];
  return DISCORD_OK;
}

int discord_cu_mask(int32_t total_cus, int32_t xccs, int32_t cus, uint32_t* words,
                    int32_t nwords) {
  if (!words || xccs < 1 || total_cus < 1 || total_cus % xccs != 0) return DISCORD_EINVAL;
  const int32_t per = total_cus / xccs;   // CUs per die
  if (per % xccs != 0 || cus < 1 || cus > total_cus || cus % xccs != 0) return DISCORD_EINVAL;
  const int32_t used = (total_cus + 31) / 32;
  if (nwords < used) return DISCORD_EINVAL;
  std::memset(words, 0, sizeof(uint32_t) * (size_t)used);
  const int32_t j = cus / xccs;           // CUs kept per die
  std::vector<int32_t> taken((size_t)xccs);
  for (int32_t x = 0; x < xccs; ++x) {
    // block x holds bits x * per .. x * per + per - 1; take j of them whose
    // residues mod xccs are (x + t) mod xccs, t = 0 .. j - 1, each residue's
    // bits in ascending order (per / xccs of them per residue, j <= per)
    std::fill(taken.begin(), taken.end(), 0);
    for (int32_t t = 0; t < j; ++t) {
      const int32_t r = (x + t) % xccs;
      const int32_t b = x * per + r + xccs * taken[(size_t)r]++;
      words[b / 32] |= 1u << (b % 32);
    }
  }
  return used;
}

int discord_stream_create_cu_limited(int32_t cus, void** stream_out) {
  if (!stream_out) return DISCORD_EINVAL;
  *stream_out = nullptr;
  int dev = 0, total = 0, xccs = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&total, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DISCORD_EDEVICE;
  if (hipDeviceGetAttribute(&xccs, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || xccs < 1)
    xccs = 1;
  std::vector<uint32_t> mask((size_t)(total + 31) / 32);
  const int used = discord_cu_mask(total, xccs, cus, mask.data(), (int32_t)mask.size());
  if (used < 0) return used;
  hipStream_t s = nullptr;
  if (hipExtStreamCreateWithCUMask(&s, (uint32_t)used, mask.data()) != hipSuccess || !s)
    return DISCORD_EDEVICE;
  std::vector<uint32_t> back(mask.size(), 0);
  int got = -1;
  if (hipExtStreamGetCUMask(s, (uint32_t)back.size(), back.data()) == hipSuccess) {
    got = 0;
    for (uint32_t w : back) got += __builtin_popcount(w);
  }
  if (got != cus) {
    (void)hipStreamDestroy(s);
    return DISCORD_EDEVICE;
  }
  *stream_out = s;
  return DISCORD_OK;
}

int discord_stream_destroy(void* stream) {
  if (!stream) return DISCORD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const bool ok = hipStreamSynchronize(s) == hipSuccess;
  return (hipStreamDestroy(s) == hipSuccess && ok) ? DISCORD_OK : DISCORD_EDEVICE;
}

}  // extern "C"

namespace dd {

int search_series_in_arena(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                           void* arena, size_t arena_bytes, hipStream_t stream,
                           discord_result* out, char* err, size_t err_len, bool timed) {
  if (err && err_len) err[0] = 0;
  discord_opts o;
  int st = check_prepare_args(T, m, n, opts, &o);
  if (st != DISCORD_OK) return st;
  // the plan lives on this stack frame: no heap object, no stream, no event
  discord_plan_s plan;
  discord_plan p = &plan;
  init_plan(p, m, n, o);
  if (!arena || p->L.total > arena_bytes || ((uintptr_t)arena % kAlign) != 0)
    return DISCORD_ERANGE;
  if (hipGetDevice(&p->device) != hipSuccess) return DISCORD_EDEVICE;
  p->stream = stream;
  p->arena = static_cast<char*>(arena);
  p->timed = timed;
  if (o.order == 1) {
    // the PhiDD order's sequences need the bucket sizes on the host first
    st = prepare_run(p, T);
    if (st == DISCORD_OK) st = discord_search(p, out);
  } else {
    // preparation and search as one sequence with one synchronisation; the
    // statistics of eq. (2) are checked from the same readback
    HostOut h;
    SearchRun run;
    run.h = &h;
    run.events = timed;
    run.with_prepare = true;
    EventPair ev(0, timed);
    if (!ev.ready()) st = fail(p, DISCORD_EDEVICE, "hipEventCreate failed");
    if (st == DISCORD_OK && ev.start(stream) != hipSuccess)
      st = fail(p, DISCORD_EDEVICE, "hipEventRecord failed");
    p->index_word = false;   // no plan is kept, and the sequences need no bucket
    if (st == DISCORD_OK) st = prepare_enqueue(p, T);
    if (st == DISCORD_OK) st = search_enqueue(p, run);
    if (st == DISCORD_OK && ev.stop(stream) != hipSuccess)
      st = fail(p, DISCORD_EDEVICE, "hipEventRecord failed");
    if (st == DISCORD_OK && hipStreamSynchronize(stream) != hipSuccess)
      st = fail(p, DISCORD_EDEVICE, "hipStreamSynchronize failed");
    if (st == DISCORD_OK) st = prepare_check(p, h);
    if (st == DISCORD_OK) st = search_finish(p, run, ev, out);
  }
  if (st != DISCORD_OK && err && err_len) std::snprintf(err, err_len, "%s", p->err);
  return st;
}

struct RequestGraph {
  discord_plan_s plan;            // host fields of the plan bound to the workspace
  const float* T = nullptr;       // the key: series pointer, sizes, options, memory, stream
  int64_t m = 0;
  int32_t n = 0;
  discord_opts opts{};
  void* arena = nullptr;
  hipStream_t stream = nullptr;
  HostOut* h = nullptr;           // pinned block the graph's copies land in
  hipGraphExec_t exec = nullptr;
  int launches = 0;
};

void request_graph_free(RequestGraph* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->h) (void)hipHostFree(g->h);
  delete g;
}

int search_series_graph(RequestGraph** cache, bool capture, const float* T, int64_t m, int32_t n,
                        const discord_opts* opts, void* arena, size_t arena_bytes,
                        hipStream_t stream, discord_result* out, char* err, size_t err_len) {
  if (err && err_len) err[0] = 0;
  discord_opts o;
  int st = check_prepare_args(T, m, n, opts, &o);
  if (st != DISCORD_OK) return st;
  RequestGraph* g = *cache;
  const bool hit = g && g->exec && g->T == T && g->m == m && g->n == n && g->arena == arena &&
                   g->stream == stream && std::memcmp(&g->opts, &o, sizeof(o)) == 0;
  if (!hit) {
    request_graph_free(g);
    *cache = nullptr;
    if (!capture || o.order == 1) {
      st = search_series_in_arena(T, m, n, &o, arena, arena_bytes, stream, out, err, err_len);
      if (st == DISCORD_OK) out->graph = 0;
      return st;
    }
    g = new (std::nothrow) RequestGraph();
    if (!g) return DISCORD_ENOMEM;
    discord_plan p = &g->plan;
    init_plan(p, m, n, o);
    auto give_up = [&](int code) {
      if (err && err_len) std::snprintf(err, err_len, "%s", p->err);
      request_graph_free(g);
      return code;
    };
    if (!arena || p->L.total > arena_bytes || ((uintptr_t)arena % kAlign) != 0)
      return give_up(DISCORD_ERANGE);
    if (hipGetDevice(&p->device) != hipSuccess) return give_up(DISCORD_EDEVICE);
    p->stream = stream;
    p->arena = static_cast<char*>(arena);
    p->timed = false;
    void* hb = nullptr;
    if (hipHostMalloc(&hb, sizeof(HostOut), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return give_up(DISCORD_ENOMEM);
    }
    g->h = static_cast<HostOut*>(hb);
    // the request's whole sequence, as the ordinary one-sequence path runs it
    SearchRun cap;
    cap.h = g->h;
    cap.events = false;
    cap.with_prepare = true;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      return give_up(fail(p, DISCORD_EDEVICE, "hipStreamBeginCapture failed"));
    }
    p->index_word = o.order == 1;   // the served request keeps no plan to inspect
    st = prepare_enqueue(p, T);
    if (st == DISCORD_OK) st = search_enqueue(p, cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &graph);
    if (st != DISCORD_OK || e != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return give_up(st != DISCORD_OK ? st
                                      : fail(p, DISCORD_EDEVICE, "stream capture failed: %s",
                                             hipGetErrorString(e)));
    }
    const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g->exec = nullptr;
      (void)hipGetLastError();
      return give_up(fail(p, DISCORD_EDEVICE, "hipGraphInstantiate failed: %s",
                          hipGetErrorString(ei)));
    }
    g->launches = cap.launches;
    g->T = T;
    g->m = m;
    g->n = n;
    g->opts = o;
    g->arena = arena;
    g->stream = stream;
    *cache = g;
  }
  discord_plan p = &g->plan;
  if (hipGraphLaunch(g->exec, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(p, DISCORD_EDEVICE, "graph launch failed");
  }
  if (st == DISCORD_OK) st = prepare_check(p, *g->h);
  if (st == DISCORD_OK) {
    SearchRun run;
    run.h = g->h;
    run.events = false;
    run.launches = g->launches;
    EventPair none(0, false);
    st = search_finish(p, run, none, out);
  }
  if (st == DISCORD_OK) out->graph = hit ? 2 : 1;
  if (st != DISCORD_OK && err && err_len) std::snprintf(err, err_len, "%s", p->err);
  return st;
}

}  // namespace dd
