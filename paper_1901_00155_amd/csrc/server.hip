// server.hip -- the GPU executor of the serving loop and discord_server_create.
//
// One device arena of the configured budget is allocated once; every admitted
// request prepares and searches inside its own block of it, so no device
// allocation happens per request.  A request's preparation and search are
// enqueued as one sequence (every decision of the search taken on the device)
// and the worker synchronises once, when the answer is on the host.  Each slot
// owns a HIP stream of default priority and a pinned host staging buffer: the
// series is copied into the staging buffer and from there to the device
// asynchronously on the slot's stream.  The kernels of different slots run
// concurrently on the GPU.
//
// A slot keeps that sequence captured as a HIP graph for its last request
// shape.  When a request has the (m, n) of the slot's previous one and got the
// same arena block (the scheduler hands a slot its previous block back when
// the footprint matches and the block is free), the second such request is
// captured and every later one replays the graph: one graph launch and one
// synchronisation per request.
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"
#include "server_core.hpp"

namespace {

struct HipSlot {
  hipStream_t stream = nullptr;
  float* staging = nullptr;   // pinned (hipHostMalloc)
  int64_t capacity = 0;       // floats
  dd::RequestGraph* graph = nullptr;   // the last shape's captured request
  int64_t last_m = -1;        // shape and block of the slot's previous request
  int32_t last_n = 0;
  void* last_ws = nullptr;
};

struct HipExecutor {
  int device = 0;
  char* arena = nullptr;
  std::vector<HipSlot> slots;
};

int set_detail(char* detail, size_t len, const char* what, const char* msg) {
  if (detail && len) std::snprintf(detail, len, "%s: %s", what, msg);
  return 0;
}

int hip_execute(void* ctx, const discord_request* rq, const discord_opts* opts,
                discord_result* out, char* detail, size_t detail_len) {
  auto* E = static_cast<HipExecutor*>(ctx);
  HipSlot& S = E->slots[rq->slot];
  hipError_t e = hipSetDevice(E->device);
  if (e == hipSuccess && !S.stream) e = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    set_detail(detail, detail_len, "stream", hipGetErrorString(e));
    return DISCORD_EDEVICE;
  }
  if (S.capacity < rq->m) {
    // grow by doubling; the previous request on this slot has completed (its
    // search synchronised the stream), so the old buffer is idle
    if (S.staging) (void)hipHostFree(S.staging);
    S.staging = nullptr;
    S.capacity = 0;
    int64_t cap = 1 << 16;
    while (cap < rq->m) cap *= 2;
    if (hipHostMalloc(reinterpret_cast<void**>(&S.staging), sizeof(float) * cap,
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      S.staging = nullptr;
      set_detail(detail, detail_len, "staging", "pinned host allocation failed");
      return DISCORD_ENOMEM;
    }
    S.capacity = cap;
  }
  std::memcpy(S.staging, rq->T, sizeof(float) * rq->m);
  // preparation and search as one sequence on the slot's stream, with one
  // synchronisation: a graph replay when the slot's previous request had the
  // same shape and block, else ordinary launches (a repeated shape is captured)
  const bool repeat = S.last_m == rq->m && S.last_n == rq->n && S.last_ws == rq->workspace;
  S.last_m = rq->m;
  S.last_n = rq->n;
  S.last_ws = rq->workspace;
  char err[256];
  const int st = dd::search_series_graph(&S.graph, repeat, S.staging, rq->m, rq->n, opts,
                                         rq->workspace, rq->ws_bytes, S.stream, out, err,
                                         sizeof(err));
  if (st != DISCORD_OK) set_detail(detail, detail_len, "request", err);
  return st;
}

void hip_fini(void* ctx) {
  auto* E = static_cast<HipExecutor*>(ctx);
  if (!E) return;
  (void)hipSetDevice(E->device);
  for (auto& S : E->slots) {
    dd::request_graph_free(S.graph);   // (synchronises the slot's stream)
    S.graph = nullptr;
    if (S.stream) {
      (void)hipStreamSynchronize(S.stream);
      (void)hipStreamDestroy(S.stream);
    }
    if (S.staging) (void)hipHostFree(S.staging);
  }
  if (E->arena) (void)hipFree(E->arena);
  delete E;
}

}  // namespace

extern "C" int discord_server_create(const discord_server_config* cfg, discord_server* out) {
  if (!out) return DISCORD_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->slots < 1 || cfg->slots > 64 || cfg->hbm_budget_bytes < 256) return DISCORD_EINVAL;
  auto* E = new (std::nothrow) HipExecutor();
  if (!E) return DISCORD_ENOMEM;
  try {
    E->slots.resize(cfg->slots);
  } catch (...) {
    delete E;
    return DISCORD_ENOMEM;
  }
  if (hipGetDevice(&E->device) != hipSuccess) {
    (void)hipGetLastError();
    delete E;
    return DISCORD_EDEVICE;
  }
  if (hipMalloc(reinterpret_cast<void**>(&E->arena), cfg->hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    E->arena = nullptr;
    delete E;
    return DISCORD_ENOMEM;
  }
  // server_create owns E from here on: it calls hip_fini on failure and at destroy
  return dd::server_create(cfg, hip_execute, E, E->arena, hip_fini, out);
}
