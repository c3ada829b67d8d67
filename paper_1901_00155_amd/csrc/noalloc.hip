// noalloc.hip -- discord_search_series_noalloc: prepare + search of one series
// with no device allocation, for callers that cannot allocate (code under
// stream capture, tight serving loops, hosts that forbid it).
//
// The plan's whole arena (padded series, preparation structures, search and
// certification state) lives in `scratch`, a static device array of
// DISCORD_NOALLOC_MAX_BYTES that every GPU the library runs on holds until the
// process ends.  Every call on a GPU uses that GPU's one copy: the preparation
// and search clear what they need themselves (as they do for any workspace),
// and calls that overlap on one GPU race.
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "internal.hpp"

static __device__ __align__(256) unsigned char scratch[DISCORD_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch`, per device

// The array's device address on the current device, taken once per device.
// In host code the name `scratch` is only a handle for the runtime; the kernels
// receive this address.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return DISCORD_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return DISCORD_EDEVICE;
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return DISCORD_OK;
}

}  // namespace

extern "C" int discord_search_series_noalloc(const float* T, int64_t m, int32_t n,
                                             const discord_opts* opts, void* stream,
                                             discord_result* out) {
  dd::set_thread_error("%s", "");
  if (!out) return DISCORD_EINVAL;
  // sizes first, with no device call: a plan that does not fit is refused
  // before anything runs
  const size_t need = discord_workspace_bytes(m, n, opts);
  if (need > DISCORD_NOALLOC_MAX_BYTES) {
    dd::set_thread_error("plan of %zu bytes exceeds the %zu-byte static workspace of "
                         "discord_search_series_noalloc", need,
                         (size_t)DISCORD_NOALLOC_MAX_BYTES);
    return DISCORD_ERANGE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DISCORD_EDEVICE;
  void* arena = nullptr;
  int st = scratch_address(dev, &arena);
  if (st != DISCORD_OK) {
    dd::set_thread_error("hipGetSymbolAddress of the static workspace failed");
    return st;
  }
  char err[256];
  st = dd::search_series_in_arena(T, m, n, opts, arena, DISCORD_NOALLOC_MAX_BYTES,
                                  static_cast<hipStream_t>(stream), out, err, sizeof(err));
  if (st != DISCORD_OK) dd::set_thread_error("%s", err);
  return st;
}
