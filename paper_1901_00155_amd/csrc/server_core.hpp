// server_core.hpp -- the request scheduler behind discord_server_* (host C++ only).
//
// The scheduler knows nothing of HIP: it queues requests, admits them first-in
// first-out by slot and arena space, runs them through an executor on worker
// threads and collects completions.  The GPU executor lives in server.hip.
#pragma once

#include <cstddef>

#include "../../include/discord.h"

namespace dd {

// First-fit allocator over [0, capacity) in 256-byte units, with coalescing of
// adjacent free blocks.  Not thread-safe: the scheduler holds its lock.
class ArenaAllocator {
 public:
  static constexpr size_t kNone = ~size_t(0);
  static constexpr size_t kAlign = 256;
  explicit ArenaAllocator(size_t capacity);
  ~ArenaAllocator();
  ArenaAllocator(const ArenaAllocator&) = delete;
  ArenaAllocator& operator=(const ArenaAllocator&) = delete;
  size_t alloc(size_t bytes);            // offset, or kNone when no free block fits
  // [off, off + bytes) if that range is free (off a multiple of kAlign), else kNone
  size_t alloc_at(size_t off, size_t bytes);
  void release(size_t offset, size_t bytes);
  size_t capacity() const { return capacity_; }
  size_t in_use() const { return in_use_; }
  size_t free_blocks() const;
  static size_t round(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

 private:
  struct Impl;
  Impl* impl_;
  size_t capacity_;
  size_t in_use_ = 0;
};

// Creates a server whose requests run through `exec`.  `arena` is the device
// base of the arena (NULL: virtual arena, offsets only); `fini(ctx)` runs once
// after every worker has stopped (may be NULL).
int server_create(const discord_server_config* cfg, discord_executor_fn exec, void* ctx,
                  void* arena, void (*fini)(void*), discord_server* out);

}  // namespace dd
