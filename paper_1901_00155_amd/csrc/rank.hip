// rank.hip -- ordering of the row groups still searched, most promising first.
//
// Between the launches of a search every item (a fixed set of consecutive rows)
// with live rows has, for each live row, a published minimum over the columns
// seen so far: an upper bound of the row's nearest-neighbour distance.  An item
// scores the largest such bound among its live rows (+inf for a row that has
// seen no column yet), and the items are put in descending score order by a counting sort on the top
// 12 bits of the score's IEEE pattern (non-negative floats order like their
// bits; bins are 1/16 of an octave wide).  Scanning the best-scored groups to
// completion first raises the best-so-far early; the order within a bin is
// arbitrary and, like every visiting order, affects only the work done.
#include <algorithm>

#include "internal.hpp"

namespace dd {
namespace {

constexpr int kBins = 4096;
constexpr int kBinShift = 19;   // 31 value bits -> 12-bit bin

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_group_score(const int32_t* __restrict__ list,
                                                     int64_t count, int64_t item_rows, int gsz,
                                                     const uint32_t* __restrict__ alive,
                                                     const uint64_t* __restrict__ best, int64_t N,
                                                     uint32_t* __restrict__ score) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= count) return;
  const int64_t r0 = (int64_t)list[k] * item_rows;
  uint32_t s = 0, live = 0;
  for (int64_t i = r0; i < r0 + item_rows && i < N; ++i) {
    const int r = (int)((i - r0) % gsz);
    if (r == 0) live = load_relaxed(&alive[i / gsz]);
    if (!((live >> r) & 1u)) continue;
    const uint64_t key = best[i];
    uint32_t bits = key == kEmptyMin ? 0x7F800000u : (uint32_t)(key >> 32);
    if (bits > 0x7F800000u) bits = 0;   // not a non-negative number: rank last
    s = bits > s ? bits : s;
  }
  score[k] = s;
}

__global__ __launch_bounds__(256) void k_rank_hist(const uint32_t* __restrict__ score,
                                                   int64_t count, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kBins];
  for (int b = threadIdx.x; b < kBins; b += 256) h[b] = 0;
  __syncthreads();
  for (int64_t k = blockIdx.x * 256ll + threadIdx.x; k < count; k += (int64_t)gridDim.x * 256)
    atomicAdd(&h[min(score[k] >> kBinShift, (uint32_t)(kBins - 1))], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += 256)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// In place: counts -> first output slot of each bin, highest bin first.
__global__ __launch_bounds__(1024) void k_rank_offsets(uint32_t* __restrict__ hist) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  // thread t owns bins kBins-1-4t .. kBins-4-4t (descending)
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    c[u] = hist[kBins - 1 - (4 * t + u)];
    sum += c[u];
  }
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan (Hillis-Steele)
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;                  // exclusive prefix of this thread
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    hist[kBins - 1 - (4 * t + u)] = run;
    run += c[u];
  }
}

__global__ __launch_bounds__(256) void k_rank_scatter(const int32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ score,
                                                      int64_t count, uint32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ out) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= count) return;
  const uint32_t slot = atomicAdd(&cursor[min(score[k] >> kBinShift, (uint32_t)(kBins - 1))], 1u);
  out[slot] = list[k];
}

}  // namespace

size_t rank_hist_bins() { return kBins; }

void launch_rank_groups(const int32_t* list, int64_t count, int64_t item_rows, int gsz,
                        const uint32_t* alive,
                        const uint64_t* best, int64_t N, uint32_t* score, uint32_t* hist,
                        int32_t* out, hipStream_t s) {
  if (count <= 0) return;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  launch_init_i32(reinterpret_cast<int32_t*>(hist), kBins, 0, s);
  hipLaunchKernelGGL(k_group_score, dim3(blocks), dim3(256), 0, s, list, count, item_rows, gsz, alive,
                     best, N, score);
  hipLaunchKernelGGL(k_rank_hist, dim3(std::min(blocks, 1024u)), dim3(256), 0, s, score, count,
                     hist);
  hipLaunchKernelGGL(k_rank_offsets, dim3(1), dim3(1024), 0, s, hist);
  hipLaunchKernelGGL(k_rank_scatter, dim3(blocks), dim3(256), 0, s, list, score, count, hist, out);
}

}  // namespace dd
