// rank.hip -- items in descending order of a score, most promising first.
//
// The search ranks its items by the mean-gap bound of their rows' NN
// (bound.hip) to choose which to complete first.  Under per-window
// normalisation, where that bound is zero, it ranks the items still searched
// after each window instead: each live row has a published minimum over the
// columns seen so far, an upper bound of its NN, and an item scores the
// largest such bound among its live rows (+inf for a row that has seen no
// column yet).  The items are put in
// descending score order by a counting sort on the top 12 bits of the score's
// IEEE pattern (non-negative floats order like their bits; bins are 1/16 of an
// octave wide); the order within a bin is arbitrary and, like every visiting
// order, affects only the work done.
#include <algorithm>

#include "internal.hpp"

namespace dd {
namespace {

constexpr int kBins = 4096;
constexpr int kBinShift = 19;   // 31 value bits -> 12-bit bin

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t row_score(const uint32_t* __restrict__ alive,
                                              const uint64_t* __restrict__ best, int64_t i,
                                              int gsz) {
  if (!((load_relaxed(&alive[i / gsz]) >> (i % gsz)) & 1u)) return 0;
  const uint64_t key = best[i];
  const uint32_t bits = key == kEmptyMin ? 0x7F800000u : (uint32_t)(key >> 32);
  return bits > 0x7F800000u ? 0 : bits;   // not a non-negative number: rank last
}

// Small items (up to 64 rows): one thread per item.
__global__ __launch_bounds__(256) void k_group_score(const int32_t* __restrict__ list,
                                                     const int64_t* __restrict__ count_p,
                                                     int64_t item_rows, int gsz,
                                                     const uint32_t* __restrict__ alive,
                                                     const uint64_t* __restrict__ best, int64_t N,
                                                     uint32_t* __restrict__ score) {
  const int64_t count = *count_p;
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= count) return;
  const int64_t r0 = (int64_t)list[k] * item_rows;
  uint32_t s = 0;
  for (int64_t i = r0; i < r0 + item_rows && i < N; ++i) {
    const uint32_t b = row_score(alive, best, i, gsz);
    s = b > s ? b : s;
  }
  score[k] = s;
}

// Large items: one wavefront per item, its lanes striding over the rows.
__global__ __launch_bounds__(256) void k_group_score_wave(const int32_t* __restrict__ list,
                                                          const int64_t* __restrict__ count_p,
                                                          int64_t item_rows, int gsz,
                                                          const uint32_t* __restrict__ alive,
                                                          const uint64_t* __restrict__ best,
                                                          int64_t N, uint32_t* __restrict__ score) {
  const int64_t count = *count_p;
  const int64_t k = blockIdx.x * 4ll + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= count) return;
  const int64_t r0 = (int64_t)list[k] * item_rows;
  const int64_t r1 = min<int64_t>(N, r0 + item_rows);
  uint32_t s = 0;
  for (int64_t i = r0 + lane; i < r1; i += 64) {
    const uint32_t b = row_score(alive, best, i, gsz);
    s = b > s ? b : s;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(s, off, 64);
    s = o > s ? o : s;
  }
  if (lane == 0) score[k] = s;
}

__global__ __launch_bounds__(256) void k_rank_hist(const uint32_t* __restrict__ score,
                                                   const int64_t* __restrict__ count_p,
                                                   uint32_t* __restrict__ hist) {
  const int64_t count = *count_p;
  if ((int64_t)blockIdx.x * 256 >= count) return;
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

// Each block ranks its items in LDS first and reserves its slots with one
// atomic per occupied bin, so a bin's global cursor sees one atomic per block
// rather than one per item.
__global__ __launch_bounds__(256) void k_rank_scatter(const int32_t* __restrict__ list,
                                                      const uint32_t* __restrict__ score,
                                                      const int64_t* __restrict__ count_p,
                                                      uint32_t* __restrict__ cursor,
                                                      int32_t* __restrict__ out) {
  const int64_t count = *count_p;
  if ((int64_t)blockIdx.x * 256 >= count) return;
  __shared__ uint32_t local[kBins];
  __shared__ uint32_t base[kBins];
  for (int b = threadIdx.x; b < kBins; b += 256) local[b] = 0;
  __syncthreads();
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  uint32_t bin = 0, pos = 0;
  if (k < count) {
    bin = min(score[k] >> kBinShift, (uint32_t)(kBins - 1));
    pos = atomicAdd(&local[bin], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += 256)
    if (local[b]) base[b] = atomicAdd(&cursor[b], local[b]);
  __syncthreads();
  if (k < count) out[base[bin] + pos] = list ? list[k] : (int32_t)k;
}

}  // namespace

size_t rank_hist_bins() { return kBins; }

void launch_rank_groups(const int32_t* list, const int64_t* count, int64_t max_count,
                        int64_t item_rows, int gsz, const uint32_t* alive, const uint64_t* best,
                        int64_t N, uint32_t* score, uint32_t* hist, int32_t* out, hipStream_t s) {
  if (max_count <= 0) return;
  const unsigned blocks = (unsigned)((max_count + 255) / 256);
  if (item_rows > 64)
    hipLaunchKernelGGL(k_group_score_wave, dim3((unsigned)((max_count + 3) / 4)), dim3(256), 0, s,
                       list, count, item_rows, gsz, alive, best, N, score);
  else
    hipLaunchKernelGGL(k_group_score, dim3(blocks), dim3(256), 0, s, list, count, item_rows, gsz,
                       alive, best, N, score);
  launch_rank_scores(list, count, max_count, score, hist, out, s);
}

void launch_rank_scores(const int32_t* list, const int64_t* count, int64_t max_count,
                        const uint32_t* score, uint32_t* hist, int32_t* out, hipStream_t s,
                        bool clear_hist) {
  if (max_count <= 0) return;
  const unsigned blocks = (unsigned)((max_count + 255) / 256);
  if (clear_hist) launch_init_i32(reinterpret_cast<int32_t*>(hist), kBins, 0, s);
  hipLaunchKernelGGL(k_rank_hist, dim3(std::min(blocks, 1024u)), dim3(256), 0, s, score, count,
                     hist);
  hipLaunchKernelGGL(k_rank_offsets, dim3(1), dim3(1024), 0, s, hist);
  hipLaunchKernelGGL(k_rank_scatter, dim3(blocks), dim3(256), 0, s, list, score, count, hist, out);
}

}  // namespace dd
