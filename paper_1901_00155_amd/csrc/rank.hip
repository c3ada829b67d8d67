// rank.hip -- items in descending order of a score, most promising first.
//
// The search ranks its items by the mean-gap bound of their rows' NN
// (bound.hip) to choose which to complete first.  The items are put in
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
