// prep.hip -- preparation stage of PhiDD (Algorithm 2, first six steps) for gfx950.
//
//   stats     eq. (2): mean and standard deviation of the series, FP64, two-pass,
//             fixed grid and fixed reduction tree (bit-reproducible run to run).
//   row stats per-row mean and centred squared norm (FP64), used by the split-BF16
//             scan and exposed for verification; with per-window normalisation
//             also the row's standard deviation.
//   sax       eqs. (3), (4), (9): PAA of each row on the z-normalised series, SAX
//             symbols by the N(0,1) breakpoints, word id = lexicographic rank.
//             One thread per row; the 256-bin word histogram (eq. 8) is built in
//             LDS and merged with global atomics.
//   cand      eq. (7): rows whose word has the minimum frequency, ascending, by a
//             stable wave-ballot compaction.
//   csr       eq. (10): Index_Word as CSR (offsets + members), a stable counting
//             sort: per-segment word counts -> scan over segments -> scatter with
//             in-wave ranks from ballots.
#include "internal.hpp"

namespace dd {
namespace {

constexpr int kSegRows = 4096;   // rows per segment of the stable compaction / counting sort

__device__ inline double block_sum_256(double v, double* sh) {
  // fixed-shape tree: wave butterfly, then the four wave sums in order
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ T, int64_t m,
                                             double* __restrict__ partials, int* __restrict__ bad) {
  __shared__ double sh[4];
  double s = 0.0;
  int nonfinite = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const float v = T[i];
    nonfinite |= !__builtin_isfinite(v);
    s += (double)v;
  }
  if (__any(nonfinite) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
  const double r = block_sum_256(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_sqdev(const float* __restrict__ T, int64_t m,
                                               const double* __restrict__ stats,
                                               double* __restrict__ partials) {
  __shared__ double sh[4];
  const double mu = stats[0];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const double d = (double)T[i] - mu;
    s += d * d;
  }
  const double r = block_sum_256(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// stats[0] = mu, stats[1] = sigma, stats[2] = sum of squared deviations
__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ partials, int nb,
                                                int64_t m, double* __restrict__ stats, int which) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += partials[b];
  const double r = block_sum_256(s, sh);
  if (threadIdx.x == 0) {
    if (which == 0) {
      stats[0] = r / (double)m;
    } else {
      stats[2] = r;
      stats[1] = sqrt(r / (double)m);
    }
  }
}

// The 256 rows of a workgroup, i0 .. i0 + 255, read the values t_{i0} ..
// t_{i0 + 254 + n}: they are copied to LDS once (coalesced), and each thread
// reads its window from there.  Rows past the series read the zero pad after
// it (the caller ignores them).  Returns this thread's window.  Windows longer
// than kStageMaxN values are read from the series itself (the copy would not
// fit in a workgroup's LDS); the barrier is taken either way, so callers may
// rely on it.
constexpr int kStageMaxN = 8192;   // 255 + n floats: at most 33.8 KB

__device__ __forceinline__ const float* stage_windows(const float* __restrict__ T, int64_t i0,
                                                      int n, float* __restrict__ sh) {
  if (n > kStageMaxN) {
    __syncthreads();
    return T + i0 + threadIdx.x;
  }
  for (int k = threadIdx.x; k < 255 + n; k += 256) sh[k] = T[i0 + k];
  __syncthreads();
  return sh + threadIdx.x;
}

size_t stage_bytes(int n) { return n > kStageMaxN ? 0 : sizeof(float) * (size_t)(255 + n); }

// Mean and centred squared norm of every row (FP64, sequential two-pass sums,
// each multiply and add rounded on its own) and, for per-window normalisation,
// the row's standard deviation sqrt(cnorm / n): eq. (2) over the window alone.
__global__ __launch_bounds__(256) void k_row_stats(const float* __restrict__ T, int64_t N, int n,
                                                   double* __restrict__ mean,
                                                   double* __restrict__ cnorm,
                                                   double* __restrict__ sigma) {
#pragma clang fp contract(off)
  extern __shared__ float stage[];
  const int64_t i0 = blockIdx.x * 256ll;
  const int64_t i = i0 + threadIdx.x;
  const float* x = stage_windows(T, i0, n, stage);
  if (i >= N) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s = s + (double)x[k];
  const double mu = s / (double)n;
  double q = 0.0;
  for (int k = 0; k < n; ++k) {
    const double d = (double)x[k] - mu;
    q = q + d * d;
  }
  mean[i] = mu;
  cnorm[i] = q;
  if (sigma) sigma[i] = sqrt(q / (double)n);
}

// FP32 row statistics of the split-BF16 scan (scan_mfma.hip) and of the
// normalised FP32 scan.  c_i = fp32(mean_i) is row i's centre; cnorm is the
// squared norm about c_i (FP64, rounded once), which differs from the norm
// about the exact mean by n (mu_i - c_i)^2, below n ulp(mu)^2; smu =
// sqrt(n) (mu - mu_T) with mu_T the series mean.  Entries N .. N+pad-1 are zero.
//
// Per-window normalisation (sigma != nullptr): r_i = fp32(1 / sigma_i) (0 for
// a flat window); the normalised operand values are x_k = (t_{i+k} - c_i) r_i,
// cnorm is their squared norm, computed with the FP32 operations the FP32
// scan uses, and smu = 0 (normalised windows have mean 0).
__global__ __launch_bounds__(256) void k_row_stats32(const float* __restrict__ T, int64_t N, int n,
                                                     int64_t padded,
                                                     const double* __restrict__ mean,
                                                     const double* __restrict__ sigma,
                                                     const double* __restrict__ stats,
                                                     float* __restrict__ c32,
                                                     float* __restrict__ smu32,
                                                     float* __restrict__ cn32,
                                                     float* __restrict__ r32) {
  extern __shared__ float stage[];
  const int64_t i0 = blockIdx.x * 256ll;
  const int64_t i = i0 + threadIdx.x;
  const float* x = stage_windows(T, i0, n, stage);
  if (i >= padded) return;
  if (i >= N) {
    c32[i] = 0.0f;
    smu32[i] = 0.0f;
    cn32[i] = 0.0f;
    if (r32) r32[i] = 0.0f;
    return;
  }
  const double mu = mean[i];
  const float c = (float)mu;
  double q = 0.0;
  if (sigma) {
    const double sg = sigma[i];
    const float r = sg > 0.0 ? (float)(1.0 / sg) : 0.0f;
    for (int k = 0; k < n; ++k) {
      const float v = (x[k] - c) * r;
      q += (double)v * (double)v;
    }
    r32[i] = r;
    smu32[i] = 0.0f;
  } else {
    const double cd = (double)c;
    for (int k = 0; k < n; ++k) {
      const double d = (double)x[k] - cd;
      q += d * d;
    }
    smu32[i] = (float)(sqrt((double)n) * (mu - stats[0]));
  }
  c32[i] = c;
  cn32[i] = (float)q;
}

struct Breakpoints {
  double b[8];
};

// Z = false: PAA of the window on the series normalised by eq. (2) once;
// Z = true: PAA of the window normalised on its own, element by element as
// (t - mu_i) / sigma_i (a flat window gives zeros), then summed per segment.
template <bool Z>
__global__ __launch_bounds__(256) void k_sax(const float* __restrict__ T, int64_t N, int n, int w,
                                             int alpha, Breakpoints bp,
                                             const double* __restrict__ stats,
                                             const double* __restrict__ zmu,
                                             const double* __restrict__ zsg,
                                             int32_t* __restrict__ words,
                                             int32_t* __restrict__ hist) {
  __shared__ int32_t lh[kMaxWords];
  extern __shared__ float stage[];
  for (int b = threadIdx.x; b < kMaxWords; b += 256) lh[b] = 0;
  const int64_t i0 = blockIdx.x * 256ll;
  const int64_t i = i0 + threadIdx.x;
  const float* x = stage_windows(T, i0, n, stage);   // (its barrier also covers lh)
  if (i < N) {
    const double mu = Z ? zmu[i] : stats[0], sigma = Z ? zsg[i] : stats[1];
    int32_t code = 0;
    for (int s = 0; s < w; ++s) {
      const int a = (int)(((int64_t)s * n) / w), e = (int)(((int64_t)(s + 1) * n) / w);
      double acc = 0.0;
      double paa;
      if (Z) {
        if (sigma > 0.0)
          for (int k = a; k < e; ++k) acc = acc + ((double)x[k] - mu) / sigma;
        paa = acc / (double)(e - a);
      } else {
        for (int k = a; k < e; ++k) acc += (double)x[k];
        // mean of the segment on the normalised series: (mean(raw) - mu) / sigma
        paa = (acc / (double)(e - a) - mu) / sigma;
      }
      int sym = 0;
      while (sym < alpha - 1 && paa >= bp.b[sym]) ++sym;   // beta_{k} <= paa < beta_{k+1}
      code = code * alpha + sym;
    }
    words[i] = code;
    atomicAdd(&lh[code], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kMaxWords; b += 256)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// min over the occurring words of their frequency (eq. 7's min_j Freq(j))
__global__ __launch_bounds__(256) void k_min_freq(const int32_t* __restrict__ hist, int dict,
                                                  int32_t* __restrict__ out) {
  __shared__ int32_t sh[4];
  int32_t v = 0x7fffffff;
  for (int b = threadIdx.x; b < dict; b += 256)
    if (hist[b] > 0) v = min(v, hist[b]);
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
}

__device__ inline uint64_t lanemask_lt() {
  const int l = threadIdx.x & 63;
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Stable compaction of {i : hist[words[i]] == minfreq}: segment counts.
__global__ __launch_bounds__(64) void k_cand_count(const int32_t* __restrict__ words,
                                                   const int32_t* __restrict__ hist,
                                                   const int32_t* __restrict__ minfreq, int64_t N,
                                                   int32_t* __restrict__ seg_counts) {
  const int64_t b = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(N, b + kSegRows);
  const int32_t mf = *minfreq;
  int32_t c = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 64) c += (hist[words[i]] == mf);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if (threadIdx.x == 0) seg_counts[blockIdx.x] = c;
}

// exclusive scan of segment counts (single block); total to *total
__global__ __launch_bounds__(256) void k_scan_segments(int32_t* __restrict__ seg, int64_t nseg,
                                                       int32_t* __restrict__ total) {
  __shared__ int32_t carry;
  __shared__ int32_t wsum[4];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nseg; base += 256) {
    const int64_t k = base + threadIdx.x;
    const int32_t v = k < nseg ? seg[k] : 0;
    // inclusive scan within the wave
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if ((threadIdx.x & 63) >= off) x += y;
    }
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    int32_t pre = carry;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += wsum[w];
    if (k < nseg) seg[k] = pre + x - v;
    __syncthreads();
    if (threadIdx.x == 255) carry = pre + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(64) void k_cand_scatter(const int32_t* __restrict__ words,
                                                     const int32_t* __restrict__ hist,
                                                     const int32_t* __restrict__ minfreq, int64_t N,
                                                     const int32_t* __restrict__ seg_base,
                                                     int32_t* __restrict__ cand) {
  const int64_t b = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(N, b + kSegRows);
  const int32_t mf = *minfreq;
  int32_t run = seg_base[blockIdx.x];
  for (int64_t i0 = b; i0 < e; i0 += 64) {
    const int64_t i = i0 + threadIdx.x;
    const bool f = i < e && hist[words[i]] == mf;
    const uint64_t mask = __ballot(f);
    if (f) cand[run + __popcll(mask & lanemask_lt())] = (int32_t)i;
    run += __popcll(mask);
  }
}

// Generic stable compaction of the indices k with flags[k] != 0 (k < count).
__global__ __launch_bounds__(64) void k_flag_count(const int32_t* __restrict__ flags, int64_t count,
                                                   int32_t* __restrict__ seg_counts) {
  const int64_t b = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(count, b + kSegRows);
  int32_t c = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 64) c += (flags[i] != 0);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if (threadIdx.x == 0) seg_counts[blockIdx.x] = c;
}

__global__ __launch_bounds__(64) void k_flag_scatter(const int32_t* __restrict__ flags,
                                                     int64_t count,
                                                     const int32_t* __restrict__ seg_base,
                                                     int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(count, b + kSegRows);
  int32_t run = seg_base[blockIdx.x];
  for (int64_t i0 = b; i0 < e; i0 += 64) {
    const int64_t i = i0 + threadIdx.x;
    const bool f = i < e && flags[i] != 0;
    const uint64_t mask = __ballot(f);
    if (f) out[run + __popcll(mask & lanemask_lt())] = (int32_t)i;
    run += __popcll(mask);
  }
}

// flags[g] = 1 for every row group g holding a Cand row
__global__ __launch_bounds__(256) void k_cand_group_flags(const int32_t* __restrict__ cand,
                                                          const int32_t* __restrict__ cand_count,
                                                          int shift, int32_t* __restrict__ flags) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k < *cand_count) flags[cand[k] >> shift] = 1;
}

// Column groups of each word's Index_Word bucket (eq. 10): the distinct values
// members[k] >> shift over the word's member range, ascending.  One block per word.
__device__ inline bool bucket_flag(const int32_t* __restrict__ members, int64_t k, int64_t first,
                                   int shift) {
  return k == first || (members[k] >> shift) != (members[k - 1] >> shift);
}

__global__ __launch_bounds__(256) void k_bucket_count(const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ members, int shift,
                                                      int32_t* __restrict__ counts) {
  __shared__ int32_t sh[4];
  const int w = blockIdx.x;
  const int64_t b = offsets[w], e = offsets[w + 1];
  int32_t c = 0;
  for (int64_t k = b + threadIdx.x; k < e; k += 256) c += bucket_flag(members, k, b, shift);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[w] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_bucket_offsets(const int32_t* __restrict__ counts, int dict,
                                 int32_t* __restrict__ goff) {
  if (threadIdx.x != 0) return;
  int32_t run = 0;
  for (int w = 0; w < dict; ++w) {
    goff[w] = run;
    run += counts[w];
  }
  goff[dict] = run;
}

__global__ void k_max_bucket(const int32_t* __restrict__ goff, int dict, int32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  int32_t m = 0;
  for (int w = 0; w < dict; ++w) m = max(m, goff[w + 1] - goff[w]);
  *out = m;
}

__global__ __launch_bounds__(256) void k_bucket_scatter(const int32_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ members,
                                                        int shift, const int32_t* __restrict__ goff,
                                                        int32_t* __restrict__ groups) {
  __shared__ int32_t wsum[4];
  const int w = blockIdx.x;
  const int64_t b = offsets[w], e = offsets[w + 1];
  int32_t run = goff[w];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = b; base < e; base += 256) {
    const int64_t k = base + threadIdx.x;
    const bool f = k < e && bucket_flag(members, k, b, shift);
    const uint64_t mask = __ballot(f);
    if (lane == 0) wsum[wv] = __popcll(mask);
    __syncthreads();
    int32_t pre = run;
    for (int q = 0; q < wv; ++q) pre += wsum[q];
    if (f) groups[pre + __popcll(mask & lanemask_lt())] = members[k] >> shift;
    run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

// CSR counting sort: per-segment word counts
__global__ __launch_bounds__(64) void k_csr_count(const int32_t* __restrict__ words, int64_t N,
                                                  int dict, int32_t* __restrict__ seg_counts) {
  __shared__ int32_t lh[kMaxWords];
  for (int b = threadIdx.x; b < kMaxWords; b += 64) lh[b] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(N, b0 + kSegRows);
  for (int64_t i = b0 + threadIdx.x; i < e; i += 64) atomicAdd(&lh[words[i]], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < dict; b += 64) seg_counts[(int64_t)blockIdx.x * dict + b] = lh[b];
}

// offsets = exclusive scan of hist; seg_counts[s][w] -> base of segment s for word w
// One workgroup per word w: offsets[w] = sum of the frequencies of the words
// before it, then the exclusive scan of w's per-segment counts (segment s at
// seg_counts[s * dict + w]) on top of it, 256 segments at a time.
__global__ __launch_bounds__(256) void k_csr_scan(const int32_t* __restrict__ hist, int dict,
                                                  int64_t nseg, int32_t* __restrict__ seg_counts,
                                                  int32_t* __restrict__ offsets) {
  __shared__ int32_t wsum[4];
  const int w = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // sum over the block of one value per thread, returned to every thread
  auto block_sum = [&](int32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();                       // wsum free again
    if (lane == 0) wsum[wv] = v;
    __syncthreads();
    return wsum[0] + wsum[1] + wsum[2] + wsum[3];
  };
  int32_t part = 0;
  for (int k = threadIdx.x; k < w; k += 256) part += hist[k];
  int32_t carry = block_sum(part);
  if (threadIdx.x == 0) {
    offsets[w] = carry;
    if (w == dict - 1) offsets[dict] = carry + hist[w];
  }
  for (int64_t s0 = 0; s0 < nseg; s0 += 256) {
    const int64_t sg = s0 + threadIdx.x;
    const int32_t v = sg < nseg ? seg_counts[sg * dict + w] : 0;
    // inclusive scan within the wave, then the wave totals
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __syncthreads();                       // wsum free again
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int32_t before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    const int32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (sg < nseg) seg_counts[sg * dict + w] = carry + before + x - v;
    carry += total;
  }
}

__global__ __launch_bounds__(64) void k_csr_scatter(const int32_t* __restrict__ words, int64_t N,
                                                    int dict, const int32_t* __restrict__ seg_base,
                                                    int32_t* __restrict__ members) {
  __shared__ int32_t run[kMaxWords];
  for (int b = threadIdx.x; b < dict; b += 64) run[b] = seg_base[(int64_t)blockIdx.x * dict + b];
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kSegRows;
  const int64_t e = min<int64_t>(N, b0 + kSegRows);
  const uint64_t lt = lanemask_lt();
  for (int64_t i0 = b0; i0 < e; i0 += 64) {
    const int64_t i = i0 + threadIdx.x;
    const bool valid = i < e;
    const int32_t wd = valid ? words[i] : -1;
    uint64_t todo = __ballot(valid);
    while (todo) {
      const int leader = __builtin_ctzll(todo);
      const int32_t w0 = __shfl(wd, leader, 64);
      const bool mine = valid && wd == w0;
      const uint64_t same = __ballot(mine);
      const int32_t base = run[w0];
      if (mine) members[base + __popcll(same & lt)] = (int32_t)i;
      __builtin_amdgcn_wave_barrier();
      if ((int)threadIdx.x == leader) run[w0] = base + __popcll(same);
      __builtin_amdgcn_wave_barrier();
      todo &= ~same;
    }
  }
}

}  // namespace

int64_t csr_waves(int64_t N) { return (N + kSegRows - 1) / kSegRows; }
int64_t compact_waves(int64_t N) { return (N + kSegRows - 1) / kSegRows; }

void launch_stats(const float* Tp, int64_t m, double* partials, double* stats, int* bad,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(kStatBlocks), dim3(256), 0, s, Tp, m, partials, bad);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partials, kStatBlocks, m, stats, 0);
  hipLaunchKernelGGL(k_sqdev, dim3(kStatBlocks), dim3(256), 0, s, Tp, m, stats, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partials, kStatBlocks, m, stats, 1);
}

void launch_row_stats(const float* Tp, int64_t N, int n, double* row_mean, double* row_cnorm,
                      double* row_sigma, hipStream_t s) {
  const int64_t blocks = (N + 255) / 256;
  hipLaunchKernelGGL(k_row_stats, dim3((unsigned)blocks), dim3(256), stage_bytes(n), s, Tp, N, n,
                     row_mean, row_cnorm, row_sigma);
}

void launch_row_stats32(const float* Tp, int64_t N, int n, int64_t padded, const double* row_mean,
                        const double* row_sigma, const double* stats, float* c32, float* smu32,
                        float* cn32, float* r32, hipStream_t s) {
  const int64_t blocks = (padded + 255) / 256;
  hipLaunchKernelGGL(k_row_stats32, dim3((unsigned)blocks), dim3(256), stage_bytes(n), s, Tp, N, n,
                     padded, row_mean, row_sigma, stats, c32, smu32, cn32, r32);
}

// Breakpoints of eq. (4): beta_k = Phi^{-1}(k / alpha), computed on the host by
// Newton's method on Phi(x) = erfc(-x / sqrt 2) / 2 from a bracketing start.
void sax_breakpoints(int alpha, double* out);

void launch_sax(const float* Tp, int64_t N, int n, int w, int alpha, const double* stats,
                const double* zmu, const double* zsg, int32_t* words, int32_t* hist,
                hipStream_t s) {
  Breakpoints bp{};
  sax_breakpoints(alpha, bp.b);
  const int64_t blocks = (N + 255) / 256;
  if (zsg)
    hipLaunchKernelGGL(k_sax<true>, dim3((unsigned)blocks), dim3(256), stage_bytes(n), s, Tp, N, n,
                       w, alpha, bp, stats, zmu, zsg, words, hist);
  else
    hipLaunchKernelGGL(k_sax<false>, dim3((unsigned)blocks), dim3(256), stage_bytes(n), s, Tp, N,
                       n, w, alpha, bp, stats, zmu, zsg, words, hist);
}

void launch_cand(const int32_t* words, const int32_t* hist, int64_t N, int dict,
                 int32_t* minfreq_scratch, int32_t* seg_counts, int32_t* cand,
                 int32_t* cand_count, hipStream_t s) {
  const int64_t nseg = compact_waves(N);
  hipLaunchKernelGGL(k_min_freq, dim3(1), dim3(256), 0, s, hist, dict, minfreq_scratch);
  hipLaunchKernelGGL(k_cand_count, dim3((unsigned)nseg), dim3(64), 0, s, words, hist,
                     minfreq_scratch, N, seg_counts);
  hipLaunchKernelGGL(k_scan_segments, dim3(1), dim3(256), 0, s, seg_counts, nseg, cand_count);
  hipLaunchKernelGGL(k_cand_scatter, dim3((unsigned)nseg), dim3(64), 0, s, words, hist,
                     minfreq_scratch, N, seg_counts, cand);
}

void launch_compact_flags(const int32_t* flags, int64_t count, int32_t* seg_counts, int32_t* out,
                          int32_t* out_count, hipStream_t s) {
  const int64_t nseg = compact_waves(count);
  hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nseg), dim3(64), 0, s, flags, count, seg_counts);
  hipLaunchKernelGGL(k_scan_segments, dim3(1), dim3(256), 0, s, seg_counts, nseg, out_count);
  hipLaunchKernelGGL(k_flag_scatter, dim3((unsigned)nseg), dim3(64), 0, s, flags, count,
                     seg_counts, out);
}

void launch_cand_group_flags(const int32_t* cand, const int32_t* cand_count, int64_t max_cand,
                             int shift, int32_t* flags, hipStream_t s) {
  const int64_t blocks = (max_cand + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_cand_group_flags, dim3((unsigned)blocks), dim3(256), 0, s, cand,
                       cand_count, shift, flags);
}

void launch_bucket_groups(const int32_t* offsets, const int32_t* members, int dict, int shift,
                          int32_t* counts, int32_t* goff, int32_t* groups, hipStream_t s) {
  hipLaunchKernelGGL(k_bucket_count, dim3(dict), dim3(256), 0, s, offsets, members, shift, counts);
  hipLaunchKernelGGL(k_bucket_offsets, dim3(1), dim3(64), 0, s, counts, dict, goff);
  hipLaunchKernelGGL(k_bucket_scatter, dim3(dict), dim3(256), 0, s, offsets, members, shift, goff,
                     groups);
}

void launch_max_bucket(const int32_t* goff, int dict, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_bucket, dim3(1), dim3(64), 0, s, goff, dict, out);
}

void launch_csr(const int32_t* words, const int32_t* hist, int64_t N, int dict,
                int32_t* seg_counts, int32_t* offsets, int32_t* members, hipStream_t s) {
  const int64_t nseg = csr_waves(N);
  hipLaunchKernelGGL(k_csr_count, dim3((unsigned)nseg), dim3(64), 0, s, words, N, dict,
                     seg_counts);
  hipLaunchKernelGGL(k_csr_scan, dim3((unsigned)dict), dim3(256), 0, s, hist, dict, nseg, seg_counts,
                     offsets);
  hipLaunchKernelGGL(k_csr_scatter, dim3((unsigned)nseg), dim3(64), 0, s, words, N, dict,
                     seg_counts, members);
}

}  // namespace dd
