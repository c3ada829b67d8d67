// bound.hip -- a cheap lower bound of every row's nearest-neighbour distance,
// used to choose which rows the search completes first.
//
// For windows a, b of length n with means mu_a, mu_b, the squared distance of
// eq. (1) splits into the centred part and the mean part,
//     |a - b|^2 = |(a - mu_a) - (b - mu_b)|^2 + n (mu_a - mu_b)^2 ,
// so d^2(i, j) >= n (mu_i - mu_j)^2 and NN(i) >= n min_j (mu_i - mu_j)^2 over
// the non-self j (|i - j| >= n).  A window whose mean lies where the series is
// rarely seen (apart from its own neighbourhood) therefore has a large NN, and
// the discord, the row with the largest NN, tends to be among the rows with
// the largest bound.  Completing those rows first raises the best-so-far close
// to its final value before the bulk of the rows are searched.  The bound only
// orders work: the search's result never depends on it.
//
// Evaluation: the row means are binned (B bins over [min, max], about 16 rows
// per bin on average, B <= 65536); each bin keeps its smallest and largest row
// index.  Bin c holds a non-self match of row i exactly when max_c >= i + n or
// min_c <= i - n, so the first such bin at distance d from row i's own bin
// bounds the nearest non-self mean below by (d - 1) bin widths.  With bins
// that dense, a row leaves the outward search after a bin or two unless its
// level is rare, which is what the bound is for.  Groups of 16 bins and
// supergroups of 256 keep the smallest and largest row index of their bins as
// well, so the search crosses a (super)group without a match in one step: a
// row at a rare level checks a few dozen slots on either side instead of
// hundreds or thousands of bins.
#include "internal.hpp"

namespace dd {
namespace {

constexpr int kBoundBins = 65536;   // most bins
constexpr int kG1 = 16;             // bins per group
constexpr int kG2 = 256;            // bins per supergroup (kG2 / kG1 groups)
// scratch arrays (smallest / largest row index): the bins, then their groups
// from kBoundBins on, then their supergroups
constexpr int kGroupBase = kBoundBins;
constexpr int kSuperBase = kBoundBins + kBoundBins / kG1;
constexpr int kBoundSlots = kSuperBase + kBoundBins / kG2;

// order-preserving map of doubles to unsigned integers
__device__ __forceinline__ uint64_t ordered(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unordered(uint64_t u) {
  return __builtin_bit_cast(double, (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u);
}

__global__ __launch_bounds__(256) void k_mean_range(const double* __restrict__ mu, int64_t N,
                                                    uint64_t* __restrict__ range) {
  __shared__ uint64_t lo_s[4], hi_s[4];
  uint64_t lo = ~0ull, hi = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const uint64_t u = ordered(mu[i]);
    lo = u < lo ? u : lo;
    hi = u > hi ? u : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t a = __shfl_xor(lo, off, 64), b = __shfl_xor(hi, off, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    lo_s[threadIdx.x >> 6] = lo;
    hi_s[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = lo_s[w] < lo ? lo_s[w] : lo;
      hi = hi_s[w] > hi ? hi_s[w] : hi;
    }
    atomicMin((unsigned long long*)&range[0], (unsigned long long)lo);
    atomicMax((unsigned long long*)&range[1], (unsigned long long)hi);
  }
}

struct Bins {
  double lo, inv_width, width;
  int count;
};

__device__ __forceinline__ Bins bins_of(const uint64_t* __restrict__ range, int count) {
  const double lo = unordered(range[0]), hi = unordered(range[1]);
  const double span = hi - lo;
  Bins b;
  b.lo = lo;
  b.width = span > 0.0 ? span / count : 1.0;
  b.inv_width = span > 0.0 ? count / span : 0.0;
  b.count = count;
  return b;
}

__device__ __forceinline__ int bin_of(const Bins& b, double x) {
  const double t = (x - b.lo) * b.inv_width;
  const int k = t > 0.0 ? (int)t : 0;
  return k < b.count - 1 ? k : b.count - 1;
}

__global__ __launch_bounds__(256) void k_bin_rows(const double* __restrict__ mu, int64_t N,
                                                  const uint64_t* __restrict__ range, int nbins,
                                                  int32_t* __restrict__ bmin,
                                                  int32_t* __restrict__ bmax) {
  const Bins b = bins_of(range, nbins);
  const int lane = threadIdx.x & 63;
  // the loop bound is uniform across the block (base steps by whole blocks), so
  // every lane of a wavefront takes each iteration and the shuffles see all 64
  for (int64_t base = blockIdx.x * 256ll; base < N; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + threadIdx.x;
    const int k = i < N ? bin_of(b, mu[i]) : -1;
    // a wavefront's rows ascend with the lane, and neighbouring windows have
    // nearly equal means: a run of lanes in one bin sends only its first row
    // (the run's smallest index) to atomicMin and its last (the largest) to
    // atomicMax, instead of every lane hitting the same address
    const int kp = __shfl_up(k, 1, 64), kn = __shfl_down(k, 1, 64);
    if (k >= 0) {
      if (lane == 0 || kp != k) atomicMin(&bmin[k], (int32_t)i);
      if (lane == 63 || kn != k) atomicMax(&bmax[k], (int32_t)i);
    }
  }
}

// the smallest / largest row index of every group (level 1) or supergroup
// (level 2) over its bins: one workgroup of kG2 threads per supergroup, whose
// threads are its bins (bins past nbins count as empty)
__global__ __launch_bounds__(kG2) void k_bin_groups(int nbins, int32_t* __restrict__ bmin,
                                                    int32_t* __restrict__ bmax) {
  __shared__ int32_t lo_s[kG2 / 64], hi_s[kG2 / 64];
  const int c = blockIdx.x * kG2 + threadIdx.x;
  int32_t lo = c < nbins ? bmin[c] : 0x7FFFFFFF, hi = c < nbins ? bmax[c] : -1;
  // groups of kG1 bins: kG1 consecutive lanes
  for (int off = 1; off < kG1; off <<= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  if ((threadIdx.x & (kG1 - 1)) == 0 && c < nbins) {
    bmin[kGroupBase + c / kG1] = lo;
    bmax[kGroupBase + c / kG1] = hi;
  }
  for (int off = kG1; off < 64; off <<= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    lo_s[threadIdx.x >> 6] = lo;
    hi_s[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kG2 / 64; ++w) {
      lo = min(lo, lo_s[w]);
      hi = max(hi, hi_s[w]);
    }
    bmin[kSuperBase + blockIdx.x] = lo;
    bmax[kSuperBase + blockIdx.x] = hi;
  }
}

// Does slot c (a bin, a group or a supergroup) hold a non-self row?
__device__ __forceinline__ bool holds_match(const int32_t* __restrict__ bmin,
                                            const int32_t* __restrict__ bmax, int c,
                                            int64_t lo_row, int64_t hi_row) {
  return bmax[c] >= hi_row || bmin[c] <= lo_row;
}

// The nearest bin at distance < limit from bin k, going down (dir < 0) or up,
// that holds a non-self row: its distance, or `limit` if none.  Bins of k's
// group one by one, then groups of k's supergroup, then supergroups; a
// (super)group that holds a match is entered (the match is in it).
__device__ int nearest_match(const int32_t* __restrict__ bmin, const int32_t* __restrict__ bmax,
                             int nbins, int k, int dir, int limit, int64_t lo_row,
                             int64_t hi_row) {
  auto dist = [&](int c) { return dir < 0 ? k - c : c - k; };
  // bins from c on (towards dir) until the edge of their group; -1 if none matches
  auto scan_bins = [&](int c) -> int {
    const int edge = dir < 0 ? c / kG1 * kG1 : min(nbins, (c / kG1 + 1) * kG1) - 1;
    for (;; c += dir) {
      if (dist(c) >= limit) return limit;
      if (holds_match(bmin, bmax, c, lo_row, hi_row)) return dist(c);
      if (c == edge) return -1;
    }
  };
  // groups from g on until the edge of their supergroup, entering the first
  // that matches; -1 if none does
  const int ngroups = (nbins + kG1 - 1) / kG1;
  auto scan_groups = [&](int g) -> int {
    const int edge = dir < 0 ? g / (kG2 / kG1) * (kG2 / kG1)
                             : min(ngroups, (g / (kG2 / kG1) + 1) * (kG2 / kG1)) - 1;
    for (;; g += dir) {
      const int first = dir < 0 ? (g + 1) * kG1 - 1 : g * kG1;   // its bin nearest to k
      if (dist(first) >= limit) return limit;
      if (holds_match(bmin, bmax, kGroupBase + g, lo_row, hi_row)) {
        const int d = scan_bins(first);
        return d >= 0 ? d : limit;   // (a matching group holds a matching bin)
      }
      if (g == edge) return -1;
    }
  };
  int d = scan_bins(k);
  if (d >= 0) return d;
  const int g = k / kG1 + dir;
  if (g >= 0 && g < ngroups && g / (kG2 / kG1) == k / kG2) {
    d = scan_groups(g);
    if (d >= 0) return d;
  }
  const int nsuper = (nbins + kG2 - 1) / kG2;
  for (int sg = k / kG2 + dir; sg >= 0 && sg < nsuper; sg += dir) {
    const int first = dir < 0 ? (sg + 1) * kG2 - 1 : sg * kG2;
    if (dist(first) >= limit) return limit;
    if (!holds_match(bmin, bmax, kSuperBase + sg, lo_row, hi_row)) continue;
    d = scan_groups(first / kG1);
    return d >= 0 ? d : limit;
  }
  return limit;
}

__global__ __launch_bounds__(256) void k_row_bound(const double* __restrict__ mu, int64_t N, int n,
                                                   const uint64_t* __restrict__ range, int nbins,
                                                   const int32_t* __restrict__ bmin,
                                                   const int32_t* __restrict__ bmax,
                                                   float* __restrict__ lb) {
  const Bins b = bins_of(range, nbins);
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const int k = bin_of(b, mu[i]);
    const int64_t lo_row = i - n, hi_row = i + n;   // non-self: j <= lo_row or j >= hi_row
    // the nearest matching bin on either side; with none at all (a row without
    // non-self matches) the distance to the farther end of the bins
    const int none = max(k + 1, nbins - k);
    const int dd = nearest_match(bmin, bmax, nbins, k, -1, min(k + 1, none), lo_row, hi_row);
    const int limit_up = dd <= k ? dd : none;
    const int du = nearest_match(bmin, bmax, nbins, k, 1, min(nbins - k, limit_up), lo_row, hi_row);
    int d = min(dd <= k ? dd : none, du < nbins - k ? du : none);
    const double gap = (d > 1 ? d - 1 : 0) * b.width;
    lb[i] = (float)(n * gap * gap);
  }
}

// item score: the largest bound among the item's rows (non-negative floats
// order like their bit patterns)
__global__ __launch_bounds__(256) void k_item_bound(const float* __restrict__ lb, int64_t N,
                                                    int64_t item_rows, int64_t n_items,
                                                    uint32_t* __restrict__ score) {
  for (int64_t t = blockIdx.x * 256ll + threadIdx.x; t < n_items; t += (int64_t)gridDim.x * 256) {
    const int64_t r0 = t * item_rows, r1 = min<int64_t>(N, r0 + item_rows);
    uint32_t s = 0;
    for (int64_t i = r0; i < r1; ++i) {
      const uint32_t v = __builtin_bit_cast(uint32_t, lb[i]);
      s = v > s ? v : s;
    }
    score[t] = s;
  }
}

// only the first min(count, win->n_groups) entries: the list holds that many
// (none when the device loop stopped before it began)
__global__ __launch_bounds__(256) void k_flag_items(const int32_t* __restrict__ list, int64_t count,
                                                    const WinDesc* __restrict__ win,
                                                    int32_t* __restrict__ flags,
                                                    int32_t* __restrict__ flags2) {
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  const int64_t c = win->n_groups < count ? win->n_groups : count;
  if (t < c) {
    const int32_t g = list[t];
    flags[g] = 1;
    if (flags2) flags2[g] = 1;
  }
}

// blocks of 256 threads for `count` items, at most `cap` (threads then stride)
unsigned blocks_for(int64_t count, int64_t cap = 1024) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

size_t bound_bins() { return kBoundSlots; }

void launch_row_bound(const double* row_mean, int64_t N, int n, uint64_t* range, int32_t* bmin,
                      int32_t* bmax, float* lb, hipStream_t s) {
  int nbins = 64;   // a power of two near N / 16, within [64, kBoundBins]
  while (nbins < kBoundBins && (int64_t)nbins * 16 < N) nbins *= 2;
  const FillOp fills[] = {
      {range, 1, ~0ull, 1},
      {range + 1, 1, 0, 1},
      {bmin, nbins, 0x7FFFFFFF, 0},
      {bmax, nbins, 0xFFFFFFFFu, 0},
  };
  launch_fill_many(fills, 4, s);
  // few workgroups: each ends with two atomics on the same two words, which the
  // memory system serialises (1024 workgroups took 26 us on 2^20 rows)
  hipLaunchKernelGGL(k_mean_range, dim3(blocks_for(N, 256)), dim3(256), 0, s, row_mean, N, range);
  hipLaunchKernelGGL(k_bin_rows, dim3(blocks_for(N, 4096)), dim3(256), 0, s, row_mean, N, range, nbins,
                     bmin, bmax);
  hipLaunchKernelGGL(k_bin_groups, dim3((unsigned)((nbins + kG2 - 1) / kG2)), dim3(kG2), 0, s,
                     nbins, bmin, bmax);
  // one thread per row: the outward search is a chain of dependent loads, so
  // many rows in flight hide its latency
  hipLaunchKernelGGL(k_row_bound, dim3(blocks_for(N, 4096)), dim3(256), 0, s, row_mean, N, n, range,
                     nbins, bmin, bmax, lb);
}

void launch_item_bound(const float* lb, int64_t N, int64_t item_rows, int64_t n_items,
                       uint32_t* score, hipStream_t s) {
  hipLaunchKernelGGL(k_item_bound, dim3(blocks_for(n_items)), dim3(256), 0, s, lb, N, item_rows,
                     n_items, score);
}

void launch_flag_items(const int32_t* list, int64_t count, const WinDesc* win, int32_t* flags,
                       int32_t* flags2, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_flag_items, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, list,
                       count, win, flags, flags2);
}

}  // namespace dd
