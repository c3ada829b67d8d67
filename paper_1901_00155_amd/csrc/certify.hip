// certify.hip -- FP64 steps of the search: the exact nearest neighbour of chosen
// rows, the witness verification that proves every other row cannot be the
// discord, and the device-wide argmax with the lowest-index tie rule.
//
// Why this is exact.  Let L be the exact NN (squared) of some row s.  Every row
// i carries a witness w(i), a non-self column found by the approximate scan
// (its approximate argmin, or the column that made it leave early).  The
// verification checks that w(i) is a column of the matrix and a non-self match
// (|i - w(i)| >= n) itself, so it does not trust the scans' masks.  Its NN is
// at most e(i) = d^2(i, w(i)) computed exactly here.  If e(i) < L, or e(i) = L
// and i > s, row i cannot be the discord under the lowest-index rule.  The rows
// that fail this test get their exact NN by a full FP64 row scan, and the final
// answer is the argmax over s and those rows.  No step relies on an error bound
// of the approximate arithmetic.
//
// FP64 distances are the sequential sum over k = 0..n-1 of (a_k - b_k)^2 with a
// separately rounded multiply and add (contraction off), i.e. the sum eq. (1)
// defines, accumulated in the order it is written; under per-window
// normalisation a_k and b_k are the normalised window elements.
#include <algorithm>

#include "internal.hpp"

namespace dd {
namespace {

#pragma clang fp contract(off)

// The two windows' values are loaded kPairBatch at a time ahead of the sum, so
// a thread has that many loads in flight instead of waiting on each one; the
// additions keep their sequential order.
constexpr int kPairBatch = 16;

__device__ inline double d2_fp64(const float* __restrict__ T, int64_t i, int64_t j, int n) {
  double s = 0.0;
  int k = 0;
  for (; k + kPairBatch <= n; k += kPairBatch) {
    float x[kPairBatch], y[kPairBatch];
#pragma unroll
    for (int u = 0; u < kPairBatch; ++u) {
      x[u] = T[i + k + u];
      y[u] = T[j + k + u];
    }
#pragma unroll
    for (int u = 0; u < kPairBatch; ++u) {
      const double d = (double)x[u] - (double)y[u];
      s = s + d * d;
    }
  }
  for (; k < n; ++k) {
    const double d = (double)T[i + k] - (double)T[j + k];
    s = s + d * d;
  }
  return s;
}

// Per-window normalisation: element k of window i is (t_{i+k} - mu_i) / sigma_i
// (a correctly rounded FP64 division), or 0 for a flat window; the distance is
// the same sequential sum over the normalised elements.
__device__ inline double zval(const float* __restrict__ T, int64_t i, int k, double mu, double sg) {
  return sg > 0.0 ? ((double)T[i + k] - mu) / sg : 0.0;
}

__device__ inline double d2_fp64_z(const float* __restrict__ T, int64_t i, int64_t j, int n,
                                   ZStats z) {
  const double mi = z.mu[i], si = z.sg[i], mj = z.mu[j], sj = z.sg[j];
  double s = 0.0;
  int k = 0;
  for (; k + kPairBatch <= n; k += kPairBatch) {
    float x[kPairBatch], y[kPairBatch];
#pragma unroll
    for (int u = 0; u < kPairBatch; ++u) {
      x[u] = T[i + k + u];
      y[u] = T[j + k + u];
    }
#pragma unroll
    for (int u = 0; u < kPairBatch; ++u) {
      const double d = (si > 0.0 ? ((double)x[u] - mi) / si : 0.0) -
                       (sj > 0.0 ? ((double)y[u] - mj) / sj : 0.0);
      s = s + d * d;
    }
  }
  for (; k < n; ++k) {
    const double d = zval(T, i, k, mi, si) - zval(T, j, k, mj, sj);
    s = s + d * d;
  }
  return s;
}

template <bool Z>
__device__ inline double pair_d2(const float* __restrict__ T, int64_t i, int64_t j, int n, ZStats z) {
  if constexpr (Z)
    return d2_fp64_z(T, i, j, n, z);
  else
    return d2_fp64(T, i, j, n);
}

__device__ inline bool has_non_self(int64_t i, int64_t N, int n) {
  return (i - n >= 0) || (i + n <= N - 1);
}

__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t v) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// Several fills in one launch: blockIdx.y selects the buffer.
__global__ void k_fill_many(FillList L) {
  const FillOp& op = L.op[blockIdx.y];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < op.count;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (op.wide)
      static_cast<uint64_t*>(op.p)[k] = op.value;
    else
      static_cast<uint32_t*>(op.p)[k] = (uint32_t)op.value;
  }
}

// Block-wide reductions that end in one atomic per block.  Device-scope
// atomics on one address are serialised in the memory system (about 10 ns
// each), so a grid that issued one per wavefront spent most of its time there.
__device__ inline uint32_t block_sum_u32(uint32_t v, uint32_t* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

__device__ inline uint64_t wave_max_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

__device__ inline uint64_t block_max_u64(uint64_t v, uint64_t* red) {
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = red[w] > t ? red[w] : t;
  return t;
}

// grid of the row-wise passes below: at most kRowPassBlocks blocks of 256,
// each thread striding over rows
constexpr int64_t kRowPassBlocks = 1024;

unsigned row_pass_blocks(int64_t N) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kRowPassBlocks, (N + 255) / 256));
}

// the witness verification: one row per thread up to 2^21 rows (each row's
// FP64 sum is a chain of dependent adds, so many rows in flight hide it)
unsigned verify_blocks(int64_t N) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (N + 255) / 256));
}

// Rows of the scan: minimum (or abandon distance) and its column; a row is
// abandoned when its bit in the group's alive mask was cleared.
__global__ __launch_bounds__(256) void k_unpack_best(const uint64_t* __restrict__ best, int64_t N,
                                                     const uint32_t* __restrict__ alive, int gsz,
                                                     float* __restrict__ nn_approx,
                                                     int32_t* __restrict__ nn_witness,
                                                     int32_t* __restrict__ row_state,
                                                     uint32_t* __restrict__ n_abandoned) {
  __shared__ uint32_t red[4];
  uint32_t ab_count = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    const uint64_t k = best[i];
    if (k == kEmptyMin) {
      nn_approx[i] = __builtin_inff();
      nn_witness[i] = -1;
      row_state[i] = kRowUnscanned;
    } else {
      const bool ab = alive && !((alive[i / gsz] >> (i % gsz)) & 1u);
      nn_approx[i] = key_dist(k);
      nn_witness[i] = (int32_t)(k & 0xFFFFFFFFu);
      row_state[i] = ab ? kRowAbandoned : kRowFull;
      ab_count += ab ? 1u : 0u;
    }
  }
  const uint32_t t = block_sum_u32(ab_count, red);
  if (threadIdx.x == 0 && t) atomicAdd(n_abandoned, t);
}

__global__ __launch_bounds__(256) void k_init_alive(uint32_t* __restrict__ alive, int64_t G,
                                                    int64_t N, int gsz) {
  const int64_t g = blockIdx.x * 256ll + threadIdx.x;
  if (g >= G) return;
  const int64_t rows = min<int64_t>(gsz, N - g * gsz);
  alive[g] = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
}

// max approximate NN over fully scanned rows, lowest row on ties
__global__ __launch_bounds__(256) void k_seed_argmax(const uint64_t* __restrict__ best,
                                                     const int32_t* __restrict__ row_state,
                                                     int64_t N, uint64_t* __restrict__ seed) {
  __shared__ uint64_t red[4];
  uint64_t key = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
    if (row_state[i] == kRowFull) {
      const uint64_t k = pack_max(key_dist(best[i]), (uint32_t)i);
      key = k > key ? k : key;
    }
  key = block_max_u64(key, red);
  if (threadIdx.x == 0 && key) atomicMax((unsigned long long*)seed, (unsigned long long)key);
}

__global__ void k_seed_row(const uint64_t* __restrict__ seed, int64_t* __restrict__ rows) {
  const uint64_t k = *seed;
  rows[0] = k ? (int64_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFu)) : 0;
}

// Exact NN of rows[y] over the columns of chunk x: block min, lowest j on ties.
template <bool Z>
__global__ __launch_bounds__(256) void k_rows_nn_fp64(const float* __restrict__ T, int n, int64_t N,
                                                      ZStats z,
                                                      const int64_t* __restrict__ rows,
                                                      int64_t nchunks,
                                                      double* __restrict__ part_d,
                                                      int64_t* __restrict__ part_j,
                                                      const uint32_t* __restrict__ count) {
  __shared__ double sd[256];
  __shared__ int64_t sj[256];
  if (count && (int64_t)blockIdx.y >= (int64_t)*count) return;   // row beyond the device count
  const int64_t i = rows[blockIdx.y];
  const int64_t cb = (int64_t)blockIdx.x * kFp64Cols;
  const int64_t ce = min<int64_t>(N, cb + kFp64Cols);
  double bd = __builtin_inf();
  int64_t bj = -1;
  for (int64_t j = cb + threadIdx.x; j < ce; j += 256) {
    const int64_t dij = i > j ? i - j : j - i;
    if (dij < n) continue;
    const double d = pair_d2<Z>(T, i, j, n, z);
    if (d < bd) {
      bd = d;
      bj = j;
    }
  }
  sd[threadIdx.x] = bd;
  sj[threadIdx.x] = bj;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double od = sd[threadIdx.x + h];
      const int64_t oj = sj[threadIdx.x + h];
      const double md = sd[threadIdx.x];
      const int64_t mj = sj[threadIdx.x];
      if (oj >= 0 && (mj < 0 || od < md || (od == md && oj < mj))) {
        sd[threadIdx.x] = od;
        sj[threadIdx.x] = oj;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_d[blockIdx.y * nchunks + blockIdx.x] = sd[0];
    part_j[blockIdx.y * nchunks + blockIdx.x] = sj[0];
  }
}

__global__ __launch_bounds__(256) void k_rows_nn_reduce(const double* __restrict__ part_d,
                                                        const int64_t* __restrict__ part_j,
                                                        int64_t nchunks, double* __restrict__ out_d,
                                                        int64_t* __restrict__ out_j,
                                                        const uint32_t* __restrict__ count) {
  __shared__ double sd[256];
  __shared__ int64_t sj[256];
  if (count && (int64_t)blockIdx.x >= (int64_t)*count) return;
  double bd = __builtin_inf();
  int64_t bj = -1;
  const double* pd = part_d + blockIdx.x * nchunks;
  const int64_t* pj = part_j + blockIdx.x * nchunks;
  for (int64_t c = threadIdx.x; c < nchunks; c += 256) {
    const double d = pd[c];
    const int64_t j = pj[c];
    if (j >= 0 && (bj < 0 || d < bd || (d == bd && j < bj))) {
      bd = d;
      bj = j;
    }
  }
  sd[threadIdx.x] = bd;
  sj[threadIdx.x] = bj;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double od = sd[threadIdx.x + h];
      const int64_t oj = sj[threadIdx.x + h];
      const double md = sd[threadIdx.x];
      const int64_t mj = sj[threadIdx.x];
      if (oj >= 0 && (mj < 0 || od < md || (od == md && oj < mj))) {
        sd[threadIdx.x] = od;
        sj[threadIdx.x] = oj;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out_d[blockIdx.x] = sd[0];
    out_j[blockIdx.x] = sj[0];
  }
}

__global__ void k_exact_from_rows(const int64_t* __restrict__ rows, const double* __restrict__ d,
                                  const int64_t* __restrict__ j, Exact* __restrict__ ex) {
  ex->d2 = d[0];
  ex->i = j[0] >= 0 ? rows[0] : -1;
  ex->j = j[0];
}

// Witness verification (see the file comment); appends failing rows.
template <bool Z>
__global__ __launch_bounds__(256) void k_verify(const float* __restrict__ T, int n, int64_t N,
                                                ZStats z,
                                                const int32_t* __restrict__ nn_witness,
                                                const float* __restrict__ nn_approx,
                                                const Exact* __restrict__ ex,
                                                int64_t* __restrict__ uncertain,
                                                uint32_t* __restrict__ count,
                                                uint32_t* __restrict__ max_rel_err_bits) {
  __shared__ uint64_t red[4];
  const double L = ex->d2;
  const int64_t s = ex->i;
  float rel = 0.0f;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
    if (i == s || !has_non_self(i, N, n)) continue;
    const int32_t w = nn_witness[i];
    bool ok = false;
    // a witness clears its row only if it is a column of the matrix and a
    // non-self match of the row (|i - w| >= n); anything else sends the row to
    // the exact rescan, so the certificate does not rest on the scans' masks
    const int64_t gap = i > (int64_t)w ? i - (int64_t)w : (int64_t)w - i;
    if (w >= 0 && (int64_t)w < N && gap >= n && s >= 0) {
      const double e = pair_d2<Z>(T, i, w, n, z);
      ok = (e < L) || (e == L && i > s);
      if (e > 0.0) rel = fmaxf(rel, (float)(fabs((double)nn_approx[i] - e) / e));
    }
    if (!ok) uncertain[atomicAdd(count, 1u)] = i;
  }
  // non-negative floats order like their bit patterns
  const uint64_t m = block_max_u64(__builtin_bit_cast(uint32_t, rel), red);
  if (threadIdx.x == 0 && m) atomicMax(max_rel_err_bits, (uint32_t)m);
}

// argmax of (ex, rows[k] with exact d[k]): larger d wins, lower row on ties.
// The exact nearest neighbours also replace the rows' witnesses, so the exported
// witness array is a complete certificate.
__global__ void k_merge_exact(const int64_t* __restrict__ rows, const double* __restrict__ d,
                              const int64_t* __restrict__ j, int64_t count, Exact* __restrict__ ex,
                              int32_t* __restrict__ nn_witness,
                              const uint32_t* __restrict__ dev_count) {
  if (dev_count) count = min<int64_t>(count, (int64_t)*dev_count);
  for (int64_t k = threadIdx.x; k < count; k += blockDim.x)
    if (j[k] >= 0) nn_witness[rows[k]] = (int32_t)j[k];
  if (threadIdx.x != 0) return;
  Exact b = *ex;
  for (int64_t k = 0; k < count; ++k) {
    if (j[k] < 0) continue;
    if (b.i < 0 || d[k] > b.d2 || (d[k] == b.d2 && rows[k] < b.i)) {
      b.d2 = d[k];
      b.i = rows[k];
      b.j = j[k];
    }
  }
  *ex = b;
}

__global__ __launch_bounds__(64) void k_sum_pairs(const uint64_t* __restrict__ slots,
                                                  uint64_t* __restrict__ total) {
  static_assert(kPairSlots <= 64, "one wavefront sums the slots");
  uint64_t v = threadIdx.x < kPairSlots ? slots[threadIdx.x * kPairStride] : 0;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (threadIdx.x == 0) *total = v;
}

}  // namespace

void launch_sum_pairs(const uint64_t* slots, uint64_t* total, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(64), 0, s, slots, total);
}

void launch_fill_many(const FillOp* ops, int count, hipStream_t s) {
  FillList L{};
  int64_t most = 0;
  for (int k = 0; k < count && k < kMaxFills; ++k) {
    L.op[L.n++] = ops[k];
    most = std::max(most, ops[k].count);
  }
  if (L.n == 0 || most <= 0) return;
  const int64_t blocks = std::min<int64_t>(4096, (most + 255) / 256);
  hipLaunchKernelGGL(k_fill_many, dim3((unsigned)blocks, (unsigned)L.n), dim3(256), 0, s, L);
}

void launch_init_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
  if (count > 0) hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
}

void launch_init_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
  if (count > 0) hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
}

void launch_unpack_best(const uint64_t* best, int64_t N, const uint32_t* alive, int gsz,
                        float* nn_approx, int32_t* nn_witness, int32_t* row_state,
                        uint32_t* n_abandoned, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_best, dim3(row_pass_blocks(N)), dim3(256), 0, s, best, N,
                     alive, gsz, nn_approx, nn_witness, row_state, n_abandoned);
}

void launch_init_alive(uint32_t* alive, int64_t G, int64_t N, int gsz, hipStream_t s) {
  if (G > 0)
    hipLaunchKernelGGL(k_init_alive, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, alive, G, N,
                       gsz);
}

void launch_seed_argmax(const uint64_t* best, const int32_t* row_state, int64_t N,
                        uint64_t* seed_key, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_argmax, dim3(row_pass_blocks(N)), dim3(256), 0, s, best,
                     row_state, N, seed_key);
}

void launch_seed_row(const uint64_t* seed_key, int64_t* rows_out, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_row, dim3(1), dim3(1), 0, s, seed_key, rows_out);
}

void launch_rows_nn_fp64(const float* Tp, int n, int64_t N, const int64_t* rows, int64_t count,
                         ZStats z, double* part_d, int64_t* part_j, double* out_d, int64_t* out_j,
                         hipStream_t s, const uint32_t* dev_count) {
  if (count <= 0) return;
  const int64_t nchunks = (N + kFp64Cols - 1) / kFp64Cols;
  if (z.sg)
    hipLaunchKernelGGL(k_rows_nn_fp64<true>, dim3((unsigned)nchunks, (unsigned)count), dim3(256), 0,
                       s, Tp, n, N, z, rows, nchunks, part_d, part_j, dev_count);
  else
    hipLaunchKernelGGL(k_rows_nn_fp64<false>, dim3((unsigned)nchunks, (unsigned)count), dim3(256), 0,
                       s, Tp, n, N, z, rows, nchunks, part_d, part_j, dev_count);
  hipLaunchKernelGGL(k_rows_nn_reduce, dim3((unsigned)count), dim3(256), 0, s, part_d, part_j,
                     nchunks, out_d, out_j, dev_count);
}

void launch_exact_from_rows(const int64_t* rows, const double* d, const int64_t* j, int64_t count,
                            Exact* ex, hipStream_t s) {
  (void)count;
  hipLaunchKernelGGL(k_exact_from_rows, dim3(1), dim3(1), 0, s, rows, d, j, ex);
}

void launch_verify(const float* Tp, int n, int64_t N, ZStats z, const int32_t* nn_witness,
                   const float* nn_approx, const Exact* ex, int64_t* uncertain,
                   uint32_t* uncertain_count, uint32_t* max_rel_err_bits, hipStream_t s) {
  if (z.sg)
    hipLaunchKernelGGL(k_verify<true>, dim3(verify_blocks(N)), dim3(256), 0, s, Tp, n, N, z,
                       nn_witness, nn_approx, ex, uncertain, uncertain_count, max_rel_err_bits);
  else
    hipLaunchKernelGGL(k_verify<false>, dim3(verify_blocks(N)), dim3(256), 0, s, Tp, n, N, z,
                       nn_witness, nn_approx, ex, uncertain, uncertain_count, max_rel_err_bits);
}

void launch_merge_exact(const int64_t* rows, const double* d, const int64_t* j, int64_t count,
                        Exact* ex, int32_t* nn_witness, hipStream_t s, const uint32_t* dev_count) {
  hipLaunchKernelGGL(k_merge_exact, dim3(1), dim3(64), 0, s, rows, d, j, count, ex, nn_witness,
                     dev_count);
}

}  // namespace dd
