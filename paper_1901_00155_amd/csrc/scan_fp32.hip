// scan_fp32.hip -- FP32 direct-form pair-distance scan for gfx950.
//
// Computes ED^2(i, j) = sum_k (t_{i+k} - t_{j+k})^2 (eq. (1) squared, the form the
// paper's PotentialDiscord/RefineDiscord loops evaluate) for blocks of rows and
// columns, keeps each row's minimum over non-self columns (|i - j| >= n) and the
// column attaining it.
//
// Layout of the work: one wavefront owns a group of 8 consecutive rows
// (i0..i0+7); each of its 64 lanes owns TN consecutive columns (j0..j0+TN-1)
// per step, so a wave covers 8 x 64 TN pairs per step: TN = 8 (512-column
// steps) in full scans and the PhiDD and matrix orders, TN = 4 (256-column
// steps) in near-first early-abandon searches, whose rows can leave only at
// the end of a step.  The subsequences are read straight from the series
// (Hankel structure: row i is t[i..i+n-1]), so no subsequence matrix is
// streamed; the row window is wave-uniform.
//
// Arithmetic reuse: the difference t_{i+k} - t_{j+k} depends only on the
// diagonal g = j - i and the position p = i + k, so inside an 8 x TN block the
// 8 TN pairs at position p need only the 7 + TN differences D_g(p).  Each
// pair's sum is still the plain sequential sum over k = 0..n-1 of its own
// squared differences (one fused multiply-add per term), so the arithmetic per
// pair is exactly the direct form; only the subtractions are shared.  Cost per
// (pair, k) term: 64 FMA + 15 SUB per 64 (about 1.23 VALU ops) at TN = 8,
// 32 FMA + 11 SUB per 32 (about 1.34) at TN = 4.
#include "internal.hpp"

namespace dd {
namespace {

constexpr int TM = kRowGroup;   // 8 rows per wave
// TN columns per lane: kColBlock (8), or kColBlockSearch (4) in early-abandon
// searches in the near-first order, whose rows can leave only at the end of a
// step of 64 lanes x TN columns (most rows there leave within their first 256
// columns, so 512-column steps did twice the work needed)
static_assert(TM == 8 && kColBlock == 8 && kColBlockSearch == 4,
              "the micro-tiles below are written for 8 x 8 and 8 x 4");

// One position p: all 64 pairs of the block that are active at p take
// acc += D^2 with D = x[p] - y[p + (c - r)].  yw[g + 7] = y[p + g].
// PRED: apply the activity test 0 <= p - r < n (first and last 7 positions).
template <bool PRED, int TN>
__device__ __forceinline__ void step(float (&acc)[TM][TN], float xp, const float* yw, int p,
                                     int n) {
  float D[TM + TN - 1];
#pragma unroll
  for (int g = 0; g < TM + TN - 1; ++g) D[g] = xp - yw[g];
#pragma unroll
  for (int r = 0; r < TM; ++r) {
    bool on = true;
    if (PRED) {
      const int k = p - r;
      on = (k >= 0) && (k < n);
    }
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      float d = D[c - r + TM - 1];
      if (PRED) d = on ? d : 0.0f;
      acc[r][c] = __builtin_fmaf(d, d, acc[r][c]);
    }
  }
}

// y loads for positions [p0, p0+8): y[p0-8 .. p0+TN+7] (TN + 16 floats, 16-byte
// aligned when y and p0 are multiples of 4 floats).
template <int TN>
__device__ __forceinline__ void load_y(const float* __restrict__ y, int p0, float (&yb)[TN + 16]) {
  const float4* v = reinterpret_cast<const float4*>(y + p0 - 8);
#pragma unroll
  for (int q = 0; q < (TN + 16) / 4; ++q) {
    const float4 f = v[q];
    yb[4 * q + 0] = f.x;
    yb[4 * q + 1] = f.y;
    yb[4 * q + 2] = f.z;
    yb[4 * q + 3] = f.w;
  }
}

__device__ __forceinline__ void load_x(const float* __restrict__ x, int p0, float (&xb)[8]) {
  const float4* v = reinterpret_cast<const float4*>(x + p0);
  const float4 a = v[0], b = v[1];
  xb[0] = a.x; xb[1] = a.y; xb[2] = a.z; xb[3] = a.w;
  xb[4] = b.x; xb[5] = b.y; xb[6] = b.z; xb[7] = b.w;
}

template <bool PRED, int TN>
__device__ __forceinline__ void steps8(float (&acc)[TM][TN], const float* __restrict__ x,
                                       const float* __restrict__ y, int p0, int n) {
  float xb[8], yb[TN + 16];
  load_x(x, p0, xb);
  load_y<TN>(y, p0, yb);
#pragma unroll
  for (int u = 0; u < 8; ++u) step<PRED, TN>(acc, xb[u], &yb[u + 1], p0 + u, n);
}

// acc[r][c] = sum_{k<n} (x[r+k] - y[c+k])^2 for the 8 x TN block at x, y.
template <int TN>
__device__ __forceinline__ void block_tile(const float* __restrict__ x, const float* __restrict__ y,
                                         int n, float (&acc)[TM][TN]) {
#pragma unroll
  for (int r = 0; r < TM; ++r)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[r][c] = 0.0f;
  steps8<true, TN>(acc, x, y, 0, n);            // positions 0..7: rows r > p not started
  int p0 = 8;
  for (; p0 + 8 <= n; p0 += 8) steps8<false, TN>(acc, x, y, p0, n);   // every row active
  for (; p0 < n + TM - 1; p0 += 8) steps8<true, TN>(acc, x, y, p0, n);  // rows finishing
}

// Per-window normalisation.  With x_{i,k} = (t_{i+k} - mu_i) / sigma_i, the
// squared distance of two normalised windows is
//     d^2 = q_i + q_j - 2 C_ij s_i s_j,   C_ij = sum_k (t_{i+k} - c_i)(t_{j+k} - c_j),
// with s = 1 / sigma and q = n (s = q = 0 for a flat window, whose normalised
// form is the zero vector); c = fp32(mu) differs from mu by less than an ulp,
// which changes C by n (mu_i - c_i)(mu_j - c_j), far below its rounding error.
// The centred products no longer share differences along diagonals, so the
// block runs over k: per position 8 row and 8 column centrings and 64 FMAs,
// 1.25 VALU ops per (pair, k) term.
__device__ __forceinline__ void load16(const float* __restrict__ p, float (&v)[16]) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const float4 f = q[h];
    v[4 * h + 0] = f.x;
    v[4 * h + 1] = f.y;
    v[4 * h + 2] = f.z;
    v[4 * h + 3] = f.w;
  }
}

// positions k0 .. k0 + kn - 1 (kn <= 8, wave-uniform)
template <bool TAIL, int TN>
__device__ __forceinline__ void zsteps8(float (&acc)[TM][TN], const float* __restrict__ x,
                                        const float* __restrict__ y, int k0, int kn,
                                        const float (&cx)[TM], const float (&cy)[TN]) {
  float xb[16], yb[16];
  load16(x + k0, xb);
  load16(y + k0, yb);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (TAIL && u >= kn) break;
    float xr[TM], yc[TN];
#pragma unroll
    for (int r = 0; r < TM; ++r) xr[r] = xb[u + r] - cx[r];
#pragma unroll
    for (int c = 0; c < TN; ++c) yc[c] = yb[u + c] - cy[c];
#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
      for (int c = 0; c < TN; ++c) acc[r][c] = __builtin_fmaf(xr[r], yc[c], acc[r][c]);
  }
}

// acc[r][c] = approximate d^2 between normalised rows x + r and columns y + c.
// x, y: TN-float aligned windows of the padded series; zx, zy: the same rows'
// and columns' entries of the centre (zc) and scale (zr) arrays.
template <int TN>
__device__ __forceinline__ void block_tile_z(const float* __restrict__ x, const float* __restrict__ y,
                                           int n, const float* __restrict__ zcx,
                                           const float* __restrict__ zrx,
                                           const float* __restrict__ zcy,
                                           const float* __restrict__ zry, float (&acc)[TM][TN]) {
  float cx[TM], sx[TM], cy[TN], sy[TN];
#pragma unroll
  for (int r = 0; r < TM; ++r) {
    cx[r] = zcx[r];
    sx[r] = zrx[r];
  }
  {
    const float4* pc = reinterpret_cast<const float4*>(zcy);
    const float4* ps = reinterpret_cast<const float4*>(zry);
#pragma unroll
    for (int h = 0; h < TN / 4; ++h) {
      const float4 c4 = pc[h], s4 = ps[h];
      cy[4 * h + 0] = c4.x; cy[4 * h + 1] = c4.y; cy[4 * h + 2] = c4.z; cy[4 * h + 3] = c4.w;
      sy[4 * h + 0] = s4.x; sy[4 * h + 1] = s4.y; sy[4 * h + 2] = s4.z; sy[4 * h + 3] = s4.w;
    }
  }
#pragma unroll
  for (int r = 0; r < TM; ++r)
#pragma unroll
    for (int c = 0; c < TN; ++c) acc[r][c] = 0.0f;
  int k0 = 0;
  for (; k0 + 8 <= n; k0 += 8) zsteps8<false, TN>(acc, x, y, k0, 8, cx, cy);
  if (k0 < n) zsteps8<true, TN>(acc, x, y, k0, n - k0, cx, cy);
  const float fn = (float)n;
#pragma unroll
  for (int r = 0; r < TM; ++r) {
    const float qx = sx[r] > 0.0f ? fn : 0.0f;
    const float m2s = -2.0f * sx[r];
#pragma unroll
    for (int c = 0; c < TN; ++c) {
      const float qy = sy[c] > 0.0f ? fn : 0.0f;
      acc[r][c] = fmaxf(__builtin_fmaf(m2s * sy[c], acc[r][c], qx + qy), 0.0f);
    }
  }
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ float wave_min_f32(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wavefront per work item (row group, chunk of its column sequence).  The
// sequence is the bucket of the group's word (Index_Word, eq. (10)), when given,
// followed by all column groups in matrix order or near-first (spiral.hpp);
// each step covers 64 column groups of 8.  With abandon on, after every step
// each live row compares its running minimum with the device best-so-far and
// leaves as soon as it is below (Algorithms 3-4); the leaving row keeps that
// column as its witness.
template <bool Z, int TN>
__device__ __forceinline__ void scan_item(const ScanJob& J, int64_t item, int lane) {
  const int64_t li = item / J.chunks;
  const int64_t ch = item - li * J.chunks;
  const int64_t g = __builtin_amdgcn_readfirstlane((int)(J.groups ? J.groups[li] : li));
  if (J.skip && J.skip[g]) return;
  const int64_t N = J.N;
  const int n = J.n;
  const int64_t i0 = g * TM;
  uint32_t valid = 0;
#pragma unroll
  for (int r = 0; r < TM; ++r) valid |= (i0 + r < N ? 1u : 0u) << r;
  uint32_t live = J.abandon ? (load_relaxed(&J.alive[g]) & valid) : valid;
  if (J.abandon && J.precheck && live) {
    // a row whose minimum over the columns of earlier launches is already below
    // the best-so-far cannot be the discord: it leaves with that witness
    const float b = __builtin_bit_cast(float, load_relaxed(J.bsf));
    bool below = false;
    if (lane < TM && ((live >> lane) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[i0 + lane]);
      below = k != kEmptyMin && key_dist(k) < b;
    }
    const uint32_t dead = (uint32_t)(__ballot(below) & 0xFFull);
    if (dead) {
      if (lane == 0) atomicAnd(&J.alive[g], ~dead);
      live &= ~dead;
    }
  }

  // column sequence: this chunk's entries of bucket ++ order
  int64_t nb = 0, b0 = 0;
  if (J.words) {
    const int w = J.words[i0];
    b0 = J.bgrp_off[w];
    nb = J.bgrp_off[w + 1] - b0;
  }
  const int64_t NQ = (N + TN - 1) / TN;
  const Spiral sp = make_spiral(i0, i0 + TM, n, NQ, TN);
  const int64_t len = nb + (J.near_first ? spiral_count(sp) : NQ);
  const int64_t e0 = J.seq_begin + ch * J.seq_chunk;
  const int64_t e1 = min<int64_t>(len, e0 + J.seq_chunk);
  const int64_t total = e1 > e0 ? e1 - e0 : 0;
  const bool final = J.seq_begin + J.chunks * J.seq_chunk >= len;
  const int64_t steps = live ? (total + 63) / 64 : 0;
  const float* x = J.Tp + i0;

  float bd[TM];
  int32_t bj[TM];
#pragma unroll
  for (int r = 0; r < TM; ++r) {
    bd[r] = __builtin_inff();
    bj[r] = -1;
  }
  uint32_t cnt = 0;
  for (int64_t s = 0; s < steps && live; ++s) {
    const int64_t e = e0 + s * 64 + lane;
    const bool in_seq = e < e1;
    const int64_t q = !in_seq ? 0
                      : e < nb ? (int64_t)J.bgrp[b0 + e]
                      : J.near_first ? spiral_block(sp, e - nb) : e - nb;
    const int32_t j0 = (int32_t)(q * TN);   // N < 2^31 (checked at prepare)
    float acc[TM][TN];
    if constexpr (Z)
      block_tile_z<TN>(x, J.Tp + j0, n, J.zc + i0, J.zr + i0, J.zc + j0, J.zr + j0, acc);
    else
      block_tile<TN>(x, J.Tp + j0, n, acc);
    // blocks inside the matrix and clear of the exclusion band need no mask:
    // each row's minimum over the 8 columns first, its column only on improvement
    const bool clean = in_seq && valid == 0xFFu && j0 + TN <= N &&
                       (j0 >= (int32_t)i0 + TM - 1 + n || j0 + TN - 1 + n <= (int32_t)i0);
    if (clean) {
      cnt += TM * TN;
#pragma unroll
      for (int r = 0; r < TM; ++r) {
        float m = acc[r][0];
#pragma unroll
        for (int c = 1; c < TN; ++c) m = fminf(m, acc[r][c]);
        if (m < bd[r]) {
          int32_t jj = j0;
#pragma unroll
          for (int c = TN - 1; c >= 0; --c)
            if (acc[r][c] == m) jj = j0 + c;
          bd[r] = m;
          bj[r] = jj;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < TM; ++r) {
        const int32_t i = (int32_t)i0 + r;
#pragma unroll
        for (int c = 0; c < TN; ++c) {
          const int32_t j = j0 + c;
          const int32_t dij = i > j ? i - j : j - i;
          const bool ok = in_seq && (j < N) && (dij >= n) && ((valid >> r) & 1u);
          cnt += ok;
          if (ok && acc[r][c] < bd[r]) {
            bd[r] = acc[r][c];
            bj[r] = j;
          }
        }
      }
    }
    if (J.abandon) {
      const float b = __builtin_bit_cast(float, load_relaxed(J.bsf));
      uint32_t dead = 0;
#pragma unroll
      for (int r = 0; r < TM; ++r)
        if ((live >> r) & 1u) dead |= (wave_min_f32(bd[r]) < b ? 1u : 0u) << r;
      if (dead) {
#pragma unroll
        for (int r = 0; r < TM; ++r) {
          if ((dead >> r) & 1u) {
            const uint64_t key = wave_min_u64(bj[r] < 0 ? kEmptyMin : pack_min(bd[r], (uint32_t)bj[r]));
            if (lane == 0) atomicMin((unsigned long long*)&J.best[i0 + r], (unsigned long long)key);
          }
        }
        if (lane == 0) atomicAnd(&J.alive[g], ~dead);
        live &= ~dead;
      }
      if (J.chunks > 1) live &= load_relaxed(&J.alive[g]);
    }
  }
  // rows still live: publish their minimum over this item's columns
#pragma unroll
  for (int r = 0; r < TM; ++r) {
    if ((live >> r) & 1u) {
      const uint64_t key = wave_min_u64(bj[r] < 0 ? kEmptyMin : pack_min(bd[r], (uint32_t)bj[r]));
      if (lane == 0 && key != kEmptyMin)
        atomicMin((unsigned long long*)&J.best[i0 + r], (unsigned long long)key);
    }
  }
  uint64_t c64 = cnt;
  for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
  if (lane == 0 && c64) atomicAdd(pair_slot(J.pairs), (unsigned long long)c64);
  if (!J.abandon) return;

  // the item's last chunk to finish decides: complete rows raise the best-so-far
  // with their minimum over the whole sequence (all launches), rows still live
  // after a non-final launch make the group a survivor
  uint32_t fin = live;
  if (J.chunks > 1) {
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&J.done[g], 1u);
    prev = __shfl(prev, 0, 64);
    if (prev + 1 != (uint32_t)J.chunks) return;
    if (lane == 0) atomicExch(&J.done[g], 0u);   // ready for the next launch
    __threadfence();
    fin = load_relaxed(&J.alive[g]) & valid;
  }
  if (!fin) return;
  if (final) {
    if (lane < TM && ((fin >> lane) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[i0 + lane]);
      if (k != kEmptyMin)
        atomicMax(J.bsf, __builtin_bit_cast(uint32_t, fmaxf(key_dist(k) * J.raise_scale - J.raise_sub, 0.0f)));
    }
  } else if (lane == 0) {
    J.survivors[atomicAdd(J.n_survivors, 1u)] = (int32_t)g;
  }
}

// Each wavefront takes work items (item, chunk) blockIdx.x * 4 + wave, then
// strides by the grid's wavefront count: a grid sized for the work gives every
// work item its own wavefront, a smaller one (the device-decided launches,
// sized for the most work they can hold) takes several per wavefront.
template <bool Z, int TN>
__global__ __launch_bounds__(256) void k_scan_fp32(ScanJob Jarg) {
  ScanJob J = Jarg;
  apply_win(J);
  const int lane = threadIdx.x & 63;
  const int64_t total = J.n_groups * J.chunks;
  for (int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); item < total;
       item += (int64_t)gridDim.x * 4)
    scan_item<Z, TN>(J, item, lane);
}

}  // namespace

void launch_scan_fp32(const ScanJob& J, hipStream_t s) {
  const int64_t items = J.win ? J.max_work : J.n_groups * J.chunks;
  if (items <= 0) return;
  const int64_t blocks = (items + 3) / 4;
  // the column width must match the one the host split the sequences with
  // (kColBlockSearch with early abandon in the near-first order, else
  // kColBlock)
  const bool fine = J.abandon && J.near_first;
  if (J.zc) {
    if (fine)
      hipLaunchKernelGGL((k_scan_fp32<true, kColBlockSearch>), dim3((unsigned)blocks), dim3(256),
                         0, s, J);
    else
      hipLaunchKernelGGL((k_scan_fp32<true, kColBlock>), dim3((unsigned)blocks), dim3(256), 0, s,
                         J);
  } else {
    if (fine)
      hipLaunchKernelGGL((k_scan_fp32<false, kColBlockSearch>), dim3((unsigned)blocks), dim3(256),
                         0, s, J);
    else
      hipLaunchKernelGGL((k_scan_fp32<false, kColBlock>), dim3((unsigned)blocks), dim3(256), 0,
                         s, J);
  }
}

}  // namespace dd
