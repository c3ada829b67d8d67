// scan_mfma.hip -- split-BF16 pair-distance scan on the gfx950 matrix cores.
//
// For rows a = T_{i,n} and columns b = T_{j,n} with means mu_a, mu_b and centred
// vectors a' = a - mu_a, b' = b - mu_b, the squared Euclidean distance (eq. (1))
// is exactly
//     d^2 = |a'|^2 + |b'|^2 - 2 a'.b' + n (mu_a - mu_b)^2 .
// The centred norms and means come from the FP64 preparation; the dot products
// run on v_mfma_f32_32x32x16_bf16 with each centred value split as
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and a'.b' ~ hi.hi + hi.lo + lo.hi,
// accumulated in FP32.  Centring first keeps the operands small, so the split
// products carry ~2^-16 relative error of |a'||b'|; every decision is then
// certified in FP64 (certify.hip), so these errors never reach the result.
//
// Operand roles (lane layout checked on the hardware): the MFMA's B operand is a
// block of 32 search rows (lane l <-> row l % 32, k-half l / 32) held in
// registers for the whole sweep; the A operand is a block of 32 candidate
// columns built per K-step straight from the series (the subsequence matrix is
// Hankel: column j is t[j .. j+n-1]) and pre-scaled by -2.  The 32x32 result
// then gives lane l the 16 columns 8(v/4) + 4(l/32) + v%4 of row l % 32, so the
// row minimum is mostly a per-lane running minimum.
#include "internal.hpp"

namespace dd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 32;   // rows per row block (one MFMA tile side)
constexpr int BN = 32;   // columns per column block

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

// 8 consecutive series values t[p .. p+7] (p only 4-byte aligned)
__device__ __forceinline__ void load8(const float* __restrict__ p, float (&v)[8]) {
  float4 a, b;
  __builtin_memcpy(&a, p, 16);
  __builtin_memcpy(&b, p + 4, 16);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wavefront per work item: RB row blocks of 32 rows (consecutive entries of
// the group list) against one column chunk; the column sequence is the first
// block's word bucket (32-column blocks) when given, then the chunk in matrix
// order, one 32-column block per step.
template <int KS, int RB>
__global__ __launch_bounds__(256) void k_scan_mfma(ScanJob J, MixedRows R) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;        // k-half of the operands
  const int rl = lane & 31;       // row (B) / column (A) within the block
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t items_per_chunk = (J.n_groups + RB - 1) / RB;
  if (item >= items_per_chunk * J.chunks) return;
  const int64_t li = item / J.chunks;
  const int64_t ch = item - li * J.chunks;
  const int64_t N = J.N;
  const int n = J.n;

  int64_t g[RB];
  uint32_t valid[RB], live[RB];
  bool any_live = false;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t e = li * RB + b;
    g[b] = -1;
    valid[b] = live[b] = 0;
    if (e < J.n_groups) {
      g[b] = __builtin_amdgcn_readfirstlane((int)(J.groups ? J.groups[e] : e));
      if (J.skip && J.skip[g[b]]) g[b] = -1;
    }
    if (g[b] >= 0) {
      const int64_t r0 = g[b] * BM;
      const int64_t rows = min<int64_t>(BM, N - r0);
      valid[b] = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
      live[b] = J.abandon ? (load_relaxed(&J.alive[g[b]]) & valid[b]) : valid[b];
      any_live |= live[b] != 0;
    }
  }
  if (!any_live) {
    // nothing to do; still count the finished chunk for completion tracking
    if (J.abandon && J.chunks > 1) {
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (g[b] >= 0 && lane == 0) atomicAdd(&J.done[g[b]], 1u);
    }
    return;
  }

  // ---- row operands, held for the whole sweep ---------------------------------
  bf16x8 bh[RB][KS], bl[RB][KS];
  float nA[RB], smr[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t row = (g[b] >= 0 ? g[b] * BM : 0) + rl;
    const float mu = R.mu[row];
    nA[b] = R.cnorm[row];
    smr[b] = R.smu[row];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k0 = 16 * s + 8 * h;
      float v[8];
      load8(J.Tp + row + k0, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k0 + e < n) ? v[e] - mu : 0.0f;
      split8(v, bh[b][s], bl[b][s]);
    }
  }

  // ---- column sequence ---------------------------------------------------------
  int64_t nb = 0, b0 = 0;
  if (J.words && ch == 0) {
    const int64_t gf = g[0] >= 0 ? g[0] : (RB > 1 ? g[RB - 1] : 0);
    const int w = J.words[gf * BM];
    b0 = J.bgrp_off[w];
    nb = J.bgrp_off[w + 1] - b0;
  }
  const int64_t cb = ch * J.cols_per_chunk;
  const int64_t ce = min<int64_t>(N, cb + J.cols_per_chunk);
  const int64_t q0 = cb / BN;
  const int64_t nm = ce > cb ? (ce + BN - 1) / BN - q0 : 0;
  const int64_t total_q = nb + nm;
  int64_t steps = total_q;
  bool exhausted = true;
  if (J.max_steps > 0 && steps > J.max_steps) {
    steps = J.max_steps;
    exhausted = false;
  }

  float rmin[RB];
  int32_t rj[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    rmin[b] = __builtin_inff();
    rj[b] = -1;
  }
  uint32_t cnt = 0;
  const float fn = (float)n;
  (void)fn;

  for (int64_t s = 0; s < steps; ++s) {
    bool go = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) go |= live[b] != 0;
    if (!go) break;
    const bool from_bucket = s < nb;
    const int64_t q = from_bucket ? (int64_t)J.bgrp[b0 + s] : q0 + (s - nb);
    const int64_t jlim = from_bucket ? N : ce;
    const int64_t j0 = q * BN;
    const int64_t col = j0 + rl;
    const float mu2 = 2.0f * R.mu[col];

    floatx16 acc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = 16 * ks + 8 * h;
      float v[8];
      load8(J.Tp + col + k0, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k0 + e < n) ? __builtin_fmaf(v[e], -2.0f, mu2) : 0.0f;
      bf16x8 ah, al;
      split8(v, ah, al);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[b][ks], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[b][ks], acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[b][ks], acc[b], 0, 0, 0);
      }
    }
    // ---- epilogue: squared distances of this lane's 16 columns ----------------
    float nB[16], smc[16];
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const int c0 = 8 * qd + 4 * h;
      const float4 a = *reinterpret_cast<const float4*>(R.cnorm + j0 + c0);
      const float4 m = *reinterpret_cast<const float4*>(R.smu + j0 + c0);
      nB[4 * qd + 0] = a.x; nB[4 * qd + 1] = a.y; nB[4 * qd + 2] = a.z; nB[4 * qd + 3] = a.w;
      smc[4 * qd + 0] = m.x; smc[4 * qd + 1] = m.y; smc[4 * qd + 2] = m.z; smc[4 * qd + 3] = m.w;
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (!live[b]) continue;
      const int64_t r0 = g[b] * BM;
      const int64_t i = r0 + rl;
      // tile needs the per-element mask near the exclusion band or the end
      const bool clean = (j0 + BN <= jlim) && ((j0 >= r0 + BM - 1 + n) || (j0 + BN - 1 + n <= r0));
      float d[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float t = smr[b] - smc[v];
        d[v] = acc[b][v] + __builtin_fmaf(t, t, nA[b] + nB[v]);
      }
      if (!clean) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t j = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int64_t dij = i > j ? i - j : j - i;
          if (!(j < jlim && dij >= n)) d[v] = __builtin_inff();
        }
      }
      float tmin = d[0];
#pragma unroll
      for (int v = 1; v < 16; ++v) tmin = fminf(tmin, d[v]);
      if (__ballot(tmin < rmin[b])) {
        if (tmin < rmin[b]) {
          int32_t jj = -1;
#pragma unroll
          for (int v = 15; v >= 0; --v)
            if (d[v] == tmin) jj = (int32_t)(j0 + 8 * (v >> 2) + 4 * h + (v & 3));
          rmin[b] = tmin;
          rj[b] = jj;
        }
      }
      if ((valid[b] >> rl) & 1u) {
        if (clean) {
          cnt += 16;
        } else {
#pragma unroll
          for (int v = 0; v < 16; ++v) cnt += d[v] < __builtin_inff();
        }
      }
    }
    if (J.abandon) {
      const float bsf = __builtin_bit_cast(float, load_relaxed(J.bsf));
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (!live[b]) continue;
        const float m = fminf(rmin[b], __shfl_xor(rmin[b], 32, 64));
        const uint32_t dead = (uint32_t)(__ballot(m < bsf && h == 0) & 0xFFFFFFFFull) & live[b];
        if (dead) {
          uint64_t key = rj[b] < 0 ? kEmptyMin : pack_min(rmin[b], (uint32_t)rj[b]);
          const uint64_t o = __shfl_xor(key, 32, 64);
          key = o < key ? o : key;
          if (h == 0 && ((dead >> rl) & 1u))
            atomicMin((unsigned long long*)&J.best[g[b] * BM + rl], (unsigned long long)key);
          if (lane == 0) atomicAnd(&J.alive[g[b]], ~dead);
          live[b] &= ~dead;
        }
        if (J.chunks > 1) live[b] &= load_relaxed(&J.alive[g[b]]);
      }
    }
  }

  // ---- publish ------------------------------------------------------------------
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (g[b] < 0) continue;
    uint64_t key = rj[b] < 0 ? kEmptyMin : pack_min(rmin[b], (uint32_t)rj[b]);
    const uint64_t o = __shfl_xor(key, 32, 64);
    key = o < key ? o : key;
    if (h == 0 && ((live[b] >> rl) & 1u) && key != kEmptyMin)
      atomicMin((unsigned long long*)&J.best[g[b] * BM + rl], (unsigned long long)key);
  }
  uint64_t c64 = cnt;
  for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
  if (lane == 0 && c64) atomicAdd((unsigned long long*)J.pairs, (unsigned long long)c64);
  if (!J.abandon) return;

#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (g[b] < 0) continue;
    if (J.chunks == 1) {
      if (exhausted) {
        const float m = fminf(rmin[b], __shfl_xor(rmin[b], 32, 64));
        if (h == 0 && ((live[b] >> rl) & 1u) && m < __builtin_inff())
          atomicMax(J.bsf, __builtin_bit_cast(uint32_t, m * J.raise_scale));
      } else if (live[b] && lane == 0) {
        J.survivors[atomicAdd(J.n_survivors, 1u)] = (int32_t)g[b];
      }
      continue;
    }
    __threadfence();
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&J.done[g[b]], 1u);
    prev = __shfl(prev, 0, 64);
    if (prev + 1 != (uint32_t)J.chunks) continue;
    __threadfence();
    const uint32_t fin = load_relaxed(&J.alive[g[b]]) & valid[b];
    if (h == 0 && ((fin >> rl) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[g[b] * BM + rl]);
      if (k != kEmptyMin) atomicMax(J.bsf, __builtin_bit_cast(uint32_t, key_dist(k) * J.raise_scale));
    }
  }
}

template <int KS>
void launch_ks(const ScanJob& J, const MixedRows& R, int rb, hipStream_t s) {
  const int64_t items = ((J.n_groups + rb - 1) / rb) * J.chunks;
  if (items <= 0) return;
  const int64_t blocks = (items + 3) / 4;
  if (rb == 2 && KS <= 16)
    hipLaunchKernelGGL((k_scan_mfma<KS, (KS <= 16 ? 2 : 1)>), dim3((unsigned)blocks), dim3(256), 0,
                       s, J, R);
  else
    hipLaunchKernelGGL((k_scan_mfma<KS, 1>), dim3((unsigned)blocks), dim3(256), 0, s, J, R);
}

}  // namespace

int mfma_row_blocks(int n) { return ((n + 15) / 16) <= 16 ? 2 : 1; }

bool launch_scan_mfma(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int ks = (J.n + 15) / 16;
  const int rb = mfma_row_blocks(J.n);
  switch (ks) {
#define DD_KS(K) \
  case K: launch_ks<K>(J, R, rb, s); return true;
    DD_KS(1) DD_KS(2) DD_KS(3) DD_KS(4) DD_KS(5) DD_KS(6) DD_KS(7) DD_KS(8)
    DD_KS(9) DD_KS(10) DD_KS(11) DD_KS(12) DD_KS(13) DD_KS(14) DD_KS(15) DD_KS(16)
    DD_KS(17) DD_KS(18) DD_KS(19) DD_KS(20) DD_KS(21) DD_KS(22) DD_KS(23) DD_KS(24)
    DD_KS(25) DD_KS(26) DD_KS(27) DD_KS(28) DD_KS(29) DD_KS(30) DD_KS(31) DD_KS(32)
#undef DD_KS
    default: return false;
  }
}

}  // namespace dd
