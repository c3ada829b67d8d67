// scan_mfma.hip -- split-BF16 pair-distance scan on the gfx950 matrix cores.
//
// For rows a = T_{i,n} and columns b = T_{j,n} with centres c_a, c_b (the FP32
// rounding of the window means mu_a, mu_b) the squared Euclidean distance of
// eq. (1) is, up to a term below n ulp(mu)^2,
//     d^2 = |a - c_a|^2 + |b - c_b|^2 - 2 (a - c_a).(b - c_b) + n (mu_a - mu_b)^2 .
// Under per-window normalisation the operands are the centred windows scaled by
// fp32(1 / sigma) and the last term is zero (normalised windows have mean 0);
// the kernels are the same, only the prepared operands and statistics differ.
// The dot products run on v_mfma_f32_32x32x16_bf16 with each centred value
// split as x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and
// a'.b' ~ hi.hi + hi.lo + lo.hi, accumulated in FP32.  Centring first keeps
// the operands small, so the split products carry ~2^-16 relative error of
// |a'||b'|; every decision is then certified in FP64 (certify.hip), so these
// errors never reach the result.
//
// The split subsequence matrix (the paper's S of eq. (5), centred and split)
// is built once by the preparation stage and stays resident in HBM, laid out
// per block of 32 rows exactly as the MFMA operand registers want it: lane l
// holds row l % 32, elements k = 16 s + 8 (l / 32) + 0..7 of K-step s.  Since
// the A and B operands share this lane layout, the same array feeds both.  One
// extra K-step per block carries the norms: as an A operand
// (P_hi, P_mid, P_lo, 1, 1, 1) with P = -|b'|^2 / 2 of the column, as a B operand
// (1, 1, 1, Q_hi, Q_mid, Q_lo) with Q = -|a'|^2 / 2 of the row (three-way bf16
// splits hold P and Q to 2^-24).  The row operands are scaled by -2 once when
// they are loaded (exact in bf16), so the accumulator ends at
// |a'|^2 + |b'|^2 - 2 a'.b' and d^2 = acc + (sqrt(n) (mu_a - mu_b))^2: two
// VALU operations per pair.
//
// Operand roles (lane layout checked on the hardware): B = a block of 32 search
// rows held in registers for the whole sweep; A = a block of 32 candidate
// columns.  The 32x32 result gives lane l the 16 columns 8(v/4) + 4(l/32) + v%4
// of row l % 32, so the row minimum is mostly a per-lane running minimum.
//
// Work sharing: a workgroup of 4 wavefronts (8 for full scans with windows of
// 129..256; see waves_for) owns two row blocks per wavefront in full scans with
// windows up to 128, else one, and sweeps a column sequence together.  Each column block is
// copied once per workgroup from HBM straight into LDS (double-buffered: the
// copy of block s+1 is issued before block s is multiplied), and every
// wavefront reads it with ds_read_b128.
#include <type_traits>

#include "internal.hpp"

namespace dd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 32;      // rows per row block (one MFMA tile side)
constexpr int BN = 32;      // columns per column block
// Work-group shapes (measured on full scans and searches).  Row blocks per
// wavefront in full scans: two while both fit in the registers of a
// two-waves-per-SIMD kernel (windows up to 128), else one; searches take one.  Wavefronts per workgroup: 4, and two
// workgroups share a CU while a wavefront fits in half the register file, so
// their steps drift apart and one's epilogue overlaps the other's MFMAs; one
// wavefront per SIMD beyond that.  The exception is a full scan with windows of
// 129..256 (one row block per wavefront): there 8 wavefronts sharing each column
// block in LDS do better (0.50 vs 0.46 of peak), while an early-abandon search
// prefers the finer 4-wavefront items (they leave sooner).
template <int KS>
constexpr int kRowBlocks = KS <= 8 ? 2 : 1;
template <int KS>
constexpr int waves_for(bool abandon) { return (KS > 8 && KS <= 16 && !abandon) ? 8 : 4; }

template <int KS>
struct Blk {
  static constexpr int SLOTS = (KS + 1) * 128;                 // 16-byte slots per block
};

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

__device__ __forceinline__ void split3(float x, __bf16& a, __bf16& b, __bf16& c) {
  a = (__bf16)x;
  const float r1 = x - (float)a;
  b = (__bf16)r1;
  c = (__bf16)(r1 - (float)b);
}

// 8 consecutive series values t[p .. p+7] (p only 4-byte aligned)
__device__ __forceinline__ void load8(const float* __restrict__ p, float (&v)[8]) {
  float4 a, b;
  __builtin_memcpy(&a, p, 16);
  __builtin_memcpy(&b, p + 4, 16);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Preparation: one thread per (block, K-step slot, lane).  KS is a template
// argument for windows up to 512 and a run-time value beyond (the body is the
// same; the constant only makes the index arithmetic cheaper).
__device__ __forceinline__ void split_blocks_body(int KS, const float* __restrict__ Tp,
                                                  int64_t nblk, int n,
                                                  const float* __restrict__ c32,
                                                  const float* __restrict__ cn32,
                                                  const float* __restrict__ r32,
                                                  bf16x8* __restrict__ out) {
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  const int64_t per_blk = (int64_t)(KS + 1) * 64;
  if (t >= nblk * per_blk) return;
  const int64_t q = t / per_blk;
  const int r = (int)(t - q * per_blk);
  const int s = r >> 6, l = r & 63;
  const int64_t row = q * BM + (l & 31);
  const int h = l >> 5;
  bf16x8* blk = out + q * ((int64_t)(KS + 1) * 128);
  if (s < KS) {
    const int k0 = 16 * s + 8 * h;
    const float c = c32[row];
    // per-window normalisation scales the centred window (1 otherwise: exact)
    const float r = r32 ? r32[row] : 1.0f;
    float v[8];
    load8(Tp + row + k0, v);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (k0 + e < n) ? (v[e] - c) * r : 0.0f;
    bf16x8 hi, lo;
    split8(v, hi, lo);
    blk[s * 128 + l] = hi;
    blk[s * 128 + 64 + l] = lo;
  } else {
    const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
    bf16x8 xa, xb;
#pragma unroll
    for (int e = 0; e < 8; ++e) xa[e] = xb[e] = zero;
    if (h == 0) {
      const float P = -0.5f * cn32[row];
      __bf16 p0, p1, p2;
      split3(P, p0, p1, p2);
      xa[0] = p0; xa[1] = p1; xa[2] = p2; xa[3] = one; xa[4] = one; xa[5] = one;
      xb[0] = one; xb[1] = one; xb[2] = one; xb[3] = p0; xb[4] = p1; xb[5] = p2;
    }
    blk[KS * 128 + l] = xa;        // extra step as an A (column) operand
    blk[KS * 128 + 64 + l] = xb;   // extra step as a B (row) operand
  }
}

template <int KS>
__global__ __launch_bounds__(256) void k_split_blocks(const float* __restrict__ Tp, int64_t nblk,
                                                      int n, const float* __restrict__ c32,
                                                      const float* __restrict__ cn32,
                                                      const float* __restrict__ r32,
                                                      bf16x8* __restrict__ out) {
  split_blocks_body(KS, Tp, nblk, n, c32, cn32, r32, out);
}

// One workgroup per (item, chunk of its column sequence).  An item is a fixed
// set of WAVES * RB consecutive row blocks (the list holds item numbers), so
// its sequence is the same in every launch and a search can resume it: the
// word bucket (32-column blocks) of its first row, when given, then the column
// blocks in matrix order or near-first (spiral.hpp) around the item's rows,
// one 32-column block per step.
template <int KS, int RB, int WAVES>
__device__ __forceinline__ void scan_item(const ScanJob& J, const MixedRows& R, int64_t wi) {
  // two stages, each a column block (Blk<KS>::SLOTS slots) followed by the
  // block's 32 column values sqrt(n) (mean - mu) (8 slots)
  extern __shared__ bf16x8 smem[];
  __shared__ uint32_t wave_live[2 * WAVES];
  constexpr int SLOTS = Blk<KS>::SLOTS;
  constexpr int PER_T = (SLOTS + WAVES * 64 - 1) / (WAVES * 64);
  constexpr int STAGE = SLOTS + 8;
  // index arithmetic of the epilogue: 32-bit, except for the 8-wavefront kernel
  // (windows of 129..256), where the 64-bit form measured 3-4% faster (the
  // register allocation differs; both are exact since N < 2^31)
  using idx_t = std::conditional_t<(WAVES == 8), int64_t, int32_t>;
  const bf16x8* __restrict__ S = reinterpret_cast<const bf16x8*>(R.sblk);

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int rl = lane & 31;
  const int64_t per_item = WAVES * RB;
  const int64_t li = wi / J.chunks;
  const int64_t ch = wi - li * J.chunks;
  if (li >= J.n_groups) return;
  const int64_t N = J.N;
  const int n = J.n;
  // the item: row blocks item * per_item .. + per_item - 1, always the same set
  const int64_t item = __builtin_amdgcn_readfirstlane((int)(J.groups ? J.groups[li] : li));
  if (J.skip && J.skip[item]) return;

  int64_t g[RB];
  uint32_t valid[RB], live[RB];
  bool any_live = false;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    g[b] = item * per_item + wv * RB + b;
    valid[b] = live[b] = 0;
    if (g[b] * BM >= N) g[b] = -1;
    if (g[b] >= 0) {
      const int64_t r0 = g[b] * BM;
      const int64_t rows = min<int64_t>(BM, N - r0);
      valid[b] = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
      live[b] = J.abandon ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g[b]]) & valid[b])
                          : valid[b];
      if (J.abandon && J.precheck && live[b]) {
        // rows whose minimum over the columns of earlier launches is already
        // below the best-so-far cannot be the discord: they leave with that witness
        const float bs = __builtin_bit_cast(float, load_relaxed(J.bsf));
        bool below = false;
        if (h == 0 && ((live[b] >> rl) & 1u)) {
          const uint64_t k = load_relaxed64(&J.best[g[b] * BM + rl]);
          below = k != kEmptyMin && key_dist(k) < bs;
        }
        const uint32_t dead = (uint32_t)(__ballot(below) & 0xFFFFFFFFull);
        if (dead) {
          if (lane == 0) atomicAnd(&J.alive[g[b]], ~dead);
          live[b] &= ~dead;
        }
      }
      any_live |= live[b] != 0;
    }
  }

  // ---- row operands, held for the whole sweep ---------------------------------
  // Scaled by -2 (exact in bf16), so the accumulator ends at
  // -2 a'.b' + |a'|^2 + |b'|^2 = d^2 - n (mu_a - mu_b)^2.
  bf16x8 bh[RB][KS], bl[RB][KS], bx[RB];
  float smr[RB];
  const __bf16 m2 = (__bf16)(-2.0f);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t gb = g[b] >= 0 ? g[b] : 0;
    const bf16x8* blk = S + gb * SLOTS;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bh[b][s] = blk[s * 128 + lane] * m2;
      bl[b][s] = blk[s * 128 + 64 + lane] * m2;
    }
    bx[b] = blk[KS * 128 + 64 + lane] * m2;
    smr[b] = R.smu[gb * BM + rl];
  }

  // ---- column sequence (uniform over the workgroup) ---------------------------
  int64_t nb = 0, b0 = 0;
  const int64_t r_first = item * per_item * BM;
  if (J.words) {
    const int w = J.words[r_first];
    b0 = J.bgrp_off[w];
    nb = J.bgrp_off[w + 1] - b0;
  }
  const int64_t NQ = (N + BN - 1) / BN;
  Spiral sp{0, -1, NQ, 0};
  if (J.near_first) sp = make_spiral(r_first, r_first + per_item * BM, n, NQ, BN);
  const int64_t len = nb + spiral_count(sp);   // spiral_count = NQ in matrix order
  const int64_t e0 = J.seq_begin + ch * J.seq_chunk;
  const int64_t e1 = min<int64_t>(len, e0 + J.seq_chunk);
  int64_t steps = e1 > e0 ? e1 - e0 : 0;
  const bool final = J.seq_begin + J.chunks * J.seq_chunk >= len;
  auto block_of = [&](int64_t s) -> int64_t {
    const int64_t e = e0 + s;
    return e < nb ? (int64_t)__builtin_amdgcn_readfirstlane(J.bgrp[b0 + e])
                  : spiral_block(sp, e - nb);
  };

  // workgroup-wide: is any row of any wavefront still live?
  if (lane == 0) wave_live[wv] = any_live ? 1u : 0u;
  __syncthreads();
  bool wg_live = false;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) wg_live |= wave_live[w] != 0;
  if (!wg_live) steps = 0;

  float rmin[RB];
  int32_t rj[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    rmin[b] = __builtin_inff();
    rj[b] = -1;
  }
  uint32_t cnt = 0;

  // column blocks go from HBM straight into LDS (global_load_lds_dwordx4: each
  // lane's 16 bytes land at its wavefront's LDS base + 16 * lane), with no
  // register staging; the barrier that closes a step waits for them
  typedef __attribute__((address_space(3))) void lds_void;
  auto fetch = [&](int64_t q, bf16x8* dst) {
    const bf16x8* src = S + q * SLOTS;
#pragma unroll
    for (int i = 0; i < PER_T; ++i) {
      const int w0 = i * WAVES * 64 + wv * 64;   // this wavefront's first slot
      if (w0 < SLOTS)                             // SLOTS is a multiple of 64
        __builtin_amdgcn_global_load_lds(src + w0 + lane, (lds_void*)(dst + w0), 16, 0, 0);
    }
    if (wv == 0 && lane < 8)
      __builtin_amdgcn_global_load_lds(R.smu + q * BN + 4 * lane, (lds_void*)(dst + SLOTS), 16, 0,
                                       0);
  };
  int64_t q_next = steps > 0 ? block_of(0) : 0;   // block of the step about to run
  if (steps > 0) fetch(q_next, smem);
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    const int cur = (int)(s & 1);
    const int64_t q_cur = q_next;
    if (s + 1 < steps) {
      q_next = block_of(s + 1);
      fetch(q_next, smem + (cur ^ 1) * STAGE);
    }
    const idx_t jlim = (idx_t)N;                  // N < 2^31 (checked at prepare)
    const idx_t j0 = (idx_t)(q_cur * BN);
    const bf16x8* buf = smem + cur * STAGE;

    bool go = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) go |= live[b] != 0;
    if (go) {
      // one accumulation chain per row block (a second, interleaved chain
      // measured no faster: dependent MFMAs issue back to back)
      floatx16 acc[RB];
      {
        const bf16x8 ax = buf[KS * 128 + lane];
        floatx16 z;
#pragma unroll
        for (int v = 0; v < 16; ++v) z[v] = 0.0f;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax, bx[b], z, 0, 0, 0);
      }
      // two wavefronts share each SIMD: the one issuing its MFMA chain goes first
      // (measured: +5% at n = 256, neutral at n = 128, a loss with one
      // wavefront per SIMD)
      if constexpr (KS <= 16) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 ah = buf[ks * 128 + lane];
        const bf16x8 al = buf[ks * 128 + 64 + lane];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[b][ks], acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[b][ks], acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[b][ks], acc[b], 0, 0, 0);
        }
      }
      if constexpr (KS <= 16) __builtin_amdgcn_s_setprio(0);
      // ---- epilogue: d^2 = acc + (smu_row - smu_col)^2 for the 16 columns -----
      float smc[16];
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        const float4 m = reinterpret_cast<const float4*>(buf + SLOTS)[2 * qd + h];
        smc[4 * qd + 0] = m.x; smc[4 * qd + 1] = m.y; smc[4 * qd + 2] = m.z; smc[4 * qd + 3] = m.w;
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (!live[b]) continue;
        const idx_t r0 = (idx_t)(g[b] * BM);
        const idx_t i = r0 + rl;
        // the per-element mask is needed only near the exclusion band or the end
        const bool clean =
            (j0 + BN <= jlim) && ((j0 >= r0 + BM - 1 + n) || (j0 + BN - 1 + n <= r0));
        float d[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float t = smr[b] - smc[v];
          d[v] = __builtin_fmaf(t, t, acc[b][v]);
        }
        if (!clean) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const idx_t j = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
            const idx_t dij = i > j ? i - j : j - i;
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
          const uint32_t dead =
              (uint32_t)(__ballot(m < bsf && h == 0) & 0xFFFFFFFFull) & live[b];
          if (dead) {
            uint64_t key = rj[b] < 0 ? kEmptyMin : pack_min(fmaxf(rmin[b], 0.0f), (uint32_t)rj[b]);
            const uint64_t o = __shfl_xor(key, 32, 64);
            key = o < key ? o : key;
            if (h == 0 && ((dead >> rl) & 1u))
              atomicMin((unsigned long long*)&J.best[g[b] * BM + rl], (unsigned long long)key);
            if (lane == 0) atomicAnd(&J.alive[g[b]], ~dead);
            live[b] &= ~dead;
          }
          if (J.chunks > 1)
            live[b] &= __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g[b]]));
        }
      }
    }
    // all wavefronts agree on leaving once no row of the workgroup is live
    bool mine = false;
#pragma unroll
    for (int b = 0; b < RB; ++b) mine |= live[b] != 0;
    // (flags alternate between two rows, so one barrier per step suffices: a
    // wavefront rewrites a row only after every wavefront has read it)
    uint32_t* flags = wave_live + ((s + 1) & 1) * WAVES;
    if (lane == 0) flags[wv] = mine ? 1u : 0u;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) any |= flags[w] != 0;
    if (!any) break;
  }

  // ---- publish ------------------------------------------------------------------
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (g[b] < 0) continue;
    // (the split products can round a near-zero distance below zero; keys hold
    // non-negative distances so that they order like the values)
    uint64_t key = rj[b] < 0 ? kEmptyMin : pack_min(fmaxf(rmin[b], 0.0f), (uint32_t)rj[b]);
    const uint64_t o = __shfl_xor(key, 32, 64);
    key = o < key ? o : key;
    if (h == 0 && ((live[b] >> rl) & 1u) && key != kEmptyMin)
      atomicMin((unsigned long long*)&J.best[g[b] * BM + rl], (unsigned long long)key);
  }
  uint64_t c64 = cnt;
  for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
  if (lane == 0 && c64) atomicAdd(pair_slot(J.pairs), (unsigned long long)c64);
  if (!J.abandon) return;

  // the item's last chunk to finish decides: complete rows raise the
  // best-so-far with their minimum over all launches; rows still live after a
  // non-final launch make the item a survivor
  __shared__ uint32_t tail[WAVES + 1];
  if (J.chunks > 1) {
    __threadfence();
    __syncthreads();                              // every wavefront has published
    if (threadIdx.x == 0) {
      const uint32_t prev = atomicAdd(&J.done[item], 1u);
      const bool last = prev + 1 == (uint32_t)J.chunks;
      if (last) atomicExch(&J.done[item], 0u);   // ready for the next launch
      tail[WAVES] = last ? 1u : 0u;
    }
    __syncthreads();
    if (!tail[WAVES]) return;
    __threadfence();
  }
  bool wave_fin = false;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (g[b] < 0) continue;
    const uint32_t fin =
        J.chunks > 1 ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g[b]])) & valid[b]
                     : live[b];
    if (!fin) continue;
    wave_fin = true;
    if (final && h == 0 && ((fin >> rl) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[g[b] * BM + rl]);
      if (k != kEmptyMin)
        atomicMax(J.bsf, __builtin_bit_cast(uint32_t, fmaxf(key_dist(k) * J.raise_scale - J.raise_sub, 0.0f)));
    }
  }
  if (final) return;
  if (lane == 0) tail[wv] = wave_fin ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    bool any = false;
    for (int w = 0; w < WAVES; ++w) any |= tail[w] != 0;
    if (any) J.survivors[atomicAdd(J.n_survivors, 1u)] = (int32_t)item;
  }
}

// One workgroup per work item (item, chunk) blockIdx.x, then striding by the
// grid size (the device-decided launches are sized for the most work they can
// hold).  Between two items every wavefront waits for its own copies into LDS
// (a sweep that ended early can leave the next block's copy in flight) and
// for the others to finish reading, before the next item's copies start.
template <int KS, int RB, int WAVES>
__global__ __launch_bounds__(WAVES * 64, (KS <= 16 ? 2 : 1)) void k_scan_mfma(ScanJob Jarg,
                                                                             MixedRows R) {
  ScanJob J = Jarg;
  apply_win(J);
  const int64_t total = J.n_groups * J.chunks;
  for (int64_t wi = blockIdx.x; wi < total; wi += gridDim.x) {
    scan_item<KS, RB, WAVES>(J, R, wi);
    if (wi + gridDim.x < total) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
}

// Full scans (no early abandon, matrix order, every item listed), software-
// pipelined: the FP32 epilogue of column block s-1 runs while the MFMAs of
// block s are in flight.  Two accumulator sets, one barrier per step.  Block
// s+1 is loading while block s feeds the MFMAs and block s-1's column values
// feed the epilogue, so the column values take three LDS stages; the operand
// part of a block takes three stages too (NST = 3, each stage a whole block)
// or, where three would not fit in LDS, two (NST = 2: block s+1 overwrites
// block s-1, whose MFMAs finished before the previous step's barrier), with
// the column values then in a ring of their own.  RB row blocks per
// wavefront, WAVES wavefronts, MINW wavefronts per SIMD (launch bound).
template <int KS, int RB, int WAVES, int MINW, int NST>
__global__ __launch_bounds__(WAVES * 64, MINW) void k_scan_mfma_full(ScanJob J, MixedRows R) {
  static_assert(NST == 2 || NST == 3, "two or three operand stages");
  extern __shared__ bf16x8 smem[];
  constexpr int SLOTS = Blk<KS>::SLOTS;
  constexpr int PER_T = (SLOTS + WAVES * 64 - 1) / (WAVES * 64);
  // NST = 3: stage t = [block | its 8 column-value slots]; NST = 2: two block
  // stages, then three 8-slot column-value stages
  constexpr int STAGE = NST == 3 ? SLOTS + 8 : SLOTS;
  const bf16x8* __restrict__ S = reinterpret_cast<const bf16x8*>(R.sblk);

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int rl = lane & 31;
  const int64_t item = blockIdx.x / J.chunks;
  const int64_t ch = blockIdx.x - item * J.chunks;
  if (item >= J.n_groups) return;
  const int64_t N = J.N;
  const int n = J.n;

  int64_t gb[RB];          // this wavefront's row blocks (0 for a block past the end)
  uint32_t valid[RB];
  bf16x8 bh[RB][KS], bl[RB][KS], bx[RB];
  float smr[RB];
  const __bf16 m2 = (__bf16)(-2.0f);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int64_t g = (item * WAVES + wv) * RB + b;
    const bool has = g * BM < N;
    gb[b] = has ? g : 0;
    const int64_t rows = has ? min<int64_t>(BM, N - g * BM) : 0;
    valid[b] = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
    const bf16x8* blk = S + gb[b] * SLOTS;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      bh[b][k] = blk[k * 128 + lane] * m2;
      bl[b][k] = blk[k * 128 + 64 + lane] * m2;
    }
    bx[b] = blk[KS * 128 + 64 + lane] * m2;
    smr[b] = R.smu[gb[b] * BM + rl];
  }

  const int64_t NQ = (N + BN - 1) / BN;
  const int64_t e0 = J.seq_begin + ch * J.seq_chunk;
  const int64_t e1 = min<int64_t>(NQ, e0 + J.seq_chunk);
  const int64_t steps = e1 > e0 ? e1 - e0 : 0;

  typedef __attribute__((address_space(3))) void lds_void;
  // step t's operand block and its 32 column values sqrt(n) (mean - mu)
  auto stage = [&](int64_t t) { return smem + (t % NST) * STAGE; };
  auto cvals = [&](int64_t t) {
    return NST == 3 ? smem + (t % 3) * STAGE + SLOTS : smem + 2 * SLOTS + (t % 3) * 8;
  };
  // step t covers column block e0 + t
  auto fetch = [&](int64_t t) {
    const int64_t q = e0 + t;
    const bf16x8* src = S + q * SLOTS;
    bf16x8* dst = stage(t);
#pragma unroll
    for (int i = 0; i < PER_T; ++i) {
      const int w0 = i * WAVES * 64 + wv * 64;
      if (w0 < SLOTS)
        __builtin_amdgcn_global_load_lds(src + w0 + lane, (lds_void*)(dst + w0), 16, 0, 0);
    }
    if (wv == 0 && lane < 8)
      __builtin_amdgcn_global_load_lds(R.smu + q * BN + 4 * lane, (lds_void*)cvals(t), 16, 0, 0);
  };

  float rmin[RB];
  int32_t rj[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    rmin[b] = __builtin_inff();
    rj[b] = -1;
  }
  uint32_t cnt = 0;
  auto mma = [&](floatx16 (&a)[RB], const bf16x8* buf) {
    const bf16x8 ax = buf[KS * 128 + lane];
    floatx16 z;
#pragma unroll
    for (int v = 0; v < 16; ++v) z[v] = 0.0f;
#pragma unroll
    for (int b = 0; b < RB; ++b) a[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax, bx[b], z, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const bf16x8 ah = buf[k * 128 + lane];
      const bf16x8 al = buf[k * 128 + 64 + lane];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        a[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[b][k], a[b], 0, 0, 0);
        a[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[b][k], a[b], 0, 0, 0);
        a[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[b][k], a[b], 0, 0, 0);
      }
    }
  };
  // epilogue, first part (straight-line, so that it can be interleaved with the
  // MFMA chain of the next block): the 16 distances of this lane per row block
  auto distances = [&](const floatx16 (&a)[RB], const bf16x8* cv, float (&d)[RB][16]) {
    float smc[16];
#pragma unroll
    for (int qd = 0; qd < 4; ++qd) {
      const float4 m = reinterpret_cast<const float4*>(cv)[2 * qd + h];
      smc[4 * qd + 0] = m.x; smc[4 * qd + 1] = m.y; smc[4 * qd + 2] = m.z; smc[4 * qd + 3] = m.w;
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float t = smr[b] - smc[v];
        d[b][v] = __builtin_fmaf(t, t, a[b][v]);
      }
  };
  // second part: exclusion mask, row minimum and witness, pair count
  auto finish = [&](float (&d)[RB][16], int64_t q) {
    const int32_t j0 = (int32_t)(q * BN);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int32_t r0 = (int32_t)(gb[b] * BM);
      const int32_t i = r0 + rl;
      const bool clean =
          (j0 + BN <= (int32_t)N) && ((j0 >= r0 + BM - 1 + n) || (j0 + BN - 1 + n <= r0));
      if (!clean) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int32_t j = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int32_t dij = i > j ? i - j : j - i;
          if (!(j < (int32_t)N && dij >= n)) d[b][v] = __builtin_inff();
        }
      }
      float tmin = d[b][0];
#pragma unroll
      for (int v = 1; v < 16; ++v) tmin = fminf(tmin, d[b][v]);
      if (__ballot(tmin < rmin[b])) {
        if (tmin < rmin[b]) {
          int32_t jj = -1;
#pragma unroll
          for (int v = 15; v >= 0; --v)
            if (d[b][v] == tmin) jj = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
          rmin[b] = tmin;
          rj[b] = jj;
        }
      }
      if ((valid[b] >> rl) & 1u) {
        if (clean) {
          cnt += 16;
        } else {
#pragma unroll
          for (int v = 0; v < 16; ++v) cnt += d[b][v] < __builtin_inff();
        }
      }
    }
  };
  auto epilogue = [&](const floatx16 (&a)[RB], int64_t t) {
    float d[RB][16];
    distances(a, cvals(t), d);
    finish(d, e0 + t);
  };
  // step t >= 1: load block t+1, multiply block t into `cur` and compute block
  // t-1's distances from `prev` in one straight-line region (the scheduler is
  // asked to interleave the two), then finish block t-1
  auto step = [&](int64_t t, floatx16 (&cur)[RB], const floatx16 (&prev)[RB]) {
    if (t + 1 < steps) fetch(t + 1);
    float d[RB][16];
    __builtin_amdgcn_s_setprio(1);
    mma(cur, stage(t));
    distances(prev, cvals(t - 1), d);
#pragma unroll
    for (int k = 0; k < 16 * RB; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);   // 3 MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // 2 VALU
    }
    __builtin_amdgcn_s_setprio(0);
    finish(d, e0 + t - 1);
    __syncthreads();
  };

  floatx16 acc0[RB], acc1[RB];
  if (steps > 0) {
    fetch(0);
    __syncthreads();
    if (steps > 1) fetch(1);
    mma(acc0, stage(0));
    __syncthreads();
  }
  int64_t t = 1;
  for (; t + 1 < steps; t += 2) {
    step(t, acc1, acc0);
    step(t + 1, acc0, acc1);
  }
  if (t < steps) {
    step(t, acc1, acc0);
    epilogue(acc1, t);
  } else if (steps > 0) {
    epilogue(acc0, steps - 1);
  }

#pragma unroll
  for (int b = 0; b < RB; ++b) {
    uint64_t key = rj[b] < 0 ? kEmptyMin : pack_min(fmaxf(rmin[b], 0.0f), (uint32_t)rj[b]);
    const uint64_t o = __shfl_xor(key, 32, 64);
    key = o < key ? o : key;
    if (h == 0 && ((valid[b] >> rl) & 1u) && key != kEmptyMin)
      atomicMin((unsigned long long*)&J.best[gb[b] * BM + rl], (unsigned long long)key);
  }
  uint64_t c64 = cnt;
  for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
  if (lane == 0 && c64) atomicAdd(pair_slot(J.pairs), (unsigned long long)c64);
}

template <int KS, int RB, int WAVES, int MINW, int NST>
void launch_full_pipelined(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int64_t blocks = J.n_groups * J.chunks;
  if (blocks <= 0) return;
  const size_t lds = sizeof(bf16x8) * (NST * Blk<KS>::SLOTS + 3 * 8);
  static const bool attr_set = [lds] {
    if (lds > 65536)
      (void)hipFuncSetAttribute(
          reinterpret_cast<const void*>(&k_scan_mfma_full<KS, RB, WAVES, MINW, NST>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL((k_scan_mfma_full<KS, RB, WAVES, MINW, NST>), dim3((unsigned)blocks),
                     dim3(WAVES * 64), lds, s, J, R);
}

template <int KS, int RB, int WAVES>
void launch_kr(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int64_t blocks = J.win ? J.max_work : J.n_groups * J.chunks;
  if (blocks <= 0) return;
  const size_t lds = sizeof(bf16x8) * 2 * (Blk<KS>::SLOTS + 8);
  // the LDS opt-in is per kernel and set once per process; the initialisation of a
  // function-local static is thread-safe, so concurrent first launches from several
  // host threads (one per serving slot) do not race
  static const bool attr_set = [lds] {
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan_mfma<KS, RB, WAVES>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL((k_scan_mfma<KS, RB, WAVES>), dim3((unsigned)blocks), dim3(WAVES * 64), lds,
                     s, J, R);
}

template <int KS>
void launch_ks(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  // full scans only (no abandon, matrix order, every item listed)
  if constexpr (KS > 8 && KS <= 16) {
    if (waves_for<KS>(J.abandon != 0) == 8) {
      launch_full_pipelined<KS, 1, 8, 2, 3>(J, R, s);
      return;
    }
  }
  if constexpr (KS > 16 && KS <= 18) {
    if (!J.abandon) {
      // two wavefronts per SIMD, two workgroups per CU (two operand stages each)
      launch_full_pipelined<KS, 1, 4, 2, 2>(J, R, s);
      return;
    }
  }
  // early-abandon searches keep one row block per wavefront at every window:
  // finer items leave sooner (8.6 -> 7.8 ms to discord on the 2^20 walk, n = 128)
  if (J.abandon)
    launch_kr<KS, 1, 4>(J, R, s);
  else
    launch_kr<KS, kRowBlocks<KS>, 4>(J, R, s);
}

template <int KS>
void launch_split(const float* Tp, int64_t nblk, int n, const float* c32, const float* cn32,
                  const float* r32, uint4* sblk, hipStream_t s) {
  const int64_t threads = nblk * (KS + 1) * 64;
  hipLaunchKernelGGL(k_split_blocks<KS>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                     Tp, nblk, n, c32, cn32, r32, reinterpret_cast<bf16x8*>(sblk));
}

}  // namespace

int mfma_row_blocks(int n, bool abandon) {
  const int ks = (n + 15) / 16;
  if (ks > 32) return 4;   // windows beyond 512: 128 rows per workgroup (scan_mfma_long.hip)
  const int waves = (ks > 8 && ks <= 16 && !abandon) ? 8 : 4;
  return waves * ((ks <= 8 && !abandon) ? 2 : 1);
}

size_t mixed_block_bytes(int n) {
  return mixed_long(n) ? 0 : (size_t)(((n + 15) / 16) + 1) * 128 * 16;
}

int64_t mixed_blocks(int64_t N) { return (N + BM - 1) / BM + 1; }

#define DD_KS_CASES(X)                                                                         \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) \
  X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

bool launch_scan_mfma(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  switch ((J.n + 15) / 16) {
#define DD_CASE(K) \
  case K: launch_ks<K>(J, R, s); return true;
    DD_KS_CASES(DD_CASE)
#undef DD_CASE
    default: return launch_scan_mfma_long(J, R, s);   // windows of 513..2048
  }
}

void launch_split_blocks(const float* Tp, int64_t N, int n, const float* c32, const float* cn32,
                         const float* r32, uint4* sblk, hipStream_t s) {
  const int64_t nblk = mixed_blocks(N);
  switch ((n + 15) / 16) {
#define DD_CASE(K) \
  case K: launch_split<K>(Tp, nblk, n, c32, cn32, r32, sblk, s); return;
    DD_KS_CASES(DD_CASE)
#undef DD_CASE
    default:
      return;   // longer windows build their operands from the series (scan_mfma_long.hip)
  }
}

}  // namespace dd
