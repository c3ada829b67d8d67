// scan_mfma_long.hip -- split-BF16 pair-distance scan for windows of 513..2048.
//
// The arithmetic is that of scan_mfma.hip: centred windows split as hi + lo
// bf16, a'.b' ~ hi.hi + hi.lo + lo.hi on v_mfma_f32_32x32x16_bf16, one extra
// K-step folding in the norms, d^2 = acc + (sqrt(n) (mu_a - mu_b))^2, and every
// decision certified in FP64 afterwards.  What changes is where the operands
// live.  A row block's operands take 8 VGPRs per K-step, so beyond 32 K-steps
// (n = 512) one wavefront cannot hold them.  Here the K-steps of ONE row block
// are split over the 4 wavefronts of a workgroup: wavefront w keeps steps
// w*KSP .. w*KSP + KSP - 1 in registers for the whole sweep (KSP <= 32) and
// reads the same steps of each column block straight from global memory (the
// column blocks are read by every row block in turn, so they are served by L2
// in matrix order and near-first order alike).  Each wavefront's partial 32x32
// accumulator goes through LDS; wavefront w then sums the four partials of the
// accumulator elements 4w..4w+3 (columns j0 + 8w + 4h + 0..3 of row rl, in the
// lane layout of the 32x32 result) and keeps the running minimum of those
// columns.  Early abandon, survivors and the best-so-far follow the short-window
// kernel; the live-row mask is made uniform over the workgroup after every
// step (a row leaves as soon as any wavefront finds a column below the
// best-so-far).
#include "internal.hpp"

namespace dd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 32;
constexpr int BN = 32;
constexpr int W = 4;   // wavefronts per workgroup, one K-part each

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per (item, chunk of its column sequence); an item is one row
// block.  KSP: K-steps per wavefront, with 4 * KSP >= KS > 4 * (KSP - 1).
template <int KSP>
__device__ __forceinline__ void scan_item(const ScanJob& J, const MixedRows& R, int64_t wi) {
  __shared__ float4 part[W][4][64];          // partial accumulators, 16 KiB
  __shared__ uint32_t live_of[2][W];         // per step parity: each wavefront's live rows
  __shared__ uint32_t tail[W + 1];
  const bf16x8* __restrict__ S = reinterpret_cast<const bf16x8*>(R.sblk);

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int rl = lane & 31;
  const int n = J.n;
  const int KS = (n + 15) / 16;
  const int64_t SLOTS = (int64_t)(KS + 1) * 128;   // 16-byte slots per block
  const int k0 = wv * KSP;                          // this wavefront's first K-step
  const int kw = min(KSP, KS - k0);                 // >= 1 (KS > 4 (KSP - 1))
  const int64_t li = wi / J.chunks;
  const int64_t ch = wi - li * J.chunks;
  if (li >= J.n_groups) return;
  const int64_t N = J.N;
  const int64_t g = __builtin_amdgcn_readfirstlane((int)(J.groups ? J.groups[li] : li));
  if (J.skip && J.skip[g]) return;
  const int64_t r0 = g * BM;
  const int64_t rows = min<int64_t>(BM, N - r0);
  const uint32_t valid = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
  uint32_t live =
      J.abandon ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g]) & valid) : valid;
  if (J.abandon && J.precheck && live) {
    // rows whose minimum over the columns of earlier launches is already below
    // the best-so-far cannot be the discord: they leave with that witness
    // (every wavefront takes the same decision from the same values)
    const float bs = __builtin_bit_cast(float, load_relaxed(J.bsf));
    bool below = false;
    if (h == 0 && ((live >> rl) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[r0 + rl]);
      below = k != kEmptyMin && key_dist(k) < bs;
    }
    const uint32_t dead = (uint32_t)(__ballot(below) & 0xFFFFFFFFull);
    if (dead) {
      if (lane == 0) atomicAnd(&J.alive[g], ~dead);
      live &= ~dead;
    }
  }

  // one live mask for the workgroup before the sweep: each wavefront read the
  // masks on its own, and another chunk of the item may have changed them
  if (lane == 0) live_of[1][wv] = live;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < W; ++w) live &= live_of[1][w];

  // ---- this wavefront's K-part of the row operands, scaled by -2 --------------
  const bf16x8* rblk = S + g * SLOTS;
  const __bf16 m2 = (__bf16)(-2.0f);
  bf16x8 bh[KSP], bl[KSP], bx;
#pragma unroll
  for (int s = 0; s < KSP; ++s) {
    if (s < kw) {
      bh[s] = rblk[(int64_t)(k0 + s) * 128 + lane] * m2;
      bl[s] = rblk[(int64_t)(k0 + s) * 128 + 64 + lane] * m2;
    } else {
      bh[s] = bl[s] = bf16x8{};
    }
  }
  bx = rblk[(int64_t)KS * 128 + 64 + lane] * m2;   // norm step (wavefront 0 uses it)
  const float smr = R.smu[r0 + rl];

  // ---- column sequence (uniform over the workgroup) ---------------------------
  int64_t nb = 0, b0 = 0;
  if (J.words) {
    const int wd = J.words[r0];
    b0 = J.bgrp_off[wd];
    nb = J.bgrp_off[wd + 1] - b0;
  }
  const int64_t NQ = (N + BN - 1) / BN;
  Spiral sp{0, -1, NQ, 0};
  if (J.near_first) sp = make_spiral(r0, r0 + BM, n, NQ, BN);
  const int64_t len = nb + spiral_count(sp);
  const int64_t e0 = J.seq_begin + ch * J.seq_chunk;
  const int64_t e1 = min<int64_t>(len, e0 + J.seq_chunk);
  int64_t steps = (e1 > e0 && live) ? e1 - e0 : 0;
  const bool final = J.seq_begin + J.chunks * J.seq_chunk >= len;
  auto block_of = [&](int64_t s) -> int64_t {
    const int64_t e = e0 + s;
    return e < nb ? (int64_t)__builtin_amdgcn_readfirstlane(J.bgrp[b0 + e])
                  : spiral_block(sp, e - nb);
  };

  float rmin = __builtin_inff();
  int32_t rj = -1;
  uint32_t cnt = 0;
  const int32_t i = (int32_t)(r0 + rl);

  // With PF > 0, column operands are read from global memory PF K-steps ahead
  // of their MFMAs: step k of a block sits in slot k % PF, refilled with step
  // k + PF once consumed; after a block's last MFMA is issued the first PF
  // steps of the next block are requested, so their latency overlaps the
  // epilogue.  The 64 registers this takes cost a wavefront per SIMD beyond 15
  // K-steps per wavefront, which measured slower (0.11 vs 0.15 of the BF16 peak
  // at n = 1024; 0.23 vs 0.19 at n = 600, where it keeps two), so there the
  // operands are loaded where they are used.
  constexpr int PF = KSP <= 15 ? 8 : 0;
  constexpr int PFS = PF > 0 ? PF : 1;
  bf16x8 pa[PFS], pl[PFS], px;
  auto prefetch_head = [&](const bf16x8* cb) {
    if constexpr (PF == 0) return;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      if (k < kw) {
        pa[k] = cb[(int64_t)(k0 + k) * 128 + lane];
        pl[k] = cb[(int64_t)(k0 + k) * 128 + 64 + lane];
      }
    }
    px = cb[(int64_t)KS * 128 + lane];
  };
  int64_t q_next = steps > 0 ? block_of(0) : 0;
  if (steps > 0) prefetch_head(S + q_next * SLOTS);

  for (int64_t s = 0; s < steps; ++s) {
    const int64_t q = q_next;
    const int32_t j0 = (int32_t)(q * BN);
    const bf16x8* cblk = S + q * SLOTS;
    if (s + 1 < steps) q_next = block_of(s + 1);
    // ---- partial product over this wavefront's K-steps ------------------------
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    if (wv == 0)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(PF > 0 ? px : cblk[(int64_t)KS * 128 + lane],
                                                    bx, acc, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < KSP; ++k) {
      if (k < kw) {
        bf16x8 ah, al;
        if constexpr (PF > 0) {
          ah = pa[k % PFS];
          al = pl[k % PFS];
          if (k + PF < kw) {
            pa[k % PFS] = cblk[(int64_t)(k0 + k + PF) * 128 + lane];
            pl[k % PFS] = cblk[(int64_t)(k0 + k + PF) * 128 + 64 + lane];
          }
        } else {
          ah = cblk[(int64_t)(k0 + k) * 128 + lane];
          al = cblk[(int64_t)(k0 + k) * 128 + 64 + lane];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[k], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[k], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[k], acc, 0, 0, 0);
      }
    }
    if (s + 1 < steps) prefetch_head(S + q_next * SLOTS);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      part[wv][c][lane] = make_float4(acc[4 * c], acc[4 * c + 1], acc[4 * c + 2], acc[4 * c + 3]);
    __syncthreads();
    // ---- this wavefront's 4 columns: sum of the partials, distance ------------
    float4 t = part[0][wv][lane];
#pragma unroll
    for (int p = 1; p < W; ++p) {
      const float4 x = part[p][wv][lane];
      t.x += x.x; t.y += x.y; t.z += x.z; t.w += x.w;
    }
    const int32_t jc = j0 + 8 * wv + 4 * h;         // this lane's first column
    const float4 sc = *reinterpret_cast<const float4*>(R.smu + jc);
    float d[4];
    {
      float u;
      u = smr - sc.x; d[0] = __builtin_fmaf(u, u, t.x);
      u = smr - sc.y; d[1] = __builtin_fmaf(u, u, t.y);
      u = smr - sc.z; d[2] = __builtin_fmaf(u, u, t.z);
      u = smr - sc.w; d[3] = __builtin_fmaf(u, u, t.w);
    }
    const bool clean = (j0 + BN <= (int32_t)N) &&
                       ((j0 >= (int32_t)r0 + BM - 1 + n) || (j0 + BN - 1 + n <= (int32_t)r0));
    if (!clean) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t j = jc + u;
        const int32_t dij = i > j ? i - j : j - i;
        if (!(j < (int32_t)N && dij >= n)) d[u] = __builtin_inff();
      }
    }
    const float tmin = fminf(fminf(d[0], d[1]), fminf(d[2], d[3]));
    if (tmin < rmin) {
      int32_t jj = -1;
#pragma unroll
      for (int u = 3; u >= 0; --u)
        if (d[u] == tmin) jj = jc + u;
      rmin = tmin;
      rj = jj;
    }
    if ((valid >> rl) & 1u) {
      if (clean) {
        cnt += 4;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) cnt += d[u] < __builtin_inff();
      }
    }
    // ---- early abandon --------------------------------------------------------
    if (J.abandon) {
      const float bsf = __builtin_bit_cast(float, load_relaxed(J.bsf));
      const float m = fminf(rmin, __shfl_xor(rmin, 32, 64));
      const uint32_t dead = (uint32_t)(__ballot(m < bsf && h == 0) & 0xFFFFFFFFull) & live;
      if (dead) {
        uint64_t key = rj < 0 ? kEmptyMin : pack_min(fmaxf(rmin, 0.0f), (uint32_t)rj);
        const uint64_t o = __shfl_xor(key, 32, 64);
        key = o < key ? o : key;
        if (h == 0 && ((dead >> rl) & 1u))
          atomicMin((unsigned long long*)&J.best[r0 + rl], (unsigned long long)key);
        if (lane == 0) atomicAnd(&J.alive[g], ~dead);
        live &= ~dead;
      }
      if (J.chunks > 1) live &= __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g]));
    }
    // ---- one live mask for the workgroup (the partials are read by now) --------
    uint32_t* lv = live_of[s & 1];
    if (lane == 0) lv[wv] = live;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; ++w) live &= lv[w];
    if (!live) break;
  }

  // ---- publish --------------------------------------------------------------------
  {
    uint64_t key = rj < 0 ? kEmptyMin : pack_min(fmaxf(rmin, 0.0f), (uint32_t)rj);
    const uint64_t o = __shfl_xor(key, 32, 64);
    key = o < key ? o : key;
    if (h == 0 && ((live >> rl) & 1u) && key != kEmptyMin)
      atomicMin((unsigned long long*)&J.best[r0 + rl], (unsigned long long)key);
  }
  uint64_t c64 = cnt;
  for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
  if (lane == 0 && c64) atomicAdd(pair_slot(J.pairs), (unsigned long long)c64);
  if (!J.abandon) return;

  // every wavefront has published its columns' minima before any is read back
  __threadfence();
  __syncthreads();
  if (J.chunks > 1) {
    // the item's last chunk to finish decides
    if (threadIdx.x == 0) {
      const uint32_t prev = atomicAdd(&J.done[g], 1u);
      const bool last = prev + 1 == (uint32_t)J.chunks;
      if (last) atomicExch(&J.done[g], 0u);   // ready for the next launch
      tail[W] = last ? 1u : 0u;
    }
    __syncthreads();
    if (!tail[W]) return;
    __threadfence();
  }
  if (wv != 0) return;
  const uint32_t fin =
      J.chunks > 1 ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g])) & valid : live;
  if (!fin) return;
  if (final) {
    // complete rows raise the best-so-far with their minimum over all launches
    if (h == 0 && ((fin >> rl) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[r0 + rl]);
      if (k != kEmptyMin)
        atomicMax(J.bsf, __builtin_bit_cast(uint32_t,
                                            fmaxf(key_dist(k) * J.raise_scale - J.raise_sub, 0.0f)));
    }
  } else if (lane == 0) {
    J.survivors[atomicAdd(J.n_survivors, 1u)] = (int32_t)g;
  }
}

// One workgroup per work item, striding by the grid size as in scan_mfma.hip.
template <int KSP>
__global__ __launch_bounds__(W * 64, 1) void k_scan_mfma_long(ScanJob Jarg, MixedRows R) {
  ScanJob J = Jarg;
  apply_win(J);
  const int64_t total = J.n_groups * J.chunks;
  for (int64_t wi = blockIdx.x; wi < total; wi += gridDim.x) {
    scan_item<KSP>(J, R, wi);
    if (wi + gridDim.x < total) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
}

template <int KSP>
void launch_long(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int64_t blocks = J.win ? J.max_work : J.n_groups * J.chunks;
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_scan_mfma_long<KSP>, dim3((unsigned)blocks), dim3(W * 64), 0, s, J, R);
}

}  // namespace

#define DD_KSP_CASES(X)                                                                       \
  X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) \
  X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

bool launch_scan_mfma_long(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int ks = (J.n + 15) / 16;
  if (ks <= 32 || ks > 4 * 32) return false;
  switch ((ks + W - 1) / W) {
#define DD_CASE(K) \
  case K: launch_long<K>(J, R, s); return true;
    DD_KSP_CASES(DD_CASE)
#undef DD_CASE
    default: return false;
  }
}

}  // namespace dd
