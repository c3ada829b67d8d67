// scan_mfma.hip -- split-BF16 pair-distance scan on the gfx950 matrix cores,
// with the operands built from the series itself (windows of 1..2048).
//
// Eq. (1)'s squared distance is expanded as |a|^2 + |b|^2 - 2 a.b.  The dot
// products run on v_mfma_f32_32x32x16_bf16, with each centred value split as
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and a.b ~ hi.hi + hi.lo +
// lo.hi, accumulated in FP32.  The split products carry ~2^-16 of |a||b|.
// Every decision is certified in FP64 afterwards (certify.hip), so these
// errors never reach the result.
//
// Operands.  The windows of a series are shifted copies of one another:
// element k of window i is t_{i+k}.  A 32 x 16 MFMA operand whose row r and
// K-index k hold x_{i0 + r + k} therefore reads, in lane (r, h), the 8
// consecutive values x_{i0 + r + 16 s + 8 h + 0..7} of one array x.  Such
// operands are built in LDS from a short stretch of the series, instead of
// being read from a per-window matrix of n values per row.  For a
// workgroup's 128 rows and a step's 128 columns that stretch is 16 KS + 128
// values each (KS = ceil(n/16) K-steps).  Every entry p of the LDS array
// holds the 8 values starting at p (hi and lo bf16 halves, 16 bytes each).
// So every operand is one aligned ds_read_b128, and the 64 lanes of a read
// touch consecutive entries.
//
// Centring.  A window cannot be centred on its own mean here (that would give
// every window its own copy of the values again), so the values of a
// workgroup's rows are centred on one offset C_R, the FP32 mean of the
// middle row, and a step's columns on C_C likewise:
//   x'_k = t_{i+k} - C_R,  y'_k = t_{j+k} - C_C,   P = x'.y'.
// With m_i = c_i - C_R and m_j = c_j - C_C (c the FP32 window means) the
// centred product is a.b = P - n m_i m_j, up to terms of order n ulp(mu) m.
// Eq. (1)'s squared distance is then
//   d^2 = |a|^2 + |b|^2 - 2 P + 2 n m_i m_j + n (mu_i - mu_j)^2 ,
// and under per-window normalisation (scales r = 1/sigma)
//   d^2 = |a r_i|^2 + |b r_j|^2 - 2 r_i r_j (P - n m_i m_j) .
// Within a workgroup the window means differ little from the offsets, so
// |x'| stays close to |a|, and the split products keep their ~2^-16 |a||b|
// error.
//
// Work sharing.  An item is 4 row blocks of 32 consecutive rows (128 rows),
// one per wavefront.  A step is 128 consecutive columns, in 4 blocks of 32.
// Wavefront w multiplies its row block by the 4 column blocks, which makes
// four 32x32 accumulators.  At K-step s, column block c needs the column
// operand at offset 16 (s + 2c), so one operand serves 4 (block, step) pairs.
// Each K-step reads one new column operand and one row operand (hi and lo)
// for 12 MFMAs.  In an early-abandon search a step in which only one row block
// is still live would leave three wavefronts idle; there the four wavefronts
// take one column block of the live row block each, and the row minima of the
// four tiles are merged through LDS by the block's own wavefront, in column
// order.  Steps visit 128-column super-blocks: the item's word bucket first
// (same-word columns, Algorithm 4), then outward from the item's rows
// (spiral.hpp), or in matrix order.
//
// Early abandon (Algorithms 3 and 4): after every step, rows whose running
// minimum is below the device best-so-far leave with that minimum and its
// column as witness; a workgroup stops once none of its rows is live.  An
// item's sequence may be split into chunks run by several workgroups and
// resumed by later launches; the last chunk of a final launch raises the
// best-so-far with its complete rows' minima, and a non-final launch lists
// items with live rows as survivors.
//
// Operand roles (lane layout checked on the hardware): B = the row block, A =
// a column block.  The 32x32 result gives lane l the 16 columns
// 8(v/4) + 4(l/32) + v%4 of row l % 32, so the row minimum is mostly a
// per-lane running minimum.
#include "internal.hpp"

namespace dd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 32;          // rows per row block
constexpr int W = 4;            // wavefronts = row blocks per item
constexpr int TR = W * BM;      // rows per item
constexpr int CB = 4;           // column blocks per step
constexpr int TC = CB * BM;     // columns per step
constexpr int THREADS = W * 64;

// LDS entries of one stretch: rows/columns 0..127 at K-steps 0..KS-1 reach
// entry 127 + 16 (KS - 1) + 8 (then 7 more values inside the entry)
__host__ __device__ constexpr int stretch_entries(int ks) { return 16 * ks + 128; }

// dynamic LDS: two stretches (hi and lo entries each), the step's columns'
// norm-step operands (2 entries per column), then two column values (128
// floats each)
__host__ __device__ constexpr size_t lds_bytes(int ks) {
  return ((size_t)2 * stretch_entries(ks) * 2 + 2 * TC) * sizeof(bf16x8) + 2 * TC * sizeof(float);
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// entries p = 0 .. L-1 of a stretch starting at series index `base`:
// hi/lo halves of (t_{base+p+e} - C) * S, e = 0..7, with S = 1 or -2 (exact).
// Reads t up to base + L + 6, inside the zero pad after the series for every
// base <= N - 1.
__device__ __forceinline__ void build_stretch(const float* __restrict__ Tp, int64_t base, float C,
                                              float S, int L, bf16x8* __restrict__ eh,
                                              bf16x8* __restrict__ el) {
  for (int p = threadIdx.x; p < L; p += THREADS) {
    const float* src = Tp + base + p;
    float4 a, b;
    __builtin_memcpy(&a, src, 16);
    __builtin_memcpy(&b, src + 4, 16);
    const float v[8] = {(a.x - C) * S, (a.y - C) * S, (a.z - C) * S, (a.w - C) * S,
                        (b.x - C) * S, (b.y - C) * S, (b.z - C) * S, (b.w - C) * S};
    bf16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 x = (__bf16)v[e];
      hi[e] = x;
      lo[e] = (__bf16)(v[e] - (float)x);
    }
    eh[p] = hi;
    el[p] = lo;
  }
}

// x = hi + mid + lo in bf16 (24 significant bits: exact for an FP32 x of
// ordinary range)
__device__ __forceinline__ void split3(float x, __bf16& a, __bf16& b, __bf16& c) {
  a = (__bf16)x;
  const float r = x - (float)a;
  b = (__bf16)r;
  c = (__bf16)(r - (float)b);
}

// The norm step, one extra K-step whose product adds the per-row and
// per-column terms to the accumulator (the row operands carry -2, so the
// K-steps of the windows add -2 P):
//   raw windows:  |a|^2 + |b|^2 + 2 n m_i m_j
//   normalised:   2 n m_i m_j      (|a r|^2 + |b r|^2 are added after scaling)
// Column (A) operand, lane half 0 / 1:  (B_hi, B_mid, B_lo, 1, 1, 1, M_hi, M_hi | M_lo, 0..)
// Row (B) operand, lane half 0 / 1:     (1, 1, 1, A_hi, A_mid, A_lo, G_hi, G_lo | G_hi, 0..)
// with B = |b|^2, A = |a|^2 (zero when normalised), M = m_j, G = 2 n m_i:
// three-way splits hold the norms to 2^-24, and M G is kept to ~2^-16 of a
// term that is itself small.
__device__ __forceinline__ void norm_col(float cn, float m, bf16x8& h0, bf16x8& h1) {
  const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
  __bf16 a, b, c;
  split3(cn, a, b, c);
  const __bf16 mh = (__bf16)m, ml = (__bf16)(m - (float)mh);
  h0 = bf16x8{a, b, c, one, one, one, mh, mh};
  h1 = bf16x8{ml, zero, zero, zero, zero, zero, zero, zero};
}

__device__ __forceinline__ bf16x8 norm_row(float cn, float g, int h) {
  const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
  __bf16 a, b, c;
  split3(cn, a, b, c);
  const __bf16 gh = (__bf16)g, gl = (__bf16)(g - (float)gh);
  return h == 0 ? bf16x8{one, one, one, a, b, c, gh, gl}
                : bf16x8{gh, zero, zero, zero, zero, zero, zero, zero};
}

__device__ __forceinline__ bf16x8 mask_bf16(bf16x8 x, uint4 m) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x &= m.x;
  u.y &= m.y;
  u.z &= m.z;
  u.w &= m.w;
  return __builtin_bit_cast(bf16x8, u);
}

// PFE > 0: the stretch has at most PFE * 256 entries, and each thread holds
// the values of its PFE entries (and a column's statistics) for the next step
// in registers: they are loaded while the current step's MFMAs run.  SHARE:
// the early-abandon instance, with the one-live-block steps (full scans never
// have a dead row block, and keep the code without them).
template <bool Z, int PFE, bool SHARE>
__device__ __forceinline__ void scan_item(const ScanJob& J, const MixedRows& R, int64_t wi,
                                          bf16x8* smem) {
  __shared__ uint32_t wave_live[2 * W];
  __shared__ uint32_t tail[W + 1];
  // one-live-block steps: each tile's row minima (early-abandon instance only)
  __shared__ float part_d[SHARE ? W * 64 : 1];
  __shared__ int32_t part_j[SHARE ? W * 64 : 1];

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int rl = lane & 31;
  const int n = J.n;
  const int KS = (n + 15) / 16;
  const int L = stretch_entries(KS);
  bf16x8* const rEh = smem;              // row stretch
  bf16x8* const rEl = smem + L;
  bf16x8* const cEh = smem + 2 * L;      // column stretch of the current step
  bf16x8* const cEl = smem + 3 * L;
  bf16x8* const cN = smem + 4 * L;                              // norm-step column operands
  float* const cst = reinterpret_cast<float*>(smem + 4 * L + 2 * TC);   // smu or r | cn

  const int64_t li = wi / J.chunks;
  const int64_t ch = wi - li * J.chunks;
  if (li >= J.n_groups) return;
  const int64_t N = J.N;
  const int64_t item = __builtin_amdgcn_readfirstlane((int)(J.groups ? J.groups[li] : li));
  if (J.skip && J.skip[item]) return;
  const int64_t r_first = item * TR;

  // ---- this wavefront's row block and its live rows ---------------------------
  const int64_t g = item * W + wv;
  const int64_t r0 = g * BM;
  uint32_t valid = 0, live = 0;
  if (r0 < N) {
    const int64_t rows = min<int64_t>(BM, N - r0);
    valid = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
    live = J.abandon ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g]) & valid) : valid;
    if (J.abandon && J.precheck && live) {
      // rows whose minimum over the columns of earlier launches is already
      // below the best-so-far cannot be the discord: they leave with that witness
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
  }

  // ---- column sequence (uniform over the workgroup) ---------------------------
  int64_t nb = 0, b0 = 0;
  if (J.words) {
    const int wd = J.words[r_first];
    b0 = J.bgrp_off[wd];
    nb = J.bgrp_off[wd + 1] - b0;
  }
  const int64_t NQ = (N + TC - 1) / TC;
  Spiral sp{0, -1, NQ, 0};
  if (J.near_first) sp = make_spiral(r_first, r_first + TR, n, NQ, TC);
  const int64_t len = nb + spiral_count(sp);
  const int64_t e0 = J.seq_begin + ch * J.seq_chunk;
  const int64_t e1 = min<int64_t>(len, e0 + J.seq_chunk);
  int64_t steps = e1 > e0 ? e1 - e0 : 0;
  const bool final = J.seq_begin + J.chunks * J.seq_chunk >= len;
  auto block_of = [&](int64_t s) -> int64_t {
    const int64_t e = e0 + s;
    return e < nb ? (int64_t)__builtin_amdgcn_readfirstlane(J.bgrp[b0 + e])
                  : spiral_block(sp, e - nb);
  };

  // workgroup-wide: is any row still live?
  if (lane == 0) wave_live[wv] = live ? 1u : 0u;
  __syncthreads();
  bool wg_live = false;
#pragma unroll
  for (int w = 0; w < W; ++w) wg_live |= wave_live[w] != 0;
  if (!wg_live) steps = 0;

  const int32_t jlim = (int32_t)N;   // N < 2^31 (checked at prepare)

  // ---- a step's column data: the stretch values, the centre and the columns'
  // statistics (prefetched one step ahead when PFE > 0) ---------------------------
  constexpr int PFN = PFE > 0 ? PFE : 1;
  float4 pa[PFN], pb[PFN];
  float pcc = 0.0f, pcn = 0.0f, pmu = 0.0f, px = 0.0f;
  int32_t pj0 = 0;
  auto fetch_cols = [&](int64_t st) {
    pj0 = (int32_t)(block_of(st) * TC);
    pcc = R.mu[min<int64_t>(pj0 + TC / 2, N - 1)];
#pragma unroll
    for (int r = 0; r < PFN; ++r) {
      const int p = threadIdx.x + THREADS * r;
      if (p < L) {
        const float* src = J.Tp + pj0 + p;
        __builtin_memcpy(&pa[r], src, 16);
        __builtin_memcpy(&pb[r], src + 4, 16);
      }
    }
    if (threadIdx.x < TC) {
      const int32_t j = pj0 + threadIdx.x;
      const bool in = j < jlim;
      pcn = in ? R.cnorm[j] : 0.0f;
      pmu = in ? R.mu[j] : 0.0f;
      px = in ? (Z ? R.r[j] : R.smu[j]) : 0.0f;
    }
  };
  // the prefetched step into LDS: hi/lo entries, norm-step operands, values
  auto store_cols = [&]() {
#pragma unroll
    for (int r = 0; r < PFN; ++r) {
      const int p = threadIdx.x + THREADS * r;
      if (p < L) {
        const float v[8] = {pa[r].x - pcc, pa[r].y - pcc, pa[r].z - pcc, pa[r].w - pcc,
                            pb[r].x - pcc, pb[r].y - pcc, pb[r].z - pcc, pb[r].w - pcc};
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const __bf16 x = (__bf16)v[e];
          hi[e] = x;
          lo[e] = (__bf16)(v[e] - (float)x);
        }
        cEh[p] = hi;
        cEl[p] = lo;
      }
    }
    if (threadIdx.x < TC) {
      const bool in = pj0 + (int32_t)threadIdx.x < jlim;
      norm_col(Z ? 0.0f : pcn, in ? pmu - pcc : 0.0f, cN[2 * threadIdx.x], cN[2 * threadIdx.x + 1]);
      cst[threadIdx.x] = px;
      if (Z) cst[TC + threadIdx.x] = pcn;
    }
  };

  // ---- the row stretch and the per-row terms -----------------------------------
  // the row stretch carries the factor -2 of -2 P (exact in bf16); the first
  // step's column loads are issued first, so that both are in flight together
  const float CR = R.mu[min<int64_t>(r_first + TR / 2, N - 1)];
  if (steps > 0) {
    if constexpr (PFE > 0) fetch_cols(0);
    build_stretch(J.Tp, r_first, CR, -2.0f, L, rEh, rEl);
  }
  const int64_t irow = min<int64_t>(r0 + rl, N - 1);
  const float ci = R.cnorm[irow];
  const float mi = R.mu[irow] - CR;
  const bf16x8 nrow = norm_row(Z ? 0.0f : ci, 2.0f * (float)n * mi, h);
  // raw: smu_i; normalised: r_i
  const float xi = Z ? R.r[irow] : R.smu[irow];
  // the last K-step holds window elements 16 (KS - 1) + 8 h + e; those >= n
  // are zeroed in the row operand (bits of each bf16: all ones, or zero)
  uint4 tail_mask;
  {
    const int lim = n - 16 * (KS - 1) - 8 * h;
    uint32_t mw[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      mw[e] = (2 * e < lim ? 0x0000FFFFu : 0u) | (2 * e + 1 < lim ? 0xFFFF0000u : 0u);
    tail_mask = make_uint4(mw[0], mw[1], mw[2], mw[3]);
  }

  float rmin = __builtin_inff();
  int32_t rj = -1;
  uint32_t cnt = 0;
  const int32_t i = (int32_t)(r0 + rl);

  for (int64_t s = 0; s < steps; ++s) {
    // every wavefront has finished reading the previous step's columns (and
    // the row stretch is complete before the first step)
    __syncthreads();
    // the row blocks live in this step (uniform over the workgroup)
    int n_live = 0, one = 0;
    if constexpr (SHARE) {
      const uint32_t* flags = wave_live + (s & 1) * W;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (flags[w] != 0) {
          ++n_live;
          one = w;
        }
      }
      if (n_live == 0) break;
    } else if (s > 0) {
      const uint32_t* flags = wave_live + (s & 1) * W;
      bool any = false;
#pragma unroll
      for (int w = 0; w < W; ++w) any |= flags[w] != 0;
      if (!any) break;
    }
    int32_t j0;
    if constexpr (PFE > 0) {
      j0 = pj0;
      store_cols();
    } else {
      j0 = (int32_t)(block_of(s) * TC);
      const float CC = R.mu[min<int64_t>(j0 + TC / 2, N - 1)];
      build_stretch(J.Tp, j0, CC, 1.0f, L, cEh, cEl);
      if (threadIdx.x < TC) {
        const int32_t j = j0 + threadIdx.x;
        const bool in = j < jlim;
        const float cn = in ? R.cnorm[j] : 0.0f;
        norm_col(Z ? 0.0f : cn, in ? R.mu[j] - CC : 0.0f, cN[2 * threadIdx.x],
                 cN[2 * threadIdx.x + 1]);
        cst[threadIdx.x] = in ? (Z ? R.r[j] : R.smu[j]) : 0.0f;
        if (Z) cst[TC + threadIdx.x] = cn;
      }
    }
    __syncthreads();
    // the next step's column loads run while this step's MFMAs do
    if constexpr (PFE > 0) {
      if (s + 1 < steps) fetch_cols(s + 1);
    }

    if (SHARE && n_live == 1) {
      // ---- one live row block: the 4 wavefronts share its 4 column blocks ----
      // Wavefront w computes the 32x32 tile of the live block `one` and column
      // block w, with the same operands and MFMA order as the owner would (so
      // the distances are the same bits); the owner then merges the 4 tiles'
      // row minima in column order and takes the abandon decision.
      const bool owner = wv == one;
      const float bsf_now = owner ? __builtin_bit_cast(float, load_relaxed(J.bsf)) : 0.0f;
      // this path's LDS addresses are formed here, not hoisted out of the step
      // loop, where they would hold registers through the 4-block K-loop
      int cw = wv;
      asm volatile("" : "+v"(cw));
      const int64_t q0 = (item * W + one) * BM;     // the live block's first row
      const uint32_t qvalid =
          N - q0 >= BM ? 0xFFFFFFFFu : ((1u << (uint32_t)(N - q0)) - 1u);
      const int64_t qrow = min<int64_t>(q0 + rl, N - 1);
      const float qc = R.cnorm[qrow];
      const bf16x8 qnrow = norm_row(Z ? 0.0f : qc, 2.0f * (float)n * (R.mu[qrow] - CR), h);
      const float qx = Z ? R.r[qrow] : R.smu[qrow];
      floatx16 a1;
      {
        floatx16 z;
#pragma unroll
        for (int v = 0; v < 16; ++v) z[v] = 0.0f;
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cN[2 * (32 * cw + rl) + h], qnrow, z, 0, 0, 0);
      }
      // column block wv at K-step k: entry 16 k + 32 wv; row block `one`: 16 k + 32 one
      const bf16x8* ph = cEh + rl + 8 * h + 32 * cw;
      const bf16x8* pl = cEl + rl + 8 * h + 32 * cw;
      const bf16x8* qh = rEh + 32 * one + rl + 8 * h;
      const bf16x8* ql = rEl + 32 * one + rl + 8 * h;
      bf16x8 oh0 = ph[0], ol0 = pl[0], bh0 = qh[0], bl0 = ql[0];
#pragma unroll 1
      for (int k = 0; k < KS; ++k) {
        const int kn = min(k + 1, KS - 1);   // the next K-step's reads, clamped
        const bf16x8 oh1 = ph[16 * kn], ol1 = pl[16 * kn], bh1 = qh[16 * kn], bl1 = ql[16 * kn];
        if (k == KS - 1) {
          bh0 = mask_bf16(bh0, tail_mask);
          bl0 = mask_bf16(bl0, tail_mask);
        }
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(oh0, bh0, a1, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(oh0, bl0, a1, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ol0, bh0, a1, 0, 0, 0);
        oh0 = oh1;
        ol0 = ol1;
        bh0 = bh1;
        bl0 = bl1;
      }
      // the tile's distances, as in the epilogue below for column block wv
      const int32_t jb = j0 + 32 * cw;
      const int32_t qi = (int32_t)(q0 + rl);
      const bool clean = (jb + BM <= jlim) && ((jb >= (int32_t)q0 + BM - 1 + n) ||
                                               (jb + BM - 1 + n <= (int32_t)q0));
      float d[16];
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        const int lc = 32 * cw + 8 * qd + 4 * h;
        const float4 xj = *reinterpret_cast<const float4*>(cst + lc);
        const float xjv[4] = {xj.x, xj.y, xj.z, xj.w};
        if (Z) {
          const float4 cn = *reinterpret_cast<const float4*>(cst + TC + lc);
          const float cnv[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            d[4 * qd + e] = __builtin_fmaf(qx * xjv[e], a1[4 * qd + e], qc + cnv[e]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float u = qx - xjv[e];
            d[4 * qd + e] = __builtin_fmaf(u, u, a1[4 * qd + e]);
          }
        }
      }
      if (!clean) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int32_t j = jb + 8 * (v >> 2) + 4 * h + (v & 3);
          const int32_t dij = qi > j ? qi - j : j - qi;
          if (!(j < jlim && dij >= n)) d[v] = __builtin_inff();
        }
      }
      float tmin = d[0];
#pragma unroll
      for (int v = 1; v < 16; ++v) tmin = fminf(tmin, d[v]);
      int32_t jj = -1;
#pragma unroll
      for (int v = 15; v >= 0; --v)
        if (d[v] == tmin) jj = jb + 8 * (v >> 2) + 4 * h + (v & 3);
      if ((qvalid >> rl) & 1u) {
        if (clean) {
          cnt += 16;
        } else {
#pragma unroll
          for (int v = 0; v < 16; ++v) cnt += d[v] < __builtin_inff();
        }
      }
      part_d[64 * cw + lane] = tmin;
      part_j[64 * cw + lane] = jj;
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const float pd = part_d[64 * c + lane];
          if (pd < rmin) {
            rmin = pd;
            rj = part_j[64 * c + lane];
          }
        }
        const float m = fminf(rmin, __shfl_xor(rmin, 32, 64));
        const uint32_t dead = (uint32_t)(__ballot(m < bsf_now && h == 0) & 0xFFFFFFFFull) & live;
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
    } else if (live) {
      // the best-so-far for this step's abandon test, read before the MFMAs so
      // that its latency overlaps them (a value read earlier is never larger)
      const float bsf_now = J.abandon ? __builtin_bit_cast(float, load_relaxed(J.bsf)) : 0.0f;
      // ---- the norm step, then -2 P for 32 rows x 128 columns ----------------------
      floatx16 acc[CB];
      {
        floatx16 z;
#pragma unroll
        for (int v = 0; v < 16; ++v) z[v] = 0.0f;
#pragma unroll
        for (int c = 0; c < CB; ++c)
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cN[2 * (32 * c + rl) + h], nrow, z, 0,
                                                          0, 0);
      }
      const bf16x8* ch_ = cEh + rl + 8 * h;          // column operand u at ch_[16 u]
      const bf16x8* cl_ = cEl + rl + 8 * h;
      const bf16x8* rh_ = rEh + 32 * wv + rl + 8 * h;   // row operand s at rh_[16 s]
      const bf16x8* rl_ = rEl + 32 * wv + rl + 8 * h;
      bf16x8 oh[8], ol[8], bh[2], bl[2];   // column operands by u mod 8, row operands by s mod 2
#pragma unroll
      for (int u = 0; u < 7; ++u) {
        oh[u] = ch_[16 * u];
        ol[u] = cl_[16 * u];
      }
      bh[0] = rh_[0];
      bl[0] = rl_[0];
      for (int kb = 0; kb < KS; kb += 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = kb + t;
          // operands of the next K-step: the column operand at u = k + 7 (its
          // block 3) and the row operand.  The reads are unconditional (indices
          // clamped into the stretch; past the last step they are not used), so
          // that every K-step waits only for the previous step's reads.
          {
            const int un = min(k + 7, KS + 5);
            const int rn = min(k + 1, KS - 1);
            oh[(t + 7) & 7] = ch_[16 * un];
            ol[(t + 7) & 7] = cl_[16 * un];
            bh[(t + 1) & 1] = rh_[16 * rn];
            bl[(t + 1) & 1] = rl_[16 * rn];
          }
          if (k < KS) {
            if (k == KS - 1) {
              bh[t & 1] = mask_bf16(bh[t & 1], tail_mask);
              bl[t & 1] = mask_bf16(bl[t & 1], tail_mask);
            }
#pragma unroll
            for (int c = 0; c < CB; ++c)
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(oh[(t + 2 * c) & 7], bh[t & 1],
                                                              acc[c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < CB; ++c)
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(oh[(t + 2 * c) & 7], bl[t & 1],
                                                              acc[c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < CB; ++c)
              acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ol[(t + 2 * c) & 7], bh[t & 1],
                                                              acc[c], 0, 0, 0);
          }
        }
      }

      // ---- epilogue: distances of the 4 column blocks ------------------------------
      // lane (rl, h), register v of block c: column j0 + 32 c + 8 (v / 4) + 4 h + v % 4
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int32_t jb = j0 + 32 * c;
        const bool clean = (jb + BM <= jlim) && ((jb >= (int32_t)r0 + BM - 1 + n) ||
                                                 (jb + BM - 1 + n <= (int32_t)r0));
        float d[16];
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
          const int lc = 32 * c + 8 * qd + 4 * h;
          const float4 xj = *reinterpret_cast<const float4*>(cst + lc);
          const float xjv[4] = {xj.x, xj.y, xj.z, xj.w};
          if (Z) {
            // |a r_i|^2 + |b r_j|^2 + r_i r_j acc,  acc = -2 (P - n m_i m_j)
            const float4 cn = *reinterpret_cast<const float4*>(cst + TC + lc);
            const float cnv[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
              d[4 * qd + e] = __builtin_fmaf(xi * xjv[e], acc[c][4 * qd + e], ci + cnv[e]);
          } else {
            // acc = |a|^2 + |b|^2 - 2 P + 2 n m_i m_j;  d^2 = acc + (smu_i - smu_j)^2
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float u = xi - xjv[e];
              d[4 * qd + e] = __builtin_fmaf(u, u, acc[c][4 * qd + e]);
            }
          }
        }
        if (!clean) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int32_t j = jb + 8 * (v >> 2) + 4 * h + (v & 3);
            const int32_t dij = i > j ? i - j : j - i;
            if (!(j < jlim && dij >= n)) d[v] = __builtin_inff();
          }
        }
        float tmin = d[0];
#pragma unroll
        for (int v = 1; v < 16; ++v) tmin = fminf(tmin, d[v]);
        if (tmin < rmin) {
          int32_t jj = -1;
#pragma unroll
          for (int v = 15; v >= 0; --v)
            if (d[v] == tmin) jj = jb + 8 * (v >> 2) + 4 * h + (v & 3);
          rmin = tmin;
          rj = jj;
        }
        if ((valid >> rl) & 1u) {
          if (clean) {
            cnt += 16;
          } else {
#pragma unroll
            for (int v = 0; v < 16; ++v) cnt += d[v] < __builtin_inff();
          }
        }
      }
      // ---- early abandon ----------------------------------------------------------
      if (J.abandon) {
        const float m = fminf(rmin, __shfl_xor(rmin, 32, 64));
        const uint32_t dead = (uint32_t)(__ballot(m < bsf_now && h == 0) & 0xFFFFFFFFull) & live;
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
    }
    // the next step's first barrier makes these flags visible; they alternate
    // between two rows, read after that barrier and rewritten only after the
    // following one
    if (lane == 0) wave_live[((s + 1) & 1) * W + wv] = live ? 1u : 0u;
  }

  // ---- publish --------------------------------------------------------------------
  if (valid) {
    // (the split products can round a near-zero distance below zero; keys hold
    // non-negative distances so that they order like the values)
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

  // the item's last chunk to finish decides: complete rows raise the
  // best-so-far with their minimum over all launches; rows still live after a
  // non-final launch make the item a survivor.  With one chunk each wavefront
  // decides on its own rows (it reads back only what it published itself), so
  // only several chunks need the fence and the barrier.
  if (J.chunks > 1) {
    __threadfence();
    __syncthreads();                            // every wavefront has published
    if (threadIdx.x == 0) {
      const uint32_t prev = atomicAdd(&J.done[item], 1u);
      const bool last = prev + 1 == (uint32_t)J.chunks;
      if (last) atomicExch(&J.done[item], 0u);   // ready for the next launch
      tail[W] = last ? 1u : 0u;
    }
    __syncthreads();
    if (!tail[W]) return;
    __threadfence();
  }
  uint32_t fin = 0;
  if (valid)
    fin = J.chunks > 1 ? __builtin_amdgcn_readfirstlane(load_relaxed(&J.alive[g])) & valid : live;
  if (final) {
    if (fin && h == 0 && ((fin >> rl) & 1u)) {
      const uint64_t k = load_relaxed64(&J.best[r0 + rl]);
      if (k != kEmptyMin)
        atomicMax(J.bsf, __builtin_bit_cast(uint32_t,
                                            fmaxf(key_dist(k) * J.raise_scale - J.raise_sub, 0.0f)));
    }
    return;
  }
  if (lane == 0) tail[wv] = fin ? 1u : 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    bool any = false;
    for (int w = 0; w < W; ++w) any |= tail[w] != 0;
    if (any) J.survivors[atomicAdd(J.n_survivors, 1u)] = (int32_t)item;
  }
}

// One workgroup per work item (item, chunk), striding by the grid size.  Every
// wavefront finishes its LDS reads before the next item rebuilds the stretches.
template <bool Z, int PFE, bool SHARE>
__global__ __launch_bounds__(THREADS, 2) void k_scan_mfma(ScanJob Jarg, MixedRows R) {
  extern __shared__ bf16x8 smem[];
  ScanJob J = Jarg;
  apply_win(J);
  const int64_t total = J.n_groups * J.chunks;
  for (int64_t wi = blockIdx.x; wi < total; wi += gridDim.x) {
    scan_item<Z, PFE, SHARE>(J, R, wi, smem);
    if (wi + gridDim.x < total) __syncthreads();
  }
}

template <bool Z, int PFE, bool SHARE>
void launch_scan(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  const int64_t blocks = J.win ? J.max_work : J.n_groups * J.chunks;
  if (blocks <= 0) return;
  const size_t lds = lds_bytes((J.n + 15) / 16);
  // the LDS opt-in is per kernel and set once per process, to the largest
  // window's need; the initialisation of a function-local static is thread-safe
  static const bool attr_set = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan_mfma<Z, PFE, SHARE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes(kMixedMaxN / 16));
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL((k_scan_mfma<Z, PFE, SHARE>), dim3((unsigned)blocks), dim3(THREADS), lds, s,
                     J, R);
}

}  // namespace

bool launch_scan_mfma(const ScanJob& J, const MixedRows& R, hipStream_t s) {
  if (J.n < 1 || J.n > kMixedMaxN) return false;
  // stretches of up to 512 entries (windows up to 384) prefetch a step ahead
  const bool pf = stretch_entries((J.n + 15) / 16) <= 2 * THREADS;
  const bool ab = J.abandon != 0;
  if (R.r) {
    if (pf)
      ab ? launch_scan<true, 2, true>(J, R, s) : launch_scan<true, 2, false>(J, R, s);
    else
      ab ? launch_scan<true, 0, true>(J, R, s) : launch_scan<true, 0, false>(J, R, s);
  } else {
    if (pf)
      ab ? launch_scan<false, 2, true>(J, R, s) : launch_scan<false, 2, false>(J, R, s);
    else
      ab ? launch_scan<false, 0, true>(J, R, s) : launch_scan<false, 0, false>(J, R, s);
  }
  return true;
}

}  // namespace dd
