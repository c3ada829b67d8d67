// spiral.hpp -- the near-first column order of the pair scan.
//
// For a work item covering rows [r0, r1) the column blocks of width W are
// visited outward from the rows: forward from the block holding column r0 + n,
// backward from the block holding column r1 - 1 - n, alternating one block from
// each side and continuing with the longer side when the shorter one runs out.
// The blocks strictly between the two starts hold only columns within n - 1 of
// every row of the item (non-self matches need |i - j| >= n), so they are left
// out; every other block is visited exactly once.  The order changes only when
// rows meet a neighbour closer than the best-so-far, never which pairs exist.
//
// constexpr functions are usable from host and device code alike.
#pragma once

#include <cstdint>

namespace dd {

struct Spiral {
  int64_t qf0;   // first forward block
  int64_t qb0;   // first backward block (blocks qb0, qb0 - 1, ..., 0)
  int64_t nf;    // forward blocks: qf0 .. NQ - 1
  int64_t nb;    // backward blocks
};

constexpr int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

constexpr Spiral make_spiral(int64_t r0, int64_t r1, int64_t n, int64_t NQ, int64_t W) {
  int64_t qf0 = floor_div(r0 + n, W);
  int64_t qb0 = floor_div(r1 - 1 - n, W);
  if (qf0 > NQ) qf0 = NQ;
  if (qb0 >= qf0) qb0 = qf0 - 1;          // wide items: no block is excluded for all rows
  Spiral s{qf0, qb0, NQ - qf0, qb0 + 1};
  if (s.nb < 0) s.nb = 0;
  return s;
}

constexpr int64_t spiral_count(const Spiral& s) { return s.nf + s.nb; }

// The p-th block of the order, 0 <= p < spiral_count(s).
constexpr int64_t spiral_block(const Spiral& s, int64_t p) {
  const int64_t m2 = s.nf < s.nb ? s.nf : s.nb;
  if (p < 2 * m2) return (p & 1) ? s.qb0 - (p >> 1) : s.qf0 + (p >> 1);
  const int64_t r = p - m2;
  return s.nf > s.nb ? s.qf0 + r : s.qb0 - r;
}

}  // namespace dd
