// Exhaustive host check of the near-first column order (csrc/spiral.hpp) on small
// sizes: the order visits every column block that holds a non-self match of
// some row of the item exactly once, visits only blocks inside the matrix,
// leaves out only blocks whose every column lies within n - 1 of every row, and
// on each side visits blocks in order of distance from the item.
//
// Build (done by tests/test_abi_cpu.py):
//   g++ -std=c++17 -O2 tests/native/spiral_check.cpp -o spiral_check
#include <cstdio>
#include <vector>

#include "../../paper_1901_00155_amd/csrc/spiral.hpp"

int main() {
  long cases = 0, errors = 0;
  for (int64_t N = 1; N <= 140; N += (N < 40 ? 1 : 7)) {
    for (int64_t W : {1, 8, 32}) {
      const int64_t NQ = (N + W - 1) / W;
      for (int64_t n = 1; n <= 40; n += (n < 10 ? 1 : 5)) {
        for (int64_t r0 = 0; r0 < N; r0 += 3) {
          for (int64_t len : {1, 8, 32, 64}) {
            const int64_t r1 = r0 + len;            // may pass N, as the last item does
            const dd::Spiral s = dd::make_spiral(r0, r1, n, NQ, W);
            ++cases;
            std::vector<int> seen(NQ, 0);
            int64_t last_f = -1, last_b = NQ;
            bool bad = false;
            for (int64_t p = 0; p < dd::spiral_count(s); ++p) {
              const int64_t q = dd::spiral_block(s, p);
              if (q < 0 || q >= NQ) { bad = true; break; }
              if (seen[q]++) bad = true;
              if (q >= s.qf0) { if (q <= last_f) bad = true; last_f = q; }
              else { if (q >= last_b) bad = true; last_b = q; }
            }
            for (int64_t q = 0; q < NQ && !bad; ++q) {
              bool needed = false;
              for (int64_t j = q * W; j < (q + 1) * W && j < N; ++j)
                for (int64_t i = r0; i < r1 && i < N; ++i)
                  if ((i > j ? i - j : j - i) >= n) needed = true;
              if (needed && !seen[q]) bad = true;
            }
            if (bad) {
              if (errors < 10)
                std::printf("FAIL N=%lld W=%lld n=%lld rows=[%lld,%lld)\n", (long long)N,
                            (long long)W, (long long)n, (long long)r0, (long long)r1);
              ++errors;
            }
          }
        }
      }
    }
  }
  std::printf("cases %ld errors %ld\n", cases, errors);
  if (!errors) std::printf("OK\n");
  return errors ? 1 : 0;
}
