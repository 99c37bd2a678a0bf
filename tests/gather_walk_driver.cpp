// Test driver (CPU): runs the gathered-update walk of hth_kernels.h
// (GatherWalk) on cases read from stdin and prints its entries, for
// tests/test_gather_walk.py to check against the definition.
//
// Input, per case: xb e0 carry_len n len_1 .. len_n.  Output, per case, in
// walk order: "B x L k off" for a block of 8^L executions starting at
// execution x, byte off of piece k (1-based); "J j s" for join j at offset s
// of the concatenation; then "N nfull nj".
#include <cstdint>
#include <cstdio>
#include <vector>

#include "hth_kernels.h"

int main() {
  unsigned long long xb, e0, carry;
  unsigned n;
  while (std::scanf("%llu %llu %llu %u", &xb, &e0, &carry, &n) == 4) {
    std::vector<unsigned long long> len(n);
    unsigned long long total = 0;
    for (unsigned k = 0; k < n; ++k) {
      if (std::scanf("%llu", &len[k]) != 1) return 1;
      total += len[k];
    }
    // the pieces in one buffer, 64 bytes apart (only addresses are used)
    std::vector<uint8_t> buf(total + 64 * (n + 1));
    std::vector<const uint8_t*> at(n);
    unsigned long long o = 0;
    for (unsigned k = 0; k < n; ++k) {
      at[k] = buf.data() + o + 64 * (k + 1);
      o += len[k];
    }
    hth::GatherWalk w(xb, e0, carry);
    unsigned k = 0;
    auto block = [&](uint64_t x, int L, const uint8_t* p) {
      std::printf("B %llu %d %u %lld\n", (unsigned long long)x, L, k + 1, (long long)(p - at[k]));
    };
    auto join = [&](uint32_t j, uint64_t s) { std::printf("J %u %llu\n", j, (unsigned long long)s); };
    for (k = 0; k < n; ++k) w.piece(at[k], len[k], block, join);
    const uint64_t nfull = w.finish(join);
    std::printf("N %llu %u\n", (unsigned long long)nfull, w.nj);
  }
  return 0;
}
