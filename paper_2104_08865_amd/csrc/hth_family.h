// HalftimeHash family constants for the GPU path (compile-time tables).
//
// The family (paper §5.1, §6.1): b = 8 words per block (the 512-bit "v4"
// block), w = 3 words per code symbol, fanout f = 8, and per output width
// (d, e, k) = (6,7,2), (7,9,3), (7,10,4), (5,9,5) for 16/24/32/40 bytes.
// The combine matrices T are the ones printed in §5.1.  The erasure codes are
// systematic GF(8) MDS codes (the paper's own codes are not printed); parity
// word u of parity item r is the sum mod 2^64 of the input words (c, v) for
// which bit u of P[r][c] * x^v is set, GF(8) = GF(2)[x]/(x^3 + x + 1).
//
// Entropy layout of one width (64-bit words):
//   [ehc: e*w][tree: k*20*7][final: k*20*7*8][tail: 8*d*w + k - 1][len: k]
// and the four widths are stored back to back in the order 16, 24, 32, 40.
#pragma once
#include <cstdint>

namespace hth {

constexpr int kBlock = 8;    // b: 64-bit words per block
constexpr int kSym = 3;      // w: words per code symbol
constexpr int kFan = 8;      // f: tree fanout
constexpr int kLevels = 20;  // tree levels that carry keys

template <int WIDTH>
struct Family;

template <>
struct Family<16> {
  static constexpr int D = 6, E = 7, K = 2;
  static constexpr uint8_t P[4][7] = {{1, 1, 1, 1, 1, 1}};
  static constexpr uint8_t T[5][10] = {{1, 0, 1, 1, 2, 1, 4}, {0, 1, 1, 2, 1, 4, 1}};
};
template <>
struct Family<24> {
  static constexpr int D = 7, E = 9, K = 3;
  static constexpr uint8_t P[4][7] = {{1, 4, 1, 2, 1, 5, 1}, {1, 5, 4, 5, 2, 4, 5}};
  static constexpr uint8_t T[5][10] = {
      {0, 0, 1, 4, 1, 1, 2, 2, 1}, {1, 1, 0, 0, 1, 4, 1, 2, 2}, {1, 4, 1, 1, 0, 0, 2, 1, 2}};
};
template <>
struct Family<32> {
  static constexpr int D = 7, E = 10, K = 4;
  static constexpr uint8_t P[4][7] = {
      {4, 3, 1, 1, 5, 1, 1}, {1, 1, 5, 4, 4, 2, 1}, {1, 5, 1, 5, 1, 6, 4}};
  static constexpr uint8_t T[5][10] = {{0, 0, 0, 1, 1, 4, 2, 4, 1, 1},
                                       {0, 1, 2, 0, 0, 1, 1, 2, 4, 1},
                                       {2, 0, 1, 0, 4, 0, 1, 1, 1, 1},
                                       {1, 1, 0, 1, 0, 0, 4, 1, 2, 8}};
};
template <>
struct Family<40> {
  static constexpr int D = 5, E = 9, K = 5;
  static constexpr uint8_t P[4][7] = {
      {1, 4, 2, 1, 5}, {6, 2, 5, 1, 1}, {1, 5, 5, 2, 4}, {2, 5, 2, 5, 2}};
  static constexpr uint8_t T[5][10] = {{1, 0, 0, 0, 0, 1, 1, 2, 4},
                                       {0, 1, 0, 0, 0, 1, 2, 1, 7},
                                       {0, 0, 1, 0, 0, 1, 3, 8, 5},
                                       {0, 0, 0, 1, 0, 1, 4, 9, 8},
                                       {0, 0, 0, 0, 1, 1, 5, 3, 9}};
};

// Product in GF(8) with modulus x^3 + x + 1 (carry-less multiply, reduce).
constexpr unsigned gf8_mul(unsigned a, unsigned b) {
  unsigned r = 0;
  for (int i = 0; i < 3; ++i)
    if ((b >> i) & 1u) r ^= a << i;
  if (r & 16u) r ^= 0x16u;  // x^4 = x^2 + x
  if (r & 8u) r ^= 0xBu;    // x^3 = x + 1
  return r & 7u;
}

// Does parity word u of (a * X) include input word v?
constexpr bool image_bit(unsigned a, int u, int v) { return (gf8_mul(a, 1u << v) >> u) & 1u; }

// Entropy layout of one width for block size B (64-bit words per block:
// 8 for the 512-bit family, 4 for the 256-bit one; §6.3): EHC keys, tree
// keys, final keys (per instance), Toeplitz tail keys, length keys.
template <int WIDTH, int B = kBlock>
struct Layout {
  using F = Family<WIDTH>;
  static constexpr int ehc = 0;
  static constexpr int tree = ehc + F::E * kSym;
  static constexpr int fin = tree + F::K * kLevels * (kFan - 1);
  static constexpr int tail = fin + F::K * kLevels * (kFan - 1) * B;
  static constexpr int len = tail + B * F::D * kSym + F::K - 1;
  static constexpr int total = len + F::K;
  static constexpr int exec_bytes = 8 * B * F::D * kSym;
  static constexpr int exec_words = B * F::D * kSym;
};

// The four widths' blocks back to back, in the order 16, 24, 32, 40.
template <int B = kBlock>
constexpr int width_offset(int width) {
  return width == 16   ? 0
         : width == 24 ? Layout<16, B>::total
         : width == 32 ? Layout<16, B>::total + Layout<24, B>::total
         : width == 40 ? Layout<16, B>::total + Layout<24, B>::total + Layout<32, B>::total
                       : -1;
}
template <int B = kBlock>
constexpr int entropy_words() {
  return Layout<16, B>::total + Layout<24, B>::total + Layout<32, B>::total + Layout<40, B>::total;
}
constexpr int kEntropyWords = entropy_words<8>();
static_assert(kEntropyWords == 18369, "entropy layout size, b = 8");
static_assert(entropy_words<4>() == 10229, "entropy layout size, b = 4");

}  // namespace hth
