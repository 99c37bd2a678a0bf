/*
 * HalftimeHash CPU oracle: public declarations.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle/hth_oracle.c form a
 * plain, slow, single-threaded reference of the hash family, written from the
 * paper's definitions.  It shares no code, header, table or generator with the
 * GPU library under paper_2104_08865_amd/.  Only tests/, the smoke check and the
 * benchmark's CPU-baseline leg load it.
 *
 * Word conventions (paper §2): a "half word" has W bits (W = 32 for the real
 * family); a data word is a pair of half words, low half first, stored in a
 * uint64_t.  All sums are taken modulo 2^(2W).  The real family uses W = 32;
 * the toy widths W = 4 and W = 8 exist only so that tests can measure
 * collision probabilities exhaustively or by Monte Carlo.
 *
 * Status returns: 0 on success, -1 on an invalid argument.
 */
#ifndef HTH_ORACLE_H
#define HTH_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fixed family shape: b = 8 words per block (the 512-bit "v4" block of §6.3),
   w = 3 words per code symbol, fanout f = 8, 20 tree levels of seed. */
#define HTH_REF_B 8u
#define HTH_REF_W 3u
#define HTH_REF_F 8u
#define HTH_REF_LMAX 20u

/* Shape of one output width (16, 24, 32 or 40 bytes).  Writes
   {d, e, k, w} to out[0..3].  Returns -1 for an unsupported width. */
int hth_ref_shape(uint32_t out_width, uint32_t out[4]);

/* The oracle's own code and combine tables of one width: P_out receives the
   (k-1) x d GF(8) parity matrix, T_out the k x e combine matrix, row-major. */
int hth_ref_tables(uint32_t out_width, uint32_t *P_out, uint32_t *T_out);

/* Number of entropy words one width needs for block size b and fanout f,
   and the offsets of its five parts.  offs = {ehc, tree, final, tail, len,
   total}.  The standard layout uses b = 8, f = 8. */
int hth_ref_layout(uint32_t out_width, uint32_t b, uint32_t f, uint64_t offs[6]);

/* Total entropy words of the standard layout (all four widths concatenated in
   the order 16, 24, 32, 40) and the offset of one width's block inside it. */
uint64_t hth_ref_entropy_words(void);
int64_t hth_ref_entropy_offset(uint32_t out_width);

/* splitmix64 expansion of a user seed into the standard entropy layout:
   words[i] = i-th output of splitmix64 started at state user_seed.
   `words` must hold hth_ref_entropy_words() words. */
void hth_ref_expand_seed(uint64_t user_seed, uint64_t *words);

/* NH on a single data word against a single seed word (§3.2), for half-word
   width W in 1..32.  out[i] = NH(x[i], s[i]). */
uint64_t hth_ref_nh(uint32_t W, uint64_t x, uint64_t s);
void hth_ref_nh_batch(uint32_t W, const uint64_t *x, const uint64_t *s,
                      uint64_t *out, size_t n);

/* GF(8) product, modulus x^3 + x + 1. */
uint32_t hth_ref_gf8_mul(uint32_t a, uint32_t b);

/* Encode step of EHC for one instance: X holds d*w words (item-major: word u
   of item c at X[c*w + u]); Y receives e*w words.  n instances back to back. */
int hth_ref_encode_batch(uint32_t out_width, uint32_t W, const uint64_t *X,
                         uint64_t *Y, size_t n);

/* Full EHC of one instance: encode, hash every code symbol with NH against
   S_ehc (e*w seed words), combine with T.  Writes k words to z. */
int hth_ref_ehc(uint32_t out_width, uint32_t W, const uint64_t *X,
                const uint64_t *S_ehc, uint64_t *z);

/* Generic form of the whole hash over a sequence of data words, for the
   test-only toy parameters (W, b, f).  `entropy` is one width's block in the
   layout hth_ref_layout(out_width, b, f) describes.  `n_exec` is the number
   of full EHC executions to run (at most nwords / (b*d*w)); the remaining
   words form the tail.  `len_value` is the length word hashed into the
   output.  Writes k words to out.  recursive != 0 selects the top-down
   recursive formulation of the tree instead of the streaming stack. */
int hth_ref_hash_words(uint32_t out_width, uint32_t W, uint32_t b, uint32_t f,
                       const uint64_t *entropy, const uint64_t *words,
                       uint64_t nwords, uint64_t n_exec, uint64_t len_value,
                       int recursive, uint64_t *out);

/* The real family on a byte string: entropy is the whole standard layout
   (hth_ref_entropy_words() words; n_words is checked), data[0, len) the
   string, out receives out_width bytes (k little-endian 64-bit words). */
int hth_ref_hash(const uint64_t *entropy, size_t n_words, const uint8_t *data,
                 uint64_t len, uint32_t out_width, uint8_t *out);

/* Many strings of one buffer: string i = data[offsets[i], +lengths[i]),
   result i at out + i*out_width.  Strings are split over `nthreads` host
   threads (each string is still hashed by the single-threaded routine). */
int hth_ref_hash_batch(const uint64_t *entropy, size_t n_words,
                       const uint8_t *data, const uint64_t *offsets,
                       const uint64_t *lengths, uint64_t count,
                       uint32_t out_width, uint8_t *out, uint32_t nthreads);

/* The same for block size b = 4 or 8 (§6.3: b is the machine's vector width
   in 64-bit words, and each b defines its own family; b = 8 is the standard
   layout above).  The layout for b has the four widths' blocks of
   hth_ref_layout(width, b, 8) back to back; the seed expansion fills it from
   one splitmix64 stream.  Invalid b: 0 words / offset -1 / status -1. */
uint64_t hth_ref_entropy_words_b(uint32_t b);
int64_t hth_ref_entropy_offset_b(uint32_t out_width, uint32_t b);
void hth_ref_expand_seed_b(uint64_t user_seed, uint32_t b, uint64_t *words);
int hth_ref_hash_b(const uint64_t *entropy, size_t n_words, const uint8_t *data,
                   uint64_t len, uint32_t out_width, uint32_t b, uint8_t *out);
int hth_ref_hash_batch_b(const uint64_t *entropy, size_t n_words,
                         const uint8_t *data, const uint64_t *offsets,
                         const uint64_t *lengths, uint64_t count,
                         uint32_t out_width, uint32_t b, uint8_t *out,
                         uint32_t nthreads);

/* Composition with a short-input family (§1: a universe-collapsing family
   reduces long strings to a few bytes that a short-input family then hashes
   as if they were the input; §7 lists pairing HalftimeHash with a fast
   short-input family as future work).  The short-input family is simple
   tabulation over c + 1 byte characters, c = inner_width (16/24/32/40):
   tables[i*256 + v] = T_i[v] for i in [0, c].  The key of a string x of L
   bytes is
     L <= c:  chars 0..c-1 = x zero-padded to c bytes, char c = L;
     L >  c:  chars 0..c-1 = the c bytes of HalftimeHash (inner width c,
              block size b) of x, char c = 255;
   and the 64-bit result is the XOR of T_i[char i] over i = 0..c.  The two
   kinds of key always differ in char c.
   hth_ref_tab_words: (c + 1) * 256, or 0 for an unsupported width.
   hth_ref_tab_expand: tables[i] = i-th output of splitmix64 started at
   user_seed (the same generator as the entropy expansion; use a seed
   independent of the hashing seed's). */
size_t hth_ref_tab_words(uint32_t inner_width);
int hth_ref_tab_expand(uint64_t user_seed, uint32_t inner_width, uint64_t *tables);
int hth_ref_hash64_b(const uint64_t *entropy, size_t n_words, const uint64_t *tables,
                     size_t n_tab, const uint8_t *data, uint64_t len,
                     uint32_t inner_width, uint32_t b, uint64_t *out);
int hth_ref_hash64_batch_b(const uint64_t *entropy, size_t n_words,
                           const uint64_t *tables, size_t n_tab,
                           const uint8_t *data, const uint64_t *offsets,
                           const uint64_t *lengths, uint64_t count,
                           uint32_t inner_width, uint32_t b, uint64_t *out,
                           uint32_t nthreads);

/* Multiplication counters of the last hth_ref_hash_words / hth_ref_hash call
   on this thread: {ehc, tree, final, tail, length}. */
void hth_ref_mul_counts(uint64_t out[5]);

#ifdef __cplusplus
}
#endif
#endif
