/*
 * HalftimeHash CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded reference of the
 * hash family H(s, x) of the paper (§1: a map from seeds and strings to a
 * 16/24/32/40-byte codomain).  It follows the paper's steps in its order and
 * notation and is deliberately unoptimised.  It shares no code with the GPU
 * library; only tests/, the smoke check and the benchmark's CPU-baseline leg
 * use it.
 *
 * Steps (one width; k = out_width / 8):
 *   1. the string is read as little-endian 64-bit words, zero padded;
 *   2. it is cut into full EHC executions of b*d*w words plus a tail (§6.1);
 *   3. each execution holds b instances; instance j owns word j of every
 *      b-word block (§2: instances are logically contiguous, physically
 *      strided);
 *   4. Encode (§3.3, §5.1): d items of w words -> e items, a systematic code
 *      of minimum distance k whose parity symbols are sums mod 2^64 of input
 *      words chosen by the binary image of a GF(8) parity matrix;
 *   5. Hash (§3.3): every encoded word goes through NH (§3.2) against its own
 *      seed word; the w NH values of an item are summed;
 *   6. Combine (§4, §5.1): the k x e matrix T printed in §5.1;
 *   7. Tree (§5.2): each of the k outputs feeds its own f-ary tree whose nodes
 *      are the NH variant of §3.2 that leaves the last word unhashed; the
 *      stack construction of Eq. (3), taken in base f, leaves one partial
 *      level per base-f digit of the number of executions;
 *   8. the leftover items of every tree are hashed by one NH (§5.2);
 *   9. the tail words are hashed by NH k times with Toeplitz-shifted keys
 *      (§6.1);
 *  10. the length is hashed by NH and added, so that strings of different
 *      lengths also separate (§2 asks for the length to be appended).
 * The readings taken where the paper leaves a choice open are listed in the
 * design notes of the repository.
 */
#include "hth_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Family tables.                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    unsigned width, d, e, k;
    /* Parity matrix over GF(8), (k-1) x d.  Row r gives parity item d + r. */
    unsigned P[4][7];
    /* Combine matrix T, k x e, exactly as printed in §5.1. */
    unsigned T[5][10];
} ref_shape;

static const ref_shape SHAPES[4] = {
    /* HalftimeHash16: distance-2 code = one parity item, the plain sum. */
    {16, 6, 7, 2,
     {{1, 1, 1, 1, 1, 1}},
     {{1, 0, 1, 1, 2, 1, 4},
      {0, 1, 1, 2, 1, 4, 1}}},
    /* HalftimeHash24: (9,7) code of distance 3. */
    {24, 7, 9, 3,
     {{1, 4, 1, 2, 1, 5, 1},
      {1, 5, 4, 5, 2, 4, 5}},
     {{0, 0, 1, 4, 1, 1, 2, 2, 1},
      {1, 1, 0, 0, 1, 4, 1, 2, 2},
      {1, 4, 1, 1, 0, 0, 2, 1, 2}}},
    /* HalftimeHash32: (10,7) code of distance 4. */
    {32, 7, 10, 4,
     {{4, 3, 1, 1, 5, 1, 1},
      {1, 1, 5, 4, 4, 2, 1},
      {1, 5, 1, 5, 1, 6, 4}},
     {{0, 0, 0, 1, 1, 4, 2, 4, 1, 1},
      {0, 1, 2, 0, 0, 1, 1, 2, 4, 1},
      {2, 0, 1, 0, 4, 0, 1, 1, 1, 1},
      {1, 1, 0, 1, 0, 0, 4, 1, 2, 8}}},
    /* HalftimeHash40: (9,5) code of distance 5. */
    {40, 5, 9, 5,
     {{1, 4, 2, 1, 5},
      {6, 2, 5, 1, 1},
      {1, 5, 5, 2, 4},
      {2, 5, 2, 5, 2}},
     {{1, 0, 0, 0, 0, 1, 1, 2, 4},
      {0, 1, 0, 0, 0, 1, 2, 1, 7},
      {0, 0, 1, 0, 0, 1, 3, 8, 5},
      {0, 0, 0, 1, 0, 1, 4, 9, 8},
      {0, 0, 0, 0, 1, 1, 5, 3, 9}}},
};

static const ref_shape *shape_of(uint32_t out_width)
{
    for (int i = 0; i < 4; i++)
        if (SHAPES[i].width == out_width) return &SHAPES[i];
    return NULL;
}

int hth_ref_tables(uint32_t out_width, uint32_t *P_out, uint32_t *T_out)
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || !P_out || !T_out) return -1;
    for (unsigned r = 0; r + 1 < sh->k; r++)
        for (unsigned c = 0; c < sh->d; c++) P_out[r * sh->d + c] = sh->P[r][c];
    for (unsigned t = 0; t < sh->k; t++)
        for (unsigned c = 0; c < sh->e; c++) T_out[t * sh->e + c] = sh->T[t][c];
    return 0;
}

int hth_ref_shape(uint32_t out_width, uint32_t out[4])
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || !out) return -1;
    out[0] = sh->d;
    out[1] = sh->e;
    out[2] = sh->k;
    out[3] = HTH_REF_W;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Entropy layout.  One width's block is                                     */
/*   [S_ehc: e*w][S_tree: k*LMAX*(f-1)][S_final: k*LMAX*(f-1)*b]              */
/*   [S_tail: b*d*w + k - 1][S_len: k]                                       */
/* (§6.2 lists the same five consumers of input entropy).                    */
/* ------------------------------------------------------------------------ */

int hth_ref_layout(uint32_t out_width, uint32_t b, uint32_t f, uint64_t offs[6])
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || !offs || b == 0 || f < 2) return -1;
    uint64_t w = HTH_REF_W, L = HTH_REF_LMAX;
    offs[0] = 0;
    offs[1] = offs[0] + (uint64_t)sh->e * w;
    offs[2] = offs[1] + (uint64_t)sh->k * L * (f - 1);
    offs[3] = offs[2] + (uint64_t)sh->k * L * (f - 1) * b;
    offs[4] = offs[3] + (uint64_t)b * sh->d * w + sh->k - 1;
    offs[5] = offs[4] + sh->k;
    return 0;
}

/* The standard layout for block size b: the four widths' blocks back to
   back, in the order 16, 24, 32, 40.  b = 8 is the 512-bit block of the
   paper's default variant, b = 4 the 256-bit one (§6.3: b follows the
   vector width of the machine, and each b is its own family). */
static int block_ok(uint32_t b) { return b == 4 || b == 8; }

uint64_t hth_ref_entropy_words_b(uint32_t b)
{
    if (!block_ok(b)) return 0;
    uint64_t total = 0, offs[6];
    for (int i = 0; i < 4; i++) {
        hth_ref_layout(SHAPES[i].width, b, HTH_REF_F, offs);
        total += offs[5];
    }
    return total;
}
int64_t hth_ref_entropy_offset_b(uint32_t out_width, uint32_t b)
{
    if (!block_ok(b)) return -1;
    uint64_t at = 0, offs[6];
    for (int i = 0; i < 4; i++) {
        if (SHAPES[i].width == out_width) return (int64_t)at;
        hth_ref_layout(SHAPES[i].width, b, HTH_REF_F, offs);
        at += offs[5];
    }
    return -1;
}
uint64_t hth_ref_entropy_words(void) { return hth_ref_entropy_words_b(HTH_REF_B); }
int64_t hth_ref_entropy_offset(uint32_t out_width) { return hth_ref_entropy_offset_b(out_width, HTH_REF_B); }
void hth_ref_expand_seed_b(uint64_t user_seed, uint32_t b, uint64_t *words)
{
    uint64_t n = hth_ref_entropy_words_b(b);
    uint64_t state = user_seed;
    for (uint64_t i = 0; i < n; i++) {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        words[i] = z ^ (z >> 31);
    }
}
void hth_ref_expand_seed(uint64_t user_seed, uint64_t *words) { hth_ref_expand_seed_b(user_seed, HTH_REF_B, words); }

/* ------------------------------------------------------------------------ */
/* Arithmetic.                                                               */
/* ------------------------------------------------------------------------ */

static uint64_t half_mask(unsigned W) { return W >= 32 ? 0xFFFFFFFFULL : ((1ULL << W) - 1); }
static uint64_t word_mask(unsigned W) { return W >= 32 ? ~0ULL : ((1ULL << (2 * W)) - 1); }

static __thread uint64_t mul_count[5];
enum { MUL_EHC, MUL_TREE, MUL_FINAL, MUL_TAIL, MUL_LEN };

/* NH (§3.2) on one pair (d_2i, d_2i+1) = (low half, high half) of a data word
   x, with seed pair (s_2i, s_2i+1) taken the same way from s:
   (d_2i + s_2i)(d_2i+1 + s_2i+1), halves added in Z_2^W, product in Z_2^2W. */
static uint64_t nh(unsigned W, uint64_t x, uint64_t s)
{
    uint64_t hm = half_mask(W);
    uint64_t lo = ((x & hm) + (s & hm)) & hm;
    uint64_t hi = (((x >> W) & hm) + ((s >> W) & hm)) & hm;
    return (lo * hi) & word_mask(W);
}

static uint64_t nh_counted(unsigned W, uint64_t x, uint64_t s, int what)
{
    mul_count[what]++;
    return nh(W, x, s);
}

uint64_t hth_ref_nh(uint32_t W, uint64_t x, uint64_t s)
{
    if (W == 0 || W > 32) return 0;
    return nh(W, x, s);
}

void hth_ref_nh_batch(uint32_t W, const uint64_t *x, const uint64_t *s, uint64_t *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = hth_ref_nh(W, x[i], s[i]);
}

/* GF(8) = GF(2)[x] / (x^3 + x + 1).  An element is a 3-bit integer whose bit
   i is the coefficient of x^i. */
uint32_t hth_ref_gf8_mul(uint32_t a, uint32_t b)
{
    uint32_t r = 0;
    for (int i = 0; i < 3; i++)
        if ((b >> i) & 1u) r ^= a << i;
    for (int i = 4; i >= 3; i--)
        if ((r >> i) & 1u) r ^= 0xBu << (i - 3);  /* 0xB = x^3 + x + 1 */
    return r & 7u;
}

/* Entry (u, v) of the binary image of multiplication by a: bit u of a * x^v.
   A code symbol of w = 3 words plays the role of a GF(8) element whose
   coefficient of x^v is word v, so parity word u of a * X sums the words v
   with a set entry (u, v). */
static unsigned mbit(unsigned a, unsigned u, unsigned v)
{
    return (hth_ref_gf8_mul(a, 1u << v) >> u) & 1u;
}

/* ------------------------------------------------------------------------ */
/* EHC (§3.3 with the generalisation of §4; code and T of §5.1).             */
/* ------------------------------------------------------------------------ */

static void encode(const ref_shape *sh, unsigned W, const uint64_t *X, uint64_t *Y)
{
    const unsigned w = HTH_REF_W;
    uint64_t m = word_mask(W);
    /* systematic part: the first d encoded items are the input items */
    for (unsigned c = 0; c < sh->d; c++)
        for (unsigned u = 0; u < w; u++) Y[c * w + u] = X[c * w + u] & m;
    /* parity items: sums mod 2^2W of the words the binary image selects */
    for (unsigned r = 0; r + 1 < sh->k; r++)
        for (unsigned u = 0; u < w; u++) {
            uint64_t sum = 0;
            for (unsigned c = 0; c < sh->d; c++)
                for (unsigned v = 0; v < w; v++)
                    if (mbit(sh->P[r][c], u, v)) sum += X[c * w + v];
            Y[(sh->d + r) * w + u] = sum & m;
        }
}

int hth_ref_encode_batch(uint32_t out_width, uint32_t W, const uint64_t *X, uint64_t *Y, size_t n)
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || W == 0 || W > 32) return -1;
    size_t in = (size_t)sh->d * HTH_REF_W, outn = (size_t)sh->e * HTH_REF_W;
    for (size_t i = 0; i < n; i++) encode(sh, W, X + i * in, Y + i * outn);
    return 0;
}

/* One EHC execution on one instance: Encode, Hash, Combine. */
static void ehc(const ref_shape *sh, unsigned W, const uint64_t *X, const uint64_t *S_ehc, uint64_t *z)
{
    const unsigned w = HTH_REF_W;
    uint64_t m = word_mask(W);
    uint64_t Y[10 * 3], h[10];
    encode(sh, W, X, Y);
    /* Hash: item c is hashed by NH over its w words with its own seed words */
    for (unsigned c = 0; c < sh->e; c++) {
        h[c] = 0;
        for (unsigned u = 0; u < w; u++)
            h[c] = (h[c] + nh_counted(W, Y[c * w + u], S_ehc[c * w + u], MUL_EHC)) & m;
    }
    /* Combine: z = T h over Z_2^2W */
    for (unsigned t = 0; t < sh->k; t++) {
        uint64_t acc = 0;
        for (unsigned c = 0; c < sh->e; c++) acc += (uint64_t)sh->T[t][c] * h[c];
        z[t] = acc & m;
    }
}

int hth_ref_ehc(uint32_t out_width, uint32_t W, const uint64_t *X, const uint64_t *S_ehc, uint64_t *z)
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || W == 0 || W > 32) return -1;
    ehc(sh, W, X, S_ehc, z);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tree (§5.2).                                                              */
/* ------------------------------------------------------------------------ */

/* Streaming form of the stack construction: leaves arrive left to right;
   level l keeps at most f-1 pending items; the f-th arrival turns the level
   into one node of level l+1, the NH variant of §3.2 over the f items (f-1
   NH products plus the last item unhashed).  The keys of a node depend only
   on its tree t and its level l (one key per child position). */
typedef struct {
    unsigned W, f, lmax;
    const uint64_t *S_tree; /* this tree's keys: S_tree[l*(f-1) + i] */
    uint64_t *items;        /* items[l*(f-1) + i] */
    unsigned *count;        /* count[l] pending items at level l */
} tree_stack;

static void stack_push(tree_stack *st, unsigned level, uint64_t v)
{
    uint64_t m = word_mask(st->W);
    for (;;) {
        if (level >= st->lmax) abort(); /* cannot happen for lengths < 2^64 */
        unsigned f1 = st->f - 1;
        if (st->count[level] < f1) {
            st->items[level * f1 + st->count[level]] = v;
            st->count[level]++;
            return;
        }
        uint64_t node = v; /* the f-th child is added without a product */
        for (unsigned i = 0; i < f1; i++)
            node += nh_counted(st->W, st->items[level * f1 + i], st->S_tree[level * f1 + i], MUL_TREE);
        st->count[level] = 0;
        v = node & m;
        level++;
    }
}

/* Recursive form, Eq. (1) taken in base f: the root of a complete subtree of
   height `level` over leaves[0, f^level). */
static uint64_t tree_root(unsigned W, unsigned f, const uint64_t *S_tree, const uint64_t *leaves,
                          uint64_t stride, unsigned level)
{
    if (level == 0) return leaves[0];
    uint64_t sub = 1;
    for (unsigned l = 1; l < level; l++) sub *= f;
    uint64_t node = 0;
    for (unsigned i = 0; i < f; i++) {
        uint64_t child = tree_root(W, f, S_tree, leaves + i * sub * stride, stride, level - 1);
        if (i + 1 < f)
            node += nh_counted(W, child, S_tree[(level - 1) * (f - 1) + i], MUL_TREE);
        else
            node += child;
    }
    return node & word_mask(W);
}

/* ------------------------------------------------------------------------ */
/* Whole hash.                                                               */
/* ------------------------------------------------------------------------ */

static int hash_words(const ref_shape *sh, unsigned W, unsigned b, unsigned f, const uint64_t *ent,
                      const uint64_t *words, uint64_t nwords, uint64_t n_exec, uint64_t len_value,
                      int recursive, uint64_t *out)
{
    const unsigned w = HTH_REF_W, d = sh->d, k = sh->k, L = HTH_REF_LMAX;
    const uint64_t m = word_mask(W);
    const uint64_t xw = (uint64_t)b * d * w; /* words per EHC execution */
    uint64_t offs[6];
    if (hth_ref_layout(sh->width, b, f, offs)) return -1;
    if (n_exec > nwords / xw) return -1;
    const uint64_t *S_ehc = ent + offs[0], *S_tree = ent + offs[1], *S_final = ent + offs[2],
                   *S_tail = ent + offs[3], *S_len = ent + offs[4];
    memset(mul_count, 0, sizeof mul_count);

    uint64_t F[5] = {0};
    const unsigned f1 = f - 1;
    /* per (tree t, instance j) leftover items at each level */
    uint64_t *items = calloc((size_t)k * b * L * f1, sizeof(uint64_t));
    unsigned *count = calloc((size_t)k * b * L, sizeof(unsigned));
    uint64_t *leaves = NULL;
    if (!items || !count) { free(items); free(count); return -1; }
    if (recursive) {
        leaves = malloc((size_t)(n_exec ? n_exec : 1) * k * b * sizeof(uint64_t));
        if (!leaves) { free(items); free(count); return -1; }
    }

    uint64_t X[7 * 3], z[5];
    for (uint64_t g = 0; g < n_exec; g++) {
        for (unsigned j = 0; j < b; j++) {
            /* instance j of execution g: word j of each of the d*w blocks */
            for (unsigned c = 0; c < d; c++)
                for (unsigned u = 0; u < w; u++)
                    X[c * w + u] = words[g * xw + (uint64_t)(c * w + u) * b + j];
            ehc(sh, W, X, S_ehc, z);
            for (unsigned t = 0; t < k; t++) {
                if (recursive) {
                    leaves[(g * k + t) * b + j] = z[t];
                } else {
                    tree_stack st = {W, f, L, S_tree + (uint64_t)t * L * f1,
                                     items + ((uint64_t)t * b + j) * L * f1,
                                     count + ((uint64_t)t * b + j) * L};
                    stack_push(&st, 0, z[t]);
                }
            }
        }
    }

    if (recursive) {
        /* Decompose the leaves into complete subtrees from the left, largest
           first: digit_l(n_exec) subtrees of height l for every level l
           (Eq. (3) in base f).  The i-th such subtree of level l is the item
           (l, i) of the tree's output sequence. */
        uint64_t pos = 0;
        unsigned top = 0;
        uint64_t pw = 1;
        while (top + 1 < L && pw <= n_exec / f) { pw *= f; top++; }
        for (int l = (int)top; l >= 0; l--) {
            uint64_t size = 1;
            for (int q = 0; q < l; q++) size *= f;
            uint64_t digit = (n_exec / size) % f;
            for (uint64_t i = 0; i < digit; i++) {
                for (unsigned t = 0; t < k; t++)
                    for (unsigned j = 0; j < b; j++) {
                        uint64_t r = tree_root(W, f, S_tree + (uint64_t)t * L * f1,
                                               leaves + (pos * k + t) * b + j, (uint64_t)k * b,
                                               (unsigned)l);
                        items[(((uint64_t)t * b + j) * L + l) * f1 + i] = r;
                        count[((uint64_t)t * b + j) * L + l] = (unsigned)digit;
                    }
                pos += size;
            }
        }
    }

    /* Final NH over every tree's leftover items (§5.2); an absent slot adds
       nothing; the seed of slot (l, i) of instance j is S_final[t][l][i][j]. */
    for (unsigned t = 0; t < k; t++)
        for (unsigned j = 0; j < b; j++)
            for (unsigned l = 0; l < L; l++) {
                unsigned cnt = count[((uint64_t)t * b + j) * L + l];
                for (unsigned i = 0; i < cnt; i++) {
                    uint64_t item = items[(((uint64_t)t * b + j) * L + l) * f1 + i];
                    uint64_t key = S_final[(((uint64_t)t * L + l) * f1 + i) * b + j];
                    F[t] = (F[t] + nh_counted(W, item, key, MUL_FINAL)) & m;
                }
            }

    /* Tail (§6.1): words not covered by a full execution, hashed k times;
       output t uses the Toeplitz keys S_tail[t, t + R). */
    uint64_t m0 = n_exec * xw, R = nwords - m0;
    for (unsigned t = 0; t < k; t++) {
        uint64_t tl = 0;
        for (uint64_t q = 0; q < R; q++)
            tl = (tl + nh_counted(W, words[m0 + q], S_tail[t + q], MUL_TAIL)) & m;
        uint64_t ln = nh_counted(W, len_value, S_len[t], MUL_LEN);
        out[t] = (F[t] + tl + ln) & m;
    }
    free(items);
    free(count);
    free(leaves);
    return 0;
}

int hth_ref_hash_words(uint32_t out_width, uint32_t W, uint32_t b, uint32_t f, const uint64_t *entropy,
                       const uint64_t *words, uint64_t nwords, uint64_t n_exec, uint64_t len_value,
                       int recursive, uint64_t *out)
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || W == 0 || W > 32 || b == 0 || f < 2 || !entropy || !out) return -1;
    if (nwords && !words) return -1;
    uint64_t tail_cap = (uint64_t)b * sh->d * HTH_REF_W;
    if (n_exec > nwords / tail_cap) return -1;
    if (nwords - n_exec * tail_cap > tail_cap) return -1; /* tail keys would run out */
    /* the stack reaches level lmax - 1 at most while n_exec < f^(lmax - 1) */
    uint64_t cap = 1;
    for (unsigned l = 0; l + 1 < HTH_REF_LMAX && cap <= UINT64_MAX / f; l++) cap *= f;
    if (n_exec >= cap) return -1;
    return hash_words(sh, W, b, f, entropy, words, nwords, n_exec, len_value, recursive, out);
}

int hth_ref_hash_b(const uint64_t *entropy, size_t n_words, const uint8_t *data, uint64_t len,
                   uint32_t out_width, uint32_t b, uint8_t *out)
{
    const ref_shape *sh = shape_of(out_width);
    if (!sh || !block_ok(b) || !entropy || !out || n_words != hth_ref_entropy_words_b(b)) return -1;
    if (len && !data) return -1;
    /* words: little-endian 64-bit, the last one zero padded */
    uint64_t nw = (len + 7) / 8;
    uint64_t *words = malloc((size_t)(nw ? nw : 1) * sizeof(uint64_t));
    if (!words) return -1;
    for (uint64_t i = 0; i < nw; i++) {
        uint64_t v = 0;
        for (unsigned q = 0; q < 8; q++) {
            uint64_t at = i * 8 + q;
            if (at < len) v |= (uint64_t)data[at] << (8 * q);
        }
        words[i] = v;
    }
    /* full executions are counted in bytes, so a final partial word never
       completes an execution */
    uint64_t xb = 8ULL * b * sh->d * HTH_REF_W;
    uint64_t n_exec = len / xb;
    uint64_t z[5];
    const uint64_t *ent = entropy + hth_ref_entropy_offset_b(out_width, b);
    int rc = hash_words(sh, 32, b, HTH_REF_F, ent, words, nw, n_exec, len, 0, z);
    free(words);
    if (rc) return rc;
    for (unsigned t = 0; t < sh->k; t++)
        for (unsigned q = 0; q < 8; q++) out[t * 8 + q] = (uint8_t)(z[t] >> (8 * q));
    return 0;
}
int hth_ref_hash(const uint64_t *entropy, size_t n_words, const uint8_t *data, uint64_t len,
                 uint32_t out_width, uint8_t *out)
{
    return hth_ref_hash_b(entropy, n_words, data, len, out_width, HTH_REF_B, out);
}

void hth_ref_mul_counts(uint64_t out[5])
{
    for (int i = 0; i < 5; i++) out[i] = mul_count[i];
}

/* ------------------------------------------------------------------------ */
/* Harness-level parallelism over strings (verification of large batches).   */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint64_t *entropy;
    size_t n_words;
    const uint8_t *data;
    const uint64_t *offsets, *lengths;
    uint64_t count;
    uint32_t out_width, b;
    uint8_t *out;
    uint32_t nthreads, id;
    int rc;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *jb = arg;
    jb->rc = 0;
    for (uint64_t i = jb->id; i < jb->count; i += jb->nthreads) {
        int rc = hth_ref_hash_b(jb->entropy, jb->n_words, jb->data + jb->offsets[i], jb->lengths[i],
                                jb->out_width, jb->b, jb->out + i * jb->out_width);
        if (rc) jb->rc = rc;
    }
    return NULL;
}

int hth_ref_hash_batch_b(const uint64_t *entropy, size_t n_words, const uint8_t *data,
                         const uint64_t *offsets, const uint64_t *lengths, uint64_t count,
                         uint32_t out_width, uint32_t b, uint8_t *out, uint32_t nthreads)
{
    if (!shape_of(out_width) || !block_ok(b) || (count && (!offsets || !lengths || !out))) return -1;
    if (nthreads == 0) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    batch_job jobs[256];
    pthread_t th[256];
    for (uint32_t i = 0; i < nthreads; i++) {
        jobs[i] = (batch_job){entropy, n_words, data, offsets, lengths, count, out_width, b, out,
                              nthreads, i, 0};
        if (nthreads == 1) batch_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, batch_worker, &jobs[i]);
    }
    int rc = 0;
    for (uint32_t i = 0; i < nthreads; i++) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
    }
    return rc;
}
int hth_ref_hash_batch(const uint64_t *entropy, size_t n_words, const uint8_t *data,
                       const uint64_t *offsets, const uint64_t *lengths, uint64_t count,
                       uint32_t out_width, uint8_t *out, uint32_t nthreads)
{
    return hth_ref_hash_batch_b(entropy, n_words, data, offsets, lengths, count, out_width, HTH_REF_B, out,
                                nthreads);
}

/* ------------------------------------------------------------------------ */
/* Composition with simple tabulation (§1, §7 future work).                  */
/* ------------------------------------------------------------------------ */

size_t hth_ref_tab_words(uint32_t inner_width)
{
    return shape_of(inner_width) ? (size_t)(inner_width + 1) * 256 : 0;
}

int hth_ref_tab_expand(uint64_t user_seed, uint32_t inner_width, uint64_t *tables)
{
    size_t n = hth_ref_tab_words(inner_width);
    if (!n || !tables) return -1;
    uint64_t state = user_seed;
    for (size_t i = 0; i < n; i++) {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        tables[i] = z ^ (z >> 31);
    }
    return 0;
}

int hth_ref_hash64_b(const uint64_t *entropy, size_t n_words, const uint64_t *tables, size_t n_tab,
                     const uint8_t *data, uint64_t len, uint32_t inner_width, uint32_t b, uint64_t *out)
{
    const uint32_t c = inner_width;
    if (!hth_ref_tab_words(c) || n_tab != hth_ref_tab_words(c) || !tables || !out) return -1;
    if (len && !data) return -1;
    /* the key: c characters and the separator character c */
    uint8_t key[41];
    if (len <= c) {
        for (uint32_t i = 0; i < c; i++) key[i] = i < len ? data[i] : 0;
        key[c] = (uint8_t)len;
    } else {
        int rc = hth_ref_hash_b(entropy, n_words, data, len, c, b, key);
        if (rc) return rc;
        key[c] = 255;
    }
    /* simple tabulation: one table per character, results XORed */
    uint64_t z = 0;
    for (uint32_t i = 0; i <= c; i++) z ^= tables[(size_t)i * 256 + key[i]];
    *out = z;
    return 0;
}

typedef struct {
    const uint64_t *entropy, *tables;
    size_t n_words, n_tab;
    const uint8_t *data;
    const uint64_t *offsets, *lengths;
    uint64_t count;
    uint32_t width, b;
    uint64_t *out;
    uint32_t nthreads, id;
    int rc;
} hash64_job;

static void *hash64_worker(void *arg)
{
    hash64_job *jb = arg;
    jb->rc = 0;
    for (uint64_t i = jb->id; i < jb->count; i += jb->nthreads) {
        int rc = hth_ref_hash64_b(jb->entropy, jb->n_words, jb->tables, jb->n_tab, jb->data + jb->offsets[i],
                                  jb->lengths[i], jb->width, jb->b, jb->out + i);
        if (rc) jb->rc = rc;
    }
    return NULL;
}

int hth_ref_hash64_batch_b(const uint64_t *entropy, size_t n_words, const uint64_t *tables, size_t n_tab,
                           const uint8_t *data, const uint64_t *offsets, const uint64_t *lengths,
                           uint64_t count, uint32_t inner_width, uint32_t b, uint64_t *out, uint32_t nthreads)
{
    if (!hth_ref_tab_words(inner_width) || !block_ok(b) || (count && (!offsets || !lengths || !out))) return -1;
    if (nthreads == 0) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    hash64_job jobs[256];
    pthread_t th[256];
    for (uint32_t i = 0; i < nthreads; i++) {
        jobs[i] = (hash64_job){entropy, tables, n_words, n_tab, data, offsets, lengths, count, inner_width, b, out,
                               nthreads, i, 0};
        if (nthreads == 1) hash64_worker(&jobs[i]);
        else pthread_create(&th[i], NULL, hash64_worker, &jobs[i]);
    }
    int rc = 0;
    for (uint32_t i = 0; i < nthreads; i++) {
        if (nthreads > 1) pthread_join(th[i], NULL);
        if (jobs[i].rc) rc = jobs[i].rc;
    }
    return rc;
}
