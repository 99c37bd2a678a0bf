"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a property stated
in the paper (AU / A-Delta-U bounds of §3.2, §4 and §6.2, the p exponents of
§5.1, the code distance of §3.3, the tree construction of Eq. (1) and
Eq. (3), the multiplication counts of §6.1), a closed form, or an
independent restatement written here from the paper's equations.  A wrong
sign, index, dropped term or transposed operand in the oracle makes at least
one of them fail.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2104_08865_amd import workloads as wl

WIDTHS = (16, 24, 32, 40)
P_EXP = {16: 2, 24: 2, 32: 3, 40: 3}  # §5.1: p of each combine matrix
M64 = (1 << 64) - 1

# The combine matrices printed in §5.1, typed from the paper.
PRINTED_T = {
    16: [[1, 0, 1, 1, 2, 1, 4],
         [0, 1, 1, 2, 1, 4, 1]],
    24: [[0, 0, 1, 4, 1, 1, 2, 2, 1],
         [1, 1, 0, 0, 1, 4, 1, 2, 2],
         [1, 4, 1, 1, 0, 0, 2, 1, 2]],
    32: [[0, 0, 0, 1, 1, 4, 2, 4, 1, 1],
         [0, 1, 2, 0, 0, 1, 1, 2, 4, 1],
         [2, 0, 1, 0, 4, 0, 1, 1, 1, 1],
         [1, 1, 0, 1, 0, 0, 4, 1, 2, 8]],
    40: [[1, 0, 0, 0, 0, 1, 1, 2, 4],
         [0, 1, 0, 0, 0, 1, 2, 1, 7],
         [0, 0, 1, 0, 0, 1, 3, 8, 5],
         [0, 0, 0, 1, 0, 1, 4, 9, 8],
         [0, 0, 0, 0, 1, 1, 5, 3, 9]],
}


def _det(M):
    """Exact integer determinant (Bareiss)."""
    M = [list(map(int, r)) for r in M]
    n = len(M)
    sign, prev = 1, 1
    for i in range(n - 1):
        if M[i][i] == 0:
            sw = next((r for r in range(i + 1, n) if M[r][i]), None)
            if sw is None:
                return 0
            M[i], M[sw] = M[sw], M[i]
            sign = -sign
        for r in range(i + 1, n):
            for c in range(i + 1, n):
                M[r][c] = (M[r][c] * M[i][i] - M[r][i] * M[i][c]) // prev
        prev = M[i][i]
    return sign * M[n - 1][n - 1]


def _v2(x):
    x = abs(x)
    return (x & -x).bit_length() - 1


# ---------------------------------------------------------------------------
# NH (§3.2)
# ---------------------------------------------------------------------------

def test_nh_closed_forms(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(7)
    x = rng.integers(0, 2**63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    zero = np.zeros_like(x)
    lo = x & np.uint64(0xFFFFFFFF)
    hi = x >> np.uint64(32)
    # zero seed: the product of the two halves
    assert (o.nh(32, x, zero) == lo * hi).all()
    # a seed whose low half cancels the low half of the input gives 0
    s = ((np.uint64(1 << 32) - lo) & np.uint64(0xFFFFFFFF))
    assert (o.nh(32, x, s) == 0).all()
    # halves wrap separately: no carry from the low half into the high half
    assert o.nh(32, [0xFFFFFFFF_FFFFFFFF], [0x00000001_00000001])[0] == 0
    assert o.nh(32, [0x00000002_FFFFFFFF], [0x00000000_00000003])[0] == 2 * 2
    # the product is the full 64-bit value
    assert o.nh(32, [0xFFFFFFFF_FFFFFFFF], [0])[0] == (0xFFFFFFFF * 0xFFFFFFFF) & M64


def test_nh_adu_exhaustive_w4(oracle_lib):
    """§3.2: NH is 2^-W almost Delta-universal.  Exhaustive at W = 4 (words in
    Z_256): for every pair x != y and every delta, at most 256 * 2^-4 = 16 of
    the 256 seeds give NH(x) - NH(y) = delta."""
    o = oracle_lib
    seeds = np.arange(256, dtype=np.uint64)
    vals = np.stack([o.nh(4, np.full(256, x, dtype=np.uint64), seeds) for x in range(256)])  # [x, s]
    worst = 0
    for x in range(256):
        diff = (vals[x][None, :].astype(np.int64) - vals.astype(np.int64)) % 256  # [y, s]
        diff[x] = -1
        cnt = np.zeros((256, 256), dtype=np.int64)
        rows = np.repeat(np.arange(256), 256)
        ok = diff.ravel() >= 0
        np.add.at(cnt, (rows[ok], diff.ravel()[ok]), 1)
        worst = max(worst, int(cnt.max()))
    assert worst <= 16, worst
    # the bound is attained, so a weaker hash would show up here
    assert worst == 16


def test_nh_adu_sampled_w8(oracle_lib):
    """W = 8: all 2^16 seeds for sampled pairs, including the adversarial
    difference 2^7 in one half."""
    o = oracle_lib
    seeds = np.arange(1 << 16, dtype=np.uint64)
    rng = np.random.default_rng(11)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, 1 << 16, (300, 2)) if a != b]
    pairs += [(0, 0x80), (0x80, 0), (0x1234, 0x12B4), (0x0034, 0x8034), (0xFFFF, 0x7F7F)]
    for x, y in pairs:
        hx = o.nh(8, np.full(seeds.size, x, dtype=np.uint64), seeds).astype(np.int64)
        hy = o.nh(8, np.full(seeds.size, y, dtype=np.uint64), seeds).astype(np.int64)
        cnt = np.bincount((hx - hy) % 65536, minlength=65536)
        assert cnt.max() <= (1 << 16) >> 8, (x, y, cnt.max())


# ---------------------------------------------------------------------------
# GF(8) and the code (§3.3, §5.1)
# ---------------------------------------------------------------------------

def test_gf8_is_the_field(oracle_lib):
    o = oracle_lib
    mul = [[o.gf8_mul(a, b) for b in range(8)] for a in range(8)]
    assert mul[2][4] == 3  # x * x^2 = x^3 = x + 1
    for a, b, c in itertools.product(range(8), repeat=3):
        assert mul[a][b] == mul[b][a]
        assert mul[mul[a][b]][c] == mul[a][mul[b][c]]
        assert mul[a][b ^ c] == mul[a][b] ^ mul[a][c]
    for a in range(1, 8):
        assert sorted(mul[a][1:]) == list(range(1, 8))  # a is invertible


@pytest.mark.parametrize("width", WIDTHS)
def test_code_shape_matches_combine(oracle_lib, width):
    """§5.1: the EHC input group length is columns + 1 - rows of T, and the
    encoded length equals the column count."""
    d, e, k, w = oracle_lib.shape(width)
    P, T = oracle_lib.tables(width)
    assert T.shape == (k, e) and e == d + k - 1 and w == 3
    assert d == {16: 6, 24: 7, 32: 7, 40: 5}[width]
    assert k == width // 8


@pytest.mark.parametrize("width", WIDTHS)
def test_combine_matrix_p(oracle_lib, width):
    """§4 theorem and §5.1: every k-column minor of T is non-zero, and the
    largest power of two dividing any of them is 2^p with p = 2, 2, 3, 3."""
    P, T = oracle_lib.tables(width)
    assert T.tolist() == PRINTED_T[width]
    k, e = T.shape
    vmax = 0
    for cols in itertools.combinations(range(e), k):
        det = _det(T[:, cols])
        assert det != 0, cols
        vmax = max(vmax, _v2(det))
    assert vmax == P_EXP[width]


def test_no_odd_minors_possible_for_3x9():
    """§4 pigeonhole lemma: any 3 x 9 matrix has three columns with an even
    determinant (checked on the printed T and on random matrices)."""
    rng = np.random.default_rng(3)
    for M in [np.array(PRINTED_T[24])] + [rng.integers(0, 9, (3, 9)) for _ in range(50)]:
        assert any(_det(M[:, c]) % 2 == 0 for c in itertools.combinations(range(9), 3))


def _item_weights(width, Y, mod):
    Y = Y % np.uint64(mod)
    return (Y.reshape(Y.shape[0], -1, 3) != 0).any(axis=2).sum(axis=1)


@pytest.mark.parametrize("width", WIDTHS)
def test_code_distance_binary_image(oracle_lib, width):
    """§3.3: the erasure code has minimum distance k.  Exhaustive over every
    non-zero input difference of the code's mod-2 image (2^(d*w) - 1 of them);
    the mod-2 image having distance k implies distance k over Z_2^64 (a
    difference 2^t * odd keeps its mod-2 pattern after dividing by 2^t)."""
    d, e, k, w = oracle_lib.shape(width)
    n = d * w
    best = 10**9
    step = 1 << 15
    for start in range(1, 1 << n, step):
        idx = np.arange(start, min(start + step, 1 << n), dtype=np.uint64)
        X = ((idx[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint64)
        Y = oracle_lib.encode(width, X)
        best = min(best, int(_item_weights(width, Y, 2).min()))
    assert best == k


@pytest.mark.parametrize("width", WIDTHS)
def test_code_distance_mod4_low_weight(oracle_lib, width):
    """Differences mod 4 supported on at most k-1 input items still reach k
    non-zero encoded items (exhaustive where small, sampled otherwise)."""
    d, e, k, w = oracle_lib.shape(width)
    rng = np.random.default_rng(5)
    for items in itertools.combinations(range(d), k - 1):
        m = len(items) * w
        if 4 ** m <= 1 << 18:
            vals = np.arange(1, 4 ** m, dtype=np.uint64)
            digits = (vals[:, None] >> (2 * np.arange(m, dtype=np.uint64))[None, :]) & np.uint64(3)
        else:
            digits = rng.integers(0, 4, (1 << 15, m)).astype(np.uint64)
            digits = digits[(digits != 0).any(axis=1)]
        X = np.zeros((digits.shape[0], d * w), dtype=np.uint64)
        for a, c in enumerate(items):
            X[:, c * w:(c + 1) * w] = digits[:, a * w:(a + 1) * w]
        Y = oracle_lib.encode(width, X)
        assert int(_item_weights(width, Y, 4).min()) >= k


@pytest.mark.parametrize("width", WIDTHS)
def test_encode_linear_and_systematic(oracle_lib, width):
    """Encode is additive mod 2^64 and keeps the input as its first d items."""
    d, e, k, w = oracle_lib.shape(width)
    rng = np.random.default_rng(9)
    a = rng.integers(0, 2**64 - 1, (20000, d * w), dtype=np.uint64, endpoint=True)
    b = rng.integers(0, 2**64 - 1, (20000, d * w), dtype=np.uint64, endpoint=True)
    with np.errstate(over="ignore"):
        s = a + b
        ya, yb, ys = (oracle_lib.encode(width, v) for v in (a, b, s))
        assert (ys == ya + yb).all()
    assert (ya[:, :d * w] == a).all()
    # full-width low-weight differences also keep distance k
    diff = np.zeros((5000, d * w), dtype=np.uint64)
    for r in range(diff.shape[0]):
        for c in rng.choice(d, size=k - 1, replace=False):
            diff[r, c * w + rng.integers(0, w)] = np.uint64(1) << np.uint64(rng.integers(0, 64))
    yd = oracle_lib.encode(width, diff)
    assert int((yd.reshape(yd.shape[0], e, w) != 0).any(axis=2).sum(axis=1).min()) >= k


# ---------------------------------------------------------------------------
# EHC (§4 theorem)
# ---------------------------------------------------------------------------

def _binom_upper(n, p, z=6.0):
    mu = n * p
    return mu + z * math.sqrt(max(mu, 1e-12)) + 6


@pytest.mark.parametrize("width", WIDTHS)
def test_ehc_collision_rate_w8(oracle_lib, width):
    """§4 theorem: EHC with NH is 2^(k(p-W))-A-Delta-U.  Monte Carlo at W = 8
    over random seeds on adversarial pairs: the collision count stays under
    the bound (6 sigma); with a code of distance k - 1 it would be ~2^(W-p)
    times larger."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    p = P_EXP[width]
    bound = 2.0 ** (k * (p - 8))
    n_seeds = 40000 if k <= 3 else 20000
    rng = np.random.default_rng(13 + width)
    S = rng.integers(0, 1 << 16, (n_seeds, e * w), dtype=np.uint64)
    base = rng.integers(0, 1 << 16, d * w, dtype=np.uint64)
    pairs = []
    y = base.copy(); y[0] ^= np.uint64(0x80); pairs.append(y)           # one word, top bit of low half
    y = base.copy(); y[w * (d - 1) + 2] ^= np.uint64(0x8000); pairs.append(y)  # last item, high half
    y = base.copy(); y[0] = (y[0] + np.uint64(1)) & np.uint64(0xFFFF); y[w] = (y[w] - np.uint64(1)) & np.uint64(0xFFFF); pairs.append(y)
    zx = np.stack([o.ehc(width, base, S[i], W=8) for i in range(n_seeds)])
    for y in pairs:
        zy = np.stack([o.ehc(width, y, S[i], W=8) for i in range(n_seeds)])
        coll = int((zx == zy).all(axis=1).sum())
        assert coll <= _binom_upper(n_seeds, bound), (width, coll, n_seeds * bound)


def test_ehc_swap_pair_w8(oracle_lib):
    """§3.3 step 2: every encoded word is hashed against its own key.  For
    HalftimeHash16 the parity item is the plain sum of the items, so swapping
    word u between two items that agree everywhere else leaves the parity
    item unchanged and the difference sits on exactly two systematic items.
    With independent keys per word the pair still obeys the §4 bound
    2^(k(p-W)); if the items shared their keys (a key picked by u alone) the
    two items' hashes would simply trade places and the pair would collide
    whenever NH(a, s) = NH(a + delta, s), about 2^-W of the time (2^4 times
    the bound at W = 8)."""
    o = oracle_lib
    width = 16
    d, e, k, w = o.shape(width)
    bound = 2.0 ** (k * (P_EXP[width] - 8))
    n_seeds = 20000
    rng = np.random.default_rng(71)
    S = rng.integers(0, 1 << 16, (n_seeds, e * w), dtype=np.uint64)
    for c1, c2, u in [(2, 3, 1), (0, 5, 0), (1, 4, 2)]:
        x = rng.integers(0, 1 << 16, d * w, dtype=np.uint64)
        x[c2 * w:(c2 + 1) * w] = x[c1 * w:(c1 + 1) * w]
        x[c2 * w + u] = (x[c1 * w + u] + np.uint64(0x80)) & np.uint64(0xFFFF)
        y = x.copy()
        y[c1 * w + u], y[c2 * w + u] = x[c2 * w + u], x[c1 * w + u]
        # the parity item (sum of the items) is the same for both
        assert (o.encode(width, x, W=8)[0, d * w:] == o.encode(width, y, W=8)[0, d * w:]).all()
        zx = np.stack([o.ehc(width, x, S[i], W=8) for i in range(n_seeds)])
        zy = np.stack([o.ehc(width, y, S[i], W=8) for i in range(n_seeds)])
        coll = int((zx == zy).all(axis=1).sum())
        assert coll <= _binom_upper(n_seeds, bound), (c1, c2, u, coll, n_seeds * bound)


def _lohi(z):
    return ((z & 0xFFFFFFFF) * (z >> 32)) & M64


@pytest.mark.parametrize("b", [8, 4])
@pytest.mark.parametrize("width", WIDTHS)
def test_ehc_single_key_closed_form(oracle_lib, width, b):
    """§3.3 step 2 with one non-zero EHC key.  All entropy zero except
    S_ehc[idx] = s, one execution of zero bytes: every instance hashes the
    zero word at idx against s (NH(0, s) = s_lo * s_hi) and every other word
    to 0, so item c = idx // w has h_c = s_lo * s_hi, z_t = T[t][c] * s_lo *
    s_hi, and the single leftover leaf of each of the b instances goes
    through the zero final key: out_t = b * lo(z_t) * hi(z_t).  A key shared
    by several words, or read by the wrong item, changes the multiplier or
    the column of T."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    P, T = o.tables(width)
    base = o.entropy_offset(width, b)
    xb = 8 * b * d * w
    s_lo, s_hi = 0x9E3779B1, 0x7F4A7C15
    for idx in range(e * w):
        ent = np.zeros(o.entropy_words(b), dtype=np.uint64)
        ent[base + idx] = np.uint64(s_lo | (s_hi << 32))
        out = np.frombuffer(o.hash_bytes(ent, bytes(xb), width, b=b).tobytes(), dtype="<u8")
        for t in range(k):
            z = int(T[t][idx // w]) * s_lo * s_hi & M64
            assert int(out[t]) == b * _lohi(z) & M64, (idx, t)


@pytest.mark.parametrize("width", WIDTHS)
def test_ehc_key_and_word_closed_form(oracle_lib, width):
    """One non-zero input word v at (item c, sub-word u, instance 0) and one
    non-zero EHC key s.  With the key on v's own position, v is hashed as
    (v_lo + s_lo)(v_hi + s_hi) while every parity word that selects v
    (binary image of P) is hashed against a zero key; with the key on a
    position holding zero in every instance, the word's key only adds
    s_lo * s_hi to that item in all b instances."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    P, T = o.tables(width)
    base = o.entropy_offset(width)
    xw = 8 * d * w
    v_lo, v_hi = 0x01234567, 0x0089ABCD
    s_lo, s_hi = 0x31415927, 0x02718281
    for c, u in [(0, 0), (d - 1, 2), (1, 1)]:
        buf = np.zeros(xw, dtype=np.uint64)
        buf[(c * w + u) * 8] = np.uint64(v_lo | (v_hi << 32))
        sel = [sum(_mbit(int(P[r][c]), uu, u) for uu in range(3)) for r in range(k - 1)]
        # (a) the key on v's own word
        ent = np.zeros(o.entropy_words(), dtype=np.uint64)
        ent[base + c * w + u] = np.uint64(s_lo | (s_hi << 32))
        out = np.frombuffer(o.hash_bytes(ent, buf.astype("<u8").tobytes(), width).tobytes(), dtype="<u8")
        own = (v_lo + s_lo) * (v_hi + s_hi)
        for t in range(k):
            z0 = (int(T[t][c]) * own + sum(int(T[t][d + r]) * sel[r] for r in range(k - 1)) * v_lo * v_hi) & M64
            zj = int(T[t][c]) * s_lo * s_hi & M64  # instances 1..7: zero word, key s
            assert int(out[t]) == (_lohi(z0) + 7 * _lohi(zj)) & M64, (c, u, t)
        # (b) the key on the next item's word u (zero in every instance)
        c2 = (c + 1) % d
        ent = np.zeros(o.entropy_words(), dtype=np.uint64)
        ent[base + c2 * w + u] = np.uint64(s_lo | (s_hi << 32))
        out = np.frombuffer(o.hash_bytes(ent, buf.astype("<u8").tobytes(), width).tobytes(), dtype="<u8")
        for t in range(k):
            ab = (int(T[t][c]) + sum(int(T[t][d + r]) * sel[r] for r in range(k - 1))) * v_lo * v_hi
            z0 = (ab + int(T[t][c2]) * s_lo * s_hi) & M64
            zj = int(T[t][c2]) * s_lo * s_hi & M64
            assert int(out[t]) == (_lohi(z0) + 7 * _lohi(zj)) & M64, (c, u, t)


# ---------------------------------------------------------------------------
# Tree (§3.1 Eq. (1), §5.2 Eq. (3))
# ---------------------------------------------------------------------------

def test_eq1_binary_tree_power_of_two(oracle_lib):
    """f = 2, b = 1: with n = 2^m executions the stack leaves exactly one item,
    the Carter-Wegman tree of Eq. (1) with the key picked by the height of the
    node, and the output is the final NH of that root plus tail and length
    terms.  Restated here directly from Eq. (1)."""
    o = oracle_lib
    width = 16
    d, e, k, w = o.shape(width)
    offs = o.layout(width, 1, 2)
    for m in range(0, 6):
        n = 1 << m
        ent = wl.splitmix64(100 + m, offs[5])
        words = wl.splitmix64(200 + m, n * d * w + 5)
        out = o.hash_words(width, ent, words, n_exec=n, len_value=12345, b=1, f=2)
        S_ehc = ent[offs[0]:offs[1]]
        leaves = [o.ehc(width, words[g * d * w:(g + 1) * d * w], S_ehc) for g in range(n)]
        for t in range(k):
            S_tree = ent[offs[1] + t * 20:offs[1] + (t + 1) * 20]  # (f-1) = 1 key per level

            def T(lo, hi):
                if hi - lo == 1:
                    return int(leaves[lo][t])
                half = (hi - lo) // 2
                height = int(math.log2(hi - lo)) - 1
                left, right = T(lo, lo + half), T(lo + half, hi)
                return (int(o.nh(32, [left], [S_tree[height]])[0]) + right) & M64

            root = T(0, n)
            fin = int(o.nh(32, [root], [ent[offs[2] + t * 20 + m]])[0])
            tail = sum(int(o.nh(32, [words[n * d * w + q]], [ent[offs[3] + t + q]])[0]) for q in range(5))
            ln = int(o.nh(32, [12345], [ent[offs[4] + t]])[0])
            assert int(out[t]) == (fin + tail + ln) & M64, (m, t)


@pytest.mark.parametrize("f,b", [(2, 1), (8, 8), (3, 2)])
def test_eq3_stack_equals_recursive(oracle_lib, f, b):
    """Eq. (3): the streaming stack and the top-down decomposition into
    complete subtrees (one per unit of each base-f digit of n) agree."""
    o = oracle_lib
    for width in WIDTHS:
        d, e, k, w = o.shape(width)
        offs = o.layout(width, b, f)
        ent = wl.splitmix64(7 * width + f, offs[5])
        ns = [0, 1, f - 1, f, f + 1, f * f - 1, f * f, f * f + 1, 2 * f * f + 3 * f + 1]
        if f == 8:
            ns = [0, 1, 7, 8, 9, 63, 64, 65, 517]
        for n in ns:
            xw = b * d * w
            words = wl.splitmix64(1000 + n, n * xw + 3)
            a = o.hash_words(width, ent, words, n_exec=n, b=b, f=f, recursive=False)
            r = o.hash_words(width, ent, words, n_exec=n, b=b, f=f, recursive=True)
            assert (a == r).all(), (width, f, b, n)


def _digits(n, f):
    out = []
    while n:
        out.append(n % f)
        n //= f
    return out


@pytest.mark.parametrize("width", WIDTHS)
def test_multiplication_counts(oracle_lib, width):
    """§6.1: each execution performs e*w products per instance; each tree node
    f-1; the stack leaves one item per unit of each base-f digit of n (for
    f = 2, one per set bit of n), each hashed once per instance by the final
    NH; the tail is hashed k times; the length once per output word."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    b, f = 8, 8
    ent = o.expand_seed(3)[o.entropy_offset(width):]
    for n in (0, 1, 7, 8, 9, 64, 100, 600):
        R = 13
        words = wl.splitmix64(n + 1, n * b * d * w + R)
        o.hash_words(width, ent, words, n_exec=n)
        c = o.mul_counts()
        assert c["ehc"] == e * w * b * n
        nodes = sum(n // f ** (l + 1) for l in range(20))
        assert c["tree"] == k * b * (f - 1) * nodes
        assert c["tree"] <= k * b * n
        assert c["final"] == k * b * sum(_digits(n, f))
        assert c["tail"] == k * R
        assert c["length"] == k
    # f = 2: one leftover item per set bit of n
    offs = o.layout(width, 1, 2)
    ent2 = wl.splitmix64(99, offs[5])
    for n in (1, 2, 3, 5, 6, 7, 11, 12):
        words = wl.splitmix64(n, n * d * w)
        o.hash_words(width, ent2, words, n_exec=n, b=1, f=2)
        assert o.mul_counts()["final"] == k * bin(n).count("1")


@pytest.mark.parametrize("width", WIDTHS)
def test_unused_entropy_is_unread(oracle_lib, width):
    """Absent stack slots add nothing (their final keys are never read) and
    tree keys above the top level are never read."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    offs = o.layout(width)
    ent = o.expand_seed(5)[o.entropy_offset(width):o.entropy_offset(width) + offs[5]].copy()
    n = 8 * 8 + 3 * 8 + 2  # digits (2, 3, 1): level 2 has one item, level 1 three, level 0 two
    words = wl.splitmix64(17, n * 8 * d * w + 40)
    ref = o.hash_words(width, ent, words, n_exec=n)
    e2 = ent.copy()
    for t in range(k):
        for l in range(20):
            used = {0: 2, 1: 3, 2: 1}.get(l, 0)
            for i in range(used, 7):
                for j in range(8):
                    e2[offs[2] + ((t * 20 + l) * 7 + i) * 8 + j] ^= np.uint64(0xDEADBEEF)
            if l >= 2:  # nodes are formed at levels 0 and 1 only
                for i in range(7):
                    e2[offs[1] + (t * 20 + l) * 7 + i] ^= np.uint64(0x12345)
    assert (o.hash_words(width, e2, words, n_exec=n) == ref).all()
    e3 = ent.copy()
    e3[offs[2]] ^= np.uint64(1 << 40)  # a used slot: output changes
    assert not (o.hash_words(width, e3, words, n_exec=n) == ref).all()


# ---------------------------------------------------------------------------
# Closed forms with zero entropy
# ---------------------------------------------------------------------------

def _mbit(a, u, v):
    """Bit u of a * x^v in GF(2)[x]/(x^3+x+1), written out independently."""
    r = 0
    for i in range(3):
        if (a >> i) & 1:
            r ^= 1 << (i + v)
    for i in (4, 3):
        if (r >> i) & 1:
            r ^= 0b1011 << (i - 3)
    return (r >> u) & 1


@pytest.mark.parametrize("width", WIDTHS)
def test_zero_entropy_closed_forms(oracle_lib, width):
    o = oracle_lib
    d, e, k, w = o.shape(width)
    P, T = o.tables(width)
    ent = np.zeros(o.entropy_words(), dtype=np.uint64)
    # tail only: every output word is the sum of lo * hi over the words
    data = bytes(range(1, 30))
    words = [int.from_bytes(data[i:i + 8].ljust(8, b"\0"), "little") for i in range(0, len(data), 8)]
    expect = sum((x & 0xFFFFFFFF) * (x >> 32) for x in words) & M64
    out = np.frombuffer(o.hash_bytes(ent, data, width).tobytes(), dtype="<u8")
    assert (out == expect).all()
    # executions are counted in bytes: one byte short of a full execution the
    # whole string (b*d*w words, the last one partial) is still tail
    xbytes = 64 * d * w
    data = wl.random_bytes(8, xbytes - 1).tobytes()
    words = [int.from_bytes(data[i:i + 8].ljust(8, b"\0"), "little") for i in range(0, len(data), 8)]
    assert len(words) == 8 * d * w
    expect = (sum((x & 0xFFFFFFFF) * (x >> 32) for x in words)
              + ((xbytes - 1) & 0xFFFFFFFF) * ((xbytes - 1) >> 32)) & M64
    out = np.frombuffer(o.hash_bytes(ent, data, width).tobytes(), dtype="<u8")
    assert (out == expect).all()
    assert o.mul_counts()["ehc"] == 0
    # one execution, one non-zero word v = a + 2^32 b at item c, sub-word u,
    # instance j: the systematic item and every parity word that selects it
    # hash to a*b; the combine gives z_t; the single leftover leaf is hashed
    # by the final NH (zero key: lo(z) * hi(z)); the length 8*b*d*w adds
    # nothing (its high half is 0).
    xw = 8 * d * w
    a_, b_ = 0x9ABCDEF1, 0x7654321
    for c, u, j in [(0, 0, 0), (d - 1, 2, 7), (1, 1, 3)]:
        buf = np.zeros(xw, dtype=np.uint64)
        buf[(c * w + u) * 8 + j] = np.uint64(a_ + (b_ << 32))
        hcount = np.zeros(e, dtype=np.int64)
        hcount[c] = 1
        for r in range(k - 1):
            hcount[d + r] = sum(_mbit(int(P[r][c]), uu, u) for uu in range(3))
        ab = a_ * b_
        out = np.frombuffer(o.hash_bytes(ent, buf.astype("<u8").tobytes(), width).tobytes(), dtype="<u8")
        for t in range(k):
            z = sum(int(T[t][q]) * int(hcount[q]) for q in range(e)) * ab & M64
            assert int(out[t]) == ((z & 0xFFFFFFFF) * (z >> 32)) & M64, (c, u, j, t)


# ---------------------------------------------------------------------------
# Whole hash
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("width", [16, 24])
def test_whole_hash_collision_rate_w8(oracle_lib, width):
    """§6.2: epsilon = 2^(-Wk) (2^(kp) + h^k + 1).  Monte Carlo at W = 8,
    b = 1 on equal-length word strings that differ in one EHC word, in one
    tail word, and in two words of different executions."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    p = P_EXP[width]
    offs = o.layout(width, 1, 8)
    n_exec, R = 9, 4
    h = 1
    eps = 2.0 ** (-8 * k) * (2 ** (k * p) + h ** k + 1)
    rng = np.random.default_rng(21)
    x = rng.integers(0, 1 << 16, n_exec * d * w + R, dtype=np.uint64)
    ys = []
    y = x.copy(); y[5] ^= np.uint64(0x80); ys.append(y)
    y = x.copy(); y[-1] ^= np.uint64(0x8000); ys.append(y)
    y = x.copy(); y[3] ^= np.uint64(1); y[d * w + 3] ^= np.uint64(1); ys.append(y)
    n_seeds = 6000
    ents = [rng.integers(0, 1 << 16, offs[5], dtype=np.uint64) for _ in range(n_seeds)]
    hx = [o.hash_words(width, s, x, n_exec=n_exec, W=8, b=1) for s in ents]
    for y in ys:
        coll = sum(int((o.hash_words(width, s, y, n_exec=n_exec, W=8, b=1) == hv).all())
                   for s, hv in zip(ents, hx))
        assert coll <= _binom_upper(n_seeds, eps), (coll, n_seeds * eps)


@pytest.mark.parametrize("width", WIDTHS)
def test_full_width_no_collisions_on_adversarial_pairs(oracle_lib, width):
    """At W = 32 epsilon is below 2^-55: no collisions over many seeds for
    pairs differing by one bit in the body, in the tail, or in the top bit."""
    o = oracle_lib
    xb = wl.execution_bytes(width)
    base = wl.random_bytes(31, 3 * xb + 100)
    flips = [0, 7, xb + 63, 3 * xb + 5, 3 * xb + 99]
    for s in range(60):
        ent = o.expand_seed(1000 + s)
        h0 = o.hash_bytes(ent, base, width)
        for pos in flips:
            y = base.copy(); y[pos] ^= 0x80
            assert not (o.hash_bytes(ent, y, width) == h0).all()


@pytest.mark.parametrize("b", [8, 4])
@pytest.mark.parametrize("width", WIDTHS)
def test_final_single_key_closed_form(oracle_lib, width, b):
    """§5.2 and §6.1 (b*f*h*k final-NH words): each leftover item (level l,
    position i) of tree t and instance j has its own final key
    S_final[t][l][i][j].  Zero bytes and zero entropy except that one key s:
    every item is 0, so out_t = s_lo * s_hi when t is the key's tree and slot
    (l, i) is occupied (i < digit_l of the execution count in base 8), and 0
    otherwise.  153 executions have digits (1, 3, 2)."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    offs = o.layout(width, b)
    base = o.entropy_offset(width, b)
    n = 153
    digits = _digits(n, 8)
    assert digits == [1, 3, 2]
    data = bytes(n * 8 * b * d * w)
    s_lo, s_hi = 0x5851F42D, 0x4C957F2D
    cases = [(0, 0, 0, 0), (k - 1, 0, 0, b - 1), (0, 1, 2, 1), (k - 1, 2, 1, b // 2),
             (0, 0, 1, 0), (0, 1, 3, 2), (k - 1, 2, 2, 0), (0, 3, 0, 0)]
    for t0, l, i, j in cases:
        ent = np.zeros(o.entropy_words(b), dtype=np.uint64)
        ent[base + offs[2] + ((t0 * 20 + l) * 7 + i) * b + j] = np.uint64(s_lo | (s_hi << 32))
        out = np.frombuffer(o.hash_bytes(ent, data, width, b=b).tobytes(), dtype="<u8")
        present = l < len(digits) and i < digits[l]
        for t in range(k):
            want = s_lo * s_hi if (t == t0 and present) else 0
            assert int(out[t]) == want, (t0, l, i, j, t)


@pytest.mark.parametrize("b", [8, 4])
@pytest.mark.parametrize("width", WIDTHS)
def test_instance_swap_no_collisions(oracle_lib, width, b):
    """Instances share the EHC and tree keys (§6.1 shares the EHC entropy
    across instances) but not the final keys, so two strings that differ only
    by trading instances j and j' (words j and j' of every block of the full
    executions swapped, tail untouched) give leftover items that trade
    places between instances, and the per-instance final keys separate them:
    no collisions at W = 32 over 60 seeds.  Were the final key shared by the
    instances, every such pair would collide."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    xb = 8 * b * d * w
    n = 9  # leftover items at levels 0 and 1
    x = wl.random_bytes(40 + width, n * xb + 100)
    pairs = [(0, 1), (2, b - 1)] if b == 8 else [(0, 3), (1, 2)]
    ys = []
    for j1, j2 in pairs:
        y = x.copy()
        blocks = y[:n * xb].view("<u8").reshape(-1, b)
        blocks[:, [j1, j2]] = blocks[:, [j2, j1]]
        assert not (y == x).all()
        ys.append(y)
    for s in range(60):
        ent = o.expand_seed(5000 + s, b=b)
        h0 = o.hash_bytes(ent, x, width, b=b)
        for y in ys:
            assert not (o.hash_bytes(ent, y, width, b=b) == h0).all(), s


@pytest.mark.parametrize("width", WIDTHS)
def test_lengths_separate_and_padding(oracle_lib, width):
    """Zero padding alone never makes two lengths collide: the length word
    separates x from x || 0 (the appended-length requirement of §2)."""
    o = oracle_lib
    ent = o.expand_seed(2)
    for n in (0, 1, 7, 8, 100, wl.execution_bytes(width) - 1):
        a = o.hash_bytes(ent, bytes(n), width)
        b = o.hash_bytes(ent, bytes(n + 1), width)
        assert not (a == b).all()


def test_batch_matches_single_and_is_offset_invariant(oracle_lib):
    o = oracle_lib
    ent = o.expand_seed(9)
    lens = np.array([0, 1, 9, 1151, 1152, 1153, 3000, 77], dtype=np.uint64)
    offs, total = wl.pack(lens)
    data = wl.random_bytes(4, total + 3)
    for width in WIDTHS:
        out = o.hash_batch(ent, data, offs + np.uint64(3), lens, width, nthreads=3)
        for i in range(lens.size):
            s = data[int(offs[i]) + 3:int(offs[i]) + 3 + int(lens[i])]
            assert (out[i] == o.hash_bytes(ent, s.tobytes(), width)).all()


def test_expand_seed_is_splitmix64(oracle_lib):
    """Seed expansion is the published splitmix64 stream (first output of
    state 0 is the well-known 0xE220A8397B1DCDAF)."""
    o = oracle_lib
    assert int(o.expand_seed(0)[0]) == 0xE220A8397B1DCDAF
    assert (o.expand_seed(12345) == wl.splitmix64(12345, o.entropy_words())).all()
    assert o.entropy_words() == 2688 + 3980 + 5245 + 6456


def test_entropy_formula_reproduces_paper_figure():
    """§6.2: HalftimeHash24 needs about 8.4 KB of entropy for strings up to one
    megabyte (ew + (f-1)hk + bfhk + bdw + k - 1 words with h = 4 levels for
    the 780 executions of 1 MiB)."""
    w, d, e, k, b, f = 3, 7, 9, 3, 8, 8
    n_exec = (1 << 20) // (8 * b * d * w)
    h = len(_digits(n_exec, f))
    words = e * w + (f - 1) * h * k + b * f * h * k + b * d * w + k - 1
    assert n_exec == 780 and h == 4
    assert round(words * 8 / 1000, 1) == 8.4


# ---------------------------------------------------------------------------
# The 256-bit block variant (b = 4; §6.3: b is the machine's vector width in
# 64-bit words, and each b is its own family)
# ---------------------------------------------------------------------------

def _nh_py(x, s):
    """NH of one word against one key, from the definition of §3.2 (halves
    added separately mod 2^32, then multiplied)."""
    lo = ((x & 0xFFFFFFFF) + (s & 0xFFFFFFFF)) & 0xFFFFFFFF
    hi = ((x >> 32) + (s >> 32)) & 0xFFFFFFFF
    return lo * hi


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_layout_sizes(oracle_lib, width):
    """With b = 4 the per-instance parts shrink to 4 instances: final keys
    k * 20 levels * 7 positions * 4 instances, Toeplitz tail keys for the
    longest tail (4*d*w words) plus k - 1; EHC and tree keys do not depend on
    b; the four widths sit back to back."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    offs = o.layout(width, 4, 8)
    sizes = np.diff(offs)
    assert list(sizes) == [e * w, k * 20 * 7, k * 20 * 7 * 4, 4 * d * w + k - 1, k]
    assert o.entropy_words(4) == sum(o.layout(x, 4, 8)[5] for x in WIDTHS)
    assert o.entropy_offset(width, 4) == sum(o.layout(x, 4, 8)[5] for x in WIDTHS if x < width)


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_tail_only_closed_form(oracle_lib, width):
    """A string shorter than one b = 4 execution (32*d*w bytes) is its tail:
    out_t = sum_m NH(word_m, S_tail[t + m]) + NH(L, S_len[t]) with the b = 4
    layout's keys; at exactly one execution it is not (the tree path runs)."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    ent = o.expand_seed(11, b=4)
    base = o.entropy_offset(width, 4)
    offs = o.layout(width, 4, 8)
    xb = 32 * d * w
    for L in (0, 1, 9, 200, xb - 1):
        data = wl.random_bytes(12, L).tobytes()
        words = [int.from_bytes(data[i:i + 8].ljust(8, b"\0"), "little") for i in range(0, L, 8)]
        out = np.frombuffer(o.hash_bytes(ent, data, width, b=4).tobytes(), dtype="<u8")
        for t in range(k):
            acc = sum(_nh_py(x, int(ent[base + offs[3] + t + m])) for m, x in enumerate(words))
            acc += _nh_py(L, int(ent[base + offs[4] + t]))
            assert int(out[t]) == acc & M64, (L, t)
    data = wl.random_bytes(12, xb).tobytes()
    words = [int.from_bytes(data[i:i + 8], "little") for i in range(0, xb, 8)]
    out = np.frombuffer(o.hash_bytes(ent, data, width, b=4).tobytes(), dtype="<u8")
    tail_form = (sum(_nh_py(x, int(ent[base + offs[3] + m])) for m, x in enumerate(words))
                 + _nh_py(xb, int(ent[base + offs[4]]))) & M64
    assert int(out[0]) != tail_form
    assert o.mul_counts()["ehc"] == e * w * 4


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_multiplication_counts(oracle_lib, width):
    """§6.1 counts with b = 4 on byte strings: e*w*b products per execution,
    (f-1)*b per tree node per output, b per leftover item per output, one per
    tail word per output, one per output for the length."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    b, f = 4, 8
    ent = o.expand_seed(5, b=4)
    xb = 8 * b * d * w
    for n, extra in ((1, 0), (8, 17), (9, 1), (64, 0), (100, 301), (600, 8)):
        L = n * xb + extra
        o.hash_bytes(ent, wl.random_bytes(n, L).tobytes(), width, b=4)
        c = o.mul_counts()
        assert c["ehc"] == e * w * b * n
        nodes = sum(n // f ** (l + 1) for l in range(20))
        assert c["tree"] == k * b * (f - 1) * nodes
        assert c["final"] == k * b * sum(_digits(n, f))
        assert c["tail"] == k * ((extra + 7) // 8)
        assert c["length"] == k


@pytest.mark.parametrize("width", WIDTHS)
def test_b4_zero_entropy_one_word(oracle_lib, width):
    """b = 4, zero entropy, one execution with a single non-zero word at
    (item c, sub-word u, instance j): the result is the b = 8 closed form with
    the execution laid out as 4-word blocks (word index (c*w + u)*4 + j)."""
    o = oracle_lib
    d, e, k, w = o.shape(width)
    P, T = o.tables(width)
    ent = np.zeros(o.entropy_words(4), dtype=np.uint64)
    xw = 4 * d * w
    a_, b_ = 0x12345679, 0x0FEDCBA9
    for c, u, j in [(0, 0, 0), (d - 1, 2, 3), (1, 1, 2)]:
        buf = np.zeros(xw, dtype=np.uint64)
        buf[(c * w + u) * 4 + j] = np.uint64(a_ + (b_ << 32))
        hcount = np.zeros(e, dtype=np.int64)
        hcount[c] = 1
        for r in range(k - 1):
            hcount[d + r] = sum(_mbit(int(P[r][c]), uu, u) for uu in range(3))
        out = np.frombuffer(o.hash_bytes(ent, buf.astype("<u8").tobytes(), width, b=4).tobytes(), dtype="<u8")
        for t in range(k):
            z = sum(int(T[t][q]) * int(hcount[q]) for q in range(e)) * (a_ * b_) & M64
            assert int(out[t]) == ((z & 0xFFFFFFFF) * (z >> 32)) & M64, (c, u, j, t)


# ---------------------------------------------------------------------------
# Composition with simple tabulation (§1: a universe-collapsing family feeds
# a short-input family; §7: pairing with a fast short-input family).
# ---------------------------------------------------------------------------

def _identity_window(width, m):
    """Tables whose XOR over a key is the little-endian word of key bytes
    8m .. 8m+7: T_i[v] = v << 8(i - 8m) inside the window, zero elsewhere."""
    t = np.zeros((width + 1, 256), dtype=np.uint64)
    for i in range(8 * m, 8 * m + 8):
        t[i] = np.arange(256, dtype=np.uint64) << np.uint64(8 * (i - 8 * m))
    return t


@pytest.mark.parametrize("b", [8, 4])
@pytest.mark.parametrize("width", WIDTHS)
def test_hash64_identity_tables_reproduce_key_bytes(oracle_lib, width, b):
    """With identity tables on window m the result is word m of the key: of
    the zero-padded string itself for L <= c, of its HalftimeHash value (inner
    width c, block size b) for L > c."""
    o = oracle_lib
    ent = o.expand_seed(9, b=b)
    for L in (0, 1, 7, 8, width - 1, width, width + 1, 1000, 3000):
        x = wl.random_bytes(L + 1, L)
        for m in range(width // 8):
            z = o.hash64(ent, _identity_window(width, m), x, width, b=b)
            if L <= width:
                key = np.zeros(width, dtype=np.uint8)
                key[:L] = x
            else:
                key = o.hash_bytes(ent, x, width, b=b)
            assert z == int(key[8 * m:8 * m + 8].view("<u8")[0]), (L, m)


@pytest.mark.parametrize("width", WIDTHS)
def test_hash64_separator_character(oracle_lib, width):
    """Only the last table non-zero, T_c[v] = v: the result is the separator
    character, L for strings of at most c bytes and 255 for longer ones."""
    o = oracle_lib
    ent = o.expand_seed(9)
    t = np.zeros((width + 1, 256), dtype=np.uint64)
    t[width] = np.arange(256, dtype=np.uint64)
    for L in list(range(0, width + 3)) + [500, 2000]:
        assert o.hash64(ent, t, wl.random_bytes(L, L), width) == (L if L <= width else 255)


@pytest.mark.parametrize("width", WIDTHS)
def test_hash64_is_xor_of_table_entries(oracle_lib, width):
    """The result is linear over XOR in the tables (and not over addition),
    two keys that differ in one character differ by exactly the two table
    entries of that character, and the empty string gives the XOR of every
    table's entry 0 with T_c[0]."""
    o = oracle_lib
    ent = o.expand_seed(10)
    t1, t2 = o.tab_expand(1, width), o.tab_expand(2, width)
    for L in (0, 3, width, width + 1, 1500):
        x = wl.random_bytes(L + 7, L)
        z1, z2 = o.hash64(ent, t1, x, width), o.hash64(ent, t2, x, width)
        assert o.hash64(ent, t1 ^ t2, x, width) == z1 ^ z2
        assert o.hash64(ent, t1 ^ t2, x, width) != (z1 + z2) & M64
    rng = np.random.default_rng(width)
    for _ in range(50):
        L = int(rng.integers(1, width + 1))
        j = int(rng.integers(0, L))
        x = rng.integers(0, 256, L).astype(np.uint8)
        y = x.copy()
        y[j] ^= np.uint8(rng.integers(1, 256))
        d = o.hash64(ent, t1, x, width) ^ o.hash64(ent, t1, y, width)
        assert d == int(t1[j, x[j]]) ^ int(t1[j, y[j]])
    expect = 0
    for i in range(width):
        expect ^= int(t1[i, 0])
    assert o.hash64(ent, t1, b"", width) == expect ^ int(t1[width, 0])


def test_hash64_short_keys_do_not_collide(oracle_lib):
    """Simple tabulation is 3-independent, so two distinct keys collide with
    probability 2^-64: none among all strings of at most two bytes (65,793
    keys), nor between them and 2,000 longer strings."""
    o = oracle_lib
    width = 16
    ent = o.expand_seed(11)
    t = o.tab_expand(12, width)
    keys = [b""] + [bytes([a]) for a in range(256)] + [bytes([a, c]) for a in range(256) for c in range(256)]
    lens = np.array([len(k) for k in keys] + [17 + i for i in range(2000)], dtype=np.uint64)
    data = np.concatenate([np.frombuffer(b"".join(keys), dtype=np.uint8), wl.random_bytes(13, int(lens[len(keys):].sum()))])
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    z = o.hash64_batch(ent, t, data, offs, lens, width, nthreads=8)
    assert np.unique(z).size == z.size
    # the batch routine agrees with the single-string one
    for i in (0, 1, 300, 65792, 65793, z.size - 1):
        assert int(z[i]) == o.hash64(ent, t, data[int(offs[i]):int(offs[i] + lens[i])], width)


def test_tab_expand_is_splitmix64(oracle_lib):
    """The tables are the first (c + 1) * 256 outputs of splitmix64 from the
    user seed: the same stream the entropy expansion is pinned to."""
    o = oracle_lib
    for width in WIDTHS:
        t = o.tab_expand(77, width)
        assert t.shape == (width + 1, 256) and o.tab_words(width) == (width + 1) * 256
        assert (t.ravel() == o.expand_seed(77)[:t.size]).all()
    with pytest.raises(ValueError):
        o.tab_words(20)
