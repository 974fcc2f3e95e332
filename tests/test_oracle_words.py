"""Pins for the oracle's word-level arithmetic (CPU only).

The oracle reduces by true division.  Here it is checked against things that
are not itself:
* Python's arbitrary-precision ``int`` (an independent big-integer library);
* the paper's single- and double-word Barrett listings (Listing 1 ``_smulmod``
  and Listing 4 ``_dmulmod``), evaluated word by word in Python with 64-bit
  words: a different reduction method that must land on the same residue;
* the identities of the paper's rewrite rules (Table 1) on 32-bit words;
* the worked rewrite of double-word modular addition (Eq. (final_addmod)).
"""
import json
import os
import random

import pytest
from hypothesis import given, settings, strategies as st

import moma_inputs as mi

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
M64 = (1 << 64) - 1
M32 = (1 << 32) - 1


# ----------------------------------------------------------------- vs Python int

@settings(max_examples=300, deadline=None)
@given(st.integers(1, 12), st.integers(1, 12), st.data())
def test_big_mul_matches_python(la, lb, data):
    import oracle
    a = data.draw(st.integers(0, (1 << (32 * la)) - 1))
    b = data.draw(st.integers(0, (1 << (32 * lb)) - 1))
    assert oracle.big_mul(a, b, la, lb) == a * b


@settings(max_examples=400, deadline=None)
@given(st.integers(1, 8), st.integers(0, 10), st.data())
def test_big_rem_matches_python(lv, extra, data):
    import oracle
    lu = lv + extra
    v = data.draw(st.integers(1, (1 << (32 * lv)) - 1))
    u = data.draw(st.integers(0, (1 << (32 * lu)) - 1))
    assert oracle.big_rem(u, v, lu, lv) == u % v


def test_big_rem_addback_branch_is_exercised():
    import oracle
    rng = random.Random(5)
    before = oracle.addback_count()
    for _ in range(2000):
        # divisor with a large second limb makes the two-limb estimate overshoot
        v = (1 << 95) | (rng.getrandbits(32) << 32) | M32
        u = rng.getrandbits(160)
        assert oracle.big_rem(u, v, 5, 3) == u % v
    assert oracle.addback_count() - before > 100


@pytest.mark.parametrize("n", [1, 2, 4, 8, 33])
def test_big_add_sub_carry_borrow(n):
    import oracle
    top = (1 << (32 * n)) - 1
    s, c = oracle.big_add(top, 1, n)
    assert (s, c) == (0, 1)                       # carry runs the whole chain
    d, b = oracle.big_sub(0, 1, n)
    assert (d, b) == (top, 1)                     # borrow runs the whole chain
    rng = random.Random(n)
    for _ in range(200):
        a, bb = rng.getrandbits(32 * n), rng.getrandbits(32 * n)
        s, c = oracle.big_add(a, bb, n)
        assert s + (c << (32 * n)) == a + bb
        d, br = oracle.big_sub(a, bb, n)
        assert d - (br << (32 * n)) == a - bb


@pytest.mark.parametrize("lam", [64, 128, 256, 384, 1024])
def test_mod_pow_and_inverse(lam):
    import oracle
    f = mi.find_prime(lam, 0)
    L = f.limbs
    rng = random.Random(lam)
    for _ in range(5):
        a, e = rng.randrange(1, f.q), rng.getrandbits(rng.choice([1, 7, 64, lam]))
        assert oracle.mod_pow(a, e, f.q, L) == pow(a, e, f.q)
        inv = oracle.mod_inv(a, f.q, L)
        assert inv * a % f.q == 1


# ----------------------------------------------------------------- paper listings

def smulmod_listing(a, b, q, mu, mbits):
    """Listing 1 _smulmod, word by word (64-bit words, 128-bit temporaries)."""
    t = a * b
    r = t >> (mbits - 2)
    r = r * mu
    r >>= (mbits + 5)
    t = t - r * q
    return t - q if t > q else t      # strict compare as printed


def test_single_word_barrett_listing_agrees_with_oracle():
    import oracle
    g = GOLDEN["barrett_single_word"]
    mbits = g["MBITS"]
    assert (mbits - 2, mbits + 5) == (g["pre_shift"], g["post_shift"])
    f = mi.find_prime(64, 0)                      # 60-bit prime: the listing's MBITS
    q = f.q
    assert q.bit_length() == mbits
    mu = (1 << (2 * mbits + 3)) // q              # reading: k = 2*MBITS + 3
    assert mu < (1 << 64)                         # mu fits one 64-bit word
    a = mi.residues(f, 2000, 2, 11)
    b = mi.residues(f, 2000, 2, 12)
    got = mi.rows_to_ints(oracle.vmul(q, 2, a, b))
    for x, y, c in zip(mi.rows_to_ints(a), mi.rows_to_ints(b), got):
        lst = smulmod_listing(x, y, q, mu, mbits)
        assert lst % q == c and 0 <= lst <= q    # one correction suffices; strict test leaves t == q


def _dmuls(a0, a1, b0, b1):
    """Listing 3: 2x2-word schoolbook product, words most-significant first."""
    s = a1 * b1; t0, t1 = s >> 64, s & M64
    s = a0 * b0; t2, t3 = s >> 64, s & M64
    s = a0 * b1; t4, t5 = s >> 64, s & M64
    s = a1 * b0; t6, t7 = s >> 64, s & M64
    # a0b1 + a1b0 as a 3-word value [t9, t10, t11]
    s = t5 + t7; t11 = s & M64; cr = s >> 64
    s = t4 + t6 + cr; t10 = s & M64; t9 = s >> 64
    # [t2, t3, t0, t1] + [t9, t10, t11, 0]
    c3 = t1
    s = t0 + t11; c2 = s & M64; cr = s >> 64
    s = t3 + t10 + cr; c1 = s & M64; cr = s >> 64
    c0 = (t2 + t9 + cr) & M64
    return c0, c1, c2, c3


def _qshr(a0, a1, a2, a3, b):
    """Listing 4 _qshr: [a0..a3] >> b for 64 <= b <= 128 -> 2 words (typos read per the text)."""
    i0, i1 = b - 64, 128 - b
    t0 = a2 >> i0
    t3 = (1 << i0) - 1
    t5 = ((a0 & t3) << i1) & M64
    t6 = a1 >> i0
    c0 = t5 | t6
    c1 = ((a1 << i1) & M64) | t0
    return c0, c1


def dmulmod_listing(a, b, q, mu, mbits=124):
    """Listing 4 _dmulmod with 64-bit words: Barrett on a double word."""
    a0, a1 = a >> 64, a & M64
    b0, b1 = b >> 64, b & M64
    q0, q1 = q >> 64, q & M64
    mu0, mu1 = mu >> 64, mu & M64
    t0, t1, t2, t3 = _dmuls(a0, a1, b0, b1)
    t4, t5 = _qshr(t0, t1, t2, t3, mbits - 2)
    t6, t7, t8, t9 = _dmuls(t4, t5, mu0, mu1)
    # [t6, t7, t8, t9] >> (MBITS + 5) = 129: keep the top two words shifted by one
    t10 = t6 >> 1
    t13 = ((t6 << 63) & M64) | (t7 >> 1)
    _, _, t16, t17 = _dmuls(t10, t13, q0, q1)
    # low double word of t minus low double word of r*q, then one conditional subtract
    low = ((t2 << 64) | t3) - ((t16 << 64) | t17)
    low &= (1 << 128) - 1
    return low - q if not low < q else low


def test_double_word_barrett_listing_agrees_with_oracle():
    import oracle
    g = GOLDEN["barrett_double_word"]
    assert (g["MBITS"] - 2, g["MBITS"] + 5) == (g["pre_shift"], g["post_shift"])
    f = mi.find_prime(128, 0)                     # 124-bit prime, the listing's MBITS
    q = f.q
    assert q.bit_length() == g["MBITS"]
    mu = (1 << (2 * g["MBITS"] + 3)) // q
    assert mu < (1 << 128)
    a = mi.residues(f, 2000, 4, 21)
    b = mi.residues(f, 2000, 4, 22)
    got = mi.rows_to_ints(oracle.vmul(q, 4, a, b))
    for x, y, c in zip(mi.rows_to_ints(a), mi.rows_to_ints(b), got):
        assert dmulmod_listing(x, y, q, mu) == c  # _dmulmod keeps t when t < q: canonical


def test_barrett_error_bound_reading():
    """The reading k = 2M+3 (M = bitlen q) gives a quotient estimate at most one short."""
    rng = random.Random(3)
    for lam in (64, 128, 256, 1024):
        q = mi.find_prime(lam, 0).q
        M = q.bit_length()
        mu = (1 << (2 * M + 3)) // q
        for _ in range(2000):
            t = rng.randrange(q) * rng.randrange(q)
            r = ((t >> (M - 2)) * mu) >> (M + 5)
            assert 0 <= t // q - r <= 1


# ----------------------------------------------------------------- rewrite rules (Table 1)

def _split(x, w=32):
    return x >> w, x & ((1 << w) - 1)


@settings(max_examples=300, deadline=None)
@given(st.integers(0, (1 << 64) - 1), st.integers(0, (1 << 64) - 1))
def test_rules_add_sub_mul_lt_eq_on_double_words(a, b):
    """Rules (addqdd)/(adc), (subddd), (mulqdd), (addqqq), (ltd), (eqd) with omega = 32."""
    import oracle
    a0, a1 = _split(a)
    b0, b1 = _split(b)
    # (addqdd) via (adc): [delta, c2] = a1 + b1 ; [c0, c1] = delta + a0 + b0
    s = a1 + b1
    delta, c2 = s >> 32, s & M32
    s = delta + a0 + b0
    c0, c1 = s >> 32, s & M32
    total, carry = oracle.big_add(a, b, 2)
    assert (carry << 64) | total == (c0 << 64) | (c1 << 32) | c2
    # (subddd): c1 = a1 - b1, delta = a1 < b1, c0 = a0 - b0 - delta (mod 2^32 each)
    d1 = (a1 - b1) & M32
    dl = int(a1 < b1)
    d0 = (a0 - b0 - dl) & M32
    diff, _ = oracle.big_sub(a, b, 2)
    assert diff == (d0 << 32) | d1
    # (ltd) and (eqd)
    assert (a < b) == ((a0 < b0) or (a0 == b0 and a1 < b1))
    assert (a == b) == (a0 == b0 and a1 == b1)
    # (mulqdd) then (addqqq): [e0,e1,d0,d1] + [h0,h1,h2,0]
    d = a1 * b1; e = a0 * b0; f_ = a0 * b1; g = a1 * b0
    h = f_ + g
    lhs = ((e >> 32) << 96) | ((e & M32) << 64) | ((d >> 32) << 32) | (d & M32)
    rhs = h << 32
    words_l = [(lhs >> (32 * k)) & M32 for k in range(4)]
    words_r = [(rhs >> (32 * k)) & M32 for k in range(4)]
    out, cr = [], 0
    for k in range(4):                             # ripple carry, least significant first
        s = words_l[k] + words_r[k] + cr
        out.append(s & M32)
        cr = s >> 32
    prod = sum(w << (32 * k) for k, w in enumerate(out))
    assert prod == oracle.big_mul(a, b, 2, 2) == a * b


def worked_addmod(a, b, q):
    """Eq. (final_addmod) with omega = 32, words most-significant first.

    The printed line for f uses q_2/q_1 and reuses delta_0; it is read as
    f1 = d2 - q1, delta = d2 < q1, f0 = d1 - q0 - delta.  Comparisons are strict
    as printed, so a + b == q yields q rather than 0.
    """
    a0, a1 = _split(a)
    b0, b1 = _split(b)
    q0, q1 = _split(q)
    s = a1 + b1
    dlt0, d2 = s >> 32, s & M32
    s = dlt0 + a0 + b0
    d0, d1 = s >> 32, s & M32
    dlt0 = (q0 < d1) or (q0 == d1 and q1 < d2)
    dlt1 = (0 < d0) or (d0 == 0 and dlt0)
    f1 = (d2 - q1) & M32
    br = int(d2 < q1)
    f0 = (d1 - q0 - br) & M32
    return (f0 << 32) | f1 if dlt1 else (d1 << 32) | d2


def test_worked_double_word_addmod_agrees_with_oracle():
    import oracle
    f = mi.find_prime(64, 0)
    q = f.q
    a = mi.residues(f, 3000, 2, 31)
    b = mi.residues(f, 3000, 2, 32)
    got = mi.rows_to_ints(oracle.vadd(q, 2, a, b))
    for x, y, c in zip(mi.rows_to_ints(a), mi.rows_to_ints(b), got):
        assert worked_addmod(x, y, q) == c
    # the strict comparison of the worked example leaves a + b == q unreduced;
    # the oracle returns the canonical residue 0
    x = q // 3
    assert worked_addmod(x, q - x, q) == q
    assert mi.rows_to_ints(oracle.vadd(q, 2, mi.ints_to_rows([x], 2), mi.ints_to_rows([q - x], 2))) == [0]


# ----------------------------------------------------------------- data-model constants

def test_paper_digit_and_word_counts():
    g = GOLDEN["decimal_example"]
    v = 0
    for dgt in g["digits_msd_first"]:
        v = v * g["base"] + dgt
    assert v == g["value"]
    w = GOLDEN["non_power_of_two_753"]
    words = -(-w["bits"] // w["machine_word"])
    assert words == w["words"]
    assert w["padded_words"] - words == w["zero_words"]
    assert -(-w["bits"] // 128) == w["words_128"] and 4 * 2 - -(-w["bits"] // 128) == w["zero_words_128"]
    assert -(-w["bits"] // 256) == w["words_256"] and 4 - w["words_256"] == w["zero_words_256"]
    r = GOLDEN["recursion_512"]
    assert r["bits"] // r["machine_word"] == r["words"] == 2 ** r["recursion_steps"]


@pytest.mark.parametrize("L", [1, 2, 3, 8, 16])
def test_digit_growth_bounds(L):
    """Adding two n-digit numbers needs n+1 digits, multiplying 2n (Section 2.2)."""
    import oracle
    top = (1 << (32 * L)) - 1
    s, c = oracle.big_add(top, top, L)
    assert c == 1 and ((c << (32 * L)) | s).bit_length() <= 32 * (L + 1)
    assert oracle.big_mul(top, top, L, L).bit_length() <= 64 * L
    assert oracle.big_mul(top, top, L, L).bit_length() > 64 * L - 32
