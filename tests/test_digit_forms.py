"""CPU model of the transform's digit-form twiddle multiply, schoolbook and
Karatsuba (Eq. (mulk)), in exact Python integers: the column sums the kernels
keep in 64-bit accumulators never overflow at any compute limb count the
kernels run them at, and the product scan returns y*w*2^(-bD) mod q in
[0, 2q).  (The GPU results themselves are compared with the oracle in the
-m gpu tests; this pins the arithmetic the kernels are written from.)"""
import random

import pytest

import moma_inputs as mi


def digits(L, fw=False):
    b = 29 if L <= 28 else 28
    D = -(-(32 * L - (0 if fw else 2)) // b)
    return b, D


def split(v, b, D):
    return [(v >> (b * i)) & ((1 << b) - 1) for i in range(D)]


def mont_digits(y, w, q, L, kara=False, fw=False):
    """The product scan of the kernels, column by column, with the carried
    accumulator checked against 2^64 after every addition."""
    b, D = digits(L, fw)
    mask = (1 << b) - 1
    a, wd, qd = split(y, b, D), split(w, b, D), split(q, b, D)
    qinvd = (-pow(q, -1, 1 << b)) % (1 << b)
    if kara:
        h, g = (D + 1) // 2, D // 2
        sa = [a[i] + (a[h + i] if i < g else 0) for i in range(h)]
        sw = [wd[i] + (wd[h + i] if i < g else 0) for i in range(h)]
        p = [0] * (2 * D - 1)
        for c in range(2 * h - 1):
            z0 = sum(a[i] * wd[c - i] for i in range(max(0, c - h + 1), min(c, h - 1) + 1))
            zm = sum(sa[i] * sw[c - i] for i in range(max(0, c - h + 1), min(c, h - 1) + 1))
            z2 = 0
            if c <= 2 * g - 2:
                z2 = sum(a[h + i] * wd[h + c - i] for i in range(max(0, c - g + 1), min(c, g - 1) + 1))
                p[c + 2 * h] += z2
            assert zm < 2 ** 64 and z0 + z2 <= zm
            p[c] += z0
            p[c + h] += zm - z0 - z2
        assert all(v < 2 ** 64 for v in p)
    else:
        p = [sum(a[j] * wd[c - j] for j in range(max(0, c - D + 1), min(c, D - 1) + 1)) for c in range(2 * D - 1)]
    m, r, acc = [0] * D, [0] * D, 0
    for i in range(D):
        acc += p[i] + sum(m[j] * qd[i - j] for j in range(i))
        assert acc < 2 ** 64
        m[i] = (acc * qinvd) & mask
        acc += m[i] * qd[0]
        assert acc < 2 ** 64 and acc & mask == 0
        acc >>= b
    for i in range(D, 2 * D - 1):
        acc += p[i] + sum(m[j] * qd[i - j] for j in range(i - D + 1, D))
        assert acc < 2 ** 64
        r[i - D] = acc & mask
        acc >>= b
    r[D - 1] = acc
    return sum(v << (b * i) for i, v in enumerate(r)), b * D, r


def stream_limbs(r, b, L, fw):
    """The kernels' result scan: each digit joins a 64-bit bit buffer and every
    32-bit limb leaves as soon as its bits are in; whatever is left after the
    last digit is the top limb (and, full width, the carry word)."""
    bits, nb, j, t = 0, 0, 0, [None] * L
    for dig in r:
        assert dig < 2 ** 32 and nb < 32
        bits |= dig << nb
        assert bits < 2 ** 64
        nb += b
        while nb >= 32 and j < L:
            t[j], j, bits, nb = bits & 0xFFFFFFFF, j + 1, bits >> 32, nb - 32
    if j < L:
        t[j], j = bits & 0xFFFFFFFF, j + 1
    assert j == L and None not in t
    top = bits & 0xFFFFFFFF if fw else 0
    return sum(v << (32 * k) for k, v in enumerate(t)) + (top << (32 * L))


@pytest.mark.parametrize("L", [2, 3, 5, 8, 9, 12, 16, 17, 23, 24])
def test_karatsuba_digit_product_matches_schoolbook_and_definition(L):
    f = mi.find_prime(32 * L, 0)
    q = f.q
    rng = random.Random(L)
    # lazy operands: y < 4q, the twiddle w < q; all-ones digits for the carry-free sums
    cases = [(4 * q - 1, q - 1), (q - 1, q - 1), ((1 << (32 * L - 2)) - 1, q - 1)]
    cases += [(rng.randrange(4 * q), rng.randrange(q)) for _ in range(20)]
    for y, w in cases:
        y = min(y, 4 * q - 1)
        t_s, bd, _ = mont_digits(y, w, q, L)
        t_k, _, _ = mont_digits(y, w, q, L, kara=True)
        assert t_s == t_k
        assert t_s < 2 * q and t_s % q == y * w * pow(2, -bd, q) % q


@pytest.mark.parametrize("L", [2, 4, 8, 10, 20, 32])
def test_full_width_digit_product_carries_the_top_bit(L):
    """A full-width modulus: digits over 32L bits, result below 2q that may
    reach 2^(32L) (the carry word the kernels keep)."""
    f = mi.find_prime(32 * L, 0, bits=32 * L)
    q = f.q
    rng = random.Random(100 + L)
    for y, w in [(q - 1, q - 1)] + [(rng.randrange(q), rng.randrange(q)) for _ in range(100)]:
        t, bd, _ = mont_digits(y, w, q, L, fw=True)
        assert t < 2 * q and t % q == y * w * pow(2, -bd, q) % q


@pytest.mark.parametrize("fw", [False, True])
def test_streamed_result_limbs_at_every_limb_count(fw):
    """The result limbs leave the product scan through a 64-bit buffer; at 10
    and 20 limbs the digits cover 32L - 1 bits only, so the top limb is still in
    the buffer after the last digit."""
    rng = random.Random(7 + fw)
    for L in range(2, 33):
        f = mi.find_prime(32 * L, 0, bits=32 * L) if fw else mi.find_prime(32 * L - 4, 0)
        q = f.q
        hi = q if fw else 4 * q
        for y, w in [(hi - 1, q - 1)] + [(rng.randrange(hi), rng.randrange(q)) for _ in range(6)]:
            t, _, r = mont_digits(y, w, q, L, fw=fw)
            b, _ = digits(L, fw)
            assert stream_limbs(r, b, L, fw) == t, L


def test_karatsuba_digit_sum_columns_fit_64_bits():
    """The widest column of digit-sum products, h (2^(b+1) - 2)^2, stays below
    2^64 at every compute limb count (the kernels run the Karatsuba form at 2
    to 24 limbs; the bound is not what limits them)."""
    for L in range(2, 33):
        b, D = digits(L)
        h = (D + 1) // 2
        assert h * (2 ** (b + 1) - 2) ** 2 < 2 ** 64, L
