"""Pins for the oracle transforms (CPU only).

Brute force in pure Python on tiny n, closed forms, linearity, the shift
theorem, the round trip and the cyclic convolution theorem, plus agreement of
the fast textbook transform with the definition.
"""
import numpy as np
import pytest

import moma_inputs as mi


def py_ntt(x, w, q):
    n = len(x)
    return [sum(x[j] * pow(w, j * k, q) for j in range(n)) % q for k in range(n)]


@pytest.mark.parametrize("lam,logn", [(64, 1), (64, 5), (128, 4), (256, 6), (1024, 3)])
def test_direct_matches_pure_python(lam, logn):
    import oracle
    f = mi.find_prime(lam, 0)
    n, L = 1 << logn, f.limbs
    w = f.root(n)
    x = mi.residues(f, n, L, 40, logn)
    assert mi.rows_to_ints(oracle.ntt_direct(f.q, L, w, x)) == py_ntt(mi.rows_to_ints(x), w, f.q)


def test_n2_is_sum_and_difference():
    import oracle
    f = mi.find_prime(256, 0)
    x = mi.residues(f, 2, 8, 41)
    x0, x1 = mi.rows_to_ints(x)
    assert f.root(2) == f.q - 1
    y = mi.rows_to_ints(oracle.ntt_radix2(f.q, 8, f.root(2), x))
    assert y == [(x0 + x1) % f.q, (x0 - x1) % f.q]


@pytest.mark.parametrize("lam,logn", [(64, 8), (256, 10), (384, 7), (1024, 6)])
def test_radix2_matches_direct(lam, logn):
    import oracle
    f = mi.find_prime(lam, 0)
    n, L = 1 << logn, f.limbs
    w = f.root(n)
    x = mi.residues(f, n, L, 42, logn)
    assert (oracle.ntt_radix2(f.q, L, w, x) == oracle.ntt_direct(f.q, L, w, x)).all()
    assert (oracle.intt_radix2(f.q, L, w, x) == oracle.intt_direct(f.q, L, w, x)).all()


@pytest.mark.parametrize("logn", [0, 1, 2, 6, 11])
def test_closed_forms(logn):
    import oracle
    f = mi.find_prime(256, 0)
    n, L, q = 1 << logn, 8, f.q
    w = f.root(n)
    ev = mi.edge_vectors(f, n, L)
    # NTT(delta_0) = all ones ; NTT(ones) = n delta_0 ; NTT(delta_1)_k = w^k
    assert mi.rows_to_ints(oracle.ntt_radix2(q, L, w, ev["delta0"])) == [1] * n
    assert mi.rows_to_ints(oracle.ntt_radix2(q, L, w, ev["ones"])) == [n % q] + [0] * (n - 1)
    if n > 1:
        assert mi.rows_to_ints(oracle.ntt_radix2(q, L, w, ev["delta1"])) == [pow(w, k, q) for k in range(n)]
    assert (oracle.ntt_radix2(q, L, w, ev["zeros"]) == 0).all()


def test_linearity_and_shift_theorem():
    import oracle
    f = mi.find_prime(384, 0)
    n, L, q = 512, 12, f.q
    w = f.root(n)
    a, b = mi.residues(f, n, L, 50), mi.residues(f, n, L, 51)
    ya, yb = oracle.ntt_radix2(q, L, w, a), oracle.ntt_radix2(q, L, w, b)
    assert (oracle.ntt_radix2(q, L, w, oracle.vadd(q, L, a, b)) == oracle.vadd(q, L, ya, yb)).all()
    # x rotated so that x'_j = x_{j-1}: y'_k = w^k y_k
    xr = np.roll(a, 1, axis=0)
    yr = mi.rows_to_ints(oracle.ntt_radix2(q, L, w, xr))
    assert yr == [(pow(w, k, q) * v) % q for k, v in enumerate(mi.rows_to_ints(ya))]


@pytest.mark.parametrize("lam,logn", [(64, 12), (256, 12), (1024, 9)])
def test_roundtrip(lam, logn):
    import oracle
    f = mi.find_prime(lam, 0)
    n, L = 1 << logn, f.limbs
    w = f.root(n)
    x = mi.residues(f, n, L, 60, logn)
    assert (oracle.intt_radix2(f.q, L, w, oracle.ntt_radix2(f.q, L, w, x)) == x).all()
    assert (oracle.ntt_radix2(f.q, L, w, oracle.intt_radix2(f.q, L, w, x)) == x).all()


@pytest.mark.parametrize("lam,logn", [(128, 6), (256, 8), (768, 5)])
def test_cyclic_convolution_theorem(lam, logn):
    import oracle
    f = mi.find_prime(lam, 0)
    n, L, q = 1 << logn, f.limbs, f.q
    w = f.root(n)
    a, b = mi.residues(f, n, L, 70), mi.residues(f, n, L, 71)
    conv = oracle.cyclic_conv(q, L, a, b)
    ai, bi = mi.rows_to_ints(a), mi.rows_to_ints(b)
    if n <= 64:   # brute force in Python as well
        assert mi.rows_to_ints(conv) == [sum(ai[i] * bi[(k - i) % n] for i in range(n)) % q for k in range(n)]
    via = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, oracle.ntt_radix2(q, L, w, a), oracle.ntt_radix2(q, L, w, b)))
    assert (via == conv).all()


def test_sampled_direct_matches_fast_at_larger_n():
    import oracle
    f = mi.find_prime(256, 0)
    n, L = 1 << 14, 8
    w = f.root(n)
    x = mi.residues(f, n, L, 80)
    y = oracle.ntt_radix2(f.q, L, w, x)
    ks = np.array([0, 1, 2, n // 2, n - 1, 12345], dtype=np.int64)
    assert (oracle.ntt_direct(f.q, L, w, x, ks) == y[ks]).all()
    js = np.array([0, 7, n - 1], dtype=np.int64)
    assert (oracle.intt_direct(f.q, L, w, y, js) == x[js]).all()


def test_root_order_is_exact():
    """omega_n has order exactly n, and omega_{2n}^2 = omega_n (the roots nest)."""
    import oracle
    f = mi.find_prime(256, 0)
    for logn in (1, 5, 20, 32):
        n = 1 << logn
        w = f.root(n)
        assert oracle.mod_pow(w, n, f.q, 8) == 1
        assert oracle.mod_pow(w, n // 2, f.q, 8) == f.q - 1
        if logn < 32:
            assert pow(f.root(2 * n), 2, f.q) == w


@pytest.mark.parametrize("lam,logn", [(64, 5), (256, 4)])
def test_full_width_modulus_direct_matches_pure_python(lam, logn):
    import oracle
    f = mi.find_prime(lam, 0, bits=lam)
    n, L = 1 << logn, f.limbs
    w = f.root(n)
    x = mi.residues(f, n, L, 42, logn)
    assert mi.rows_to_ints(oracle.ntt_radix2(f.q, L, w, x)) == py_ntt(mi.rows_to_ints(x), w, f.q)
