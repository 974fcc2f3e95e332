"""Seeded input generator: SplitMix64, primes, roots, residues (CPU only)."""
import numpy as np
import pytest
import sympy

import moma_inputs as mi


def test_splitmix64_reference_outputs():
    # First outputs of SplitMix64 seeded with 1234567, as printed by the
    # reference C implementation (Steele, Lea, Flood 2014; Vigna's splitmix64.c).
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [int(v) for v in mi.splitmix64(1234567, 0, 5)] == want


def test_splitmix64_vector_matches_scalar():
    key = mi.stream_key(3, 1, 4)
    v = mi.splitmix64(key, 100, 1000)
    assert all(int(v[i]) == mi.splitmix64_scalar(key, 100 + i) for i in range(0, 1000, 37))


@pytest.mark.parametrize("lam", [64, 96, 128, 256, 384, 512, 768, 1024])
def test_prime_shape(lam):
    f = mi.find_prime(lam, 0)
    assert f.q.bit_length() == lam - 4
    assert (f.q - 1) % (1 << 32) == 0
    assert sympy.isprime(f.q)
    assert pow(f.z, (f.q - 1) // 2, f.q) == f.q - 1
    for n in (2, 1 << 10, 1 << 24):
        w = f.root(n)
        assert pow(w, n, f.q) == 1 and pow(w, n // 2, f.q) == f.q - 1


def test_prime_deterministic_and_distinct():
    assert mi.find_prime(256, 0).q == mi.find_prime(256, 0).q
    assert mi.find_prime(256, 0).q != mi.find_prime(256, 1).q


def test_miller_rabin_against_sympy():
    rng = np.random.default_rng(7)
    for _ in range(300):
        n = int(rng.integers(2, 1 << 62)) | 1
        assert mi.is_probable_prime(n) == sympy.isprime(n)
    # Carmichael numbers and squares of primes
    for n in (561, 1105, 1729, 2465, 2821, 6601, 8911, 41041, 7919 ** 2):
        assert not mi.is_probable_prime(n)


@pytest.mark.parametrize("lam,L", [(64, 2), (256, 8), (384, 12), (256, 10)])
def test_residues_uniform_range_and_deterministic(lam, L):
    f = mi.find_prime(lam, 0)
    x = mi.residues(f, 4096, L, 9, 9)
    vals = mi.rows_to_ints(x)
    assert all(0 <= v < f.q for v in vals)
    assert len(set(vals)) == len(vals)
    assert (mi.residues(f, 4096, L, 9, 9) == x).all()
    top = max(vals)
    assert top.bit_length() == f.q.bit_length()
    # zero upper limbs when L exceeds the limbs of q
    Lq = (f.q.bit_length() + 31) // 32
    assert (x[:, Lq:] == 0).all()


def test_planar_roundtrip():
    f = mi.find_prime(256, 0)
    x = mi.residues(f, 100, 8, 1)
    p = mi.to_planar(x)
    assert p.shape == (8, 100) and (mi.from_planar(p) == x).all()
    assert p[3, 17] == x[17, 3]
