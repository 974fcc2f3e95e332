"""Pins for the oracle's elementwise operations (CPU only): Python int and edge cases."""
import numpy as np
import pytest

import moma_inputs as mi


@pytest.mark.parametrize("lam,L", [(64, 2), (128, 4), (256, 8), (384, 12), (768, 24), (1024, 32), (256, 10)])
def test_blas_matches_python_int(lam, L):
    import oracle
    f = mi.find_prime(lam, 0)
    q = f.q
    n = 300
    a, b, y = (mi.residues(f, n, L, k) for k in (1, 2, 3))
    alpha = mi.scalar_residue(f, 4)
    ai, bi, yi = mi.rows_to_ints(a), mi.rows_to_ints(b), mi.rows_to_ints(y)
    assert mi.rows_to_ints(oracle.vadd(q, L, a, b)) == [(u + v) % q for u, v in zip(ai, bi)]
    assert mi.rows_to_ints(oracle.vsub(q, L, a, b)) == [(u - v) % q for u, v in zip(ai, bi)]
    assert mi.rows_to_ints(oracle.vmul(q, L, a, b)) == [(u * v) % q for u, v in zip(ai, bi)]
    assert mi.rows_to_ints(oracle.axpy(q, L, alpha, a, y)) == [(alpha * u + v) % q for u, v in zip(ai, yi)]


@pytest.mark.parametrize("lam", [64, 256, 768])
def test_blas_edge_cases(lam):
    import oracle
    f = mi.find_prime(lam, 0)
    q, L = f.q, f.limbs
    ev = mi.edge_vectors(f, 16, L)
    for name, a in ev.items():
        for name2, b in ev.items():
            ai, bi = mi.rows_to_ints(a), mi.rows_to_ints(b)
            assert mi.rows_to_ints(oracle.vadd(q, L, a, b)) == [(u + v) % q for u, v in zip(ai, bi)], (name, name2)
            assert mi.rows_to_ints(oracle.vsub(q, L, a, b)) == [(u - v) % q for u, v in zip(ai, bi)], (name, name2)
            assert mi.rows_to_ints(oracle.vmul(q, L, a, b)) == [(u * v) % q for u, v in zip(ai, bi)], (name, name2)
    a, b = mi.sum_to_q_pair(f, 64, L, 7)
    assert (oracle.vadd(q, L, a, b) == 0).all()          # a + b == q reduces to 0 (canonical)
    assert (oracle.vsub(q, L, a, a) == 0).all()
    qm1 = q - 1
    assert mi.rows_to_ints(oracle.axpy(q, L, qm1, ev["all_qm1"], ev["all_qm1"])) == [(qm1 * qm1 + qm1) % q] * 16


def test_blas_empty_vectors():
    import oracle
    f = mi.find_prime(256, 0)
    z = np.zeros((0, 8), dtype=np.uint32)
    assert oracle.vadd(f.q, 8, z, z).shape == (0, 8)
    assert oracle.axpy(f.q, 8, 5, z, z).shape == (0, 8)


@pytest.mark.parametrize("lam", [64, 256, 992])
def test_full_width_modulus_matches_python_int(lam):
    """A modulus as wide as its storage (bitlen(q) = 32 limbs): the oracle's
    products and sums still equal Python's."""
    import oracle
    f = mi.find_prime(lam, 0, bits=lam)
    q, L = f.q, f.limbs
    assert q.bit_length() == 32 * L
    a, b = mi.residues(f, 200, L, 8, 1), mi.residues(f, 200, L, 8, 2)
    ai, bi = mi.rows_to_ints(a), mi.rows_to_ints(b)
    assert mi.rows_to_ints(oracle.vadd(q, L, a, b)) == [(u + v) % q for u, v in zip(ai, bi)]
    assert mi.rows_to_ints(oracle.vsub(q, L, a, b)) == [(u - v) % q for u, v in zip(ai, bi)]
    assert mi.rows_to_ints(oracle.vmul(q, L, a, b)) == [(u * v) % q for u, v in zip(ai, bi)]
