"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/moma.h declares, and rejects invalid arguments on the host before any
HIP call (every case here fails validation, so no kernel is ever launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "moma.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(moma_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("moma_ntt_fwd", "moma_ntt_inv", "moma_vadd", "moma_vsub", "moma_vmul", "moma_axpy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2501_07535_amd as moma
    lib = moma.library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(moma.EXPORTED) <= set(declared_functions())


def test_product_path_does_not_reference_oracle():
    pkg = os.path.join(ROOT, "paper_2501_07535_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def _w(v, L):
    return (ctypes.c_uint32 * L)(*[(v >> (32 * j)) & 0xFFFFFFFF for j in range(L)])


DUMMY = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def test_error_codes_and_strings():
    import paper_2501_07535_amd as moma
    lib = moma.library()
    assert lib.moma_strerror(0) == b"MOMA_OK"
    for code in (-1, -2, -3, -4, -5, -6):
        assert lib.moma_strerror(code).startswith(b"MOMA_E_")
    assert b"gfx950" in lib.moma_version()


@pytest.mark.parametrize("case", ["limbs_low", "limbs_high", "q_even", "q_too_wide", "q_null", "q_small"])
def test_blas_rejects_bad_modulus(case):
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    L, q = 8, f.q
    if case == "limbs_low":
        rc = lib.moma_vadd(_w(q, 8), 1, 10, DUMMY, DUMMY, DUMMY, None)
        assert rc == moma.MOMA_E_ARG
    elif case == "limbs_high":
        rc = lib.moma_vadd(_w(q, 33), 33, 10, DUMMY, DUMMY, DUMMY, None)
        assert rc == moma.MOMA_E_ARG
    elif case == "q_even":
        rc = lib.moma_vmul(_w(q + 1, L), L, 10, DUMMY, DUMMY, DUMMY, None)
        assert rc == moma.MOMA_E_MODULUS
    elif case == "q_too_wide":
        # full width (no headroom) is accepted up to 1024 bits (n = 0: validation only)
        assert lib.moma_vsub(_w((1 << 1023) + 1, 32), 32, 0, None, None, None, None) == 0
        assert lib.moma_vsub(_w((1 << 255) + 1, L), L, 0, None, None, None, None) == 0
    elif case == "q_null":
        rc = lib.moma_vadd(None, L, 10, DUMMY, DUMMY, DUMMY, None)
        assert rc == moma.MOMA_E_ARG
    elif case == "q_small":
        rc = lib.moma_vadd(_w(1, L), L, 10, DUMMY, DUMMY, DUMMY, None)
        assert rc == moma.MOMA_E_MODULUS
    assert lib.moma_last_error_detail()


def test_blas_rejects_null_vectors_and_bad_alpha():
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    assert lib.moma_vadd(_w(f.q, 8), 8, 10, None, DUMMY, DUMMY, None) == moma.MOMA_E_ARG
    assert lib.moma_axpy(_w(f.q, 8), 8, 10, None, DUMMY, DUMMY, DUMMY, None) == moma.MOMA_E_ARG
    assert lib.moma_axpy(_w(f.q, 8), 8, 10, _w(f.q, 8), DUMMY, DUMMY, DUMMY, None) == moma.MOMA_E_ARG
    assert lib.moma_vadd(_w(f.q, 8), 8, (1 << 31) + 1, DUMMY, DUMMY, DUMMY, None) == moma.MOMA_E_ARG
    # n == 0 is a no-op that touches nothing
    assert lib.moma_vmul(_w(f.q, 8), 8, 0, None, None, None, None) == 0


@pytest.mark.parametrize("case", ["n_not_pow2", "n_too_big", "n_one", "omega_order", "omega_ge_q", "omega_null",
                                  "n_not_dividing"])
def test_ntt_rejects_bad_arguments(case):
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    q, L, n = f.q, 8, 1 << 10
    w = f.root(n)
    want = moma.MOMA_E_ARG
    if case == "n_not_pow2":
        args = (_w(q, L), _w(w, L), 1000)
    elif case == "n_too_big":
        args = (_w(q, L), _w(w, L), 1 << 27)
    elif case == "n_one":
        args = (_w(q, L), _w(w, L), 1)
    elif case == "omega_order":
        args, want = (_w(q, L), _w(f.root(n // 2), L), n), moma.MOMA_E_ROOT   # order n/2, not n
    elif case == "omega_ge_q":
        args, want = (_w(q, L), _w(q, L), n), moma.MOMA_E_ROOT
    elif case == "omega_null":
        args = (_w(q, L), None, n)
    else:   # n = 2^33 does not divide q - 1 (2-adicity 33) -> too big anyway; use a prime with small 2-adicity
        q2 = 1000000007                                 # q2 - 1 = 2 * 500000003
        args, want = (_w(q2, 2), _w(q2 - 1, 2), 4), moma.MOMA_E_ROOT
        assert lib.moma_ntt_fwd(*args, 2, DUMMY, DUMMY, None) == want
        return
    assert lib.moma_ntt_fwd(*args, L, DUMMY, DUMMY, None) == want
    assert lib.moma_ntt_inv(*args, L, DUMMY, DUMMY, None) == want
    assert lib.moma_ntt_cyclic_mul(*args, L, DUMMY, DUMMY, DUMMY, None) == want
    assert lib.moma_ntt_prepare(*args, L) == want


def test_cyclic_mul_rejects_null_buffers():
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    q, w = _w(f.q, 8), _w(f.root(64), 8)
    for bufs in ((None, DUMMY, DUMMY), (DUMMY, None, DUMMY), (DUMMY, DUMMY, None)):
        assert lib.moma_ntt_cyclic_mul(q, w, 64, 8, *bufs, None) == moma.MOMA_E_ARG


def test_vmul_variant_validation():
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    assert lib.moma_vmul_set_variant(_w(f.q, 8), 8, 2) == moma.MOMA_E_ARG
    assert lib.moma_vmul_get_variant(_w(f.q, 8), 8, None) == moma.MOMA_E_ARG
    # a 27-bit modulus computes in one limb: no Karatsuba split
    small = (1 << 27) - (1 << 12) + 1   # odd, 27 bits
    assert lib.moma_vmul_set_variant(_w(small, 2), 2, 1) == moma.MOMA_E_UNSUPPORTED
    assert moma.vmul_get_variant(f.q, 8) == moma.VMUL_SCHOOLBOOK
    moma.vmul_set_variant(f.q, 8, moma.VMUL_KARATSUBA)
    assert moma.vmul_get_variant(f.q, 8) == moma.VMUL_KARATSUBA
    assert moma.vmul_get_variant(f.q, 9) == moma.VMUL_KARATSUBA     # same compute limb count
    moma.vmul_set_variant(f.q, 8, moma.VMUL_SCHOOLBOOK)
    buf = (ctypes.c_float * 2)()
    assert lib.moma_vmul_tune(_w(f.q, 8), 8, 0, 3, buf, None) == moma.MOMA_E_ARG
    assert lib.moma_vmul_tune(_w(f.q, 8), 8, 16, 3, None, None) == moma.MOMA_E_ARG


def test_input_check_rejects_bad_arguments_on_the_host():
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0)
    L, q = f.limbs, f.q
    bad = ctypes.c_uint64(7)
    assert lib.moma_check_canonical(_w(q, L), L, 16, DUMMY, None, None) == moma.MOMA_E_ARG
    assert lib.moma_check_canonical(_w(q, L), L, (1 << 31) + 1, DUMMY, ctypes.byref(bad), None) == moma.MOMA_E_ARG
    assert lib.moma_check_canonical(_w(q, L), L, 16, None, ctypes.byref(bad), None) == moma.MOMA_E_ARG
    assert lib.moma_check_canonical(_w(q + 1, L), L, 16, DUMMY, ctypes.byref(bad), None) == moma.MOMA_E_MODULUS
    assert lib.moma_check_canonical(_w(q, L), 1, 16, DUMMY, ctypes.byref(bad), None) == moma.MOMA_E_ARG
    assert lib.moma_check_canonical(_w(q, L), L, 0, None, ctypes.byref(bad), None) == moma.MOMA_OK
    assert bad.value == 0                                       # an empty vector has nothing to count
    assert lib.moma_set_input_check(1) == moma.MOMA_OK and lib.moma_set_input_check(0) == moma.MOMA_OK


def test_layout_conversion_rejects_bad_arguments_on_the_host():
    import paper_2501_07535_amd as moma
    lib = moma.library()
    other = ctypes.c_void_p(0x2000)
    for fn in (lib.moma_pack_planar, lib.moma_unpack_planar):
        assert fn(1, 16, DUMMY, other, None) == moma.MOMA_E_ARG             # limbs below 2
        assert fn(33, 16, DUMMY, other, None) == moma.MOMA_E_ARG            # limbs above 32
        assert fn(8, (1 << 31) + 1, DUMMY, other, None) == moma.MOMA_E_ARG
        assert fn(8, 16, None, other, None) == moma.MOMA_E_ARG
        assert fn(8, 16, DUMMY, DUMMY, None) == moma.MOMA_E_ARG             # in place
        assert fn(8, 0, None, None, None) == moma.MOMA_OK                   # nothing to move
