"""The allocation-free cyclic product (moma_ntt_cyclic_mul_noalloc), called
through the raw C ABI: bit for bit the same output as moma_ntt_cyclic_mul on
two calls in a row (the second smaller, so it runs over what the first left in
the shared scratch array), device free memory unchanged by the calls, the
oracle's definition on the small case, and its host-side refusals (no plan,
more scratch than the fixed array holds)."""
import ctypes

import numpy as np
import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _w(v, L):
    return (ctypes.c_uint32 * L)(*[(v >> (32 * j)) & 0xFFFFFFFF for j in range(L)])


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(lib, f, L, n, w, da, db, dc):
    return lib.moma_ntt_cyclic_mul_noalloc(_w(f.q, L), _w(w, L), n, L, ctypes.c_void_p(da.data_ptr()),
                                           ctypes.c_void_p(db.data_ptr()), ctypes.c_void_p(dc.data_ptr()), _stream())


def _plain(lib, f, L, n, w, da, db, dc):
    return lib.moma_ntt_cyclic_mul(_w(f.q, L), _w(w, L), n, L, ctypes.c_void_p(da.data_ptr()),
                                   ctypes.c_void_p(db.data_ptr()), ctypes.c_void_p(dc.data_ptr()), _stream())


@pytest.mark.parametrize("lam,big,small", [(256, 20, 9), (1024, 13, 6), (64, 16, 12)])
def test_noalloc_matches_cyclic_mul_on_two_calls(lam, big, small):
    import torch

    import oracle
    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(lam, 0)
    L = f.limbs
    cases = []
    for logn in (big, small):
        n = 1 << logn
        w = f.root(n)
        a, b = mi.residues(f, n, L, 930, logn), mi.residues(f, n, L, 931, logn)
        assert lib.moma_ntt_prepare(_w(f.q, L), _w(w, L), n, L) == 0
        cases.append((logn, n, w, a, b, to_dev(a), to_dev(b)))
    outs = [torch.full_like(c[5], -1) for c in cases]
    # one untimed call first: the code object holding the scratch array is
    # loaded (and its memory taken) on first use, once per process
    logn, n, w, a, b, da, db = cases[1]
    assert _noalloc(lib, f, L, n, w, da, db, outs[1]) == 0
    torch.cuda.synchronize()
    outs[1].fill_(-1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (logn, n, w, a, b, da, db), dc in zip(cases, outs):
        say(f"noalloc cyclic product lam={lam} logn={logn}")
        assert _noalloc(lib, f, L, n, w, da, db, dc) == 0, moma.library().moma_last_error_detail()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0  # nothing allocated on the device by either call
    for (logn, n, w, a, b, da, db), dc in zip(cases, outs):
        ref = torch.empty_like(dc)
        say(f"plain cyclic product lam={lam} logn={logn}")
        assert _plain(lib, f, L, n, w, da, db, ref) == 0
        torch.cuda.synchronize()
        assert torch.equal(dc, ref), f"logn={logn}: differs from moma_ntt_cyclic_mul"
    logn, n, w, a, b, da, db = cases[1]
    got = from_dev(outs[1])
    if logn <= 9:
        assert (got == oracle.cyclic_conv(f.q, L, a, b)).all()
    else:
        want = oracle.intt_radix2(f.q, L, w, oracle.vmul(f.q, L, oracle.ntt_radix2(f.q, L, w, a),
                                                          oracle.ntt_radix2(f.q, L, w, b)))
        assert (got == want).all()


def test_noalloc_full_width_and_in_place():
    """A full-width modulus with the output over one input, against the plain
    call."""
    import torch

    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 0, bits=256)
    L = f.limbs
    for logn in (14, 7):
        n = 1 << logn
        w = f.root(n)
        a, b = mi.residues(f, n, L, 932, logn), mi.residues(f, n, L, 933, logn)
        assert lib.moma_ntt_prepare(_w(f.q, L), _w(w, L), n, L) == 0
        da, db = to_dev(a), to_dev(b)
        ref = torch.empty_like(da)
        say(f"noalloc full width logn={logn}")
        assert _plain(lib, f, L, n, w, da, db, ref) == 0
        assert _noalloc(lib, f, L, n, w, da, db, da) == 0  # out == a
        torch.cuda.synchronize()
        assert torch.equal(da, ref)


def test_noalloc_refusals():
    import torch

    import paper_2501_07535_amd as moma
    lib = moma.library()
    f = mi.find_prime(256, 1)
    L = f.limbs
    d = torch.zeros((L, 1 << 21), dtype=torch.int32, device="cuda:0")
    # no plan yet for this (q, omega, n): refused, nothing enqueued
    n = 1 << 10
    w = f.root(n)
    dv = d[:, :n].contiguous()
    assert _noalloc(lib, f, L, n, w, dv, dv, dv) == moma.MOMA_E_ARG
    assert b"moma_ntt_prepare" in lib.moma_last_error_detail()
    # 2 n L words above the fixed array: refused on the host
    n = 1 << 21
    w = f.root(n)
    assert lib.moma_ntt_prepare(_w(f.q, L), _w(w, L), n, L) == 0
    assert 2 * n * L > moma.NOALLOC_SCRATCH_WORDS
    assert _noalloc(lib, f, L, n, w, d, d, d) == moma.MOMA_E_ARG
    assert b"scratch" in lib.moma_last_error_detail()
    torch.cuda.synchronize()
    assert not (d != 0).any()
