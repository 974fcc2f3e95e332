"""Transforms at every compute limb count and at the largest sizes, bit-exact
against the oracle (Eq. (ntt); the paper's non-power-of-two widths, Section 4,
are limb counts that are not powers of two).

Every compute limb count L from 2 to 32 (a (32L - 4)-bit prime, the paper's
class width less four bits) runs a multi-pass forward and inverse transform
under its default launch shape and under sampled feasible shapes of every
register radix the limb count allows; whole vectors are compared with the
oracle's radix-2 transforms.  L = 10 and 11 sit on the boundary of three
kernel paths (the store fused into the last round and 16-byte stores, up to
10 limbs; the radix-2 round that loads its second operand late, from 11
limbs), L = 16 and 17 on that of the radix-4 units (up to 16 limbs), so these
get explicit shapes that take each path.
"""
import random

import numpy as np
import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _field(L):
    return mi.find_prime(32 * L, 0)


def _shapes(moma, L, logn, extra=()):
    """The default shape, the given ones, and one sampled multi-pass shape per
    register radix (seeded by L)."""
    cands = [tuple(s) for s in moma.ntt_candidates(L, logn)]
    multi = [s for s in cands if s[0] < logn]
    rng = random.Random(1000 + L)
    rng.shuffle(multi)
    picks = [tuple(moma.ntt_default_schedule(L, logn))] + [tuple(s) for s in extra]
    for r in sorted({s[3] for s in multi}):
        picks.append(next(s for s in multi if s[3] == r))
    # two more of any radix, for the column counts and thread counts
    picks += multi[:2]
    out = []
    for s in picks:
        if s not in out:
            out.append(s)
    return out


def _check_shapes(L, logn, shapes, seed):
    import oracle
    import paper_2501_07535_amd as moma
    f = _field(L)
    assert (f.q.bit_length() + 4 + 31) // 32 == L
    n, q = 1 << logn, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, seed, L, logn)
    want_f = oracle.ntt_radix2(q, L, w, x)
    want_i = oracle.intt_radix2(q, L, w, x)
    dx = to_dev(x)
    ran = 0
    try:
        for s in shapes:
            try:
                moma.ntt_set_schedule(q, w, n, L, s)
            except moma.MomaError as e:
                assert e.code in (moma.MOMA_E_UNSUPPORTED, moma.MOMA_E_ARG), (s, e)
                continue
            passes = moma.ntt_describe(q, w, n, L)["passes"]
            say(f"limbs L={L} logn={logn} sched={s} passes={passes}")
            assert (from_dev(moma.ntt_fwd(dx, q, w)) == want_f).all(), s
            assert (from_dev(moma.ntt_inv(dx, q, w)) == want_i).all(), s
            ran += 1
        # in place, under the last shape
        d = dx.clone()
        moma.ntt_fwd(d, q, w, out=d)
        assert (from_dev(d) == want_f).all()
        moma.ntt_inv(d, q, w, out=d)
        assert (from_dev(d) == x).all()
    finally:
        moma.ntt_set_schedule(q, w, n, L, None)
    return ran


@pytest.mark.parametrize("L", list(range(2, 33)))
def test_every_compute_limb_count(L):
    import paper_2501_07535_amd as moma
    logn = 13 if L <= 16 else 12
    shapes = _shapes(moma, L, logn)
    ran = _check_shapes(L, logn, shapes, 500)
    assert ran >= 2


# (tile_log, col_log, threads, radix_log) at n = 2^14, two or three passes:
# 16 or 32 columns (later passes store from the last round's registers up to
# 10 limbs), 4 or 8 columns (16-byte stores from LDS up to 10 limbs, one word
# per lane above), radix-4 units (up to 16 limbs) and radix-2 units
BOUNDARY_SHAPES = [(10, 4, 256, 2), (10, 5, 256, 2), (10, 3, 256, 2), (10, 2, 128, 2),
                   (10, 4, 256, 1), (10, 5, 256, 1), (10, 3, 256, 1), (10, 2, 128, 1)]


@pytest.mark.parametrize("L", [9, 10, 11, 12, 16, 17])
def test_kernel_path_boundary_limb_counts(L):
    ran = _check_shapes(L, 14, BOUNDARY_SHAPES, 501)
    # radix-4 shapes are refused above 16 limbs; the radix-2 ones always run
    assert ran == (8 if L <= 16 else 4)


@pytest.mark.parametrize("logn,nsamp", [(25, 6), (26, 4)])
def test_largest_sizes_64bit(logn, nsamp):
    """n = 2^25 and 2^26 (the largest transform the library takes) at 64 bits:
    sampled outputs against the definition, and the whole vector through the
    round trip."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(64, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 2, logn)
    say(f"largest size 64-bit logn={logn}")
    dx = to_dev(x)
    y = moma.ntt_fwd(dx, q, w)
    rng = np.random.default_rng(logn)
    ks = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, nsamp - 3)]).astype(np.int64))
    got = mi.from_planar(y[:, torch.from_numpy(ks).to("cuda:0")].cpu().numpy().view(np.uint32))
    assert (got == oracle.ntt_direct(q, L, w, x, ks)).all()
    z = moma.ntt_inv(y, q, w)
    assert torch.equal(z, dx)
    del y, z, dx
    moma.shutdown()
    torch.cuda.empty_cache()
