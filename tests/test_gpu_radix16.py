"""Radix-16 register units (two-limb moduli): every such launch shape, alone, in
the fused cyclic product and inside a batch, gives the oracle's transform."""
import random

import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _r16(moma, L, logn):
    return [s for s in moma.ntt_candidates(L, logn) if s[3] == 4]


@pytest.mark.parametrize("logn,limit", [(4, 99), (9, 99), (13, 12), (17, 8)])
def test_radix16_shapes_agree_with_oracle(logn, limit):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(64, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    assert L == 2
    w = f.root(n)
    cands = _r16(moma, L, logn)
    assert cands, logn
    random.Random(logn).shuffle(cands)
    x = mi.residues(f, n, L, 310, logn)
    want_f = oracle.ntt_radix2(q, L, w, x)
    want_i = oracle.intt_radix2(q, L, w, x)
    dx = to_dev(x)
    for s in cands[:limit]:
        moma.ntt_set_schedule(q, w, n, L, s)
        say(f"radix16 logn={logn} sched={s}")
        assert (from_dev(moma.ntt_fwd(dx, q, w)) == want_f).all(), s
        assert (from_dev(moma.ntt_inv(dx, q, w)) == want_i).all(), s
    moma.ntt_set_schedule(q, w, n, L, None)


def test_radix16_fused_cyclic_product():
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(64, 0)
    L, logn = f.limbs, 10
    n, q, w = 1 << logn, f.q, f.root(1 << logn)
    a, b = mi.residues(f, n, L, 311, 1), mi.residues(f, n, L, 311, 2)
    want = oracle.cyclic_conv(q, L, a, b)
    for s in _r16(moma, L, logn):
        moma.ntt_set_schedule(q, w, n, L, s)
        say(f"radix16 cyclic product sched={s}")
        assert (from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), q, w)) == want).all(), s
    moma.ntt_set_schedule(q, w, n, L, None)


def test_radix16_inside_a_batch():
    """Jobs above 2^18 points keep their plan's schedule in a batch, so a 2^19
    two-limb job set to a radix-16 shape runs the batch kernel's radix-16
    instantiation; small jobs beside it take the batch rule."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(64, 0)
    L, logn = f.limbs, 19
    n, q, w = 1 << logn, f.q, f.root(1 << logn)
    s = (12, 4, 256, 4)
    assert s + (0,) in moma.ntt_candidates(L, logn)
    moma.ntt_set_schedule(q, w, n, L, s)
    big = [mi.residues(f, n, L, 312, k) for k in range(2)]
    g = mi.find_prime(128, 3)
    small = [(g, 1 << 11, mi.residues(g, 1 << 11, g.limbs, 313, 0)), (f, 1 << 13, mi.residues(f, 1 << 13, L, 313, 1))]
    specs, outs, wants = [], [], []
    for k, x in enumerate(big):
        inv = k == 1
        dx = to_dev(x)
        o = torch.empty_like(dx)
        specs.append((dx, o, q, w, inv))
        outs.append(o)
        wants.append((oracle.intt_radix2 if inv else oracle.ntt_radix2)(q, L, w, x))
    for fld, m, x in small:
        dx = to_dev(x)
        o = torch.empty_like(dx)
        specs.append((dx, o, fld.q, fld.root(m), False))
        outs.append(o)
        wants.append(oracle.ntt_radix2(fld.q, fld.limbs, fld.root(m), x))
    say("radix16 batch")
    bt = moma.Batch(specs)
    bt.run()
    torch.cuda.synchronize()
    for k, (o, want) in enumerate(zip(outs, wants)):
        assert (from_dev(o) == want).all(), k
    bt.close()
    moma.ntt_set_schedule(q, w, n, L, None)
