"""GPU parity for the Karatsuba form of the butterfly's twiddle multiply (one
level of Karatsuba on the digit product, Eq. (mulk)), a launch-shape choice of
the autotuner: whole vectors against the oracle at compute limb counts 2 to 24,
one and several passes, the inverse and the cyclic product; the shapes it does
not run are refused."""
import random

import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

# compute limbs 2..24: even and odd digit counts, both halves of the split
CASES = [(64, 12), (96, 11), (160, 13), (256, 12), (288, 10), (384, 11), (512, 12), (544, 9), (736, 10), (768, 11)]


def _kara_shapes(L, logn, seed, k=3):
    import paper_2501_07535_amd as moma
    cands = [c for c in moma.ntt_candidates(L, logn) if c[4] == 1]
    assert cands and all(c[3] == 1 for c in cands)
    rng = random.Random(seed)
    one = [c for c in cands if c[0] >= logn]
    multi = [c for c in cands if c[0] < logn]
    pick = (rng.sample(one, 1) if one else []) + rng.sample(multi, min(k, len(multi)))
    return pick


@pytest.mark.parametrize("lam,logn", CASES)
def test_karatsuba_butterfly_matches_oracle(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q, L, n = f.q, f.limbs, 1 << logn
    w = f.root(n)
    x = mi.residues(f, n, L, 700, logn)
    want = oracle.ntt_radix2(q, L, w, x)
    dx = to_dev(x)
    for s in _kara_shapes(L, logn, lam + logn):
        moma.ntt_set_schedule(q, w, n, L, s)
        assert moma.ntt_get_schedule(q, w, n, L) == s
        say(f"karatsuba lam={lam} L={L} logn={logn} sched={s}")
        y = moma.ntt_fwd(dx, q, w)
        assert (from_dev(y) == want).all(), s
        assert (from_dev(moma.ntt_inv(y, q, w)) == x).all(), s
    moma.ntt_set_schedule(q, w, n, L, None)


@pytest.mark.parametrize("lam,logn", [(128, 10), (256, 13), (768, 9)])
def test_karatsuba_cyclic_product_and_in_place(lam, logn):
    """The fused pointwise product of a cyclic product with Karatsuba butterflies
    around it, and an in-place transform, against the oracle."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q, L, n = f.q, f.limbs, 1 << logn
    w = f.root(n)
    a, b = mi.residues(f, n, L, 701, 1), mi.residues(f, n, L, 701, 2)
    s = _kara_shapes(L, logn, 3 * lam + logn, k=1)[-1]
    moma.ntt_set_schedule(q, w, n, L, s)
    say(f"karatsuba cyclic product lam={lam} logn={logn} sched={s}")
    fa = oracle.ntt_radix2(q, L, w, a)
    want = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, fa, oracle.ntt_radix2(q, L, w, b)))
    assert (from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), q, w)) == want).all()
    da = to_dev(a)
    moma.ntt_fwd(da, q, w, out=da)
    assert (from_dev(da) == fa).all()
    moma.ntt_set_schedule(q, w, n, L, None)


def test_karatsuba_edge_vectors():
    """All q - 1, alternating 0 / q - 1 and full carry runs through the digit sums."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    q, L, n = f.q, f.limbs, 1 << 11
    w = f.root(n)
    s = _kara_shapes(L, 11, 5, k=1)[-1]
    moma.ntt_set_schedule(q, w, n, L, s)
    for name, x in mi.edge_vectors(f, n, L).items():
        say(f"karatsuba edge {name}")
        assert (from_dev(moma.ntt_fwd(to_dev(x), q, w)) == oracle.ntt_radix2(q, L, w, x)).all(), name
    moma.ntt_set_schedule(q, w, n, L, None)


def test_karatsuba_refusals():
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    q, L, n = f.q, f.limbs, 1 << 12
    w = f.root(n)
    with pytest.raises(moma.MomaError):
        moma.ntt_set_schedule(q, w, n, L, (10, 4, 256, 2, 1))   # radix 4
    g = mi.find_prime(256, 0, bits=256)                          # full width
    with pytest.raises(moma.MomaError):
        moma.ntt_set_schedule(g.q, g.root(n), n, 8, (10, 4, 256, 1, 1))
    h = mi.find_prime(800, 0)                                    # 25 compute limbs
    with pytest.raises(moma.MomaError):
        moma.ntt_set_schedule(h.q, h.root(n), n, h.limbs, (10, 4, 256, 1, 1))
    assert not [c for c in moma.ntt_candidates(25, 12) if c[4] == 1]


def test_tuner_times_both_multiply_forms():
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(128, 0)
    q, L, n = f.q, f.limbs, 1 << 12
    w = f.root(n)
    moma.tune_db_clear()
    say("tune with both multiply forms")
    r = moma.ntt_tune(q, w, n, L, reps=1, warmup=1)
    rows = moma.tune_db_rows()
    assert r["timed"] == len(moma.ntt_candidates(L, 12)) == len(rows)
    assert {row["sched"][4] for row in rows} == {0, 1}
    x = mi.residues(f, n, L, 702, 1)
    assert (from_dev(moma.ntt_fwd(to_dev(x), q, w)) == oracle.ntt_radix2(q, L, w, x)).all()
    moma.tune_db_clear()
    moma.ntt_set_schedule(q, w, n, L, None)
