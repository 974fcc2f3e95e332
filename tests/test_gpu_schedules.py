"""Every launch shape computes the same transform: sampled schedules vs the oracle."""
import itertools
import random

import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def all_schedules():
    return list(itertools.product(range(5, 15), (2, 3, 4, 5), (64, 128, 256, 512, 1024), (1, 2, 3, 4)))


@pytest.mark.parametrize("lam,logn", [(256, 11), (256, 14), (128, 16), (384, 13), (64, 15), (1024, 11)])
def test_schedules_agree_with_oracle(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 300, logn)
    want_f = oracle.ntt_radix2(q, L, w, x)
    want_i = oracle.intt_radix2(q, L, w, x)
    rng = random.Random(lam * 100 + logn)
    cands = all_schedules()
    rng.shuffle(cands)
    tried = 0
    dx = to_dev(x)
    for s in cands:
        try:
            moma.ntt_set_schedule(q, w, n, L, s)
        except moma.MomaError as e:
            assert e.code in (moma.MOMA_E_UNSUPPORTED, moma.MOMA_E_ARG)
            continue
        assert moma.ntt_get_schedule(q, w, n, L) == s + (0,)  # a 4-tuple sets the schoolbook multiply
        say(f"schedule lam={lam} logn={logn} sched={s}")
        assert (from_dev(moma.ntt_fwd(dx, q, w)) == want_f).all(), s
        assert (from_dev(moma.ntt_inv(dx, q, w)) == want_i).all(), s
        tried += 1
        if tried >= 30:
            break
    moma.ntt_set_schedule(q, w, n, L, None)
    assert tried >= 10
