"""The input check: counting non-canonical elements (value >= q) on the GPU, and
the checking mode that makes every call refuse such inputs before it enqueues
any work.  The expected counts are the definition, evaluated with Python
integers on the planted vectors."""
import numpy as np
import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _value(row):
    return sum(int(w) << (32 * j) for j, w in enumerate(row))


def _words(v, L):
    return np.array([(v >> (32 * j)) & 0xFFFFFFFF for j in range(L)], dtype=np.uint32)


def _planted(f, n, L, seed):
    """Canonical residues with q, q + 1, all-ones and q - 1 planted at the
    first, a middle, the last and another index (the last three are >= q
    unless they do not fit the storage width)."""
    x = mi.residues(f, n, L, seed)
    top = (1 << (32 * L)) - 1
    for i, v in ((0, f.q), (n // 2, f.q + 1), (n - 1, top), (n // 3, f.q - 1)):
        if v <= top:
            x[i] = _words(v, L)
    return x


@pytest.mark.parametrize("lam,bits,n", [(64, None, 1000), (256, None, 4096), (384, None, 257), (256, 256, 4096),
                                        (1024, None, 70001)])
def test_count_matches_the_definition(lam, bits, n):
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0, bits=bits)
    L = lam // 32
    clean = mi.residues(f, n, L, 720)
    say(f"check_canonical lam={lam} bits={bits} n={n}")
    assert moma.check_canonical(to_dev(clean), f.q) == 0
    x = _planted(f, n, L, 721)
    want = sum(1 for row in x if _value(row) >= f.q)
    assert want >= 2
    assert moma.check_canonical(to_dev(x), f.q) == want


def test_checking_mode_refuses_noncanonical_inputs():
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n = f.limbs, 1 << 12
    w = f.root(n)
    good, good2 = mi.residues(f, n, L, 722, 1), mi.residues(f, n, L, 722, 2)
    bad = _planted(f, n, L, 723)
    dg, dg2, db = to_dev(good), to_dev(good2), to_dev(bad)
    say("input check mode")
    moma.set_input_check(True)
    try:
        calls = [lambda a, b: moma.ntt_fwd(a, f.q, w), lambda a, b: moma.ntt_inv(a, f.q, w),
                 lambda a, b: moma.vmul(b, a, f.q), lambda a, b: moma.vadd(a, b, f.q),
                 lambda a, b: moma.axpy(3, b, a, f.q), lambda a, b: moma.ntt_cyclic_mul(b, a, f.q, w)]
        for k, call in enumerate(calls):
            with pytest.raises(moma.MomaError) as e:
                call(db, dg)
            assert e.value.code == moma.MOMA_E_ARG, k
            assert "elements >= q" in str(e.value), k
        # a batch names the job whose input is not canonical
        o1, o2 = torch.empty_like(dg), torch.empty_like(dg)
        bt = moma.Batch([(dg, o1, f.q, w, False), (db, o2, f.q, w, False)])
        with pytest.raises(moma.MomaError) as e:
            bt.run()
        assert e.value.code == moma.MOMA_E_ARG and "job 1" in str(e.value)
        bt.close()
        # canonical inputs still give the oracle's results with the check on
        assert (from_dev(moma.ntt_fwd(dg, f.q, w)) == oracle.ntt_radix2(f.q, L, w, good)).all()
        assert (from_dev(moma.vmul(dg, dg2, f.q)) == oracle.vmul(f.q, L, good, good2)).all()
        bt = moma.Batch([(dg, o1, f.q, w, False), (dg2, o2, f.q, w, True)])
        bt.run()
        torch.cuda.synchronize()
        assert (from_dev(o1) == oracle.ntt_radix2(f.q, L, w, good)).all()
        assert (from_dev(o2) == oracle.intt_radix2(f.q, L, w, good2)).all()
        bt.close()
    finally:
        moma.set_input_check(False)
