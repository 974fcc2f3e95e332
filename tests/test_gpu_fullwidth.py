"""GPU parity for full-width moduli (bitlen(q) = 32 x storage limbs): the
library computes in one more internal limb and stages the transforms' vectors
through buffers of that width; outputs are bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

WIDTHS = [64, 96, 256, 512, 992]


@pytest.mark.parametrize("lam", WIDTHS)
def test_full_width_blas(lam):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0, bits=lam)
    q, L, n = f.q, f.limbs, 1537
    a, b = mi.residues(f, n, L, 500, 1), mi.residues(f, n, L, 500, 2)
    alpha = mi.scalar_residue(f, 500, 3)
    da, db = to_dev(a), to_dev(b)
    say(f"full-width blas lam={lam}")
    assert (from_dev(moma.vadd(da, db, q)) == oracle.vadd(q, L, a, b)).all()
    assert (from_dev(moma.vsub(da, db, q)) == oracle.vsub(q, L, a, b)).all()
    assert (from_dev(moma.vmul(da, db, q)) == oracle.vmul(q, L, a, b)).all()
    assert (from_dev(moma.axpy(alpha, da, db, q)) == oracle.axpy(q, L, alpha, a, b)).all()
    ev = mi.edge_vectors(f, 64, L)
    for name, x in ev.items():
        dx = to_dev(x)
        assert (from_dev(moma.vmul(dx, dx, q)) == oracle.vmul(q, L, x, x)).all(), name
        assert (from_dev(moma.vadd(dx, dx, q)) == oracle.vadd(q, L, x, x)).all(), name


@pytest.mark.parametrize("lam,logn", [(64, 6), (64, 14), (256, 9), (256, 13), (512, 12), (992, 10)])
def test_full_width_ntt(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0, bits=lam)
    q, L, n = f.q, f.limbs, 1 << logn
    w = f.root(n)
    x = mi.residues(f, n, L, 501, logn)
    say(f"full-width ntt lam={lam} logn={logn} plan={moma.ntt_describe(q, w, n, L)}")
    dx = to_dev(x)
    y = moma.ntt_fwd(dx, q, w)
    want = oracle.ntt_radix2(q, L, w, x)
    assert (from_dev(y) == want).all()
    assert (from_dev(moma.ntt_inv(y, q, w)) == x).all()
    moma.ntt_fwd(dx, q, w, out=dx)                       # in place
    assert (from_dev(dx) == want).all()
    b = mi.residues(f, n, L, 501, 100 + logn)
    c = from_dev(moma.ntt_cyclic_mul(to_dev(x), to_dev(b), q, w))
    want_c = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, want, oracle.ntt_radix2(q, L, w, b)))
    assert (c == want_c).all()


def test_full_width_batch_jobs():
    """Full-width jobs mixed with ordinary ones in one graph launch."""
    import oracle
    import paper_2501_07535_amd as moma
    specs, checks, keep = [], [], []
    for k, (lam, bits, logn, kind) in enumerate([(256, 256, 11, 0), (256, 252, 12, 1), (128, 128, 13, 1),
                                                  (64, 64, 10, 2), (512, 512, 9, 0), (96, 96, 12, 2)]):
        f = mi.find_prime(lam, 0, bits=bits)
        q, L, n = f.q, f.limbs, 1 << logn
        w = f.root(n)
        x, y = mi.residues(f, n, L, 502, k), mi.residues(f, n, L, 503, k)
        dx, dy = to_dev(x), to_dev(y)
        out = torch.full_like(dx, -1)
        keep += [dx, dy, out]
        specs.append(((dx, dy) if kind == 2 else dx, out, q, w, kind))
        if kind == 0:
            want = oracle.ntt_radix2(q, L, w, x)
        elif kind == 1:
            want = oracle.intt_radix2(q, L, w, x)
        else:
            want = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, oracle.ntt_radix2(q, L, w, x),
                                                           oracle.ntt_radix2(q, L, w, y)))
        checks.append((out, want, lam, bits, kind))
    say("full-width batch")
    bt = moma.Batch(specs)
    bt.run()
    torch.cuda.synchronize()
    for out, want, lam, bits, kind in checks:
        assert (from_dev(out) == want).all(), (lam, bits, kind)
    bt.close()
