"""GPU parity for full-width moduli (bitlen(q) = 32 x storage limbs, no
headroom for lazy reduction): the library computes in the storage limbs with
canonical operands and Montgomery products that carry out of the top limb;
outputs are bit-exact against the oracle, up to a full 1024-bit modulus."""
import random

import numpy as np
import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

WIDTHS = [64, 96, 256, 320, 512, 640, 992, 1024]


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


@pytest.mark.parametrize("lam,logn", [(64, 6), (64, 14), (256, 9), (256, 13), (320, 12), (512, 12), (992, 10),
                                      (1024, 8), (1024, 12)])
def test_full_width_ntt(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0, bits=lam)
    q, L, n = f.q, f.limbs, 1 << logn
    w = f.root(n)
    x = mi.residues(f, n, L, 501, logn)
    d = moma.ntt_describe(q, w, n, L)
    say(f"full-width ntt lam={lam} logn={logn} plan={d}")
    assert d["compute_limbs"] == L
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
                                                  (64, 64, 10, 2), (512, 512, 9, 0), (96, 96, 12, 2),
                                                  (1024, 1024, 11, 0), (1024, 1024, 10, 2)]):
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


@pytest.mark.parametrize("lam,logn", [(64, 13), (128, 14), (256, 12), (320, 11), (512, 11)])
def test_full_width_sampled_schedules(lam, logn):
    """Radix-2 and radix-4 units (radix 4 up to 16 limbs), one and several
    passes, 4 to 32 columns: sampled launch shapes of the full-width kernels
    against the oracle; radix-8 shapes and the Karatsuba multiply refused."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0, bits=lam)
    q, L, n = f.q, f.limbs, 1 << logn
    w = f.root(n)
    x = mi.residues(f, n, L, 504, logn)
    want = oracle.ntt_radix2(q, L, w, x)
    dx = to_dev(x)
    rng = random.Random(lam * 7 + logn)
    rmax = 2 if L <= 16 else 1  # the full-width kernels' register units
    cands = [c for c in moma.ntt_candidates(L, logn) if c[3] <= rmax and c[4] == 0]
    rng.shuffle(cands)
    seen = set()
    for c in cands:
        key = (c[3], c[1])
        if key in seen:
            continue
        seen.add(key)
        moma.ntt_set_schedule(q, w, n, L, c)
        say(f"full-width schedule lam={lam} logn={logn} sched={c}")
        y = moma.ntt_fwd(dx, q, w)
        assert (from_dev(y) == want).all(), c
        assert (from_dev(moma.ntt_inv(y, q, w)) == x).all(), c
    # radix-8 shapes and the Karatsuba multiply are refused for a full-width modulus
    refused = [c for c in moma.ntt_candidates(L, logn) if c[3] > rmax][:1] + \
        [c for c in moma.ntt_candidates(L, logn) if c[4] == 1][:1]
    assert refused
    for c in refused:
        with pytest.raises(moma.MomaError):
            moma.ntt_set_schedule(q, w, n, L, c)
    moma.ntt_set_schedule(q, w, n, L, None)


def test_full_width_tuner_keeps_radix_limit():
    """The tuner's candidates for a full-width plan stop at radix 4, and the
    tuned plan still equals the oracle."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(128, 0, bits=128)
    q, L, n = f.q, f.limbs, 1 << 12
    w = f.root(n)
    x = mi.residues(f, n, L, 505, 1)
    say("full-width tune lam=128 logn=12")
    r = moma.ntt_tune(q, w, n, L, reps=1, warmup=1, max_candidates=24)
    assert r["best"][3] <= 2
    assert (from_dev(moma.ntt_fwd(to_dev(x), q, w)) == oracle.ntt_radix2(q, L, w, x)).all()
