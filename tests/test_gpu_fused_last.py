"""Passes whose last three stages run as one radix-4 round plus a final stage
whose partners are exchanged across lanes (v_permlane32_swap / 16_swap), not
through LDS, and whose first round reads straight from HBM: transforms,
inverses and cyclic products in launch shapes that take those paths (first and
later passes, 16 and 32 groups per tile, radix-4 and radix-8 units, 2 to 8
limbs) equal the oracle's."""
import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [(256, 15, (10, 5, 256, 2)), (256, 13, (9, 4, 128, 2)), (64, 15, (9, 4, 128, 2)),
         (160, 17, (10, 5, 256, 2)), (256, 14, (11, 4, 256, 2)), (128, 15, (10, 5, 128, 2)),
         # radix-8 units: last 4 stages fused (k = 7) and the direct first round
         (128, 14, (11, 4, 256, 3)), (64, 14, (11, 4, 256, 3)), (160, 19, (11, 5, 256, 3))]


@pytest.mark.parametrize("lam,logn,sched", CASES)
def test_fused_last_stage_matches_oracle(lam, logn, sched):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    w = f.root(n)
    assert sched + (0,) in moma.ntt_candidates(L, logn)  # (schoolbook multiply)
    moma.ntt_set_schedule(q, w, n, L, sched)
    x = mi.residues(f, n, L, 730, logn)
    dx = to_dev(x)
    say(f"fused last stage lam={lam} logn={logn} sched={sched}")
    assert (from_dev(moma.ntt_fwd(dx, q, w)) == oracle.ntt_radix2(q, L, w, x)).all()
    assert (from_dev(moma.ntt_inv(dx, q, w)) == oracle.intt_radix2(q, L, w, x)).all()
    inpl = dx.clone()
    moma.ntt_fwd(inpl, q, w, out=inpl)
    assert (from_dev(inpl) == oracle.ntt_radix2(q, L, w, x)).all()
    moma.ntt_set_schedule(q, w, n, L, None)


def test_fused_last_stage_in_the_cyclic_product():
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, logn = f.limbs, 15
    n, q, w = 1 << logn, f.q, f.root(1 << logn)
    moma.ntt_set_schedule(q, w, n, L, (10, 5, 256, 2))
    a, b = mi.residues(f, n, L, 731, 1), mi.residues(f, n, L, 731, 2)
    want = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, oracle.ntt_radix2(q, L, w, a), oracle.ntt_radix2(q, L, w, b)))
    say("fused last stage cyclic product")
    assert (from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), q, w)) == want).all()
    moma.ntt_set_schedule(q, w, n, L, None)


def test_variant_passes_inside_a_batch():
    """Batch jobs whose passes take the variant (odd stage counts with 16 or 32
    groups under the batch's own launch shapes): forward, inverse and cyclic
    products equal the oracle."""
    import torch

    import oracle
    import paper_2501_07535_amd as moma
    specs, checks, keep = [], [], []
    for lam, logn, kind in ((256, 15, moma.JOB_FORWARD), (256, 15, moma.JOB_CYCLIC_MUL), (128, 14, moma.JOB_INVERSE),
                            (128, 14, moma.JOB_CYCLIC_MUL), (64, 17, moma.JOB_FORWARD), (160, 13, moma.JOB_CYCLIC_MUL)):
        f = mi.find_prime(lam, 2)
        L, n, q = f.limbs, 1 << logn, f.q
        w = f.root(n)
        a, b = mi.residues(f, n, L, 732, logn, 1), mi.residues(f, n, L, 732, logn, 2)
        da, db = to_dev(a), to_dev(b)
        o = torch.empty_like(da)
        keep += [da, db]
        specs.append(((da, db) if kind == moma.JOB_CYCLIC_MUL else da, o, q, w, kind))
        if kind == moma.JOB_FORWARD:
            want = oracle.ntt_radix2(q, L, w, a)
        elif kind == moma.JOB_INVERSE:
            want = oracle.intt_radix2(q, L, w, a)
        else:
            want = oracle.intt_radix2(q, L, w, oracle.vmul(q, L, oracle.ntt_radix2(q, L, w, a), oracle.ntt_radix2(q, L, w, b)))
        checks.append((o, want, lam, logn, kind))
    say("variant passes in a batch")
    bt = moma.Batch(specs)
    bt.run()
    torch.cuda.synchronize()
    for o, want, lam, logn, kind in checks:
        assert (from_dev(o) == want).all(), (lam, logn, kind)
    bt.close()
