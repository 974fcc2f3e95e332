"""Batched transforms: every job of one graph launch equals the plain call and the oracle."""
import numpy as np
import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def test_batch_mixed_jobs_match_plain_and_oracle():
    import oracle
    import paper_2501_07535_amd as moma
    jobs = mi.batch_jobs(40, config=33)
    xs = mi.batch_inputs(jobs, config=33)
    dx = [to_dev(x) for x in xs]
    outs, specs = [], []
    for k, (j, x) in enumerate(zip(jobs, dx)):
        inv = k % 3 == 2
        inplace = k % 5 == 4
        o = x.clone() if inplace else torch.empty_like(x)
        outs.append(o)
        specs.append((o if inplace else x, o, j.field.q, j.omega, inv))
    say("batch create 40 jobs")
    b = moma.Batch(specs)
    info = b.info()
    assert info["launches"] >= 1 and info["items"] >= len(jobs)
    b.run()
    torch.cuda.synchronize()
    for k, (j, x) in enumerate(zip(jobs, xs)):
        inv = k % 3 == 2
        got = from_dev(outs[k])
        plain = moma.ntt_inv(dx[k], j.field.q, j.omega) if inv else moma.ntt_fwd(dx[k], j.field.q, j.omega)
        assert (got == from_dev(plain)).all(), (k, j.lam, j.logn)
        want = (oracle.intt_radix2 if inv else oracle.ntt_radix2)(j.field.q, j.limbs, j.omega, x)
        assert (got == want).all(), (k, j.lam, j.logn)
    # running again from the same inputs gives the same outputs (in-place jobs excepted: their input changed)
    first = [o.clone() for o in outs]
    b.run()
    torch.cuda.synchronize()
    for k in range(len(jobs)):
        if k % 5 != 4:
            assert torch.equal(outs[k], first[k])
    b.close()


def test_batch_shape_recipe():
    shapes = [mi.batch_shape(i) for i in range(4096)]
    lams = {s[0] for s in shapes}
    logns = {s[1] for s in shapes}
    assert lams == {64, 128, 256, 384} and logns == set(range(10, 17))
    counts = np.bincount([s[1] for s in shapes])[10:]
    assert counts.min() > 4096 / 7 * 0.8


def test_batch_rejects_bad_job():
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    x = to_dev(mi.residues(f, 64, 8, 1))
    with pytest.raises(moma.MomaError):
        moma.Batch([(x, torch.empty_like(x), f.q, f.root(32), False)])   # root of the wrong order
