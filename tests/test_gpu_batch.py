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


def test_batch_large_jobs_run_in_groups():
    """Jobs of 16 MiB or more run in groups of at most 256 MiB of data, one group
    after another: eight 2^20-point 256-bit transforms (32 MiB each; forward,
    inverse and in place) fill the first group, a ninth and a cyclic product of
    two 2^19-point vectors the second, and small jobs run beside the first.
    Every output equals the plain call's, sampled outputs the oracle's
    definition, and a second run the first."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, q = f.limbs, f.q
    big, half, small = 1 << 20, 1 << 19, 1 << 12
    wb, wh, ws = f.root(big), f.root(half), f.root(small)
    specs, checks, host = [], [], []
    for k in range(9):
        xh = mi.residues(f, big, L, 71, k)
        x = to_dev(xh)
        inv, inplace = k % 3 == 1, k == 5
        o = x.clone() if inplace else torch.empty_like(x)
        checks.append((o, (moma.ntt_inv if inv else moma.ntt_fwd)(x, q, wb), not inplace))
        specs.append((o if inplace else x, o, q, wb, inv))
        host.append((xh, inv))
    a, bv = to_dev(mi.residues(f, half, L, 72, 0)), to_dev(mi.residues(f, half, L, 72, 1))
    o = torch.empty_like(a)
    checks.append((o, moma.ntt_cyclic_mul(a, bv, q, wh), True))
    specs.append(((a, bv), o, q, wh, moma.JOB_CYCLIC_MUL))
    for k in range(6):
        x = to_dev(mi.residues(f, small, L, 73, k))
        o = torch.empty_like(x)
        checks.append((o, moma.ntt_fwd(x, q, ws), True))
        specs.append((x, o, q, ws, False))
    torch.cuda.synchronize()
    say("batch: nine 2^20-point jobs, a 2^19-point cyclic product, six 2^12-point jobs")
    b = moma.Batch(specs)
    assert b.info()["launches"] >= 8  # two groups of at least four passes each
    b.run()
    torch.cuda.synchronize()
    for i, (o, want, _) in enumerate(checks):
        assert torch.equal(o, want), i
    ks = np.array([0, 1, 777, big - 1], dtype=np.int64)
    for k in (0, 1, 8):  # one forward and one inverse job of the first group, one job of the second
        xh, inv = host[k]
        got = from_dev(checks[k][0][:, torch.from_numpy(ks).to("cuda:0")].contiguous())
        want = (oracle.intt_direct if inv else oracle.ntt_direct)(q, L, wb, xh, ks)
        assert (got == want).all(), k
    first = [o.clone() for o, _, _ in checks]
    b.run()
    torch.cuda.synchronize()
    for i, (o, _, rerun_same) in enumerate(checks):
        if rerun_same:
            assert torch.equal(o, first[i]), i
    b.close()


def test_batch_jobs_larger_than_a_group():
    """A job of more than 256 MiB makes a group of its own: two 2^24-point
    256-bit transforms (512 MiB each, one forward, one inverse in place) run
    one after the other in one batch, beside a 2^20-point job; every output
    equals the plain call's."""
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, q = f.limbs, f.q
    n, m = 1 << 24, 1 << 20
    wn, wm = f.root(n), f.root(m)
    x0 = to_dev(mi.residues(f, n, L, 74, 0))
    x1 = to_dev(mi.residues(f, n, L, 74, 1))
    x2 = to_dev(mi.residues(f, m, L, 74, 2))
    o0, o2 = torch.empty_like(x0), torch.empty_like(x2)
    want = [moma.ntt_fwd(x0, q, wn), moma.ntt_inv(x1, q, wn), moma.ntt_fwd(x2, q, wm)]
    torch.cuda.synchronize()
    say("batch: two 2^24-point jobs of 512 MiB and a 2^20-point job")
    b = moma.Batch([(x0, o0, q, wn, False), (x1, x1, q, wn, True), (x2, o2, q, wm, False)])
    b.run()
    torch.cuda.synchronize()
    for i, got in enumerate((o0, x1, o2)):
        assert torch.equal(got, want[i]), i
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


def test_batch_blas_jobs_with_transforms():
    """vadd / vsub / vmul / axpy jobs of mixed widths and ragged lengths (and a
    full-width modulus, and in-place outputs) captured with transform jobs in
    one graph: each output equals the plain call and the oracle."""
    import oracle
    import paper_2501_07535_amd as moma
    kinds = [moma.JOB_VADD, moma.JOB_VSUB, moma.JOB_VMUL, moma.JOB_AXPY]
    ref = {moma.JOB_VADD: "vadd", moma.JOB_VSUB: "vsub", moma.JOB_VMUL: "vmul"}
    cases = [(64, None, 1000), (96, None, 257), (256, None, 70001), (256, 256, 4096), (384, None, 1),
             (512, None, 3000), (768, None, 513), (1024, None, 200), (128, 128, 999), (256, None, 0)]
    specs, checks, keep = [], [], []
    f8 = mi.find_prime(256, 0)
    moma.vmul_set_variant(f8.q, 8, moma.VMUL_KARATSUBA)      # one width runs the Karatsuba products
    try:
        for k, (lam, bits, n) in enumerate(cases):
            f = mi.find_prime(lam, 0, bits=bits) if bits else mi.find_prime(lam, 0)
            q, L = f.q, f.limbs
            for kind in kinds:
                a, b = mi.residues(f, n, L, 700 + k, kind), mi.residues(f, n, L, 750 + k, kind)
                alpha = mi.scalar_residue(f, 800 + k, kind)
                da, db = to_dev(a), to_dev(b)
                inplace = (k + kind) % 3 == 0
                out = da if inplace else torch.full_like(da, -1)
                keep += [da, db, out]
                specs.append(((da, db), out, q, alpha, kind))
                want = oracle.axpy(q, L, alpha, a, b) if kind == moma.JOB_AXPY else getattr(oracle, ref[kind])(q, L, a, b)
                checks.append((out, want, a, b, alpha, q, kind, lam, n))
        # and two transforms in the same graph
        f = mi.find_prime(256, 0)
        x = mi.residues(f, 1 << 12, 8, 900)
        dx = to_dev(x)
        ox = torch.empty_like(dx)
        keep += [dx, ox]
        specs.append((dx, ox, f.q, f.root(1 << 12), moma.JOB_FORWARD))
        say(f"batch with {len(specs)} jobs (BLAS and transforms)")
        bt = moma.Batch(specs)
        bt.run()
        torch.cuda.synchronize()
        assert (from_dev(ox) == oracle.ntt_radix2(f.q, 8, f.root(1 << 12), x)).all()
        for out, want, a, b, alpha, q, kind, lam, n in checks:
            if n == 0:
                continue
            assert (from_dev(out) == want).all(), (lam, kind, n)
            da, db = to_dev(a), to_dev(b)
            plain = moma.axpy(alpha, da, db, q) if kind == moma.JOB_AXPY else getattr(moma, ref[kind])(da, db, q)
            assert (from_dev(plain) == want).all(), (lam, kind, n)
        bt.close()
    finally:
        moma.vmul_set_variant(f8.q, 8, moma.VMUL_SCHOOLBOOK)


def test_batch_4096_job_workload_sampled_against_oracle():
    """The benchmarked workload itself (4096 forward transforms, 64..384 bits,
    2^10..2^16 points, a prime each, one graph launch): 64 seeded jobs, 16 of
    each width, compared element by element with the oracle's transform; every
    job equal to its plain call."""
    import oracle
    import paper_2501_07535_amd as moma
    jobs = mi.batch_jobs(4096)
    xs = mi.batch_inputs(jobs)
    dx = [to_dev(x) for x in xs]
    outs = [torch.empty_like(x) for x in dx]
    say("batch create 4096 jobs (the benchmarked workload)")
    b = moma.Batch([(x, o, j.field.q, j.omega, False) for j, x, o in zip(jobs, dx, outs)])
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(4096)
    picks = []
    for lam in mi.BATCH_WIDTHS:
        idx = [j.index for j in jobs if j.lam == lam]
        picks += list(rng.choice(idx, size=16, replace=False))
    say(f"batch 4096: oracle check of {len(picks)} jobs")
    for k in picks:
        j = jobs[k]
        want = oracle.ntt_radix2(j.field.q, j.limbs, j.omega, xs[k])
        assert (from_dev(outs[k]) == want).all(), (k, j.lam, j.logn)
    say("batch 4096: every job against its plain call")
    for j, x, o in zip(jobs, dx, outs):
        assert torch.equal(moma.ntt_fwd(x, j.field.q, j.omega), o), (j.index, j.lam, j.logn)
    b.close()
