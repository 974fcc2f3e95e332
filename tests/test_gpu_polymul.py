"""GPU parity for the cyclic product a * b mod (x^n - 1, q): bit-exact against
the oracle's direct O(n^2) definition at small n, and against the oracle's
forward / pointwise / inverse transforms (its convolution theorem, pinned by the
definition on the CPU) at larger n."""
import random

import numpy as np
import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _pair(lam, logn, seed, L=None):
    f = mi.find_prime(lam, 0)
    n = 1 << logn
    L = L or f.limbs
    return f, L, n, f.root(n), mi.residues(f, n, L, seed, 1), mi.residues(f, n, L, seed, 2)


def _theorem(q, L, w, a, b):
    import oracle
    return oracle.intt_radix2(q, L, w, oracle.vmul(q, L, oracle.ntt_radix2(q, L, w, a), oracle.ntt_radix2(q, L, w, b)))


@pytest.mark.parametrize("lam,logn", [(64, 1), (64, 5), (128, 8), (256, 2), (256, 6), (256, 9), (384, 7),
                                      (512, 8), (768, 6), (1024, 5), (1024, 8)])
def test_cyclic_mul_matches_definition(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f, L, n, w, a, b = _pair(lam, logn, 400)
    say(f"cyclic_mul lam={lam} logn={logn}")
    c = from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), f.q, w))
    assert (c == oracle.cyclic_conv(f.q, L, a, b)).all()


@pytest.mark.parametrize("lam,logn", [(256, 7), (1024, 6)])
def test_full_polynomial_product_by_zero_padding(lam, logn):
    """The paper's polynomial product (Section 2.3), sum_i a_i b_{j-i} x^j up to
    degree 2m-2, from the cyclic product of length n = 2m of the zero-padded
    coefficient vectors, against that sum in Python integers."""
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    m = n // 2
    a, b = mi.residues(f, n, L, 407, 1), mi.residues(f, n, L, 407, 2)
    a[m:] = 0
    b[m:] = 0
    say(f"full product lam={lam} logn={logn}")
    c = mi.rows_to_ints(from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), q, f.root(n))))
    ai, bi = mi.rows_to_ints(a), mi.rows_to_ints(b)
    want = [sum(ai[i] * bi[j - i] for i in range(max(0, j - m + 1), min(j, m - 1) + 1)) % q for j in range(2 * m - 1)]
    assert c[:2 * m - 1] == want and c[2 * m - 1] == 0


@pytest.mark.parametrize("lam,logn", [(256, 12), (256, 13), (256, 16), (64, 15), (128, 14), (384, 13),
                                      (768, 12), (1024, 11)])
def test_cyclic_mul_multi_pass(lam, logn):
    import paper_2501_07535_amd as moma
    f, L, n, w, a, b = _pair(lam, logn, 401)
    say(f"cyclic_mul multi-pass lam={lam} logn={logn} plan={moma.ntt_describe(f.q, w, n, L)}")
    c = from_dev(moma.ntt_cyclic_mul(to_dev(a), to_dev(b), f.q, w))
    assert (c == _theorem(f.q, L, w, a, b)).all()


@pytest.mark.parametrize("lam,logn", [(256, 10), (256, 14), (768, 11), (128, 13)])
def test_cyclic_mul_every_load_path(lam, logn):
    """Sampled launch shapes: one pass with 4-row vector loads, 4+ column tiles
    (vector loads), 2-column tiles (scalar loads), radix 2 / 4 / 8 units."""
    import paper_2501_07535_amd as moma
    f, L, n, w, a, b = _pair(lam, logn, 402)
    want = _theorem(f.q, L, w, a, b)
    da, db = to_dev(a), to_dev(b)
    rng = random.Random(lam * 31 + logn)
    cands = [(t, c, th, r) for t in range(5, 15) for c in (1, 2, 3, 4) for th in (64, 128, 256, 512)
             for r in (1, 2, 3)]
    rng.shuffle(cands)
    tried = 0
    for s in cands:
        try:
            moma.ntt_set_schedule(f.q, w, n, L, s)
        except moma.MomaError as e:
            assert e.code in (moma.MOMA_E_UNSUPPORTED, moma.MOMA_E_ARG)
            continue
        say(f"cyclic_mul lam={lam} logn={logn} sched={s}")
        assert (from_dev(moma.ntt_cyclic_mul(da, db, f.q, w)) == want).all(), s
        tried += 1
        if tried >= 16:
            break
    moma.ntt_set_schedule(f.q, w, n, L, None)
    assert tried >= 8


def test_cyclic_mul_aliasing_and_wide_storage():
    """out may be a or b; a 252-bit q stored in 10 limbs gives zero upper planes."""
    import paper_2501_07535_amd as moma
    f, L, n, w, a, b = _pair(256, 13, 403, L=10)
    want = _theorem(f.q, L, w, a, b)
    say("cyclic_mul out=a")
    da, db = to_dev(a), to_dev(b)
    moma.ntt_cyclic_mul(da, db, f.q, w, out=da)
    assert (from_dev(da) == want).all()
    say("cyclic_mul out=b")
    da = to_dev(a)
    moma.ntt_cyclic_mul(da, db, f.q, w, out=db)
    assert (from_dev(db) == want).all()
    say("cyclic_mul wide storage, dirty out")
    out = torch.full((L, n), -1, dtype=torch.int32, device="cuda:0")
    moma.ntt_cyclic_mul(to_dev(a), to_dev(b), f.q, w, out=out)
    assert (from_dev(out) == want).all()


@pytest.mark.parametrize("logn", [3, 12])
def test_cyclic_mul_closed_forms(logn):
    """x^s * a is a rotated by s; 1 * a = a; (q-1)-vectors; a * 0 = 0."""
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n, q = 8, 1 << logn, f.q
    w = f.root(n)
    a = mi.residues(f, n, L, 404, 1)
    ev = mi.edge_vectors(f, n, L)
    da = to_dev(a)
    say(f"cyclic_mul closed forms logn={logn}")
    assert (from_dev(moma.ntt_cyclic_mul(da, to_dev(ev["delta0"]), q, w)) == a).all()
    assert (from_dev(moma.ntt_cyclic_mul(da, to_dev(ev["zeros"]), q, w)) == 0).all()
    d1 = from_dev(moma.ntt_cyclic_mul(da, to_dev(ev["delta1"]), q, w))
    assert (d1 == np.roll(a, 1, axis=0)).all()
    # all (q-1): every output is n (q-1)^2 mod q = n
    allq = from_dev(moma.ntt_cyclic_mul(to_dev(ev["all_qm1"]), to_dev(ev["all_qm1"]), q, w))
    assert mi.rows_to_ints(allq) == [n % q] * n


@pytest.mark.parametrize("lam,logn", [(256, 20), (128, 18), (1024, 16)])
def test_cyclic_mul_full_size(lam, logn):
    """Large n: a shift by s against the rotation (any size), and a random product
    checked at sampled outputs against the definition."""
    import paper_2501_07535_amd as moma
    f, L, n, w, a, b = _pair(lam, logn, 405)
    q = f.q
    da, db = to_dev(a), to_dev(b)
    s = 12345 % n
    sh = np.zeros_like(a)
    sh[s, 0] = 1
    say(f"cyclic_mul full shift lam={lam} logn={logn}")
    got = from_dev(moma.ntt_cyclic_mul(da, to_dev(sh), q, w))
    assert (got == np.roll(a, s, axis=0)).all()
    say(f"cyclic_mul full random lam={lam} logn={logn}")
    c = from_dev(moma.ntt_cyclic_mul(da, db, q, w))
    ai, bi = mi.rows_to_ints(a), mi.rows_to_ints(b)
    for k in (0, 1, n // 3, n - 1):
        want = sum(ai[i] * bi[(k - i) % n] for i in range(n)) % q
        assert mi.rows_to_ints(c[k:k + 1])[0] == want, k


def test_batch_cyclic_mul_jobs():
    """Cyclic products mixed with forward and inverse jobs in one graph: each equals
    the plain call and the oracle."""
    import paper_2501_07535_amd as moma
    jobs = mi.batch_jobs(18, config=34)
    xs = mi.batch_inputs(jobs, config=34)
    ys = mi.batch_inputs(jobs, config=35)
    specs, outs, kinds, keep = [], [], [], []
    for k, (j, x, y) in enumerate(zip(jobs, xs, ys)):
        kind = (moma.JOB_CYCLIC_MUL, moma.JOB_FORWARD, moma.JOB_CYCLIC_MUL, moma.JOB_INVERSE)[k % 4]
        dx, dy = to_dev(x), to_dev(y)
        keep += [dx, dy]
        alias = k % 8 == 2
        o = dx if alias else torch.empty_like(dx)
        outs.append(o)
        kinds.append(kind)
        specs.append(((dx, dy) if kind == moma.JOB_CYCLIC_MUL else dx, o, j.field.q, j.omega, kind))
    say("batch create cyclic-mul jobs")
    bt = moma.Batch(specs)
    bt.run()
    torch.cuda.synchronize()
    import oracle
    for k, (j, x, y) in enumerate(zip(jobs, xs, ys)):
        got = from_dev(outs[k])
        if kinds[k] == moma.JOB_CYCLIC_MUL:
            plain = from_dev(moma.ntt_cyclic_mul(to_dev(x), to_dev(y), j.field.q, j.omega))
            want = _theorem(j.field.q, j.limbs, j.omega, x, y)
        elif kinds[k] == moma.JOB_INVERSE:
            plain = from_dev(moma.ntt_inv(to_dev(x), j.field.q, j.omega))
            want = oracle.intt_radix2(j.field.q, j.limbs, j.omega, x)
        else:
            plain = from_dev(moma.ntt_fwd(to_dev(x), j.field.q, j.omega))
            want = oracle.ntt_radix2(j.field.q, j.limbs, j.omega, x)
        assert (got == plain).all(), (k, j.lam, j.logn)
        assert (got == want).all(), (k, j.lam, j.logn)
    bt.close()


def test_cyclic_mul_rejects_bad_args():
    import ctypes
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    a = to_dev(mi.residues(f, 64, 8, 1))
    with pytest.raises(moma.MomaError) as e:
        moma.ntt_cyclic_mul(a, a, f.q, f.root(32))
    assert e.value.code == moma.MOMA_E_ROOT
    # a cyclic-product job without its second input, through the C ABI
    qw, ww = moma._words(f.q, 8), moma._words(f.root(64), 8)
    job = moma._Job(ctypes.cast(qw, moma._u32p), ctypes.cast(ww, moma._u32p), 64, 8, moma.JOB_CYCLIC_MUL,
                    a.data_ptr(), a.data_ptr(), None)
    h = ctypes.c_void_p()
    assert moma.library().moma_batch_create(ctypes.byref(job), 1, ctypes.byref(h)) == moma.MOMA_E_ARG
    assert not h.value
    job.kind = 7
    assert moma.library().moma_batch_create(ctypes.byref(job), 1, ctypes.byref(h)) == moma.MOMA_E_ARG
