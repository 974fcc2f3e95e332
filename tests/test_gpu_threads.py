"""Calls from several host threads at once, each on its own stream: the plan
cache is shared (several threads create and use the same plans), and every
result still equals the oracle's.  ctypes releases the GIL during a library
call, so the calls really overlap on the host."""
import threading

import pytest
import torch

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

NTHREADS = 6
ITERS = 6


def test_threads_share_plans_and_get_oracle_results():
    import oracle
    import paper_2501_07535_amd as moma
    moma.shutdown()                                   # every plan is created under contention
    # shared plans: out-of-place transforms of the same (q, n) from every thread
    shared = []
    for lam, logn in ((256, 12), (128, 15), (384, 10)):
        f = mi.find_prime(lam, 0)
        n, w = 1 << logn, f.root(1 << logn)
        x = mi.residues(f, n, f.limbs, 700, logn)
        shared.append((f, w, x, oracle.ntt_radix2(f.q, f.limbs, w, x), oracle.intt_radix2(f.q, f.limbs, w, x)))
    # private plans: in-place transforms and cyclic products use the plan's scratch,
    # so each thread has its own (q, n)
    private = []
    for t in range(NTHREADS):
        f = mi.find_prime(64 + 64 * (t % 4), 10 + t)
        logn = 9 + t % 3
        n, w = 1 << logn, f.root(1 << logn)
        a, b = mi.residues(f, n, f.limbs, 701, t, 1), mi.residues(f, n, f.limbs, 701, t, 2)
        private.append((f, w, a, b, oracle.ntt_radix2(f.q, f.limbs, w, a), oracle.cyclic_conv(f.q, f.limbs, a, b),
                        oracle.vmul(f.q, f.limbs, a, b)))
    dev_shared = [(to_dev(x), f, w) for f, w, x, _, _ in shared]
    dev_private = [(to_dev(a), to_dev(b)) for _, _, a, b, *_ in private]
    torch.cuda.synchronize()

    results = [None] * NTHREADS
    errors = []
    start = threading.Barrier(NTHREADS)

    def work(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                f, w, a, b, *_ = private[t]
                da, db = dev_private[t]
                got = []
                start.wait()
                for it in range(ITERS):
                    dx, g, gw = dev_shared[(t + it) % len(dev_shared)]
                    y = moma.ntt_fwd(dx, g.q, gw)
                    z = moma.ntt_inv(dx, g.q, gw)
                    inpl = da.clone()
                    moma.ntt_fwd(inpl, f.q, w, out=inpl)
                    c = moma.ntt_cyclic_mul(da, db, f.q, w)
                    p = moma.vmul(da, db, f.q)
                    got.append(((t + it) % len(dev_shared), y, z, inpl, c, p))
                # a failing call reports its own error on this thread
                with pytest.raises(moma.MomaError) as e:
                    moma.ntt_fwd(da, f.q, 2)
                assert e.value.code == moma.MOMA_E_ROOT
                s.synchronize()
                results[t] = [(k, from_dev(y), from_dev(z), from_dev(i), from_dev(c), from_dev(p))
                              for k, y, z, i, c, p in got]
        except BaseException as ex:  # reported from the main thread
            errors.append((t, repr(ex)))
            start.abort()

    say(f"threads: {NTHREADS} threads x {ITERS} iterations")
    th = [threading.Thread(target=work, args=(t,)) for t in range(NTHREADS)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not any(x.is_alive() for x in th), "a thread did not finish"
    assert not errors, errors
    for t in range(NTHREADS):
        _, _, _, _, fwd, cyc, prod = private[t]
        for k, y, z, inpl, c, p in results[t]:
            assert (y == shared[k][3]).all(), (t, k)
            assert (z == shared[k][4]).all(), (t, k)
            assert (inpl == fwd).all(), t
            assert (c == cyc).all(), t
            assert (p == prod).all(), t
