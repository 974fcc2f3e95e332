"""GPU parity for the forward and inverse NTT: bit-exact against the oracle."""
import numpy as np
import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def _case(lam, logn, seed=200):
    f = mi.find_prime(lam, 0)
    n = 1 << logn
    return f, f.limbs, n, f.root(n), mi.residues(f, n, f.limbs, seed, logn)


@pytest.mark.parametrize("logn", list(range(1, 16)))
def test_ntt_256_all_small_sizes(logn):
    """Single-pass (LDS) sizes up to 2^11 and multi-pass sizes from 2^12 at 256 bits."""
    import oracle
    import paper_2501_07535_amd as moma
    f, L, n, w, x = _case(256, logn)
    say(f"ntt lam=256 logn={logn}")
    y = moma.ntt_fwd(to_dev(x), f.q, w)
    want = oracle.ntt_radix2(f.q, L, w, x)
    assert (from_dev(y) == want).all()
    z = moma.ntt_inv(to_dev(want), f.q, w)
    assert (from_dev(z) == oracle.intt_radix2(f.q, L, w, want)).all()


@pytest.mark.parametrize("lam,logn", [(64, 12), (64, 14), (96, 13), (128, 12), (128, 15), (384, 11), (384, 13),
                                      (512, 12), (768, 10), (768, 12), (1024, 9), (1024, 12)])
def test_ntt_other_widths(lam, logn):
    import oracle
    import paper_2501_07535_amd as moma
    f, L, n, w, x = _case(lam, logn)
    say(f"ntt lam={lam} logn={logn}")
    y = from_dev(moma.ntt_fwd(to_dev(x), f.q, w))
    assert (y == oracle.ntt_radix2(f.q, L, w, x)).all()
    assert (from_dev(moma.ntt_inv(to_dev(y), f.q, w)) == x).all()


@pytest.mark.parametrize("logn", [4, 11, 13])
def test_ntt_in_place(logn):
    import oracle
    import paper_2501_07535_amd as moma
    f, L, n, w, x = _case(256, logn, 201)
    say(f"ntt in place logn={logn}")
    d = to_dev(x)
    moma.ntt_fwd(d, f.q, w, out=d)
    assert (from_dev(d) == oracle.ntt_radix2(f.q, L, w, x)).all()
    moma.ntt_inv(d, f.q, w, out=d)
    assert (from_dev(d) == x).all()


@pytest.mark.parametrize("logn", [3, 12])
def test_ntt_closed_forms_and_edges(logn):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n, q = 8, 1 << logn, f.q
    w = f.root(n)
    ev = mi.edge_vectors(f, n, L)
    say(f"ntt edges logn={logn}")
    assert mi.rows_to_ints(from_dev(moma.ntt_fwd(to_dev(ev["delta0"]), q, w))) == [1] * n
    assert mi.rows_to_ints(from_dev(moma.ntt_fwd(to_dev(ev["ones"]), q, w))) == [n] + [0] * (n - 1)
    assert mi.rows_to_ints(from_dev(moma.ntt_fwd(to_dev(ev["delta1"]), q, w))) == [pow(w, k, q) for k in range(n)]
    for name in ("zeros", "all_qm1", "alt_0_qm1", "carry_run"):
        x = ev[name]
        assert (from_dev(moma.ntt_fwd(to_dev(x), q, w)) == oracle.ntt_radix2(q, L, w, x)).all(), name
        assert (from_dev(moma.ntt_inv(to_dev(x), q, w)) == oracle.intt_radix2(q, L, w, x)).all(), name


def test_ntt_storage_wider_than_modulus():
    """q of 252 bits stored in 10 limbs: the upper planes come back zero."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n = 10, 1 << 12
    w = f.root(n)
    x = mi.residues(f, n, L, 202)
    say("ntt wide storage")
    out = torch.full((L, n), -1, dtype=torch.int32, device="cuda:0")
    y = from_dev(moma.ntt_fwd(to_dev(x), f.q, w, out=out))
    assert (y == oracle.ntt_radix2(f.q, L, w, x)).all()


def test_ntt_convolution_theorem_on_gpu():
    """inv(fwd(a) * fwd(b)) is the cyclic convolution, computed by the oracle's definition."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(384, 0)
    L, n, q = 12, 256, f.q
    w = f.root(n)
    a, b = mi.residues(f, n, L, 203, 1), mi.residues(f, n, L, 203, 2)
    say("ntt convolution")
    ya, yb = moma.ntt_fwd(to_dev(a), q, w), moma.ntt_fwd(to_dev(b), q, w)
    c = from_dev(moma.ntt_inv(moma.vmul(ya, yb, q), q, w))
    assert (c == oracle.cyclic_conv(q, L, a, b)).all()


FULL = [(256, 16), (256, 17), (256, 18), (256, 19), (256, 20), (256, 21), (256, 22), (256, 23), (256, 24),
        (128, 20), (384, 20), (1024, 20)]


@pytest.mark.parametrize("lam,logn", FULL)
def test_ntt_full_size_sampled(lam, logn):
    """The sweep sizes: outputs checked at sampled k against the definition, and
    the whole vector through the round trip."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 2, logn)
    say(f"ntt full lam={lam} logn={logn}")
    dx = to_dev(x)
    y = moma.ntt_fwd(dx, q, w)
    rng = np.random.default_rng(logn * 1000 + lam)
    nsamp = 8 if n * L >= (1 << 25) else 16
    ks = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, nsamp)]).astype(np.int64))
    got = mi.from_planar(y[:, torch.from_numpy(ks).to("cuda:0")].cpu().numpy().view(np.uint32))
    assert (got == oracle.ntt_direct(q, L, w, x, ks)).all()
    z = moma.ntt_inv(y, q, w)
    assert torch.equal(z, dx)


@pytest.mark.parametrize("sched", [(10, 5, 256, 2), (11, 5, 256, 2)])
def test_headline_size_in_the_benchmarked_launch_shape(sched):
    """256 bits, n = 2^20, in the launch shapes the benchmark times (the
    autotuner's picks): sampled outputs against the definition, the whole
    vector against the oracle's fast transform, the round trip, and the
    in-place call."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n, q = 8, 1 << 20, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 2, 20)          # the benchmark's input stream
    moma.ntt_set_schedule(q, w, n, L, sched)
    try:
        say(f"headline shape {sched}")
        dx = to_dev(x)
        y = moma.ntt_fwd(dx, q, w)
        ks = np.array([0, 1, 12345, n // 3, n - 1], dtype=np.int64)
        got = mi.from_planar(y[:, torch.from_numpy(ks).to("cuda:0")].cpu().numpy().view(np.uint32))
        assert (got == oracle.ntt_direct(q, L, w, x, ks)).all()
        assert (from_dev(y) == oracle.ntt_radix2(q, L, w, x)).all()
        assert torch.equal(moma.ntt_inv(y, q, w), dx)
        moma.ntt_fwd(dx, q, w, out=dx)
        assert torch.equal(dx, y)
    finally:
        moma.ntt_set_schedule(q, w, n, L, None)
