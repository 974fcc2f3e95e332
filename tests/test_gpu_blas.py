"""GPU parity for the modular BLAS kernels: bit-exact against the oracle."""
import numpy as np
import pytest

import moma_inputs as mi
from gpu_util import from_dev, sample_indices, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [  # (class bits, storage limbs, n): several 256-lane blocks plus a ragged tail
    (64, 2, 5000), (128, 4, 1), (256, 8, 1000), (256, 8, 70001), (384, 12, 4097), (512, 16, 300),
    (768, 24, 777), (1024, 32, 513), (96, 3, 2049), (256, 10, 1500),  # last: storage wider than q
]


@pytest.mark.parametrize("lam,L,n", CASES)
def test_blas_matches_oracle(lam, L, n):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q = f.q
    a, b, y = (mi.residues(f, n, L, 100, k) for k in (1, 2, 3))
    alpha = mi.scalar_residue(f, 100, 4)
    da, db, dy = to_dev(a), to_dev(b), to_dev(y)
    say(f"blas lam={lam} L={L} n={n}")
    got = {
        "vadd": from_dev(moma.vadd(da, db, q)),
        "vsub": from_dev(moma.vsub(da, db, q)),
        "vmul": from_dev(moma.vmul(da, db, q)),
        "axpy": from_dev(moma.axpy(alpha, da, dy, q)),
    }
    assert (got["vadd"] == oracle.vadd(q, L, a, b)).all()
    assert (got["vsub"] == oracle.vsub(q, L, a, b)).all()
    assert (got["vmul"] == oracle.vmul(q, L, a, b)).all()
    assert (got["axpy"] == oracle.axpy(q, L, alpha, a, y)).all()


@pytest.mark.parametrize("lam", [64, 256, 384, 1024])
def test_blas_edge_vectors(lam):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q, L, n = f.q, f.limbs, 300
    ev = mi.edge_vectors(f, n, L)
    names = list(ev)
    say(f"blas edges lam={lam}")
    for i, na in enumerate(names):
        nb = names[(i + 3) % len(names)]
        a, b = ev[na], ev[nb]
        da, db = to_dev(a), to_dev(b)
        for op in ("vadd", "vsub", "vmul"):
            assert (from_dev(getattr(moma, op)(da, db, q)) == getattr(oracle, op)(q, L, a, b)).all(), (op, na, nb)
        for alpha in (0, 1, q - 1):
            assert (from_dev(moma.axpy(alpha, da, db, q)) == oracle.axpy(q, L, alpha, a, b)).all(), (alpha, na, nb)
    a, b = mi.sum_to_q_pair(f, n, L, 101)
    assert (from_dev(moma.vadd(to_dev(a), to_dev(b), q)) == 0).all()      # a + b == q -> 0
    assert (from_dev(moma.vsub(to_dev(a), to_dev(a), q)) == 0).all()


def test_blas_in_place_and_empty():
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(384, 0)
    q, L, n = f.q, 12, 3001
    a, b = mi.residues(f, n, L, 102, 1), mi.residues(f, n, L, 102, 2)
    da, db = to_dev(a), to_dev(b)
    say("blas in place")
    moma.vmul(da, db, q, out=da)
    assert (from_dev(da) == oracle.vmul(q, L, a, b)).all()
    db2 = to_dev(b)
    moma.axpy(7, to_dev(a), db2, q, out=db2)
    assert (from_dev(db2) == oracle.axpy(q, L, 7, a, b)).all()
    e = torch.zeros((L, 0), dtype=torch.int32, device="cuda:0")
    assert moma.vadd(e, e, q).shape == (L, 0)


@pytest.mark.parametrize("lam,L", [(256, 8), (384, 12), (768, 24)])
def test_blas_full_size_sampled(lam, L):
    """The workload size: 2^24 elements; outputs checked at sampled positions."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q, n = f.q, 1 << 24
    a, b = mi.residues(f, n, L, 1, 1), mi.residues(f, n, L, 1, 2)
    alpha = mi.scalar_residue(f, 1, 3)
    idx = sample_indices(n, 4000, lam)
    da, db = to_dev(a), to_dev(b)
    say(f"blas full lam={lam} n=2^24")
    for op in ("vadd", "vsub", "vmul"):
        out = getattr(moma, op)(da, db, q)
        got = mi.from_planar(out[:, torch.from_numpy(idx).to("cuda:0")].cpu().numpy().view(np.uint32))
        assert (got == getattr(oracle, op)(q, L, a[idx], b[idx])).all(), op
        del out
    out = moma.axpy(alpha, da, db, q)
    got = mi.from_planar(out[:, torch.from_numpy(idx).to("cuda:0")].cpu().numpy().view(np.uint32))
    assert (got == oracle.axpy(q, L, alpha, a[idx], b[idx])).all()


KARA_CASES = [(64, 2, 3000), (96, 3, 1025), (128, 4, 700), (160, 5, 513), (256, 8, 2049), (384, 12, 999),
              (512, 16, 257), (768, 24, 300), (992, 31, 130), (1024, 32, 129)]


@pytest.mark.parametrize("lam,L,n", KARA_CASES)
def test_vmul_karatsuba_matches_oracle(lam, L, n):
    """The Karatsuba product variant (even and odd limb counts) gives the oracle's
    products, on random residues and on the edge vectors."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q = f.q
    a, b = mi.residues(f, n, L, 102, 1), mi.residues(f, n, L, 102, 2)
    ev = mi.edge_vectors(f, n, L)
    say(f"vmul karatsuba lam={lam} L={L} n={n}")
    moma.vmul_set_variant(q, L, moma.VMUL_KARATSUBA)
    try:
        assert (from_dev(moma.vmul(to_dev(a), to_dev(b), q)) == oracle.vmul(q, L, a, b)).all()
        names = list(ev)
        for i, na in enumerate(names):
            x, y = ev[na], ev[names[(i + 2) % len(names)]]
            assert (from_dev(moma.vmul(to_dev(x), to_dev(y), q)) == oracle.vmul(q, L, x, y)).all(), na
    finally:
        moma.vmul_set_variant(q, L, moma.VMUL_SCHOOLBOOK)


def test_vmul_tune_installs_a_variant():
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(768, 0)
    q, L = f.q, f.limbs
    say("vmul tune 768")
    r = moma.vmul_tune(q, L, 1 << 16, reps=3)
    assert r["chosen"] in (moma.VMUL_SCHOOLBOOK, moma.VMUL_KARATSUBA)
    assert r["schoolbook_us"] > 0 and r["karatsuba_us"] > 0
    assert moma.vmul_get_variant(q, L) == r["chosen"]
    a, b = mi.residues(f, 4097, L, 103, 1), mi.residues(f, 4097, L, 103, 2)
    assert (from_dev(moma.vmul(to_dev(a), to_dev(b), q)) == oracle.vmul(q, L, a, b)).all()
    moma.vmul_set_variant(q, L, moma.VMUL_SCHOOLBOOK)


@pytest.mark.parametrize("lam,n", [(256, 4096), (384, 2048), (128, 1024)])
def test_blas_unaligned_buffers(lam, n):
    """Planes that are not 16-byte aligned (a buffer starting one word into an
    allocation) take the one-element-per-lane kernels; results are unchanged."""
    import oracle
    import torch
    import paper_2501_07535_amd as moma
    f = mi.find_prime(lam, 0)
    q, L = f.q, f.limbs
    a, b = mi.residues(f, n, L, 104, 1), mi.residues(f, n, L, 104, 2)

    def shifted(x):
        flat = torch.empty(L * n + 1, dtype=torch.int32, device="cuda:0")
        v = flat[1:].view(L, n)
        v.copy_(to_dev(x))
        return v

    da, db = shifted(a), shifted(b)
    out = torch.empty(L * n + 1, dtype=torch.int32, device="cuda:0")[1:].view(L, n)
    say(f"blas unaligned lam={lam} n={n}")
    for op in ("vadd", "vsub", "vmul"):
        getattr(moma, op)(da, db, q, out=out)
        assert (from_dev(out) == getattr(oracle, op)(q, L, a, b)).all(), op
    moma.axpy(7, da, db, q, out=out)
    assert (from_dev(out) == oracle.axpy(q, L, 7, a, b)).all()
