"""Autotuner, timing database and learned cost model on the GPU."""
import os

import numpy as np
import pytest

import moma_inputs as mi
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


def test_tune_exhaustive_installs_the_fastest(tmp_path):
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    L, n = 8, 1 << 12
    w = f.root(n)
    moma.tune_db_clear()
    say("tune exhaustive 256-bit 2^12")
    r = moma.ntt_tune(f.q, w, n, L, reps=3, warmup=1)
    assert r["timed"] == r["feasible"] == len(moma.ntt_candidates(L, 12)) > 5
    rows = moma.tune_db_rows()
    assert len(rows) == r["timed"]
    best = min(rows, key=lambda x: x["us"])
    assert best["sched"] == r["best"] == moma.ntt_get_schedule(f.q, w, n, L)
    assert abs(best["us"] - r["best_us"]) < 1e-6 * max(1.0, best["us"])
    x = mi.residues(f, n, L, 400)
    assert (from_dev(moma.ntt_fwd(to_dev(x), f.q, w)) == oracle.ntt_radix2(f.q, L, w, x)).all()
    path = str(tmp_path / "db.csv")
    moma.tune_db_save(path)
    moma.tune_db_clear()
    assert moma.tune_db_rows() == []
    moma.tune_db_load(path)
    assert len(moma.tune_db_rows()) == len(rows)


def test_costmodel_ranks_and_top_k(tmp_path):
    import paper_2501_07535_amd as moma
    moma.tune_db_clear()
    f = mi.find_prime(128, 0)
    shapes = [(11, ), (13, ), (14, )]
    for (logn,) in shapes:
        say(f"tune 128-bit 2^{logn}")
        moma.ntt_tune(f.q, f.root(1 << logn), 1 << logn, f.limbs, reps=3, warmup=1)
    rows = moma.tune_db_rows()
    feats = np.array([moma.costmodel_features(r["limbs"], r["log2_n"], r["sched"]) for r in rows], np.float32)
    y = np.log(np.array([r["us"] for r in rows], np.float32))
    mse = moma.costmodel_train(feats, y, epochs=300, batch=64, lr=3e-3, seed=3)
    assert mse < np.var(y)                      # better than predicting the mean
    pred = moma.costmodel_predict(feats)
    assert np.corrcoef(pred, y)[0, 1] > 0.5
    path = str(tmp_path / "cm.txt")
    moma.costmodel_save(path)
    moma.costmodel_clear()
    with pytest.raises(moma.MomaError):
        moma.costmodel_predict(feats)
    moma.costmodel_load(path)
    assert np.allclose(moma.costmodel_predict(feats), pred, rtol=1e-5, atol=1e-5)
    r = moma.ntt_tune(f.q, f.root(1 << 12), 1 << 12, f.limbs, reps=3, warmup=1, top_k=3)
    assert r["timed"] == 3 and r["feasible"] > 3
    moma.costmodel_clear()
    with pytest.raises(moma.MomaError):
        moma.ntt_tune(f.q, f.root(1 << 12), 1 << 12, f.limbs, top_k=3)
    moma.load_packaged_costmodel()


def test_new_plans_take_the_models_pick():
    """With the packaged model loaded and no timings for a shape, a new plan
    starts from the candidate with the lowest predicted time; the transform is
    still the oracle's."""
    import oracle
    import paper_2501_07535_amd as moma
    if not moma.load_packaged_costmodel():
        pytest.skip("no packaged cost model")
    moma.tune_db_clear()
    moma.shutdown()
    f = mi.find_prime(384, 7)
    L, logn = f.limbs, 15
    n, w = 1 << logn, f.root(1 << logn)
    cands = moma.ntt_candidates(L, logn)
    feats = np.array([moma.costmodel_features(L, logn, s) for s in cands], np.float32)
    pick = tuple(cands[int(np.argmin(moma.costmodel_predict(feats)))])
    say(f"model pick 384-bit 2^{logn}: {pick}")
    assert moma.ntt_get_schedule(f.q, w, n, L) == pick
    x = mi.residues(f, n, L, 602)
    assert (from_dev(moma.ntt_fwd(to_dev(x), f.q, w)) == oracle.ntt_radix2(f.q, L, w, x)).all()
    moma.ntt_set_schedule(f.q, w, n, L, moma.ntt_default_schedule(L, logn))
    moma.ntt_set_schedule(f.q, w, n, L, None)                 # back to the model's pick
    assert moma.ntt_get_schedule(f.q, w, n, L) == pick


def test_tuners_with_storage_wider_than_the_modulus():
    """The tuners' own buffers hold the caller's storage planes (a transform
    zero-fills the planes above the compute limbs), here 10 planes for a
    252-bit modulus; the tuned plan still gives the oracle's transform."""
    import oracle
    import paper_2501_07535_amd as moma
    f = mi.find_prime(256, 0)
    q, n, Ls = f.q, 1 << 12, 10
    w = f.root(n)
    say("tune wide storage")
    r = moma.ntt_tune(q, w, n, Ls, reps=1, warmup=1, max_candidates=6)
    assert r["timed"] >= 1 and r["best_us"] > 0
    x = mi.residues(f, n, Ls, 600)
    assert (from_dev(moma.ntt_fwd(to_dev(x), q, w)) == oracle.ntt_radix2(q, Ls, w, x)).all()
    v = moma.vmul_tune(q, Ls, 4096, reps=2)
    assert v["schoolbook_us"] > 0 and v["karatsuba_us"] > 0
    a, b = mi.residues(f, 999, Ls, 601, 1), mi.residues(f, 999, Ls, 601, 2)
    assert (from_dev(moma.vmul(to_dev(a), to_dev(b), q)) == oracle.vmul(q, Ls, a, b)).all()
    moma.vmul_set_variant(q, Ls, moma.VMUL_SCHOOLBOOK)
    moma.ntt_set_schedule(q, w, n, Ls, None)


def _random_k_expected(times, k):
    """Expected best time of k distinct candidates drawn uniformly at random:
    the i-th fastest (0-based) is the best of the draw with probability
    C(N-1-i, k-1) / C(N, k)."""
    from math import comb
    t = sorted(times)
    N = len(t)
    return sum(t[i] * comb(N - 1 - i, k - 1) for i in range(N)) / comb(N, k)


def test_learned_model_gains_over_default_rule_and_random_picks():
    """What the trained network gains over the method without it.  Sixteen
    shapes (4 widths x 4 sizes) are tuned exhaustively; a fresh network is
    trained on the GPU from twelve of them; on the four held-out shapes,
    timing only the network's top 3 candidates must cost less (geometric mean
    regret against the exhaustive best) than the fixed default rule and than
    3 random candidates."""
    import paper_2501_07535_amd as moma
    widths, sizes = (64, 128, 256, 384), (10, 12, 14, 16)
    held = {(128, 12), (256, 14), (64, 14), (384, 12)}
    moma.tune_db_clear()
    shapes = {}
    try:
        for lam in widths:
            f = mi.find_prime(lam, 0)
            for logn in sizes:
                n = 1 << logn
                say(f"gain test: tune {lam}-bit 2^{logn}")
                moma.ntt_tune(f.q, f.root(n), n, f.limbs, reps=3, warmup=1)
                shapes[(lam, logn)] = f.limbs
        rows = moma.tune_db_rows()
        by_shape = {}
        for r in rows:
            by_shape.setdefault((r["limbs"], r["log2_n"]), {})[tuple(r["sched"])] = r["us"]
        train = [r for r in rows if (32 * r["limbs"], r["log2_n"]) not in held]
        feats = np.array([moma.costmodel_features(r["limbs"], r["log2_n"], r["sched"]) for r in train], np.float32)
        y = np.log(np.array([r["us"] for r in train], np.float32))
        say(f"gain test: train on {len(train)} timings")
        moma.costmodel_train(feats, y, epochs=300, batch=128, lr=3e-3, seed=11)
        model, default, rand3 = [], [], []
        for lam, logn in sorted(held):
            L = shapes[(lam, logn)]
            t = by_shape[(L, logn)]
            cands = list(t)
            best = min(t.values())
            pf = np.array([moma.costmodel_features(L, logn, s) for s in cands], np.float32)
            order = np.argsort(moma.costmodel_predict(pf), kind="stable")
            model.append(min(t[cands[i]] for i in order[:3]) / best)
            default.append(t[tuple(moma.ntt_default_schedule(L, logn))] / best)
            rand3.append(_random_k_expected(list(t.values()), 3) / best)
        g = {name: float(np.exp(np.mean(np.log(v)))) - 1 for name, v in
             (("model_top3", model), ("default_rule", default), ("random_3", rand3))}
        say(f"gain test: held-out geomean regret {g}; per shape model {model} default {default} random {rand3}")
        assert g["model_top3"] < g["random_3"]
        assert g["model_top3"] <= g["default_rule"]
    finally:
        moma.tune_db_clear()
        moma.costmodel_clear()
        moma.load_packaged_costmodel()
        moma.shutdown()
