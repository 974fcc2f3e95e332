"""Host-side logic of the library that needs no GPU: the launch-shape
enumeration and its constraints, the fixed default rule, cost-model features,
the packaged model file and the timing-database file format."""
import math

import pytest

MAX_RADIX = {**{L: 4 for L in range(1, 3)}, **{L: 3 for L in range(3, 6)}, **{L: 2 for L in range(6, 17)}, **{L: 1 for L in range(17, 33)}}


def _max_threads(L, r):
    live = L << r
    return 1024 if live <= 16 else (512 if live <= 32 else 256)


def _passes(L, logn, s):
    """Stages per pass of a schedule, as the header documents the split."""
    tile, col, threads, r = s[:4]
    if logn <= tile:
        return [logn]
    kmax = tile - col
    P = -(-logn // kmax)
    return [logn // P + (1 if i < logn % P else 0) for i in range(P)]


@pytest.mark.parametrize("L", [1, 2, 5, 8, 11, 16, 24, 32])
@pytest.mark.parametrize("logn", [1, 4, 10, 12, 16, 20, 26])
def test_candidates_respect_the_documented_limits(L, logn):
    import paper_2501_07535_amd as moma
    cands = moma.ntt_candidates(L, logn)
    assert cands, (L, logn)
    assert len(set(cands)) == len(cands)
    for s in cands:
        tile, col, threads, r, mv = s
        assert threads % 64 == 0 and 64 <= threads <= _max_threads(L, r), s
        assert 1 <= r <= MAX_RADIX[L], s
        # the Karatsuba butterfly: radix 2, 2 to 24 limbs
        assert mv == 0 or (mv == 1 and r == 1 and 2 <= L <= 24), s
        assert 4 * L * (1 << tile) <= 160 * 1024, s
        ps = _passes(L, logn, s)
        if logn > tile:
            assert sum(ps) == logn and max(ps) <= tile - col, s
    # every radix-2 shape comes once more with the Karatsuba multiply, after the schoolbook ones
    school = [s for s in cands if s[4] == 0]
    kara = [s for s in cands if s[4] == 1]
    assert cands == school + kara
    assert kara == ([s[:4] + (1,) for s in school if s[3] == 1] if 2 <= L <= 24 else [])


@pytest.mark.parametrize("L", list(range(1, 33)))
def test_default_rule_is_a_candidate_for_every_size(L):
    import paper_2501_07535_amd as moma
    for logn in range(1, 27):
        d = moma.ntt_default_schedule(L, logn)
        assert d in moma.ntt_candidates(L, logn), (L, logn, d)


def test_costmodel_features_follow_their_definition():
    import paper_2501_07535_amd as moma
    L, logn, s = 8, 20, (10, 5, 256, 2)
    f = moma.costmodel_features(L, logn, s)
    assert len(f) == 7 and f[6] == 0.0                  # schoolbook multiply
    assert moma.costmodel_features(L, logn, (10, 5, 256, 1, 1))[6] == 1.0
    assert f[:3] == [20.0, 8.0, 2.0]
    assert f[3] == 5.0                                 # stages of the longest pass
    assert f[4] == pytest.approx(math.log2(256))
    assert f[5] == pytest.approx(math.log2(4 * 8 * 2 ** 10))
    g = moma.costmodel_features(4, 9, (12, 4, 128, 3))  # one pass: the whole transform in LDS
    assert g[3] == 9.0 and g[5] == pytest.approx(math.log2(4 * 4 * 2 ** 9))


def test_packaged_costmodel_file_loads_and_bad_files_are_rejected(tmp_path):
    import paper_2501_07535_amd as moma
    with open(moma.COSTMODEL_PATH) as fh:
        head = fh.readline().split()
    assert head[:2] == ["moma-costmodel", "1"] and int(head[2]) == moma.mlp_nparams()
    moma.costmodel_load(moma.COSTMODEL_PATH)
    bad = tmp_path / "bad.txt"
    bad.write_text("moma-costmodel 1 12\n1 2\n")
    with pytest.raises(moma.MomaError) as e:
        moma.costmodel_load(str(bad))
    assert e.value.code == moma.MOMA_E_ARG
    with pytest.raises(moma.MomaError):
        moma.costmodel_load(str(tmp_path / "missing.txt"))
    moma.load_packaged_costmodel()


def test_timing_database_file_round_trip(tmp_path):
    import paper_2501_07535_amd as moma
    src = tmp_path / "db.csv"
    src.write_text("device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps\n"
                   "gfx950/256cu,8,20,10,5,256,2,139.5,3\n"
                   "gfx950/256cu,4,12,12,0,512,2,8.25,3\n")
    moma.tune_db_clear()
    moma.tune_db_load(str(src))
    rows = moma.tune_db_rows()
    assert [(r["limbs"], r["log2_n"], r["sched"], r["reps"]) for r in rows] == \
        [(8, 20, (10, 5, 256, 2, 0), 3), (4, 12, (12, 0, 512, 2, 0), 3)]
    assert rows[0]["us"] == pytest.approx(139.5)
    out = tmp_path / "out.csv"
    moma.tune_db_save(str(out))
    moma.tune_db_clear()
    moma.tune_db_load(str(out))
    assert [(r["limbs"], r["log2_n"], r["sched"]) for r in moma.tune_db_rows()] == \
        [(r["limbs"], r["log2_n"], r["sched"]) for r in rows]
    moma.tune_db_clear()


def test_timing_database_keeps_the_multiply_variant(tmp_path):
    import paper_2501_07535_amd as moma
    src = tmp_path / "db.csv"
    src.write_text("device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps,mul_variant\n"
                   "gfx950/256cu,8,12,12,0,256,1,30.5,3,1\n"
                   "gfx950/256cu,8,12,12,0,256,1,20.5,3,0\n")
    moma.tune_db_clear()
    moma.tune_db_load(str(src))
    assert [r["sched"] for r in moma.tune_db_rows()] == [(12, 0, 256, 1, 1), (12, 0, 256, 1, 0)]
    out = tmp_path / "out.csv"
    moma.tune_db_save(str(out))
    assert open(out).readline().strip().endswith(",mul_variant")
    moma.tune_db_clear()
    bad = tmp_path / "bad.csv"
    bad.write_text("device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps,mul_variant\n"
                   "gfx950/256cu,8,12,12,0,256,1,30.5,3,2\n")
    with pytest.raises(moma.MomaError):
        moma.tune_db_load(str(bad))
    moma.tune_db_clear()
