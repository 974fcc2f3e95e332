"""Host logic of the tuning tool (no GPU): reading timing databases and the
width-sweep report."""
import json

import pytest


def _db(path, rows):
    with open(path, "w") as fh:
        fh.write("device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps\n")
        for r in rows:
            fh.write(",".join(str(v) for v in r) + "\n")


def test_load_rows_keeps_latest_measurement(tmp_path):
    from paper_2501_07535_amd import tuning
    p = tmp_path / "db.csv"
    _db(p, [("dev", 8, 12, 10, 5, 256, 2, 50.0, 3), ("dev", 8, 12, 10, 5, 256, 2, 40.0, 3),
            ("dev", 8, 12, 9, 4, 128, 1, 45.0, 3)])
    rows = sorted(tuning.load_rows([str(p)]))
    assert rows == [(8, 12, (9, 4, 128, 1, 0), 45.0), (8, 12, (10, 5, 256, 2, 0), 40.0)]


def test_load_rows_reads_the_multiply_variant_column(tmp_path):
    """Rows with the mul_variant column keep it; rows without read as schoolbook."""
    from paper_2501_07535_amd import tuning
    p = tmp_path / "db.csv"
    with open(p, "w") as fh:
        fh.write("device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps,mul_variant\n")
        fh.write("dev,8,12,9,4,128,1,45.0,3,1\n")
        fh.write("dev,8,12,9,4,128,1,41.0,3,0\n")
        fh.write("dev,8,12,9,4,128,1,47.0,3\n")
    rows = sorted(tuning.load_rows([str(p)]))
    assert rows == [(8, 12, (9, 4, 128, 1, 0), 47.0), (8, 12, (9, 4, 128, 1, 1), 45.0)]


def test_widths_report_best_time_and_doublings(tmp_path):
    from paper_2501_07535_amd import tuning
    p = tmp_path / "db.csv"
    rows = []
    for L, base in ((2, 10.0), (4, 20.0), (8, 50.0), (16, 150.0), (32, 600.0), (3, 15.0)):
        rows.append(("dev", L, 12, 10, 5, 256, 2, base * 1.5, 3))
        rows.append(("dev", L, 12, 9, 4, 128, 1, base, 3))      # the fastest schedule of the shape
        rows.append(("dev", L, 16, 10, 5, 256, 2, base * 4, 3))
    _db(p, rows)
    out = tmp_path / "w.json"
    rep = tuning.widths([str(p)], str(out))
    assert json.load(open(out)) == json.loads(json.dumps(rep))
    s12 = rep["sizes"]["12"]
    assert s12["us_by_width"][64] == 10.0 and s12["us_by_width"][96] == 15.0
    assert s12["slowdown_per_doubling"] == {"64->128": 2.0, "128->256": 2.5, "256->512": 3.0, "512->1024": 4.0}
    assert rep["sizes"]["16"]["slowdown_per_doubling"]["64->128"] == pytest.approx(2.0)
