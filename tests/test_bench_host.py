"""Host logic of bench.py, on the CPU: the op model that prices the roofline
(Section 5.3's butterfly as the unit of work), the choice of the committed
counter record, and the one-GPU refusal."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

RATES = ("add_u32", "add_co_addc_u32", "mad_u64_u32", "mad_addc_u32", "mul_lo_u32", "mul_hi_u32")


def _rates(scale=1.0):
    return {k: bench.PEAK_INT_OPS * scale for k in RATES}


@pytest.mark.parametrize("L", [2, 4, 8, 10, 12, 20, 24, 32])
def test_multiply_forms_count_their_instructions(L):
    """At rates equal to the peak every instruction costs one lane-op: the word
    form is P(L) products with a carry step each, the digit form 2D^2 products,
    D reduction multiplies and two add-class ops per column."""
    f = bench.multiply_forms(L, _rates())
    b = 29 if L <= 28 else 28
    D = -(-(32 * L - 2) // b)
    assert f["digits"] == D
    assert f["word"] == pytest.approx(2 * (2 * L * L + L))
    assert f["digit"] == pytest.approx(2 * D * D + D + 2 * (2 * D - 1))
    assert bench.butterfly_slots(L, _rates()) == pytest.approx(min(f["word"], f["digit"]) + 6 * L)


def test_op_costs_scale_with_the_measured_rates():
    """Twice the issue rate, half the lane-ops: achieved / peak is time at the
    measured rates over the measured time."""
    for L in (4, 8, 32):
        assert bench.butterfly_slots(L, _rates(2.0)) == pytest.approx(bench.butterfly_slots(L, _rates()) / 2)
    cm, ca = bench.issue_costs(_rates(0.5))
    assert (cm, ca) == (pytest.approx(4.0), pytest.approx(2.0))


def test_digit_form_is_the_cheaper_from_eight_limbs_at_measured_rates():
    """With the rates gfx950 measures (mad 33, mad+addc pair 37.6, add/addc
    chain 36.3, mul_lo 38 T/s) the digit form is priced below the word form
    from 8 limbs on and above it at 2 limbs, as the kernels' choice implies."""
    r = {"add_u32": 54.3e12, "add_co_addc_u32": 36.3e12, "mad_u64_u32": 32.3e12, "mad_addc_u32": 37.6e12,
         "mul_lo_u32": 38.0e12, "mul_hi_u32": 37.9e12}
    for L in (8, 12, 16, 24, 32):
        f = bench.multiply_forms(L, r)
        assert f["digit"] < f["word"], L
    f = bench.multiply_forms(2, r)
    assert f["word"] < f["digit"]


def _fake_repo(tmp_path, records, sources_text=b"kernel source"):
    src = tmp_path / "k.hpp"
    src.write_bytes(sources_text)
    h = hashlib.sha256(sources_text).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    top = {"kernel_sources_sha256": h, "sources": ["k.hpp"], "records": records}
    (prof / "ntt_counters_L8_256bit_n2e20.json").write_text(json.dumps(top))
    return src


def test_counter_record_matches_the_tuned_launches(tmp_path, monkeypatch):
    recs = [{"schedule": [10, 5, 256, 2, 0], "pass_stages": [5, 5, 5, 5], "traffic_bytes_per_launch": 1},
            {"schedule": [11, 5, 128, 2, 0], "pass_stages": [5, 5, 5, 5], "traffic_bytes_per_launch": 2}]
    src = _fake_repo(tmp_path, recs)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the tile size bound does not change the launches; threads, columns, radix and passes do
    assert bench.committed_counters(256, 20, (11, 5, 256, 2, 0), [5, 5, 5, 5])["traffic_bytes_per_launch"] == 1
    assert bench.committed_counters(256, 20, (10, 5, 128, 2, 0), [5, 5, 5, 5])["traffic_bytes_per_launch"] == 2
    assert bench.committed_counters(256, 20, (10, 4, 256, 2, 0), [5, 5, 5, 5]) is None
    assert bench.committed_counters(256, 20, (10, 5, 256, 2, 1), [5, 5, 5, 5]) is None
    assert bench.committed_counters(256, 20, (10, 5, 256, 2, 0), [4, 4, 4, 4, 4]) is None
    # other kernel sources: no record applies
    src.write_bytes(b"changed kernel source")
    assert bench.committed_counters(256, 20, (10, 5, 256, 2, 0), [5, 5, 5, 5]) is None


def test_counter_file_without_records_is_ignored(tmp_path, monkeypatch):
    _fake_repo(tmp_path, [])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_counters(256, 20, (10, 5, 256, 2, 0), [5, 5, 5, 5]) is None
    assert bench.committed_counters(128, 20, (10, 5, 256, 2, 0), [5, 5, 5, 5]) is None  # no file at all


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
