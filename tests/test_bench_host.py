"""Host-side logic of bench.py: the counter ingestion behind roofline.traffic."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, FIELDS)
        w.writeheader()
        w.writerows(rows)


def _runs(tmp_path, tile_read_factor, tile_write_factor, steps=1):
    """Fake FETCH_SIZE / WRITE_SIZE runs: case 0 of each step is a plain copy whose
    counters read 1/2 (fetch) and 1/1 (write) of its bytes; the rest are tiles
    moving the given multiples of their bytes.  A torch kernel is interleaved."""
    cases = bench.dense_cases()
    fr, wr = [], []
    d = 0
    for s in range(steps):
        for i, c in enumerate(cases):
            nb = c[4]
            if i == 0:
                k, rf, wf = "void rr::k_copy<16>(rr::CopyArgs)", 0.5, 1.0
            else:
                k, rf, wf = "void rr::k_tile<4, 4>(rr::TileArgs)", 0.5 * tile_read_factor, tile_write_factor
            d += 1
            fr.append(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name="FETCH_SIZE", Counter_Value=nb * rf / 1024))
            wr.append(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name="WRITE_SIZE", Counter_Value=nb * wf / 1024))
            d += 1
            fr.append(dict(Dispatch_Id=d, Kernel_Name="void at::native::fill(...)", Counter_Name="FETCH_SIZE",
                           Counter_Value=1))
            wr.append(dict(Dispatch_Id=d, Kernel_Name="void at::native::fill(...)", Counter_Name="WRITE_SIZE",
                           Counter_Value=1))
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(f, fr)
    _write(w, wr)
    return str(f), str(w), cases


@pytest.mark.parametrize("steps", [1, 2])
def test_ingest_calibrates_on_plain_copies(tmp_path, steps):
    f, w, cases = _runs(tmp_path, 1.5, 1.25, steps)
    out = tmp_path / "counters.json"
    prof = bench.ingest_counters(f, w, str(out))
    assert json.loads(out.read_text()) == prof
    assert prof["source_hash"] == bench.kernel_source_hash()
    assert prof["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert prof["calibration"]["write_scale"] == pytest.approx(1.0)
    c = prof["kernels"]["k_copy<16>"]
    assert c["launches"] == steps and c["traffic_over_algorithmic"] == pytest.approx(1.0)
    t = prof["kernels"]["k_tile<4,4>"]
    assert t["launches"] == (len(cases) - 1) * steps
    algo = 2 * sum(x[4] for x in cases[1:]) / (len(cases) - 1)
    assert t["algorithmic_bytes_per_launch"] == pytest.approx(algo, rel=1e-9)
    assert t["hbm_bytes_per_launch"] == pytest.approx(algo / 2 * (1.5 + 1.25), rel=1e-6)
    assert t["traffic_over_algorithmic"] == pytest.approx((1.5 + 1.25) / 2, abs=1e-4)


def test_ingest_rejects_mismatched_runs(tmp_path):
    f, w, _ = _runs(tmp_path, 1.0, 1.0)
    rows = list(csv.DictReader(open(w)))[:-3]
    _write(tmp_path / "short.csv", rows)
    with pytest.raises(SystemExit):
        bench.ingest_counters(f, str(tmp_path / "short.csv"), str(tmp_path / "o.json"))


def test_committed_counters_are_plausible():
    """Committed counters taken from the current kernels show each kernel moving
    about its algorithmic bytes."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        pytest.skip("no counters committed")
    prof = json.load(open(path))
    if prof["source_hash"] != bench.kernel_source_hash():
        pytest.skip("counters predate the current kernel sources: bench.py reports traffic as null")
    for k, v in prof["kernels"].items():
        assert 0.99 < v["traffic_over_algorithmic"] < 2.0, (k, v)
