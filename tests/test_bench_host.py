"""bench.py's host logic (no GPU): the single-GPU contract of --gpus, the
counter-to-traffic scaling of the step kernels, and the gate that reports
roofline.traffic only while the step kernels' sources and flags hash to the
value recorded with the counters."""
import csv
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=str(ROOT), timeout=300)
    assert r.returncode != 0
    assert "single MI355X" in (r.stdout + r.stderr)


def _pmc_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": kib})


def test_counters_scaled_by_the_state_restore_copies(tmp_path):
    mixed, fp64 = bench.STATE_BYTES["mixed"], bench.STATE_BYTES["fp64"]
    # a counter that reads half the true bytes (as FETCH_SIZE does) and one that reads them exactly
    for name, f in (("fetch", 0.5), ("write", 1.0)):
        _pmc_csv(tmp_path / (name + ".csv"), [
            ("__amd_rocclr_copyBuffer", f * fp64 / 1024), ("__amd_rocclr_copyBuffer", f * mixed / 1024),
            ("__amd_rocclr_copyBuffer", 10.0),                                   # too small: ignored
            ("void ionic::sdc_kernel<ionic::TT06, ionic::Fp64, 3, 0, 1>(ionic::LaunchArgs)", f * 3e9 / 1024),
            ("void ionic::sdc_kernel<ionic::TT06, ionic::Mixed, 3, 0, 1>(ionic::LaunchArgs)", f * 2e8 / 1024),
            ("void ionic::sdc_kernel<ionic::TT06, ionic::Mixed, 2, 1, 2>(ionic::LaunchArgs)", 1e9),  # ROS2: ignored
            ("void ionic::sdc_kernel<ionic::LR91, ionic::Fp64, 3, 0, 2>(ionic::LaunchArgs)", 1e9),  # LR91: ignored
        ])
    t = bench.traffic_from_counters(tmp_path / "fetch.csv", tmp_path / "write.csv")
    assert t["fp64"]["fetch"] == pytest.approx(3e9) and t["fp64"]["write"] == pytest.approx(3e9)
    assert t["mixed"]["fetch"] == pytest.approx(2e8) and t["mixed"]["write"] == pytest.approx(2e8)
    assert t["mixed"]["fetch_scale"] == pytest.approx(2.0) and t["mixed"]["write_scale"] == pytest.approx(1.0)


def test_traffic_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    good.write_text("source_hash: %s\nmixed_fetch_bytes: 1.0e8\nmixed_write_bytes: 2.0e8\n"
                    % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.read_traffic("mixed") == pytest.approx(3.0e8)
    stale = tmp_path / "stale.txt"
    stale.write_text("source_hash: 0000000000000000\nmixed_fetch_bytes: 1.0e8\nmixed_write_bytes: 2.0e8\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.read_traffic("mixed") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic("mixed") is None


def test_step_kernel_names():
    assert bench.step_kernel_args("void ionic::sdc_kernel<ionic::TT06, ionic::Mixed, 3, 0, 1>(x)") == [
        "ionic::TT06", "ionic::Mixed", "3", "0", "1"]
    assert bench.is_tt06_newton_step("void ionic::sdc_kernel<ionic::TT06, ionic::Fp64, 3, 0>(x)")
    assert not bench.is_tt06_newton_step("void ionic::sdc_kernel<ionic::TT06, ionic::Mixed, 2, 1, 2>(x)")
    assert not bench.is_tt06_newton_step("void ionic::sdc_kernel<ionic::LR91, ionic::Fp64, 3, 0, 2>(x)")
    assert bench.step_kernel_args("ionic::cg_q_kernel(ionic::CgParams)") is None
