"""Host logic of the counter-based traffic summary (paper_0911_4498_amd/pmc_traffic.py)."""
import csv

import pytest

from paper_0911_4498_amd import pmc_traffic


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, v) in enumerate(rows):
            w.writerow([i, i, k, counter, v])


def test_summary_scales_by_the_copy(tmp_path):
    copy = "at::native::vectorized_elementwise_kernel<neg_kernel>"
    kern = "ssa::k_pass2_matvec<4>(ssa::ConvGeom, ...)"
    # the counters read the 256 MiB copy as 0.5x / 2x its size; the kernel's reads scale alike
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 131072.0), (kern, 100.0), (kern, 300.0), ("other", 5.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 524288.0), (kern, 400.0), (kern, 400.0)])
    s = pmc_traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_pass2_matvec")
    assert s["copy_fetch_factor"] == pytest.approx(2.0)
    assert s["copy_write_factor"] == pytest.approx(0.5)
    assert s["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert s["write_bytes_per_launch"] == pytest.approx(400.0 * 1024 * 0.5)
    assert s["traffic_bytes_per_launch"] == pytest.approx(200.0 * 2048 + 400.0 * 512)
    out = tmp_path / "sum.txt"
    pmc_traffic.write_summary(str(out), s, "rocprofv3 ...", "test")
    back = pmc_traffic.load_summary(str(out))
    assert back["kernel"] == "k_pass2_matvec"
    assert back["traffic_bytes_per_launch"] == pytest.approx(s["traffic_bytes_per_launch"])
    assert back["source_sha256"] == pmc_traffic.source_hash()


def test_summary_needs_the_copy(tmp_path):
    _write(tmp_path / "f.csv", "FETCH_SIZE", [("k", 1.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [("k", 1.0)])
    with pytest.raises(ValueError):
        pmc_traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k")


def test_idle_dispatches_can_be_skipped(tmp_path):
    """Gated launches that return at once count only with skip_idle off."""
    copy = "neg_kernel"
    kern = "ssa::k_cgs_project(ssa::ReduceArgs)"
    _write(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 131072.0), (kern, 1000.0), (kern, 0.1), (kern, 3000.0), (kern, 0.0)])
    _write(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 262144.0), (kern, 50.0), (kern, 0.0), (kern, 50.0), (kern, 0.0)])
    s = pmc_traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_cgs_project", skip_idle=True)
    assert s["idle_dispatches_skipped"] == 2 and s["dispatches_fetch"] == 2
    assert s["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    s_all = pmc_traffic.summarize(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_cgs_project")
    assert s_all["dispatches_fetch"] == 4 and s_all["fetch_bytes_per_launch"] < s["fetch_bytes_per_launch"]
