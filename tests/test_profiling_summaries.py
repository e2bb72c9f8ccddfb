"""Host-side checks of the rocprofv3 summaries (paper_2604_11659_amd/profiling.py) on synthetic CSVs."""
import csv

from paper_2604_11659_amd import profiling as pf


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_busy_union_bins_and_gaps(tmp_path):
    p = tmp_path / "x_kernel_trace.csv"
    # two overlapping kernels, a 60 ms gap, two back-to-back kernels
    _write(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["a", 0, 40_000_000], ["b", 30_000_000, 90_000_000], ["c", 150_000_000, 160_000_000],
            ["d", 160_000_000, 260_000_000]])
    merged = pf.busy_intervals(str(p))
    assert merged == [[0, 90_000_000], [150_000_000, 260_000_000]]
    assert [round(b, 6) for b in pf.busy_bins(merged, 100e6)] == [0.9, 0.5, 0.6]
    text = pf.busy_markdown(str(p), "T", "cmd", gap_ms=5.0)
    # every bin is at least half busy: the compute phase is the whole trace, gap included
    assert "0.090 s: 60.0 ms" in text and "(0.769)" in text and "0.0-0.3 s" in text
    assert "* none" in pf.busy_markdown(str(p), "T", "cmd", gap_ms=100.0)
    # with a higher threshold the phase is the first bin only, which holds no gap
    t2 = pf.busy_markdown(str(p), "T", "cmd", gap_ms=5.0, active=0.8)
    assert "0.0-0.1 s" in t2 and "* none" in t2


def test_traffic_scaled_by_the_copy_kernel(tmp_path):
    """Counter KiB per dispatch scaled so the 1 GiB copy-like kernel reads and writes 1 GiB."""
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the calibration kernel under-reports FETCH_SIZE by 2x; the kernel of interest has two dispatches
    _write(f, hdr, [["bitwise_not", "FETCH_SIZE", 512 * 1024], ["k_inner<A>", "FETCH_SIZE", 100.0],
                    ["k_inner<A>", "FETCH_SIZE", 300.0], ["other", "FETCH_SIZE", 9e9]])
    _write(w, hdr, [["bitwise_not", "WRITE_SIZE", 1024 * 1024], ["k_inner<A>", "WRITE_SIZE", 50.0],
                    ["k_inner<A>", "WRITE_SIZE", 50.0]])
    t = pf.traffic(str(f), str(w), r"k_inner", "bitwise", float(1 << 30))
    assert t["dispatches"] == 2
    assert abs(t["fetch_scale"] - 2.0) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    assert abs(t["fetch_bytes_per_launch"] - 200.0 * 1024 * 2.0) < 1e-6
    assert abs(t["bytes_per_launch"] - (200.0 * 1024 * 2.0 + 50.0 * 1024)) < 1e-6


def test_traffic_block_only_for_the_current_kernel_source(tmp_path):
    """A traffic summary is used only while kernels.hip has the SHA-256 it was measured on."""
    t = {"dispatches": 1, "fetch_bytes_per_launch": 1.0, "write_bytes_per_launch": 2.0, "bytes_per_launch": 3.0,
         "fetch_scale": 2.0, "write_scale": 1.0, "raw_fetch_kib_per_launch": 0.5, "raw_write_kib_per_launch": 2.0}
    (tmp_path / "a_traffic.md").write_text(pf.traffic_markdown(t, "inner", "T", "cmd"))
    got = pf.load_traffic(str(tmp_path), "inner")
    assert got is not None and got["bytes_per_launch"] == 3.0 and got["file"] == "a_traffic.md"
    assert pf.load_traffic(str(tmp_path), "other") is None
    stale = (tmp_path / "a_traffic.md").read_text().replace(pf.kernel_source_sha256(), "0" * 64)
    (tmp_path / "a_traffic.md").write_text(stale)
    assert pf.load_traffic(str(tmp_path), "inner") is None
