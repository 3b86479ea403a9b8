"""The rocprofv3 summary tool: counter calibration and per-kernel averages on
small synthetic CSV files (no GPU)."""
import csv

from paper_1708_01613_amd import profsum


def _counters(path, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(cols)
        for r in rows:
            w.writerow(r)


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    gib = 1 << 30
    # a 1 GiB copy reads FETCH_SIZE = half its bytes (two dispatches), a small
    # copy with a smaller grid is ignored; the kernel reads 3 and 5 KiB
    _counters(fd / "run_counter_collection.csv", [
        (1, "__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", gib / 2 / 1024),
        (2, "__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", gib / 2 / 1024),
        (3, "__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", 1.0),
        (4, "void flb::k_step<X>(args)", 4096, "FETCH_SIZE", 3.0),
        (5, "void flb::k_step<X>(args)", 4096, "FETCH_SIZE", 5.0),
    ])
    _counters(wd / "run_counter_collection.csv", [
        (1, "__amd_rocclr_copyBuffer", 131072, "WRITE_SIZE", gib / 1024),
        (4, "void flb::k_step<X>(args)", 4096, "WRITE_SIZE", 2.0),
    ])
    out = profsum.traffic(str(fd), str(wd), "void flb::k_step<X>", gib, 1024)
    vals = dict(line[2:].split(": ", 1) for line in out.splitlines() if line.startswith("- "))
    assert float(vals["hbm_read_bytes_per_launch"]) == 2 * 4 * 1024  # mean 4 KiB, scaled by 2
    assert float(vals["hbm_write_bytes_per_launch"]) == 2 * 1024
    assert float(vals["hbm_bytes_per_launch"]) == 10 * 1024
    assert vals["hbm_bytes_per_update"].startswith("10.00")


def test_stats_table_orders_by_total_time(tmp_path):
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"])
        w.writerow(["small", 10, 1000, 100, 90, 110, 10.0])
        w.writerow(["big", 2, 9000, 4500, 4000, 5000, 90.0])
    lines = profsum.stats(str(tmp_path), 5).splitlines()
    assert lines[2].startswith("| `big` | 2 | 4.5 |") and lines[3].startswith("| `small` | 10 | 0.1 |")


def test_traffic_calibrates_on_the_library_copy_kernel(tmp_path):
    # with k_copy16 dispatches present they calibrate (every one copies the
    # full size), whatever other copies the program made
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    gib = 1 << 30
    name = "void flb::k_copy16<4>(float __vector(4) const*, float __vector(4)*, long long)"
    _counters(fd / "run_counter_collection.csv", [
        (1, name, 8192 * 256, "FETCH_SIZE", gib / 1024),
        (2, name, 32768 * 256, "FETCH_SIZE", gib / 1024),
        (3, "__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", 7.0),
        (4, "void flb::k_step<X>(args)", 4096, "FETCH_SIZE", 6.0),
    ])
    _counters(wd / "run_counter_collection.csv", [
        (1, name, 8192 * 256, "WRITE_SIZE", gib / 2 / 1024),
        (4, "void flb::k_step<X>(args)", 4096, "WRITE_SIZE", 2.0),
    ])
    out = profsum.traffic(str(fd), str(wd), "void flb::k_step<X>", gib, 0)
    vals = dict(line[2:].split(": ", 1) for line in out.splitlines() if line.startswith("- "))
    assert float(vals["hbm_read_bytes_per_launch"]) == 6 * 1024
    assert float(vals["hbm_write_bytes_per_launch"]) == 2 * 2 * 1024
