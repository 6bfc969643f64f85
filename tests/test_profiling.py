"""Host-side parsing of rocprofv3 counter output (no GPU): copy calibration,
per-launch HBM bytes, and the staleness check on the source digest."""
from __future__ import annotations

import csv
import os

from paper_0908_4403_amd import profiling as P

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
KERNEL = "void heget::me2_kernel<float, 4, 4, 16, 2, 1>(double const*, long, int const*)"
CALIB = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>(int)"


def write_csv(path, counter, kernel_kib, calib_kib):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        w.writerow(dict(Dispatch_Id=1, Kernel_Name=CALIB, Grid_Size=1 << 24, Counter_Name=counter,
                        Counter_Value=calib_kib))
        # autotune-sized launch (smaller grid) is ignored; the two full launches average
        w.writerow(dict(Dispatch_Id=2, Kernel_Name=KERNEL, Grid_Size=1 << 18, Counter_Name=counter,
                        Counter_Value=1.0))
        for d, v in ((3, kernel_kib - 10), (4, kernel_kib + 10)):
            w.writerow(dict(Dispatch_Id=d, Kernel_Name=KERNEL, Grid_Size=1 << 20, Counter_Name=counter,
                            Counter_Value=v))


def test_short_name():
    assert P.short_name(KERNEL) == "me2_kernel<float,4,4,16,2,1>"


def test_traffic_is_copy_calibrated(tmp_path):
    mib = P.CALIB_BYTES / 1024.0  # the copy moves CALIB_BYTES each way, in KiB
    write_csv(str(tmp_path / "f"), "FETCH_SIZE", 1000.0, 1.25 * mib)   # counter over-reads by 25%
    write_csv(str(tmp_path / "w"), "WRITE_SIZE", 500.0, 0.5 * mib)     # under-reads by half
    t = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "me2_kernel<float,4,4,16,2,1>")
    assert t["fetch"]["launches"] == 2 and t["fetch"]["grid"] == 1 << 20
    assert abs(t["fetch"]["bytes_per_launch"] - 1000.0 * 1024 / 1.25) < 1e-6
    assert abs(t["write"]["bytes_per_launch"] - 500.0 * 1024 / 0.5) < 1e-6
    assert abs(t["bytes_per_launch"] - (819200.0 + 1024000.0)) < 1e-6


def test_read_traffic_checks_kernel_and_sources(tmp_path):
    mib = P.CALIB_BYTES / 1024.0
    write_csv(str(tmp_path / "f"), "FETCH_SIZE", 1000.0, mib)
    write_csv(str(tmp_path / "w"), "WRITE_SIZE", 500.0, mib)
    k = "me2_kernel<float,4,4,16,2,1>"
    t = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), k)
    md = tmp_path / "s.md"
    md.write_text(P.traffic_markdown(k, t, "cmd", "title"))
    assert P.read_traffic(str(md), k) == float("%.6e" % (1500.0 * 1024))
    assert P.read_traffic(str(md), "me2_kernel<float,4,4,16,2,4>") is None
    md.write_text(md.read_text().replace(P.source_digest(), "0" * 16))
    assert P.read_traffic(str(md), k) is None
    assert P.read_traffic(str(tmp_path / "missing.md"), k) is None
