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


def test_short_name_of_anonymous_namespace_kernels():
    name = "void heget::(anonymous namespace)::me2_frame_kernel<float, 5>(double const*, long)"
    assert P.short_name(name) == "me2_frame_kernel<float,5>"


def test_issue_summary_relates_valu_issue_to_the_probe(tmp_path):
    """Counters of two passes average per dispatch (largest launch only) and
    the VALU issue of a kernel is read relative to the FMA probe's."""
    probe = "void heget::fma_peak_kernel<float>(float*, float, float, int)"
    rows = [  # pass A
        (probe, 1 << 20, "SQ_ACTIVE_INST_VALU", 800.0), (probe, 1 << 20, "SQ_BUSY_CYCLES", 100.0),
        (KERNEL, 1 << 20, "SQ_ACTIVE_INST_VALU", 600.0), (KERNEL, 1 << 20, "SQ_BUSY_CYCLES", 100.0),
        (KERNEL, 1 << 20, "SQ_INSTS_VALU", 4000.0), (KERNEL, 1 << 20, "SQ_WAVES", 10.0),
        (KERNEL, 1 << 20, "SQ_WAVE_CYCLES", 1000.0), (KERNEL, 1 << 20, "SQ_WAIT_INST_ANY", 50.0),
        (KERNEL, 1 << 18, "SQ_INSTS_VALU", 1.0),  # a smaller launch: ignored
        (CALIB, 1 << 24, "SQ_WAVES", 5.0),         # not a kernel of the path: ignored
    ]
    for name, data in (("a", rows), ("b", [(KERNEL, 1 << 20, "SQ_WAIT_ANY", 120.0),
                                           (KERNEL, 1 << 20, "SQ_WAVE_CYCLES", 1000.0)])):
        os.makedirs(tmp_path / name)
        with open(tmp_path / name / "run_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=FIELDS)
            w.writeheader()
            for i, (k, g, c, v) in enumerate(data):
                w.writerow(dict(Dispatch_Id=i, Kernel_Name=k, Grid_Size=g, Counter_Name=c, Counter_Value=v))
    st = P.issue([str(tmp_path / "a"), str(tmp_path / "b")])
    assert set(st) == {"fma_peak_kernel<float>", "me2_kernel<float,4,4,16,2,1>"}
    k = st["me2_kernel<float,4,4,16,2,1>"]
    assert k["SQ_INSTS_VALU"] == 4000.0 and k["SQ_WAIT_ANY"] == 120.0
    md = P.issue_markdown(st, "cmd", "title")
    row = next(l for l in md.splitlines() if l.startswith("| `me2_kernel"))
    assert "| 400 | 75.0% | 5.0% | 12.0% |" in row  # 4000/10 per wave, (600/100)/(800/100)
