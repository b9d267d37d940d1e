"""The rocprofv3 summary tools that feed the bench's roofline record:
kernel names normalised as the bench looks them up, per-dispatch counter
means, the copy-kernel calibration of FETCH_SIZE / WRITE_SIZE, and the
source-hash guard that drops traffic measured on other kernel code."""
import csv

from paper_2606_06617_amd import profiling

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
       "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
       "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for i, (name, val) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 64, 7, name, 64, 0, 0, 8, 0, 16, counter, val, 0, 1])


def test_short_names():
    assert profiling.short_name("void pswf::k_spread<8, 4>(pswf::Geo, pswf::Tables, pswf::Work, int, int)") \
        == "k_spread<8,4>"
    assert profiling.short_name("pswf::k_zero_int(int*, int)") == "k_zero_int"


def test_kernel_stats(tmp_path):
    p = tmp_path / "s.csv"
    p.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
                 '"void pswf::k_gather<8>(pswf::Geo)",4,4000000,1000000.0,50.0,900000,1100000,1.0\n')
    r = profiling.kernel_stats(str(p))
    assert r[0]["kernel"] == "k_gather<8>" and r[0]["calls"] == 4
    assert abs(r[0]["avg_us"] - 1000.0) < 1e-9 and abs(r[0]["total_ms"] - 4.0) < 1e-12


def test_traffic_calibration_and_hash_guard(tmp_path):
    copy = profiling.COPY_KERNEL
    # the copy of 2 MiB reads 1 MiB and writes 1 MiB; the counters read half
    # of the bytes for fetch and all of them for write
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 512.0), ("pswf::k_zfwd(int)", 100.0),
                                                 ("pswf::k_zfwd(int)", 300.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 1024.0), ("pswf::k_zfwd(int)", 50.0),
                                                 ("pswf::k_zfwd(int)", 50.0)])
    tr, ff, fw = profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 2 << 20)
    assert abs(ff - 2.0) < 1e-12 and abs(fw - 1.0) < 1e-12
    z = tr["k_zfwd"]
    assert abs(z["fetch_bytes"] - 200.0 * 1024 * 2) < 1e-6     # mean of 100 and 300 KiB, x2
    assert abs(z["write_bytes"] - 50.0 * 1024) < 1e-6
    out = tmp_path / "t.txt"
    profiling.write_traffic(tr, ff, fw, 2 << 20, str(out), "cmd")
    rows, sha = profiling.read_traffic(str(out))
    assert sha == profiling.source_hash()
    assert abs(rows["k_zfwd"] - z["bytes"]) < 1.0
    assert profiling.read_traffic(str(tmp_path / "missing.txt")) == (None, None)
